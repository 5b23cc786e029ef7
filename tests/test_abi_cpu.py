"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and rejects bad arguments before touching
a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfkde.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfk_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2601_20758_amd import _lib
    return _lib.lib()


def test_header_declares_expected_entry_points():
    names = _declared()
    for required in ["sfk_ctx_create", "sfk_ctx_destroy", "sfk_build_tree", "sfk_tree_info",
                     "sfk_tree_destroy", "sfk_eval_roi", "sfk_submit", "sfk_poll", "sfk_wait",
                     "sfk_cancel", "sfk_status_string", "sfk_last_error",
                     "sfk_debug_candidates", "sfk_debug_point_h2", "sfk_debug_eval_count",
                     "sfk_debug_mbe", "sfk_serve", "sfk_autotune"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_declares_every_export():
    from paper_2601_20758_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_status_strings(lib):
    for code in range(9):
        assert lib.sfk_status_string(code)
    assert lib.sfk_status_string(0) == b"ok"
    assert b"gfx950" in lib.sfk_version()


def test_null_arguments_rejected(lib):
    from paper_2601_20758_amd import _lib
    # NULL out pointer
    assert lib.sfk_ctx_create(0, None, 0, None) == 1
    assert lib.sfk_last_error(None)
    # NULL context everywhere
    assert lib.sfk_build_tree(None, None, 0, None, None, None, None) == 1
    assert lib.sfk_eval_roi(None, None, None, None) == 1
    t = C.c_int64()
    assert lib.sfk_submit(None, None, None, 0, C.byref(t)) == 1
    d = C.c_int32()
    assert lib.sfk_poll(None, 1, C.byref(d)) == 1
    assert lib.sfk_tree_info(None, None, None, None) == 1
    assert lib.sfk_ctx_destroy(None) == 0
    assert lib.sfk_tree_destroy(None) == 0
    # allocator with a missing callback
    a = _lib.Allocator()
    h = C.c_void_p()
    assert lib.sfk_ctx_create(0, C.byref(a), 0, C.byref(h)) == 1


def test_no_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = lib.sfk_ctx_create(0, None, 0, C.byref(h))
    assert st == 4 and not h.value
    assert b"device" in lib.sfk_last_error(None)


def test_roi_marshalling():
    import synth
    from paper_2601_20758_amd import roi_struct
    r = roi_struct(synth.c2_roi(), 1234)
    assert (r.kernel, r.bw, r.norm, r.set) == (1, 2, 0, 0)
    assert list(r.res) == [128, 128, 128] and r.d_out == 1234
    with pytest.raises(ValueError):
        roi_struct(synth.c1_roi().replace(kernel="triangle"), 1)


def test_marching_cubes_table_matches_oracle(lib):
    # the library's case table (the one its kernels use, read on the host)
    # against the oracle's own derivation of the same rule, all 256 cases
    import ctypes as C
    import numpy as np
    import oracle
    buf = (C.c_int8 * 15)()
    n = C.c_int32()
    for cs in range(256):
        assert lib.sfk_debug_mc_case(cs, buf, C.byref(n)) == 0
        got = np.array(buf[:3 * n.value], dtype=np.int32).reshape(-1, 3)
        assert np.array_equal(got, oracle.mc_case(cs)), cs
    assert lib.sfk_debug_mc_case(256, buf, C.byref(n)) == 1


def test_header_constants_match_the_binding():
    text = open(HEADER).read()
    from paper_2601_20758_amd import _lib
    m = re.search(r"#define SFK_NUM_TILE_SHAPES (\d+)", text)
    assert m and int(m.group(1)) == _lib.NUM_TILE_SHAPES
    m = re.search(r"#define SFK_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and (int(m.group(1)) << int(m.group(2))) == _lib.NOALLOC_SCRATCH_BYTES
