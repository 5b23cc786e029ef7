"""Parity of the grid consumers (density at points, selection by a density
threshold, Marching Cubes cell classification) through the C ABI against the
oracle, on seeded synthetic grids and points. Both sides evaluate the
interpolation in double in the same operation order, so sampled densities,
selections and cell cases are compared for exact equality.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import Roi

from gpu_common import ctx, dev, say, sfk, torch  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = [
    (Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (2, 2, 2)), 1000, 1),
    (Roi((0.1, -0.3, 0.25), (0.9, 0.55, 1.4), (37, 29, 23)), 20000, 2),
    (Roi((-2.0, 1.0, 0.0), (3.0, 1.5, 0.125), (64, 17, 9)), 20000, 3),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sample_select_iso_exact(ctx, torch, case):
    roi, n, seed = CASES[case]
    grid = synth.random_grid(roi.res, seed)
    pts = synth.probe_points(roi, n, seed + 100)
    g_d, p_d = dev(torch, grid), dev(torch, pts)
    say("case", case, roi.res, "points", len(pts))
    got = ctx.sample_density(roi, g_d, p_d).cpu().numpy()
    ref = oracle.sample_density(grid, roi, pts).astype(np.float32)
    assert np.array_equal(got, ref), np.max(np.abs(got - ref))
    inside = ref > 0
    for q in (0.1, 0.5, 0.9):
        iso = float(np.quantile(ref[inside], q))
        sel = ctx.select_points(roi, g_d, iso, p_d).cpu().numpy()
        assert np.array_equal(sel, oracle.select_points(grid, roi, iso, pts)), (case, q)
        cells, cases = ctx.iso_cells(roi, g_d, iso)
        rc, rk = oracle.iso_cells(grid, roi, iso)
        assert np.array_equal(cells.cpu().numpy(), rc) and np.array_equal(cases.cpu().numpy(), rk)
    # a threshold equal to a point's own density selects it (>=)
    one = pts[-roi.res[0]:][roi.res[0] // 2:roi.res[0] // 2 + 1]
    v = float(oracle.sample_density(grid, roi, one)[0])
    assert v > 0.0
    sel = ctx.select_points(roi, g_d, v, dev(torch, one)).cpu().numpy()
    assert list(sel) == list(oracle.select_points(grid, roi, v, one)) == [0]
    sel = ctx.select_points(roi, g_d, float(np.nextafter(v, 10.0)), dev(torch, one)).cpu().numpy()
    assert list(sel) == []


def test_edge_cases(ctx, torch):
    roi = Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (5, 4, 3))
    grid = synth.random_grid(roi.res, 7)
    g_d = dev(torch, grid)
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    assert ctx.sample_density(roi, g_d, empty).numel() == 0
    assert ctx.select_points(roi, g_d, 1.0, empty).numel() == 0
    # non-finite coordinates are outside every box
    bad = np.array([[np.nan, 0.5, 0.5], [0.5, np.inf, 0.5], [0.5, 0.5, 0.5]], np.float32)
    got = ctx.sample_density(roi, g_d, dev(torch, bad)).cpu().numpy()
    assert got[0] == 0 and got[1] == 0 and got[2] == np.float32(oracle.sample_density(grid, roi, bad)[2])
    # thresholds outside the field's range: no active cell
    assert ctx.iso_cells(roi, g_d, -1.0)[0].numel() == 0
    assert ctx.iso_cells(roi, g_d, 10.0)[0].numel() == 0
    # a capacity smaller than the count: the full count, the first cap indices
    pts = synth.probe_points(roi, 5000, 8)
    p_d = dev(torch, pts)
    ref = oracle.select_points(grid, roi, 1.0, pts)
    idx = torch.full((10,), -7, dtype=torch.int64, device="cuda")
    import ctypes as C
    import paper_2601_20758_amd as sfk_mod
    import paper_2601_20758_amd._lib as L
    cnt = C.c_int64()
    r = sfk_mod.roi_struct(roi, 0)
    st = L.lib().sfk_select_points(ctx._h, C.byref(r), g_d.data_ptr(), 1.0, p_d.data_ptr(),
                                   len(pts), idx.data_ptr(), 10, C.byref(cnt), None)
    assert st == 0 and cnt.value == len(ref) and np.array_equal(idx.cpu().numpy(), ref[:10])
    # invalid geometry is rejected
    with pytest.raises(sfk_mod.SfkError):
        ctx.sample_density(Roi((0.0, 0.0, 0.0), (0.0, 1.0, 1.0), (5, 4, 3)), g_d, p_d)


def test_full_size(ctx, torch):
    """A 256^3 field (16.8M nodes) sampled at 10M points: every value, the
    selection at two thresholds and the active cells, exactly."""
    roi = Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (256, 256, 256))
    grid = synth.random_grid(roi.res, 9)
    pts = synth.probe_points(roi, 10_000_000, 10, margin=0.02)
    g_d, p_d = dev(torch, grid), dev(torch, pts)
    say("sampling 10M points on a 256^3 field")
    got = ctx.sample_density(roi, g_d, p_d).cpu().numpy()
    ref = oracle.sample_density(grid, roi, pts)
    assert np.array_equal(got, ref.astype(np.float32))
    for iso in (1.0, 2.5):
        say("selection and iso cells at", iso)
        sel = ctx.select_points(roi, g_d, iso, p_d).cpu().numpy()
        assert np.array_equal(sel, oracle.select_points(grid, roi, iso, pts))
        cells, cases = ctx.iso_cells(roi, g_d, iso)
        rc, rk = oracle.iso_cells(grid, roi, iso)
        assert np.array_equal(cells.cpu().numpy(), rc) and np.array_equal(cases.cpu().numpy(), rk)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_iso_surface_exact(ctx, torch, case):
    # every triangle vertex equal to the oracle's (same case table, same
    # double interpolation), in the same order
    roi, _, seed = CASES[case]
    grid = synth.random_grid(roi.res, seed)
    g_d = dev(torch, grid)
    for q in (0.2, 0.5, 0.8):
        iso = float(np.quantile(grid, q))
        got = ctx.iso_surface(roi, g_d, iso).cpu().numpy()
        ref = oracle.iso_surface(grid, roi, iso)
        assert got.shape == ref.shape, (case, q, got.shape, ref.shape)
        assert np.array_equal(got, ref), (case, q)
    # a capacity below the count writes a prefix and still reports the count
    iso = float(np.quantile(grid, 0.5))
    full = oracle.iso_surface(grid, roi, iso)
    if len(full) > 3:
        part = ctx.iso_surface(roi, g_d, iso, cap=3).cpu().numpy()
        assert np.array_equal(part, full[:3])


def test_iso_surface_of_density_grid(ctx, torch):
    # the selection volume of an evaluated density field (C1 cloud, 48^3):
    # the surface at a tenth of the peak, exact against the oracle on the
    # GPU's grid, closed (every edge used once in each direction)
    pts = synth.c1_cloud(1)
    roi = Roi((0, 0, 0), (1, 1, 1), (48, 48, 48), kernel="epanechnikov", bw="fixed",
              h=(0.04, 0.04, 0.04))
    tree = ctx.build_tree(dev(torch, pts))
    g = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    gh = g.cpu().numpy()
    iso = 0.1 * float(gh.max())
    got = ctx.iso_surface(roi, g, iso).cpu().numpy()
    ref = oracle.iso_surface(gh, roi, iso)
    assert len(got) > 1000 and np.array_equal(got, ref)
    # outward normals: the enclosed volume is positive
    t = got.astype(np.float64)
    vol = np.einsum("ij,ij->i", t[:, 0], np.cross(t[:, 1], t[:, 2])).sum() / 6.0
    assert vol > 0
    tree.close()
