"""MI355X (gfx950) ROI kernel density estimation: Python binding of libsfkde.

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of libsfkde.so. PyTorch supplies device memory (optionally through
its caching allocator) and streams. The names follow the C ABI in
include/sfkde.h (sfk_build_tree -> Context.build_tree, ...).
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from typing import Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import NOALLOC_SCRATCH_BYTES, NUM_TILE_SHAPES

__all__ = ["SfkError", "Context", "Tree", "curve_keys", "roi_struct", "version",
           "NOALLOC_SCRATCH_BYTES", "NUM_TILE_SHAPES"]


class SfkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (L.STATUS.get(status, status), msg))
        self.status = status
        self.name = L.STATUS.get(status, str(status))


def version() -> str:
    return L.lib().sfk_version().decode()


def curve_keys(curve, bits: int, cells) -> np.ndarray:
    """sfk_debug_curve_keys (host only): the tree build's sort key of each
    (x, y, z) lattice cell of an (n, 3) integer array, 2^bits cells per axis."""
    c = np.ascontiguousarray(cells, dtype=np.uint32).reshape(-1, 3)
    out = np.zeros(max(len(c), 1), dtype=np.uint64)
    st = L.lib().sfk_debug_curve_keys(_enum(L.CURVES, curve, "curve"), int(bits),
                                      c.ctypes.data, len(c), out.ctypes.data)
    if st != 0:
        raise SfkError(st, L.lib().sfk_last_error(None).decode())
    return out[:len(c)]


def _enum(table, v, what):
    if isinstance(v, str):
        if v not in table:
            raise ValueError("unknown %s %r" % (what, v))
        return table[v]
    return int(v)


def roi_struct(roi, d_out: int) -> L.RoiC:
    """Marshal an ROI description (fields lo, hi, res, kernel, bw, norm, set,
    h, tag) and a device output pointer into the C descriptor."""
    r = L.RoiC()
    for k in range(3):
        r.lo[k] = float(roi.lo[k])
        r.hi[k] = float(roi.hi[k])
        r.res[k] = int(roi.res[k])
        r.h[k] = float(roi.h[k]) if roi.h is not None else 0.0
    r.kernel = _enum(L.KERNEL, roi.kernel, "kernel")
    r.bw = _enum(L.BW, roi.bw, "bandwidth mode")
    r.norm = _enum(L.NORM, roi.norm, "norm")
    r.set = _enum(L.SET, roi.set, "set")
    r.d_out = d_out
    r.tag = int(getattr(roi, "tag", 0) or 0)
    return r


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """sfk_ctx_create / sfk_ctx_destroy. allocator: "torch" routes device
    memory through torch's caching allocator, "hip" uses hipMalloc."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, allocator: str = "torch"):
        self._lib = L.lib()
        self._h = C.c_void_p()
        self._trees = weakref.WeakSet()
        self._views = weakref.WeakSet()
        self.device = device
        self._alloc = None
        # tests: while True, the allocator callback returns NULL (as when the
        # device is out of memory), which the library reports as SFK_E_NOMEM
        self.fail_allocations = False
        ap = None
        if allocator == "torch":
            import torch

            alloc_fn = torch.cuda.caching_allocator_alloc
            free_fn = torch.cuda.caching_allocator_delete

            def _a(nbytes, user):
                if self.fail_allocations:
                    return None
                try:
                    return alloc_fn(int(nbytes), device)
                except Exception:  # out of memory -> NULL -> SFK_E_NOMEM
                    return None

            def _f(ptr, nbytes, user):
                try:
                    free_fn(ptr)
                except Exception:  # interpreter shutdown: the process frees it
                    pass

            self._alloc = L.Allocator(L.Allocator.ALLOC(_a), L.Allocator.FREE(_f), None)
            ap = C.byref(self._alloc)
        elif allocator != "hip":
            raise ValueError("allocator must be 'torch' or 'hip'")
        st = self._lib.sfk_ctx_create(device, ap, int(budget_bytes), C.byref(self._h))
        if st != L.SFK_OK:
            raise SfkError(st, self._lib.sfk_last_error(None).decode())
        # release device memory while torch is still alive
        atexit.register(self.close)

    # -- helpers
    def _check(self, st):
        if st != L.SFK_OK:
            raise SfkError(st, self.last_error())

    def last_error(self) -> str:
        return self._lib.sfk_last_error(self._h).decode()

    def close(self):
        for v in list(self._views):
            v.close()
        for t in list(self._trees):
            t.close()
        if self._h:
            self._lib.sfk_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- tree
    def build_tree(self, xyz, knn_k: int = 0, h=None, key_bits: int = 0,
                   curve: str = "hilbert", stream=None) -> "Tree":
        """sfk_build_tree on an (n, 3) float32 device tensor (and an optional
        per-particle bandwidth tensor h of n floats); curve is "hilbert" or
        "morton"."""
        import torch
        if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.float32):
            raise TypeError("xyz must be a float32 device tensor")
        if xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
            raise ValueError("xyz must be a contiguous (n, 3) tensor")
        hp = None
        if h is not None:
            if not (h.is_cuda and h.dtype == torch.float32 and h.is_contiguous()
                    and h.numel() == xyz.shape[0]):
                raise ValueError("h must be n contiguous float32 device values")
            hp = h.data_ptr()
        opts = L.TreeOpts(0, int(knn_k), int(key_bits), _enum(L.CURVES, curve, "curve"))
        out = C.c_void_p()
        self._check(self._lib.sfk_build_tree(self._h, xyz.data_ptr() if xyz.numel() else None,
                                             int(xyz.shape[0]), hp, C.byref(opts),
                                             _stream_ptr(stream), C.byref(out)))
        t = Tree(self, out)
        self._trees.add(t)
        return t

    # -- evaluation
    def eval_roi(self, tree: "Tree", roi, out=None, stream=None):
        """sfk_eval_roi: stream-ordered evaluation into `out` (allocated if None)."""
        out = self._out_for(roi, out)
        r = roi_struct(roi, out.data_ptr())
        self._check(self._lib.sfk_eval_roi(self._h, tree._h, C.byref(r), _stream_ptr(stream)))
        return out

    def eval_roi_noalloc(self, tree: "Tree", roi, out, stream=None):
        """sfk_eval_roi_noalloc: sfk_eval_roi with the workspace in the
        library's static scratch array (no allocation); `out` is required."""
        out = self._out_for(roi, out)
        r = roi_struct(roi, out.data_ptr())
        self._check(self._lib.sfk_eval_roi_noalloc(self._h, tree._h, C.byref(r),
                                                   _stream_ptr(stream)))
        return out

    def submit(self, tree: "Tree", rois: Sequence, outs: Sequence) -> int:
        """sfk_submit of a batch; outs[i] receives rois[i]."""
        arr = (L.RoiC * len(rois))()
        for i, (roi, o) in enumerate(zip(rois, outs)):
            arr[i] = roi_struct(roi, o.data_ptr())
        t = C.c_int64()
        self._check(self._lib.sfk_submit(self._h, tree._h, arr, len(rois), C.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        self._check(self._lib.sfk_poll(self._h, ticket, C.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, timeout_us: int = -1):
        self._check(self._lib.sfk_wait(self._h, ticket, int(timeout_us)))

    def cancel(self, ticket: int):
        self._check(self._lib.sfk_cancel(self._h, ticket))

    def set_eval_opts(self, tile_shape: int = 0, chunk_leaves: int = 0,
                      persistent_waves_per_cu: int = 0, list_capacity: int = 0,
                      disable_graphs: bool = False, partial_capacity: int = 0):
        o = L.EvalOpts(int(tile_shape), int(chunk_leaves), int(persistent_waves_per_cu),
                       int(list_capacity), 1 if disable_graphs else 0, int(partial_capacity))
        self._check(self._lib.sfk_set_eval_opts(self._h, C.byref(o)))

    def autotune(self, tree: "Tree", rois: Sequence, outs: Sequence):
        arr = (L.RoiC * len(rois))()
        for i, (roi, o) in enumerate(zip(rois, outs)):
            arr[i] = roi_struct(roi, o.data_ptr())
        self._check(self._lib.sfk_autotune(self._h, tree._h, arr, len(rois)))

    def autotune_table(self) -> dict:
        n = C.c_int32()
        self._check(self._lib.sfk_autotune_table(self._h, None, None, 0, C.byref(n)))
        keys = (C.c_int32 * max(1, n.value))()
        shapes = (C.c_int32 * max(1, n.value))()
        self._check(self._lib.sfk_autotune_table(self._h, keys, shapes, n.value, C.byref(n)))
        return {keys[i]: shapes[i] for i in range(n.value)}

    def autotune_costs(self) -> dict:
        """sfk_autotune_costs: key -> [ms of shapes 1..NUM_TILE_SHAPES]."""
        n = C.c_int32()
        self._check(self._lib.sfk_autotune_costs(self._h, None, None, 0, C.byref(n)))
        keys = (C.c_int32 * max(1, n.value))()
        S = NUM_TILE_SHAPES
        ms = (C.c_double * (S * max(1, n.value)))()
        self._check(self._lib.sfk_autotune_costs(self._h, keys, ms, n.value, C.byref(n)))
        return {keys[i]: [ms[S * i + j] for j in range(S)] for i in range(n.value)}

    def autotune_save(self, path: str):
        self._check(self._lib.sfk_autotune_save(self._h, path.encode()))

    def autotune_load(self, path: str):
        self._check(self._lib.sfk_autotune_load(self._h, path.encode()))

    def serve(self, tree: "Tree", arrivals: Sequence[float], rois: Sequence, outs: Sequence,
              mode: int = 0, n_slots: int = 4, max_batch: int = 64, budget_bytes: float = 0.0,
              max_batch_work: float = 0.0, interleave: bool = False):
        """sfk_serve over a request trace; returns (per-request results, summary)."""
        n = len(rois)
        reqs = (L.Request * n)()
        for i in range(n):
            reqs[i].arrival_s = float(arrivals[i])
            reqs[i].roi = roi_struct(rois[i], outs[i].data_ptr())
        opts = L.ServeOpts(int(mode), int(n_slots), int(max_batch), 1 if interleave else 0,
                           float(budget_bytes), float(max_batch_work))
        res = (L.RequestResult * n)()
        summ = L.ServeSummary()
        self._check(self._lib.sfk_serve(self._h, tree._h, reqs, n, C.byref(opts), res,
                                        C.byref(summ)))
        return res, summ

    def _out_for(self, roi, out):
        import torch
        m = int(roi.res[0]) * int(roi.res[1]) * int(roi.res[2])
        if out is None:
            out = torch.empty(m, dtype=torch.float32, device="cuda:%d" % self.device)
        if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
                and out.numel() == m):
            raise ValueError("out must be a contiguous float32 device tensor of %d values" % m)
        return out

    # -- profiling
    def profile_enable(self, on: bool = True):
        self._check(self._lib.sfk_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, reset: bool = False) -> dict:
        pr = L.Profile()
        self._check(self._lib.sfk_profile_read(self._h, C.byref(pr), 1 if reset else 0))
        return {name: getattr(pr, name) for name, _ in L.Profile._fields_}

    # -- test exports
    def debug_candidates(self, tree: "Tree", roi, node_begin: int, node_end: int):
        """Support sets of nodes [node_begin, node_end): (offsets, original indices)."""
        nn = node_end - node_begin
        offs = np.zeros(nn + 1, dtype=np.int64)
        need = C.c_int64()
        r = roi_struct(roi, 1)
        self._check(self._lib.sfk_debug_candidates(self._h, tree._h, C.byref(r), node_begin,
                                                    node_end, offs.ctypes.data, None, 0,
                                                    C.byref(need)))
        idx = np.zeros(max(need.value, 1), dtype=np.int64)
        self._check(self._lib.sfk_debug_candidates(self._h, tree._h, C.byref(r), node_begin,
                                                    node_end, offs.ctypes.data, idx.ctypes.data,
                                                    idx.shape[0], C.byref(need)))
        return offs, idx[:need.value]

    # ---- adaptive resolution ----

    def eval_adaptive(self, tree: "Tree", roi, brick: int = 8, max_level: int = 2,
                      threshold: float = 0.1, cap_floats: int = 1 << 24, cap_bricks: int = 1 << 16,
                      out=None, stream=None):
        """sfk_eval_adaptive: (base grid, brick values, [brick dicts], result dict). Brick i's
        grid is bricks[b['offset'] : b['offset'] + prod(b['res'])], x fastest."""
        import torch
        out = self._out_for(roi, out)
        r = roi_struct(roi, out.data_ptr())
        o = L.AdaptiveOpts(int(brick), int(max_level), float(threshold), 0)
        vals = torch.empty(max(1, int(cap_floats)), dtype=torch.float32, device=out.device)
        hb = (L.Brick * max(1, int(cap_bricks)))()
        res = L.AdaptiveResult()
        self._check(self._lib.sfk_eval_adaptive(self._h, tree._h, C.byref(r), C.byref(o),
                                                vals.data_ptr(), int(cap_floats), hb,
                                                int(cap_bricks), C.byref(res),
                                                _stream_ptr(stream)))
        bricks = [{"level": hb[i].level, "parent": hb[i].parent, "cell0": tuple(hb[i].cell0),
                   "res": tuple(hb[i].res), "lo": tuple(hb[i].lo), "hi": tuple(hb[i].hi),
                   "offset": hb[i].offset} for i in range(res.n_bricks)]
        info = {"n_bricks": res.n_bricks, "levels": res.levels, "complete": bool(res.complete),
                "peak": res.peak, "floats_used": res.floats_used}
        return out, vals[:res.floats_used], bricks, info

    # ---- view cache (recomputation policy, reuse across frames) ----

    def view(self, tree: "Tree", kernel: str = "epanechnikov", bw: str = "fixed", h=(0.01,) * 3,
             res: int = 64, block: int = 32, scale_threshold: float = 1.0, margin: float = 0.0,
             max_blocks: int = 512, norm: str = "paper") -> "View":
        """sfk_view_create: a device-resident block cache over lattices of nodes."""
        hh = tuple(float(x) for x in h) if h is not None else (1.0, 1.0, 1.0)
        if len(hh) == 1:
            hh = hh * 3
        o = L.ViewOpts(L.KERNEL[kernel], L.BW[bw], L.NORM[norm], int(res), (C.c_float * 3)(*hh),
                       int(block), float(scale_threshold), float(margin), int(max_blocks))
        out = C.c_void_p()
        self._check(self._lib.sfk_view_create(self._h, tree._h, C.byref(o), C.byref(out)))
        v = View(self, tree, out, int(block) or 32)
        self._views.add(v)
        return v

    # ---- consumers of a density grid (all on the device) ----

    @staticmethod
    def _grid_args(roi, grid, xyz=None):
        import torch
        if not (isinstance(grid, torch.Tensor) and grid.is_cuda and grid.dtype == torch.float32
                and grid.is_contiguous() and grid.numel() == roi.n_nodes):
            raise ValueError("grid must be a contiguous float32 device tensor of the ROI's nodes")
        if xyz is not None and not (isinstance(xyz, torch.Tensor) and xyz.is_cuda
                                    and xyz.dtype == torch.float32 and xyz.is_contiguous()
                                    and xyz.dim() == 2 and xyz.shape[1] == 3):
            raise ValueError("points must be a contiguous (n, 3) float32 device tensor")

    def sample_density(self, roi, grid, xyz, out=None, stream=None):
        """sfk_sample_density: trilinear density of `grid` (the nodes of `roi`) at each point."""
        import torch
        self._grid_args(roi, grid, xyz)
        n = xyz.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=xyz.device)
        r = roi_struct(roi, 0)
        self._check(self._lib.sfk_sample_density(self._h, C.byref(r), grid.data_ptr(),
                                                 xyz.data_ptr(), n, out.data_ptr(),
                                                 _stream_ptr(stream)))
        return out

    def select_points(self, roi, grid, iso: float, xyz, stream=None):
        """sfk_select_points: ascending int64 indices of the points in the box with density >= iso."""
        import torch
        self._grid_args(roi, grid, xyz)
        n = xyz.shape[0]
        cap = n
        idx = torch.empty(max(1, cap), dtype=torch.int64, device=xyz.device)
        cnt = C.c_int64()
        r = roi_struct(roi, 0)
        self._check(self._lib.sfk_select_points(self._h, C.byref(r), grid.data_ptr(), float(iso),
                                                xyz.data_ptr(), n, idx.data_ptr(), cap,
                                                C.byref(cnt), _stream_ptr(stream)))
        return idx[:cnt.value]

    def iso_cells(self, roi, grid, iso: float, stream=None):
        """sfk_iso_cells: (active cells ascending, their Marching Cubes cases) as device tensors."""
        import torch
        self._grid_args(roi, grid)
        nc = (roi.res[0] - 1) * (roi.res[1] - 1) * (roi.res[2] - 1)
        cells = torch.empty(max(1, nc), dtype=torch.int64, device=grid.device)
        cases = torch.empty(max(1, nc), dtype=torch.uint8, device=grid.device)
        cnt = C.c_int64()
        r = roi_struct(roi, 0)
        self._check(self._lib.sfk_iso_cells(self._h, C.byref(r), grid.data_ptr(), float(iso),
                                            cells.data_ptr(), cases.data_ptr(), nc, C.byref(cnt),
                                            _stream_ptr(stream)))
        return cells[:cnt.value], cases[:cnt.value]

    def iso_surface(self, roi, grid, iso: float, cap: Optional[int] = None, stream=None):
        """sfk_iso_surface: the Marching Cubes triangles as an (n, 3, 3)
        float32 device tensor (a first call counts them when cap is None)."""
        import torch
        self._grid_args(roi, grid)
        cnt = C.c_int64()
        r = roi_struct(roi, 0)
        if cap is None:
            self._check(self._lib.sfk_iso_surface(self._h, C.byref(r), grid.data_ptr(),
                                                  float(iso), None, 0, C.byref(cnt),
                                                  _stream_ptr(stream)))
            cap = cnt.value
        tris = torch.empty((max(1, cap), 3, 3), dtype=torch.float32, device=grid.device)
        self._check(self._lib.sfk_iso_surface(self._h, C.byref(r), grid.data_ptr(), float(iso),
                                              tris.data_ptr(), cap, C.byref(cnt),
                                              _stream_ptr(stream)))
        return tris[:min(cnt.value, cap)]

    def debug_poison(self, bits: int):
        """sfk_debug_poison: test-only out-of-range leaf ids (see the header)."""
        self._check(self._lib.sfk_debug_poison(self._h, int(bits)))

    def debug_tile_leaves(self, tree: "Tree", roi, out=None):
        """sfk_debug_tile_leaves: (tile shape, per-tile leaf counts, the
        concatenated per-tile leaf lists)."""
        out = self._out_for(roi, out)
        r = roi_struct(roi, out.data_ptr())
        nt, tot = C.c_int64(), C.c_int64()
        shape = np.zeros(3, dtype=np.int32)
        self._check(self._lib.sfk_debug_tile_leaves(self._h, tree._h, C.byref(r),
                                                    shape.ctypes.data, None, 0, None, 0,
                                                    C.byref(nt), C.byref(tot)))
        cnt = np.zeros(max(1, nt.value), dtype=np.int64)
        leaves = np.zeros(max(1, tot.value), dtype=np.int32)
        self._check(self._lib.sfk_debug_tile_leaves(self._h, tree._h, C.byref(r),
                                                    shape.ctypes.data, cnt.ctypes.data, nt.value,
                                                    leaves.ctypes.data, tot.value,
                                                    C.byref(nt), C.byref(tot)))
        return tuple(int(v) for v in shape), cnt[:nt.value], leaves[:tot.value]

    def debug_leaf_boxes(self, tree: "Tree") -> np.ndarray:
        """sfk_debug_leaf_boxes: (n_leaves, 6) float32 (lo xyz, hi xyz)."""
        n_leaves = (tree.info()[0] + 63) // 64
        b = np.zeros((max(1, n_leaves), 6), dtype=np.float32)
        self._check(self._lib.sfk_debug_leaf_boxes(self._h, tree._h, b.ctypes.data))
        return b[:n_leaves]

    def debug_point_h2(self, tree: "Tree") -> np.ndarray:
        n = tree.info()[0]
        out = np.zeros(max(n, 1), dtype=np.float32)
        self._check(self._lib.sfk_debug_point_h2(self._h, tree._h, out.ctypes.data))
        return out[:n]

    def debug_tree_order(self, tree: "Tree") -> np.ndarray:
        """Original index of each particle in the tree's leaf order."""
        n = tree.info()[0]
        out = np.zeros(max(n, 1), dtype=np.int32)
        self._check(self._lib.sfk_debug_tree_order(self._h, tree._h, out.ctypes.data))
        return out[:n]

    def debug_particle_estimate(self, tree: "Tree", lo, hi) -> float:
        """sfk_debug_particle_estimate: the tree's particle estimate for the
        closed box [lo, hi]."""
        a = np.ascontiguousarray(lo, dtype=np.float64)
        b = np.ascontiguousarray(hi, dtype=np.float64)
        out = C.c_double()
        self._check(self._lib.sfk_debug_particle_estimate(self._h, tree._h, a.ctypes.data,
                                                          b.ctypes.data, C.byref(out)))
        return out.value

    def debug_eval_count(self, tree: "Tree", roi):
        u = C.c_int64()
        t = C.c_int64()
        r = roi_struct(roi, 1)
        self._check(self._lib.sfk_debug_eval_count(self._h, tree._h, C.byref(r), C.byref(u),
                                                    C.byref(t)))
        return u.value, t.value

    def debug_support_counts(self, tree: "Tree", roi, out=None, stream=None):
        out = self._out_for(roi, out)
        r = roi_struct(roi, out.data_ptr())
        self._check(self._lib.sfk_debug_support_counts(self._h, tree._h, C.byref(r),
                                                       out.data_ptr(), _stream_ptr(stream)))
        return out

    def debug_mbe(self, tree: "Tree", roi, out=None, cap_b: Optional[int] = None,
                  per_particle: bool = True):
        """MBE stages of one ROI: dict of ell0, n_b, idx_b, pilot, pden,
        aveden, ell_j and the final grid (device tensor). per_particle=False
        returns ell0, n_b, pilot, aveden and the grid only (no per-particle
        host arrays)."""
        out = self._out_for(roi, out)
        n = tree.info()[0]
        cap = (n if cap_b is None else cap_b) if per_particle else 0
        m = out.numel()
        ell0 = np.zeros(3, dtype=np.float32)
        nb = C.c_int64()
        pilot = np.zeros(m, dtype=np.float32)
        ave = C.c_double()
        if per_particle:
            idx = np.zeros(max(cap, 1), dtype=np.int64)
            pden = np.zeros(max(cap, 1), dtype=np.float32)
            ellj = np.zeros((max(cap, 1), 3), dtype=np.float32)
            ptrs = (idx.ctypes.data, pden.ctypes.data, ellj.ctypes.data)
        else:
            ptrs = (None, None, None)
        r = roi_struct(roi, out.data_ptr())
        self._check(self._lib.sfk_debug_mbe(self._h, tree._h, C.byref(r), ell0.ctypes.data,
                                            C.byref(nb), ptrs[0], pilot.ctypes.data, ptrs[1],
                                            C.byref(ave), ptrs[2], cap))
        k = nb.value
        res = {"ell0": ell0, "n_b": k, "pilot": pilot, "aveden": ave.value, "final": out}
        if per_particle:
            res.update(idx_b=idx[:k], pden=pden[:k], ell_j=ellj[:k])
        return res


class View:
    """An interactive view's block cache (sfk_view). frame(lo, hi) returns the
    grid of lattice nodes covering the box and what the frame did."""

    def __init__(self, ctx: Context, tree: "Tree", h: C.c_void_p, block: int):
        self._ctx = ctx
        self._tree = tree  # the tree must outlive the view
        self._h = h
        self.block = block

    @staticmethod
    def _info(inf) -> dict:
        return {"lo": tuple(inf.lo), "hi": tuple(inf.hi), "g0": tuple(inf.g0),
                "res": tuple(inf.res), "new_lattice": bool(inf.new_lattice),
                "spacing": inf.spacing, "lattice_id": inf.lattice_id,
                "blocks_needed": inf.blocks_needed, "blocks_evaluated": inf.blocks_evaluated}

    def plan(self, lo, hi) -> dict:
        """What frame(lo, hi) would do (no device work, no state change)."""
        a, b = (C.c_double * 3)(*lo), (C.c_double * 3)(*hi)
        inf = L.ViewFrameInfo()
        self._ctx._check(L.lib().sfk_view_frame(self._h, a, b, None, 0, C.byref(inf), None))
        return self._info(inf)

    def frame(self, lo, hi, out=None, stream=None):
        """sfk_view_frame: (grid tensor (x fastest, nodes of info['res']), info)."""
        import torch
        need = self.plan(lo, hi)
        n = need["res"][0] * need["res"][1] * need["res"][2]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device="cuda:%d" % self._ctx.device)
        if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()):
            raise ValueError("out must be a contiguous float32 device tensor")
        a, b = (C.c_double * 3)(*lo), (C.c_double * 3)(*hi)
        inf = L.ViewFrameInfo()
        self._ctx._check(L.lib().sfk_view_frame(self._h, a, b, out.data_ptr(), out.numel(),
                                                C.byref(inf), _stream_ptr(stream)))
        return out[:n], self._info(inf)

    def close(self):
        if self._h:
            L.lib().sfk_view_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """A device-resident spatial index (sfk_tree)."""

    def __init__(self, ctx: Context, h: C.c_void_p):
        self._ctx = ctx
        self._h = h

    def info(self):
        n = C.c_int64()
        bb = (C.c_double * 6)()
        nb = C.c_size_t()
        self._ctx._check(L.lib().sfk_tree_info(self._h, C.byref(n), bb, C.byref(nb)))
        return n.value, list(bb), nb.value

    def close(self):
        if self._h:
            for v in list(self._ctx._views):  # views of this tree go first
                if v._tree is self:
                    v.close()
            L.lib().sfk_tree_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
