"""Plain FP64 brute-force oracle for ROI kernel density estimation.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product library. It shares no
code with the HIP implementation; only the seeded input generators (package
`synth`) serve both.

Everything here is a definition evaluated directly over every particle
(ScaleFree, arXiv 2601.20758, Section 3.1): Eq. 2 / Eq. 7 densities, the
Eq. 4 kernel, Eq. 1 initial smoothing length, the Eq. 5 mean and the Eq. 6
adaptive smoothing length. The readings of points the paper leaves open are
documented in kde_oracle.c and in the design notes. Every function is pinned
by tests/test_oracle_pins.py against closed forms, invariants, library
routines or brute force on tiny inputs.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_KERNELS = {"epanechnikov": 0, "gauss_trunc3": 1, "count": 2}
_LIB = None

f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        lib = C.CDLL(path)
        vp = C.c_void_p
        lib.orc_density_nodes.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_double, vp, C.c_int,
                                          vp, vp, vp, C.c_double, vp, C.c_int64, vp]
        lib.orc_density_nodes.restype = None
        lib.orc_candidates.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_int, vp, vp, vp,
                                       vp, C.c_int64, vp, vp]
        lib.orc_candidates.restype = None
        lib.orc_knn_h2.argtypes = [vp, C.c_int64, C.c_int, vp, C.c_int64, vp]
        lib.orc_knn_h2.restype = C.c_int
        lib.orc_mbe_initial_ell.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
        lib.orc_mbe_initial_ell.restype = None
        lib.orc_mbe_asl.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_mbe_asl.restype = None
        lib.orc_point_params_from_h2.argtypes = [vp, C.c_int64, vp, vp]
        lib.orc_params_from_ell.argtypes = [vp, C.c_int64, vp, vp]
        lib.orc_trilinear.argtypes = [vp, vp, vp, vp, vp]
        lib.orc_trilinear.restype = C.c_double
        lib.orc_percentile.argtypes = [vp, C.c_int64, C.c_int, C.c_double]
        lib.orc_percentile.restype = C.c_double
        lib.orc_node_coord.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int]
        lib.orc_node_coord.restype = C.c_double
        lib.orc_u2.argtypes = [C.c_double] * 3 + [C.c_float] * 6
        lib.orc_u2.restype = C.c_double
        lib.orc_d2_f32.argtypes = [vp, vp]
        lib.orc_d2_f32.restype = C.c_float
        for name in ("orc_ck_epanechnikov", "orc_ck_gauss_trunc3", "orc_p_chi2_3_below_9"):
            getattr(lib, name).argtypes = []
            getattr(lib, name).restype = C.c_double
        lib.orc_kernel_ck.argtypes = [C.c_int]
        lib.orc_kernel_ck.restype = C.c_double
        lib.orc_sample_points.argtypes = [vp, vp, vp, vp, vp, C.c_int64, vp]
        lib.orc_sample_points.restype = None
        lib.orc_select_points.argtypes = [vp, vp, vp, vp, C.c_double, vp, C.c_int64, vp]
        lib.orc_select_points.restype = C.c_int64
        lib.orc_iso_cells.argtypes = [vp, vp, C.c_double, vp, vp]
        lib.orc_iso_cells.restype = C.c_int64
        lib.orc_mc_case.argtypes = [C.c_int, vp]
        lib.orc_mc_case.restype = C.c_int
        lib.orc_iso_surface.argtypes = [vp, vp, vp, vp, C.c_double, vp, C.c_int64]
        lib.orc_iso_surface.restype = C.c_int64
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_set_threads.restype = None
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = C.c_int
        _LIB = lib
    return _LIB


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (timing only; results do not
    depend on it)."""
    _lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_lib().orc_max_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# constants and geometry
# ---------------------------------------------------------------------------

def kernel_ck(kernel: str) -> float:
    """Normalisation constant C_K of a kernel (Eq. 2's 15/(8 pi) for
    Epanechnikov; 1/((2 pi)^{3/2} P(chi2_3 < 9)) for the truncated Gaussian)."""
    return _lib().orc_kernel_ck(_KERNELS[kernel])


def p_chi2_3_below_9() -> float:
    return _lib().orc_p_chi2_3_below_9()


def node_coord(lo: float, hi: float, res: int, i: int) -> float:
    return _lib().orc_node_coord(lo, hi, res, i)


def axis_coords(lo: float, hi: float, res: int) -> np.ndarray:
    return np.array([node_coord(lo, hi, res, i) for i in range(res)], dtype=np.float64)


def node_positions(roi, nodes: np.ndarray) -> np.ndarray:
    rx, ry, _ = (int(v) for v in roi.res)
    ax = [axis_coords(roi.lo[k], roi.hi[k], int(roi.res[k])) for k in range(3)]
    ix = nodes % rx
    iy = (nodes // rx) % ry
    iz = nodes // (rx * ry)
    return np.stack([ax[0][ix], ax[1][iy], ax[2][iz]], axis=1)


def u2(node, p, ih) -> float:
    """Canonical squared scaled distance (double, on float32 particle and
    inverse-bandwidth inputs): the membership and kernel-value quantity."""
    return _lib().orc_u2(float(node[0]), float(node[1]), float(node[2]),
                         float(p[0]), float(p[1]), float(p[2]),
                         float(ih[0]), float(ih[1]), float(ih[2]))


def roi_h(roi) -> np.ndarray:
    """Bandwidth per axis (float32) of a uniform-bandwidth ROI.

    fixed:      h_k as given.
    roi_scaled: h_k = h0 * (hi_k - lo_k), in double, rounded once.
    """
    if roi.bw == "fixed":
        return np.array(roi.h, dtype=np.float32)
    if roi.bw == "roi_scaled":
        h0 = np.float32(roi.h[0])
        return np.array([np.float64(h0) * (float(roi.hi[k]) - float(roi.lo[k]))
                         for k in range(3)], dtype=np.float64).astype(np.float32)
    raise ValueError("uniform bandwidth only for fixed / roi_scaled")


def uniform_params(h: np.ndarray):
    """(ih, w): ih_k = (float)(1/h_k); w = 1/(h_x h_y h_z) in double."""
    h64 = h.astype(np.float64)
    ih = (1.0 / h64).astype(np.float32)
    w = 1.0 / (h64[0] * h64[1] * h64[2])
    return ih, float(w)


def in_box_mask(pts: np.ndarray, lo, hi) -> np.ndarray:
    """Closed-box membership, compared in double."""
    p = pts.astype(np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return np.all((p >= lo) & (p <= hi), axis=1)


def _all_nodes(roi) -> np.ndarray:
    return np.arange(int(roi.res[0]) * int(roi.res[1]) * int(roi.res[2]), dtype=np.int64)


def _geom(roi):
    lo = _f64(roi.lo)
    hi = _f64(roi.hi)
    res = np.ascontiguousarray(roi.res, dtype=np.int32)
    return lo, hi, res


# ---------------------------------------------------------------------------
# core brute-force evaluation
# ---------------------------------------------------------------------------

def density_raw(pts, roi, kernel: str, scale: float, ih_u=None, w_u=0.0,
                ih_pp=None, w_pp=None, include=None, nodes=None) -> np.ndarray:
    """rho(n) = scale * sum_j [u2 < c2] w_j K(u2) at the listed nodes (FP64)."""
    pts = _f32(pts)
    n = pts.shape[0]
    nodes = _all_nodes(roi) if nodes is None else np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros(nodes.shape[0], dtype=np.float64)
    if nodes.shape[0] == 0:
        return out
    lo, hi, res = _geom(roi)
    ih_u = None if ih_u is None else _f32(ih_u)
    ih_pp = None if ih_pp is None else _f32(ih_pp)
    w_pp = None if w_pp is None else _f64(w_pp)
    inc = None if include is None else np.ascontiguousarray(include, dtype=np.uint8)
    _lib().orc_density_nodes(_ptr(pts), n, _ptr(ih_pp), _ptr(w_pp), _ptr(ih_u), float(w_u),
                             _ptr(inc), _KERNELS[kernel], _ptr(lo), _ptr(hi), _ptr(res),
                             float(scale), _ptr(nodes), nodes.shape[0], _ptr(out))
    return out


def candidates_raw(pts, roi, kernel: str, ih_u=None, ih_pp=None, include=None,
                   nodes=None):
    """Support sets S(n): (offsets[len(nodes)+1], original indices)."""
    pts = _f32(pts)
    n = pts.shape[0]
    nodes = _all_nodes(roi) if nodes is None else np.ascontiguousarray(nodes, dtype=np.int64)
    lo, hi, res = _geom(roi)
    offs = np.zeros(nodes.shape[0] + 1, dtype=np.int64)
    ih_u = None if ih_u is None else _f32(ih_u)
    ih_pp = None if ih_pp is None else _f32(ih_pp)
    inc = None if include is None else np.ascontiguousarray(include, dtype=np.uint8)
    args = (_ptr(pts), n, _ptr(ih_pp), _ptr(ih_u), _ptr(inc), _KERNELS[kernel], _ptr(lo),
            _ptr(hi), _ptr(res), _ptr(nodes), nodes.shape[0])
    _lib().orc_candidates(*args, _ptr(offs), None)
    idx = np.zeros(int(offs[-1]), dtype=np.int64)
    _lib().orc_candidates(*args, _ptr(offs), _ptr(idx))
    return offs, idx


# ---------------------------------------------------------------------------
# per-point bandwidth (k-th nearest neighbour)
# ---------------------------------------------------------------------------

def knn_h2(pts, k: int = 32, queries: Optional[np.ndarray] = None) -> np.ndarray:
    """h_j^2 = k-th smallest canonical float32 squared distance to the other
    particles (self excluded by index), for each queried particle."""
    pts = _f32(pts)
    n = pts.shape[0]
    q = np.arange(n, dtype=np.int64) if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    out = np.zeros(q.shape[0], dtype=np.float32)
    rc = _lib().orc_knn_h2(_ptr(pts), n, int(k), _ptr(q), q.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("k-NN bandwidth needs at least k+1 particles")
    return out


def params_from_h2(h2: np.ndarray):
    """Per-point (ih[n,3] float32, w[n] double) of an isotropic bandwidth sqrt(h2)."""
    h2 = _f32(h2)
    n = h2.shape[0]
    ih = np.zeros((n, 3), dtype=np.float32)
    w = np.zeros(n, dtype=np.float64)
    _lib().orc_point_params_from_h2(_ptr(h2), n, _ptr(ih), _ptr(w))
    return ih, w


def params_from_h(h: np.ndarray):
    """Per-point (ih[n,3] float32, w[n] double) of a given isotropic bandwidth:
    ih = (float)(1/h), w = 1/h^3 in double."""
    h64 = _f32(h).astype(np.float64)
    ih = np.repeat((1.0 / h64).astype(np.float32)[:, None], 3, axis=1)
    return np.ascontiguousarray(ih), 1.0 / (h64 * h64 * h64)


def params_from_ell(ell: np.ndarray):
    """Per-point (ih[n,3] float32, w[n] double) of per-axis smoothing lengths."""
    ell = _f32(ell).reshape(-1, 3)
    n = ell.shape[0]
    ih = np.zeros((n, 3), dtype=np.float32)
    w = np.zeros(n, dtype=np.float64)
    _lib().orc_params_from_ell(_ptr(ell), n, _ptr(ih), _ptr(w))
    return ih, w


# ---------------------------------------------------------------------------
# MBE stages (Section 3.1, Eqs. 1-8)
# ---------------------------------------------------------------------------

def percentile(x: np.ndarray, q: float) -> float:
    """Type-7 percentile (linear interpolation between order statistics)."""
    x = _f32(x)
    return _lib().orc_percentile(_ptr(x), x.shape[0], 1, float(q))


def mbe_initial_ell(pts_b: np.ndarray, roi):
    """Eq. 1 over the particles inside B: (ell[3] float32, degenerate flags)."""
    pts_b = _f32(pts_b).reshape(-1, 3)
    lo, hi, res = _geom(roi)
    ell = np.zeros(3, dtype=np.float32)
    flags = C.c_int(0)
    _lib().orc_mbe_initial_ell(_ptr(pts_b), pts_b.shape[0], _ptr(lo), _ptr(hi), _ptr(res),
                               _ptr(ell), C.byref(flags))
    return ell, flags.value


def trilinear(grid: np.ndarray, roi, p) -> float:
    grid = _f64(grid)
    lo, hi, res = _geom(roi)
    p = _f32(p)
    return _lib().orc_trilinear(_ptr(grid), _ptr(lo), _ptr(hi), _ptr(res), _ptr(p))


def mbe_asl(pts_b: np.ndarray, roi, pilot: np.ndarray, ell0: np.ndarray):
    """Eqs. 5-6 given a pilot grid: (pden[n_b], aveden, ell_j[n_b, 3])."""
    pts_b = _f32(pts_b).reshape(-1, 3)
    n_b = pts_b.shape[0]
    lo, hi, res = _geom(roi)
    pilot = _f64(pilot)
    ell0 = _f32(ell0)
    pden = np.zeros(n_b, dtype=np.float64)
    ave = C.c_double(0.0)
    ell_j = np.zeros((n_b, 3), dtype=np.float32)
    _lib().orc_mbe_asl(_ptr(pts_b), n_b, _ptr(pilot), _ptr(lo), _ptr(hi), _ptr(res),
                       _ptr(ell0), _ptr(pden), C.byref(ave), _ptr(ell_j))
    return pden, ave.value, ell_j


def _nu(roi, n_eff: int) -> float:
    if roi.norm == "count":
        return 1.0
    return 1.0 / n_eff if n_eff > 0 else 0.0


def mbe(pts, roi, nodes=None, pilot_in=None, ell_j_in=None) -> dict:
    """The full MBE chain for one ROI (Section 3.1):
    B and N_B -> Eq. 1 -> pilot grid (Eq. 2) -> pden by trilinear
    interpolation -> aveDen (Eq. 5) -> l_kj (Eq. 6) -> final grid (Eq. 7).

    pilot_in / ell_j_in substitute an upstream stage's result (stage-wise
    parity: a verified upstream array is fed to the next stage)."""
    if roi.kernel != "epanechnikov":
        raise ValueError("MBE is defined for the Epanechnikov kernel")
    pts = _f32(pts)
    inc = in_box_mask(pts, roi.lo, roi.hi)
    idx_b = np.nonzero(inc)[0]
    pts_b = np.ascontiguousarray(pts[idx_b])
    n_b = pts_b.shape[0]
    out = {"idx_b": idx_b, "n_b": n_b}
    m = int(roi.res[0]) * int(roi.res[1]) * int(roi.res[2])
    if n_b == 0:
        out.update(ell0=np.zeros(3, np.float32), pilot=np.zeros(m), pden=np.zeros(0),
                   aveden=0.0, ell_j=np.zeros((0, 3), np.float32),
                   final=np.zeros(m if nodes is None else len(nodes)), flags=0)
        return out
    ell0, flags = mbe_initial_ell(pts_b, roi)
    ck = kernel_ck("epanechnikov")
    scale = ck * _nu(roi, n_b)
    if pilot_in is None:
        ih, w = uniform_params(ell0)
        pilot = density_raw(pts_b, roi, "epanechnikov", scale, ih_u=ih, w_u=w)
    else:
        pilot = _f64(pilot_in)
    pden, ave, ell_j = mbe_asl(pts_b, roi, pilot, ell0)
    if ell_j_in is not None:
        ell_j = _f32(ell_j_in).reshape(-1, 3)
    ihp, wp = params_from_ell(ell_j)
    final = density_raw(pts_b, roi, "epanechnikov", scale, ih_pp=ihp, w_pp=wp, nodes=nodes)
    out.update(ell0=ell0, flags=flags, pilot=pilot, pden=pden, aveden=ave, ell_j=ell_j,
               final=final)
    return out


# ---------------------------------------------------------------------------
# one-call front end per ROI
# ---------------------------------------------------------------------------

def _setup(pts, roi, h2=None):
    """Resolve a ROI into (kernel, scale, ih_u, w_u, ih_pp, w_pp, include)."""
    pts = _f32(pts)
    n = pts.shape[0]
    include = None
    n_eff = n
    if roi.set == "in_roi":
        include = in_box_mask(pts, roi.lo, roi.hi)
        n_eff = int(include.sum())
    kernel = roi.kernel
    ck = kernel_ck(kernel) if kernel != "count" else 1.0
    scale = ck * _nu(roi, n_eff)
    ih_u = w_u = ih_pp = w_pp = None
    if roi.bw in ("fixed", "roi_scaled"):
        ih_u, w_u = uniform_params(roi_h(roi))
    elif roi.bw == "per_point":
        if h2 is None:
            raise ValueError("per_point bandwidth needs h2")
        ih_pp, w_pp = params_from_h2(h2)
    else:
        raise ValueError(roi.bw)
    return kernel, scale, ih_u, (w_u or 0.0), ih_pp, w_pp, include


def density(pts, roi, nodes=None, h2=None) -> np.ndarray:
    """Grid density (FP64) of one ROI at the listed node indices (all if None)."""
    if roi.bw == "mbe":
        return mbe(pts, roi, nodes=nodes)["final"]
    kernel, scale, ih_u, w_u, ih_pp, w_pp, include = _setup(pts, roi, h2)
    return density_raw(pts, roi, kernel, scale, ih_u=ih_u, w_u=w_u, ih_pp=ih_pp,
                       w_pp=w_pp, include=include, nodes=nodes)


def support_counts(pts, roi, nodes=None, h2=None) -> np.ndarray:
    """#S(n) per node (exact integer counts, with the ROI kernel's support)."""
    kernel, _, ih_u, _, ih_pp, _, include = _setup(pts, roi, h2)
    pts = _f32(pts)
    nodes = _all_nodes(roi) if nodes is None else np.ascontiguousarray(nodes, dtype=np.int64)
    lo, hi, res = _geom(roi)
    offs = np.zeros(nodes.shape[0] + 1, dtype=np.int64)
    ih_u = None if ih_u is None else _f32(ih_u)
    ih_pp = None if ih_pp is None else _f32(ih_pp)
    inc = None if include is None else np.ascontiguousarray(include, dtype=np.uint8)
    _lib().orc_candidates(_ptr(pts), pts.shape[0], _ptr(ih_pp), _ptr(ih_u), _ptr(inc),
                          _KERNELS[kernel], _ptr(lo), _ptr(hi), _ptr(res), _ptr(nodes),
                          nodes.shape[0], _ptr(offs), None)
    return np.diff(offs)


def candidates(pts, roi, nodes, h2=None):
    """Support sets (offsets, original indices ascending) of the listed nodes."""
    kernel, _, ih_u, _, ih_pp, _, include = _setup(pts, roi, h2)
    return candidates_raw(pts, roi, kernel, ih_u=ih_u, ih_pp=ih_pp, include=include,
                          nodes=nodes)


# ---------------------------------------------------------------------------
# consumers of a density grid (Section 3.1 after Eq. 8; Section 4.1)
# ---------------------------------------------------------------------------

def sample_density(grid: np.ndarray, roi, pts: np.ndarray) -> np.ndarray:
    """Trilinear density of the node grid at each point; 0 outside the closed box."""
    grid = _f64(grid).ravel()
    lo, hi, res = _geom(roi)
    pts = _f32(pts).reshape(-1, 3)
    out = np.zeros(pts.shape[0], dtype=np.float64)
    _lib().orc_sample_points(_ptr(grid), _ptr(lo), _ptr(hi), _ptr(res), _ptr(pts),
                             pts.shape[0], _ptr(out))
    return out


def select_points(grid: np.ndarray, roi, iso: float, pts: np.ndarray) -> np.ndarray:
    """Ascending indices of the points in the closed box whose density is >= iso."""
    grid = _f64(grid).ravel()
    lo, hi, res = _geom(roi)
    pts = _f32(pts).reshape(-1, 3)
    idx = np.zeros(max(1, pts.shape[0]), dtype=np.int64)
    m = _lib().orc_select_points(_ptr(grid), _ptr(lo), _ptr(hi), _ptr(res), float(iso),
                                 _ptr(pts), pts.shape[0], _ptr(idx))
    return idx[:m].copy()


def iso_cells(grid: np.ndarray, roi, iso: float):
    """Active Marching Cubes cells (ascending) and their 8-bit cases."""
    grid = _f64(grid).ravel()
    _, _, res = _geom(roi)
    n_cells = int(np.prod(np.asarray(roi.res, dtype=np.int64) - 1))
    cells = np.zeros(max(1, n_cells), dtype=np.int64)
    cases = np.zeros(max(1, n_cells), dtype=np.uint8)
    m = _lib().orc_iso_cells(_ptr(grid), _ptr(res), float(iso), _ptr(cells), _ptr(cases))
    return cells[:m].copy(), cases[:m].copy()


def mc_case(case: int) -> np.ndarray:
    """Marching Cubes triangles of one 8-bit case as (n, 3) edge ids."""
    e = np.zeros(36, dtype=np.int32)
    n = _lib().orc_mc_case(int(case), _ptr(e))
    return e[:3 * n].reshape(n, 3).copy()


def iso_surface(grid: np.ndarray, roi, iso: float) -> np.ndarray:
    """Marching Cubes iso-surface of a node grid: (n, 3, 3) float32
    triangles (vertex, xyz), cells in ascending order."""
    grid = _f64(grid).ravel()
    lo, hi, res = _geom(roi)
    n = _lib().orc_iso_surface(_ptr(grid), _ptr(lo), _ptr(hi), _ptr(res), float(iso), None, 0)
    out = np.zeros((max(1, n), 3, 3), dtype=np.float32)
    _lib().orc_iso_surface(_ptr(grid), _ptr(lo), _ptr(hi), _ptr(res), float(iso), _ptr(out), n)
    return out[:n]
