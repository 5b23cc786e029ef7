"""Seeded particle clouds and ROI workloads.

Every generator takes an explicit seed and draws from numpy's PCG64, so a
cloud is a pure function of its arguments. Coordinates are float32 in
[0, 1]^3 (samples that fall outside the unit box are redrawn), laid out as
an (N, 3) C-contiguous array.

The paper's datasets (cosmological N-body and filament clouds of 76k-442k
points, Section 3.3) are not available; `clumpy_cloud` stands in for them
with a multiscale clustered structure, and `paperlike_cloud` gives clouds of
the paper's three sizes from the same recipe.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Roi", "c1_cloud", "clumpy_cloud", "clumpy_cloud_device", "lattice_cloud", "uniform_cloud",
    "blob_cloud", "paperlike_cloud", "c1_roi", "c2_roi", "nested_zoom_rois",
    "random_batch_rois", "serving_trace",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclasses.dataclass
class Roi:
    """One region-of-interest request: a closed box, a grid and a bandwidth.

    kernel: "epanechnikov" | "gauss_trunc3" | "count"
    bw:     "fixed" | "roi_scaled" | "per_point" | "mbe"
    norm:   "paper" (times 1/N) | "count" (no 1/N)
    set:    "cloud" (every particle) | "in_roi" (particles inside the box)
    h:      bandwidth per axis for "fixed"; the factor h0 for "roi_scaled"
    """
    lo: Sequence[float]
    hi: Sequence[float]
    res: Sequence[int]
    kernel: str = "epanechnikov"
    bw: str = "fixed"
    norm: str = "paper"
    set: str = "cloud"
    h: Sequence[float] = (0.02, 0.02, 0.02)
    tag: int = 0

    @property
    def n_nodes(self) -> int:
        return int(self.res[0]) * int(self.res[1]) * int(self.res[2])

    def replace(self, **kw) -> "Roi":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# clouds
# ---------------------------------------------------------------------------

def _in_unit_box(p: np.ndarray) -> np.ndarray:
    return np.all((p >= 0.0) & (p <= 1.0), axis=1)


def uniform_cloud(n: int, seed: int) -> np.ndarray:
    """n points uniform in [0, 1)^3."""
    return _rng(seed).random((n, 3), dtype=np.float64).astype(np.float32)


def c1_cloud(seed: int = 1, n_uniform: int = 10_000, n_clusters: int = 8,
             per_cluster: int = 1_250, sigma: float = 0.03) -> np.ndarray:
    """The small correctness workload: half uniform, half in isotropic clusters.

    Cluster centres are U[0.1, 0.9]^3; cluster samples falling outside the
    unit box are redrawn from the same cluster.
    """
    g = _rng(seed)
    uni = g.random((n_uniform, 3))
    centres = g.uniform(0.1, 0.9, size=(n_clusters, 3))
    parts = [uni]
    for c in centres:
        pts = c + sigma * g.standard_normal((per_cluster, 3))
        bad = ~_in_unit_box(pts)
        while bad.any():
            pts[bad] = c + sigma * g.standard_normal((int(bad.sum()), 3))
            bad = ~_in_unit_box(pts)
        parts.append(pts)
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def _quat_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices from unit quaternions (w, x, y, z), shape (K, 3, 3)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = np.empty((q.shape[0], 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


@dataclasses.dataclass
class ClumpInfo:
    centres: np.ndarray   # (K, 3)
    masses: np.ndarray    # (K,)
    sigma1: np.ndarray    # (K,)
    counts: np.ndarray    # (K,)


_CHUNK = 1 << 22  # points per generation chunk (fixed: part of the recipe)


def clumpy_cloud(n: int, seed: int, n_clumps: int = 2000, bg_frac: float = 0.2,
                 m_lo: float = 1.0, m_hi: float = 1e3, index: float = -1.8,
                 with_info: bool = False):
    """Cosmology-like clustered cloud.

    Recipe: a fraction `bg_frac` of the points is uniform in [0,1]^3; the rest
    sit in `n_clumps` anisotropic Gaussian clumps. Clump masses follow a
    truncated power law (pdf proportional to m**index on [m_lo, m_hi], drawn
    by inverse CDF); point counts are multinomial in proportion to mass;
    centres are U[0.05, 0.95]^3; the principal width is
    0.02 * (m / m_hi)**(1/3) and the two others are that times U[0.3, 1];
    every clump has a uniformly random orientation. Out-of-box samples are
    redrawn from their clump.
    """
    g = _rng(seed)
    a = index + 1.0
    u = g.random(n_clumps)
    masses = (m_lo ** a + u * (m_hi ** a - m_lo ** a)) ** (1.0 / a)
    centres = g.uniform(0.05, 0.95, size=(n_clumps, 3))
    s1 = 0.02 * (masses / m_hi) ** (1.0 / 3.0)
    q = g.uniform(0.3, 1.0, size=(n_clumps, 2))
    sig = np.stack([s1, s1 * q[:, 0], s1 * q[:, 1]], axis=1)
    quat = g.standard_normal((n_clumps, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    rot = _quat_rot(quat)
    n_bg = int(round(bg_frac * n))
    n_cl = n - n_bg
    counts = g.multinomial(n_cl, masses / masses.sum())

    out = np.empty((n, 3), dtype=np.float32)
    # background, in fixed-size chunks
    pos = 0
    while pos < n_bg:
        k = min(_CHUNK, n_bg - pos)
        out[pos:pos + k] = g.random((k, 3))
        pos += k
    # clumps, grouped into chunks of whole clumps
    cid = 0
    while cid < n_clumps:
        stop = cid
        tot = 0
        while stop < n_clumps and (tot == 0 or tot + counts[stop] <= _CHUNK):
            tot += counts[stop]
            stop += 1
        ids = np.repeat(np.arange(cid, stop), counts[cid:stop])
        pts = _clump_points(g, ids, centres, sig, rot)
        bad = ~_in_unit_box(pts)
        while bad.any():
            pts[bad] = _clump_points(g, ids[bad], centres, sig, rot)
            bad = ~_in_unit_box(pts)
        out[pos:pos + tot] = pts
        pos += tot
        cid = stop
    assert pos == n
    if with_info:
        return out, ClumpInfo(centres, masses, s1, counts)
    return out


def _clump_points(g, ids, centres, sig, rot):
    z = g.standard_normal((ids.shape[0], 3)) * sig[ids]
    return centres[ids] + np.einsum("nij,nj->ni", rot[ids], z)


def paperlike_cloud(n: int, seed: int) -> np.ndarray:
    """Clumpy cloud at one of the paper's dataset sizes (76k, 164k, 442k)."""
    return clumpy_cloud(n, seed)


def lattice_cloud(m: int, a: float, origin: float = 0.0) -> np.ndarray:
    """Cubic lattice of m^3 points with spacing a (exact in float32 when a
    and origin are dyadic)."""
    i = np.arange(m, dtype=np.float64) * a + origin
    x, y, z = np.meshgrid(i, i, i, indexing="ij")
    return np.ascontiguousarray(
        np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float32))


def blob_cloud(n: int, centre: Sequence[float], sigma: float, seed: int) -> np.ndarray:
    """n points from an isotropic Gaussian N(centre, sigma^2 I) (no redraw)."""
    g = _rng(seed)
    return np.ascontiguousarray(
        (np.asarray(centre) + sigma * g.standard_normal((n, 3))).astype(np.float32))


# ---------------------------------------------------------------------------
# ROI workloads
# ---------------------------------------------------------------------------

def c1_roi() -> Roi:
    """Full unit box, 32^3 grid, Epanechnikov, fixed h = 0.02."""
    return Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (32, 32, 32),
               kernel="epanechnikov", bw="fixed", h=(0.02, 0.02, 0.02))


def c2_roi(res: int = 128) -> Roi:
    """Full unit box, res^3 grid, Gaussian truncated at 3h, per-point h."""
    return Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (res, res, res),
               kernel="gauss_trunc3", bw="per_point", h=(0.0, 0.0, 0.0))


def box_around(centre, side):
    """(lo, hi) of the cube of the given side centred on `centre`, moved
    inside the unit box."""
    c = np.clip(np.asarray(centre, dtype=np.float64), side / 2, 1.0 - side / 2)
    return tuple(float(v) for v in c - side / 2), tuple(float(v) for v in c + side / 2)


_clamped_box = box_around


def nested_zoom_rois(info: ClumpInfo, seed: int, n_steps: int = 11,
                     resolutions: Sequence[int] = (64, 128, 256),
                     h0: float = 0.01) -> List[Roi]:
    """Zoom sequence: sides 2^-i (i = 0..n_steps-1) around a clump drawn with
    the seed from the 10 most massive; each box at every resolution."""
    g = _rng(seed)
    top = np.argsort(-info.masses)[:10]
    c = info.centres[top[g.integers(0, len(top))]]
    rois = []
    for i in range(n_steps):
        side = 2.0 ** (-i)
        lo, hi = _clamped_box(c, side)
        for r in resolutions:
            rois.append(Roi(lo, hi, (r, r, r), kernel="epanechnikov",
                            bw="roi_scaled", h=(h0, h0, h0), tag=len(rois)))
    return rois


def random_batch_rois(n: int, seed: int, side_lo: float = 1e-3,
                      side_hi: float = 1.0, res_lo: int = 16, res_hi: int = 128,
                      h0: float = 0.01, res_choices: Optional[Sequence[int]] = None
                      ) -> List[Roi]:
    """n cubic ROIs: side log-uniform, centre uniform with the box inside
    [0,1]^3, resolution uniform on an integer range (or a choice list)."""
    g = _rng(seed)
    sides = np.exp(g.uniform(math.log(side_lo), math.log(side_hi), size=n))
    rois = []
    for t in range(n):
        s = float(sides[t])
        c = g.uniform(s / 2, 1.0 - s / 2, size=3)
        if res_choices is None:
            r = int(g.integers(res_lo, res_hi + 1))
        else:
            r = int(res_choices[int(g.integers(0, len(res_choices)))])
        lo, hi = _clamped_box(c, s)
        rois.append(Roi(lo, hi, (r, r, r), kernel="epanechnikov",
                        bw="roi_scaled", h=(h0, h0, h0), tag=t))
    return rois


def serving_trace(seed: int, duration_s: float, n_streams: int = 8,
                  rate_hz: float = 90.0, side_lo: float = 1e-4, side_hi: float = 1.0,
                  res_choices: Sequence[int] = (32, 48, 64, 96, 128),
                  h0: float = 0.01):
    """VR-like request trace: each stream has Poisson arrivals at rate_hz and
    a panning centre (a Gaussian step of 0.25 * side per request, kept inside
    the unit box). Returns (arrival_seconds, stream_ids, rois) sorted by time."""
    g = _rng(seed)
    arrivals, streams, rois = [], [], []
    for s in range(n_streams):
        t = 0.0
        centre = g.uniform(0.0, 1.0, size=3)
        while True:
            t += g.exponential(1.0 / rate_hz)
            if t >= duration_s:
                break
            side = float(np.exp(g.uniform(math.log(side_lo), math.log(side_hi))))
            centre = np.clip(centre + g.normal(0.0, 0.25 * side, size=3),
                             side / 2, 1.0 - side / 2)
            r = int(res_choices[int(g.integers(0, len(res_choices)))])
            lo, hi = _clamped_box(centre, side)
            arrivals.append(t)
            streams.append(s)
            rois.append(Roi(lo, hi, (r, r, r), kernel="epanechnikov",
                            bw="roi_scaled", h=(h0, h0, h0)))
    order = np.argsort(np.asarray(arrivals), kind="stable")
    arr = np.asarray(arrivals)[order]
    st = np.asarray(streams)[order]
    rs = [rois[i] for i in order]
    for k, r in enumerate(rs):
        r.tag = k
    return arr, st, rs


def view_path(info: ClumpInfo, seed: int, n_frames: int = 180, fps: float = 90.0,
              side0: float = 0.2, zoom_octaves: float = 1.5, zoom_period_s: float = 2.0,
              pan_radius: float = 0.15):
    """A smooth camera path of an interactive view (one box per frame at fps):
    the centre circles a massive clump (three incommensurate sinusoids of
    amplitude pan_radius), the side breathes between side0 * 2^-zoom_octaves
    and side0 * 2^zoom_octaves over zoom_period_s. Returns [(lo, hi), ...]."""
    g = _rng(seed)
    top = np.argsort(-np.asarray(info.masses))[:10]
    c0 = np.asarray(info.centres[int(top[int(g.integers(0, len(top)))])], dtype=np.float64)
    ph = g.uniform(0.0, 2.0 * math.pi, size=4)
    boxes = []
    for i in range(n_frames):
        t = i / fps
        side = side0 * 2.0 ** (zoom_octaves * math.sin(2.0 * math.pi * t / zoom_period_s + ph[3]))
        c = c0 + pan_radius * np.array([math.sin(2.0 * math.pi * t / 2.7 + ph[0]),
                                        math.sin(2.0 * math.pi * t / 3.1 + ph[1]),
                                        math.sin(2.0 * math.pi * t / 3.7 + ph[2])])
        boxes.append((tuple(float(v) for v in c - side / 2), tuple(float(v) for v in c + side / 2)))
    return boxes


def clumpy_cloud_device(n: int, seed: int, device="cuda", n_clumps: int = 2000,
                        bg_frac: float = 0.2, m_lo: float = 1.0, m_hi: float = 1e3,
                        index: float = -1.8, chunk: int = 1 << 25):
    """The `clumpy_cloud` recipe drawn on the GPU with torch's seeded Philox
    generator, for clouds too large to draw on the host (1e8-1e9 points).
    Same distribution, different random stream: the points differ from
    `clumpy_cloud(n, seed)`. Returns an (n, 3) float32 device tensor; the
    clump metadata is drawn on the host with numpy (seeded) and returned.
    Out-of-box samples are redrawn."""
    import torch
    g = _rng(seed)
    a = index + 1.0
    u = g.random(n_clumps)
    masses = (m_lo ** a + u * (m_hi ** a - m_lo ** a)) ** (1.0 / a)
    centres = g.uniform(0.05, 0.95, size=(n_clumps, 3))
    s1 = 0.02 * (masses / m_hi) ** (1.0 / 3.0)
    q = g.uniform(0.3, 1.0, size=(n_clumps, 2))
    sig = np.stack([s1, s1 * q[:, 0], s1 * q[:, 1]], axis=1)
    quat = g.standard_normal((n_clumps, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    rot = _quat_rot(quat)
    n_bg = int(round(bg_frac * n))
    counts = g.multinomial(n - n_bg, masses / masses.sum())
    tg = torch.Generator(device=device)
    tg.manual_seed(int(seed))
    out = torch.empty((n, 3), dtype=torch.float32, device=device)
    pos = 0
    while pos < n_bg:
        k = min(chunk, n_bg - pos)
        out[pos:pos + k] = torch.rand((k, 3), generator=tg, device=device, dtype=torch.float32)
        pos += k
    c_t = torch.as_tensor(centres, dtype=torch.float64, device=device)
    s_t = torch.as_tensor(sig, dtype=torch.float64, device=device)
    r_t = torch.as_tensor(rot, dtype=torch.float64, device=device)
    cum = np.concatenate([[0], np.cumsum(counts)])
    cid = 0
    while cid < n_clumps:
        stop = cid
        while stop < n_clumps and (stop == cid or cum[stop + 1] - cum[cid] <= chunk):
            stop += 1
        tot = int(cum[stop] - cum[cid])
        ids = torch.repeat_interleave(torch.arange(cid, stop, device=device),
                                      torch.as_tensor(counts[cid:stop], device=device))

        def draw(sel):
            z = torch.randn((sel.shape[0], 3), generator=tg, device=device,
                            dtype=torch.float64) * s_t[sel]
            r = r_t[sel]
            rz = r[:, :, 0] * z[:, 0:1] + r[:, :, 1] * z[:, 1:2] + r[:, :, 2] * z[:, 2:3]
            return c_t[sel] + rz

        pts = draw(ids)
        bad = ~((pts >= 0) & (pts <= 1)).all(dim=1)
        while bool(bad.any()):
            pts[bad] = draw(ids[bad])
            bad = ~((pts >= 0) & (pts <= 1)).all(dim=1)
        out[pos:pos + tot] = pts.to(torch.float32)
        pos += tot
        cid = stop
    assert pos == n
    return out, ClumpInfo(centres, masses, s1, counts)


def random_grid(res: Sequence[int], seed: int, scale: float = 3.0) -> np.ndarray:
    """A seeded float32 node field of res[0] * res[1] * res[2] values (x
    fastest), uniform in [0, scale): an input for the grid consumers."""
    g = _rng(seed)
    return (g.random(int(np.prod(res))) * scale).astype(np.float32)


def probe_points(roi: Roi, n: int, seed: int, margin: float = 0.1) -> np.ndarray:
    """n float32 points uniform in the ROI box grown by `margin` of its side
    on every face, plus the box corners and one row of node x-positions on
    the box's middle y and z planes (points on faces, near nodes, outside)."""
    g = _rng(seed)
    lo = np.asarray(roi.lo, np.float64)
    hi = np.asarray(roi.hi, np.float64)
    side = hi - lo
    p = g.uniform(lo - margin * side, hi + margin * side, size=(n, 3))
    corners = np.array([[lo[0] if b & 1 == 0 else hi[0], lo[1] if b & 2 == 0 else hi[1],
                         lo[2] if b & 4 == 0 else hi[2]] for b in range(8)])
    row = np.column_stack([np.linspace(lo[0], hi[0], roi.res[0]),
                           np.full(roi.res[0], 0.5 * (lo[1] + hi[1])),
                           np.full(roi.res[0], 0.5 * (lo[2] + hi[2]))])
    return np.vstack([p, corners, row]).astype(np.float32)
