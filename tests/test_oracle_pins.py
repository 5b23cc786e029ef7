"""Pins of the FP64 oracle against facts other than itself.

Each test checks the oracle against a closed form, an invariant, a library
routine, a hand-derived fixture (tests/golden/) or brute force on a tiny
input, chosen so that a dropped term, a wrong constant, a sign error, a
transposed axis or a non-strict support boundary fails at least one of them.
All run on the CPU.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.spatial
import scipy.stats

import oracle
import synth
from synth import Roi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows, extra = [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0].isalpha():
                extra[parts[0]] = [float(v) for v in parts[1:]]
            else:
                rows.append([float(v) for v in parts])
    return rows, extra


# ---------------------------------------------------------------------------
# kernel constants: the normalised kernel integrates to one
# ---------------------------------------------------------------------------

def test_epanechnikov_constant_unit_mass():
    # radial integral of (1 - r^2) over the unit ball, by quadrature
    m, _ = si.quad(lambda r: (1 - r * r) * 4 * math.pi * r * r, 0.0, 1.0)
    assert oracle.kernel_ck("epanechnikov") * m == pytest.approx(1.0, abs=1e-13)


def test_gauss_trunc3_constant_unit_mass():
    assert oracle.p_chi2_3_below_9() == pytest.approx(scipy.stats.chi2.cdf(9.0, 3), abs=1e-14)
    m, _ = si.quad(lambda r: math.exp(-0.5 * r * r) * 4 * math.pi * r * r, 0.0, 3.0)
    assert oracle.kernel_ck("gauss_trunc3") * m == pytest.approx(1.0, abs=1e-13)


# ---------------------------------------------------------------------------
# node placement
# ---------------------------------------------------------------------------

def test_node_coords_dyadic_and_endpoints():
    ax = oracle.axis_coords(0.0, 1.0, 33)
    assert np.array_equal(ax, np.arange(33) / 32.0)
    ax = oracle.axis_coords(0.1, 0.7, 17)
    assert ax[0] == 0.1 and ax[-1] == 0.7
    assert np.all(np.diff(ax) > 0)
    np.testing.assert_allclose(np.diff(ax), 0.6 / 16, rtol=1e-13)


# ---------------------------------------------------------------------------
# single particle: kernel profile at exact dyadic distances, per axis
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["epanechnikov", "gauss_trunc3"])
def test_single_particle_profile_anisotropic(kernel):
    # box [0,1]^3, res (33, 17, 65): spacings 1/32, 1/16, 1/64 (exact)
    roi = Roi((0, 0, 0), (1, 1, 1), (33, 17, 65), kernel=kernel, bw="fixed",
              h=(0.25, 0.125, 0.5), norm="count")
    p = np.array([[0.5, 0.5, 0.5]], dtype=np.float32)
    rho = oracle.density(p, roi).reshape(65, 17, 33)  # [z, y, x]
    ck = oracle.kernel_ck(kernel)
    w = 1.0 / (0.25 * 0.125 * 0.5)
    c2 = 1.0 if kernel == "epanechnikov" else 9.0

    def prof(u2):
        if u2 >= c2:
            return 0.0
        return (1.0 - u2) if kernel == "epanechnikov" else math.exp(-0.5 * u2)

    # along x: node 16 + k at distance k/32 -> u = k/8
    for k in range(0, 30):
        ix = 16 + k
        if ix > 32:
            break
        u2 = (k / 8.0) ** 2
        assert rho[32, 8, ix] == pytest.approx(ck * w * prof(u2), rel=1e-14, abs=1e-300)
    # along y: node 8 + k at distance k/16 -> u = k/2
    for k in range(0, 9):
        u2 = (k / 2.0) ** 2
        assert rho[32, 8 + k, 16] == pytest.approx(ck * w * prof(u2), rel=1e-14, abs=1e-300)
    # along z: node 32 + k at distance k/64 -> u = k/32
    for k in range(0, 33):
        u2 = (k / 32.0) ** 2
        assert rho[32 + k, 8, 16] == pytest.approx(ck * w * prof(u2), rel=1e-14, abs=1e-300)
    # off-axis node: (dx, dy, dz) = (2/32, 1/16, 4/64) -> u2 = 1/16 + 1/4 + 1/64
    u2 = (2 / 32 * 4) ** 2 + (1 / 16 * 8) ** 2 + (4 / 64 * 2) ** 2
    assert rho[36, 9, 18] == pytest.approx(ck * w * prof(u2), rel=1e-14)


# closed-form constants, written out here rather than taken from the oracle
_CK_EPAN = 15.0 / (8.0 * math.pi)
_CK_GAUSS3 = 1.0 / ((2.0 * math.pi) ** 1.5 * scipy.stats.chi2.cdf(9.0, 3))


def _profile(kernel, r2_over_h2):
    if kernel == "epanechnikov":
        return max(0.0, 1.0 - r2_over_h2)
    return math.exp(-0.5 * r2_over_h2) if r2_over_h2 < 9.0 else 0.0


@pytest.mark.parametrize("kernel", ["epanechnikov", "gauss_trunc3"])
@pytest.mark.parametrize("norm", ["paper", "count"])
def test_single_particle_profile_per_point(kernel, norm):
    # Per-point bandwidth (Eq. 7: each particle carries its own 1/(l_x l_y l_z)
    # and its own scaled distance). Two particles far apart with given squared
    # bandwidths 1/16 and 1/64 (h = 1/4 and 1/8, exact): along x from each
    # particle the density is C_K / h^3 * K(r^2 / h^2), with C_K and K written
    # out here; with norm = paper it is divided by N = 2.
    roi = Roi((0, 0, 0), (3, 1, 1), (97, 33, 33), kernel=kernel, bw="per_point", norm=norm)
    pts = np.array([[0.5, 0.5, 0.5], [2.5, 0.5, 0.5]], dtype=np.float32)
    h = [0.25, 0.125]
    h2 = np.array([h[0] ** 2, h[1] ** 2], dtype=np.float32)
    rho = oracle.density(pts, roi, h2=h2).reshape(33, 33, 97)  # [z, y, x]
    ck = _CK_EPAN if kernel == "epanechnikov" else _CK_GAUSS3
    nu = 0.5 if norm == "paper" else 1.0
    reach = 1.0 if kernel == "epanechnikov" else 3.0
    for j, (ix0, hj) in enumerate(zip((16, 80), h)):
        # node ix0 + k sits at distance k/32 from particle j on the x axis
        for k in range(0, min(32, 97 - ix0)):
            r = k / 32.0
            other = 2.0 - r  # distance to the other particle, beyond its reach
            assert other >= reach * h[1 - j]
            want = nu * ck / hj ** 3 * _profile(kernel, (r / hj) ** 2)
            got = rho[16, 16, ix0 + k]
            assert got == pytest.approx(want, rel=1e-14, abs=1e-300), (j, k)
    # an off-axis node of particle 0: (dx, dy, dz) = (1/32, 2/32, 2/32)
    r2 = (1 / 32) ** 2 + 2 * (2 / 32) ** 2
    want = nu * ck / h[0] ** 3 * _profile(kernel, r2 / h[0] ** 2)
    assert rho[18, 18, 17] == pytest.approx(want, rel=1e-14)


def test_given_bandwidth_params_profile():
    # a given per-particle bandwidth h (not squared): ih = 1/h, w = 1/h^3
    roi = Roi((0, 0, 0), (1, 1, 1), (33, 33, 33), kernel="epanechnikov", bw="per_point",
              norm="count")
    p = np.array([[0.5, 0.5, 0.5]], dtype=np.float32)
    ih, w = oracle.params_from_h(np.array([0.5], dtype=np.float32))
    rho = oracle.density_raw(p, roi, "epanechnikov", _CK_EPAN, ih_pp=ih, w_pp=w)
    rho = rho.reshape(33, 33, 33)
    for k in range(0, 17):
        r = k / 32.0
        want = _CK_EPAN / 0.5 ** 3 * _profile("epanechnikov", (r / 0.5) ** 2)
        assert rho[16, 16, 16 + k] == pytest.approx(want, rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("kernel", ["epanechnikov", "gauss_trunc3"])
def test_per_point_total_mass(kernel):
    # a compact cloud with per-particle bandwidths spanning 2-4 node spacings:
    # every support lies inside the grid, so the field integrates to 1
    # (norm = paper) whatever each particle's h is
    g = np.random.default_rng(11)
    n = 300
    pts = g.normal(0.5, 0.04, size=(n, 3)).astype(np.float32)
    s = 1.0 / 60.0
    h = g.uniform(2.0 * s, 4.0 * s, size=n)
    if kernel == "gauss_trunc3":
        h = h / 1.5
    h2 = (h * h).astype(np.float32)
    roi = Roi((0, 0, 0), (1, 1, 1), (61, 61, 61), kernel=kernel, bw="per_point")
    mass = oracle.density(pts, roi, h2=h2).sum() * s ** 3
    assert mass == pytest.approx(1.0, abs=2e-3)


def test_support_boundary_golden():
    rows, _ = _golden("support_boundary.txt")
    roi = Roi((0, 0, 0), (1, 1, 1), (5, 5, 5), kernel="epanechnikov", bw="fixed",
              h=(0.25, 0.25, 0.25), norm="count")
    node = 2 + 5 * (2 + 5 * 2)
    ih = np.float32(4.0)
    for px, py, pz, member, u2 in rows:
        p = np.array([[px, py, pz]], dtype=np.float32)
        assert oracle.u2((0.5, 0.5, 0.5), p[0], (ih, ih, ih)) == u2
        cnt = oracle.support_counts(p, roi, nodes=np.array([node]))
        assert int(cnt[0]) == int(member), (px, py, pz)
        # density is zero exactly on the boundary
        d = oracle.density(p, roi, nodes=np.array([node]))
        assert (d[0] > 0) == bool(member)
    # one float32 ulp inside the boundary is a member
    p = np.array([[np.nextafter(np.float32(0.75), np.float32(0))], [0.5], [0.5]],
                 dtype=np.float32).reshape(1, 3)
    assert int(oracle.support_counts(p, roi, nodes=np.array([node]))[0]) == 1


# ---------------------------------------------------------------------------
# total mass: the grid sum times the cell volume integrates the KDE
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel,h,norm", [
    ("epanechnikov", (0.1, 0.1, 0.1), "paper"),
    ("epanechnikov", (0.12, 0.07, 0.09), "count"),
    ("gauss_trunc3", (0.035, 0.035, 0.035), "paper"),
])
def test_total_mass(kernel, h, norm):
    # particles well inside so every support lies inside the grid; random
    # sub-cell positions make the lattice sum exact in expectation
    g = np.random.default_rng(5)
    n = 400
    pts = g.uniform(0.35, 0.65, size=(n, 3)).astype(np.float32)
    res = (41, 37, 45)
    roi = Roi((0, 0, 0), (1, 1, 1), res, kernel=kernel, bw="fixed", h=h, norm=norm)
    rho = oracle.density(pts, roi)
    cell = 1.0 / ((res[0] - 1) * (res[1] - 1) * (res[2] - 1))
    mass = rho.sum() * cell
    target = 1.0 if norm == "paper" else float(n)
    assert mass == pytest.approx(target, rel=2e-3)


# ---------------------------------------------------------------------------
# Gaussian blob: expected density at the centre is N (K * G)(0)
# ---------------------------------------------------------------------------

def _radial_kg(kernel, h, sig):
    ck = oracle.kernel_ck(kernel)
    rmax = h if kernel == "epanechnikov" else 3 * h

    def kval(s):
        u2 = (s / h) ** 2
        return ck / h ** 3 * ((1 - u2) if kernel == "epanechnikov" else math.exp(-0.5 * u2))

    def g(s):
        return (2 * math.pi * sig * sig) ** -1.5 * math.exp(-s * s / (2 * sig * sig))

    mu1, _ = si.quad(lambda s: kval(s) * g(s) * 4 * math.pi * s * s, 0, rmax, epsabs=0, epsrel=1e-12)
    mu2, _ = si.quad(lambda s: kval(s) ** 2 * g(s) * 4 * math.pi * s * s, 0, rmax, epsabs=0, epsrel=1e-12)
    return mu1, mu2


@pytest.mark.parametrize("kernel,h", [("epanechnikov", 0.05), ("gauss_trunc3", 0.02)])
def test_gaussian_blob_centre(kernel, h):
    sig = 0.04
    n = 40_000
    zs = []
    for seed in (11, 12, 13):
        pts = synth.blob_cloud(n, (0.5, 0.5, 0.5), sig, seed)
        roi = Roi((0.25, 0.25, 0.25), (0.75, 0.75, 0.75), (3, 3, 3), kernel=kernel,
                  bw="fixed", h=(h, h, h), norm="count")
        centre = 1 + 3 * (1 + 3 * 1)
        rho = oracle.density(pts, roi, nodes=np.array([centre]))[0]
        mu1, mu2 = _radial_kg(kernel, h, sig)
        zs.append((rho - n * mu1) / math.sqrt(n * (mu2 - mu1 * mu1)))
    assert max(abs(z) for z in zs) < 5.0
    # and the untruncated identity (K_h * G_sig)(0) = G_{sqrt(sig^2+h^2)}(0)
    # is approached when the truncation is negligible
    if kernel == "gauss_trunc3":
        mu1, _ = _radial_kg(kernel, h, sig)
        full = (2 * math.pi * (sig * sig + h * h)) ** -1.5
        assert mu1 == pytest.approx(full, rel=0.03)


# ---------------------------------------------------------------------------
# uniform interior: E[rho] = N for COUNT normalisation away from the faces
# ---------------------------------------------------------------------------

def test_uniform_interior_constant():
    n = 30_000
    pts = synth.uniform_cloud(n, 7)
    h = 0.08
    roi = Roi((0, 0, 0), (1, 1, 1), (21, 21, 21), kernel="epanechnikov", bw="fixed",
              h=(h, h, h), norm="count")
    ax = np.arange(21) / 20.0
    inner = np.nonzero((ax >= h) & (ax <= 1 - h))[0]
    ii, jj, kk = np.meshgrid(inner, inner, inner, indexing="ij")
    nodes = (ii + 21 * (jj + 21 * kk)).ravel()
    rho = oracle.density(pts, roi, nodes=nodes)
    # per-node sd = sqrt(N int K^2), int K^2 = 15 / (14 pi h^3)
    sd = math.sqrt(n * 15.0 / (14.0 * math.pi * h ** 3))
    assert abs(rho.mean() - n) < 5 * sd / math.sqrt(len(nodes) / 8.0)
    assert np.all(np.abs(rho - n) < 6 * sd)


# ---------------------------------------------------------------------------
# candidate sets: brute force in numpy float32 on tiny adversarial clouds
# ---------------------------------------------------------------------------

def _np_members(pts, node, ih, c2):
    d = np.asarray(node, dtype=np.float64) - pts.astype(np.float64)
    u = d * ih.astype(np.float64)
    s = u * u
    u2 = (s[:, 0] + s[:, 1]) + s[:, 2]
    return np.nonzero(u2 < c2)[0]


@pytest.mark.parametrize("kernel", ["epanechnikov", "gauss_trunc3"])
def test_candidates_brute_force(kernel):
    g = np.random.default_rng(3)
    base = g.uniform(0.2, 0.8, size=(60, 3)).astype(np.float32)
    extra = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.75, 0.5, 0.5],
                      [0.2, 0.2, 0.2], [1.2, 0.5, 0.5], [0.0, 0.0, 0.0]], dtype=np.float32)
    pts = np.concatenate([base, extra])
    h = (0.25, 0.2, 0.3) if kernel == "epanechnikov" else (0.08, 0.07, 0.1)
    roi = Roi((0.2, 0.2, 0.2), (0.8, 0.8, 0.8), (5, 4, 6), kernel=kernel, bw="fixed", h=h)
    nodes = np.arange(5 * 4 * 6)
    offs, idx = oracle.candidates(pts, roi, nodes)
    pos = oracle.node_positions(roi, nodes)
    ih = (1.0 / np.asarray(h, dtype=np.float32).astype(np.float64)).astype(np.float32)
    c2 = 1.0 if kernel == "epanechnikov" else 9.0
    for q in range(len(nodes)):
        ref = _np_members(pts, pos[q], ih, c2)
        assert np.array_equal(idx[offs[q]:offs[q + 1]], ref)


def test_permutation_invariance():
    pts = synth.c1_cloud(1)[:3000]
    roi = Roi((0, 0, 0), (1, 1, 1), (12, 12, 12), kernel="epanechnikov", bw="fixed",
              h=(0.07, 0.07, 0.07))
    perm = np.random.default_rng(0).permutation(len(pts))
    a = oracle.density(pts, roi)
    b = oracle.density(pts[perm], roi)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)
    nodes = np.arange(0, 12 ** 3, 37)
    oa, ia = oracle.candidates(pts, roi, nodes)
    ob, ib = oracle.candidates(pts[perm], roi, nodes)
    for q in range(len(nodes)):
        assert np.array_equal(np.sort(perm[ib[ob[q]:ob[q + 1]]]), ia[oa[q]:oa[q + 1]])


def test_in_roi_set_excludes_outside_particles():
    # a particle outside the box contributes to CLOUD but not to IN_ROI
    pts = np.array([[0.45, 0.5, 0.5], [0.52, 0.5, 0.5], [0.61, 0.5, 0.5]], dtype=np.float32)
    roi = Roi((0.4, 0.4, 0.4), (0.6, 0.6, 0.6), (3, 3, 3), kernel="epanechnikov",
              bw="fixed", h=(0.1, 0.1, 0.1), norm="count")
    node = np.array([2 + 3 * (1 + 3 * 1)])  # (0.6, 0.5, 0.5)
    c_all = oracle.support_counts(pts, roi, nodes=node)[0]
    c_in = oracle.support_counts(pts, roi.replace(set="in_roi"), nodes=node)[0]
    assert (c_all, c_in) == (2, 1)
    # the box is closed: a particle exactly on a face is inside B
    pts2 = np.array([[0.6, 0.5, 0.5], [0.5, 0.5, 0.5]], dtype=np.float32)
    lo = np.float32(0.4).astype(np.float64)
    hi = np.float32(0.6).astype(np.float64)
    roi2 = roi.replace(lo=(lo, lo, lo), hi=(hi, hi, hi), set="in_roi", h=(0.15, 0.15, 0.15))
    assert oracle.in_box_mask(pts2, roi2.lo, roi2.hi).tolist() == [True, True]
    assert oracle.support_counts(pts2, roi2, nodes=node)[0] == 2


# ---------------------------------------------------------------------------
# k-NN bandwidth
# ---------------------------------------------------------------------------

def test_knn_lattice_golden():
    rows, _ = _golden("knn_lattice.txt")
    pts = synth.lattice_cloud(9, 0.0625, 0.25)
    centre = 4 + 9 * (4 + 9 * 4)
    assert np.all(pts[centre] == np.float32(0.5))
    for k, expect in rows:
        h2 = oracle.knn_h2(pts, int(k), queries=np.array([centre]))
        assert h2[0] == np.float32(expect), k


def test_knn_matches_kdtree():
    pts = synth.c1_cloud(2)[::10].copy()
    q = np.arange(0, len(pts), 7)
    h2 = oracle.knn_h2(pts, 32, queries=q)
    d, _ = scipy.spatial.cKDTree(pts.astype(np.float64)).query(pts[q].astype(np.float64), k=33)
    np.testing.assert_allclose(h2, d[:, 32] ** 2, rtol=2e-6)


def test_knn_self_excluded_duplicates_count():
    pts = np.array([[0.1, 0.1, 0.1], [0.1, 0.1, 0.1], [0.3, 0.1, 0.1], [0.1, 0.6, 0.1]],
                   dtype=np.float32)
    h2 = oracle.knn_h2(pts, 1)
    assert h2[0] == 0.0 and h2[1] == 0.0
    assert h2[2] == np.float32(np.float32(0.2) ** 2) or abs(h2[2] - 0.04) < 1e-7
    h2 = oracle.knn_h2(pts, 3)
    with pytest.raises(ValueError):
        oracle.knn_h2(pts, 4)


# ---------------------------------------------------------------------------
# MBE stages
# ---------------------------------------------------------------------------

def test_percentile_golden_and_numpy():
    rows, extra = _golden("percentile_type7.txt")
    v = np.array(extra["values"], dtype=np.float32)
    for q, expect in rows:
        assert oracle.percentile(v, q) == pytest.approx(expect, abs=1e-15)
    x = np.random.default_rng(1).normal(size=1001).astype(np.float32)
    for q in (0.2, 0.8, 0.37):
        assert oracle.percentile(x, q) == pytest.approx(np.percentile(x.astype(np.float64), 100 * q),
                                                        abs=1e-15)


def test_eq1_uniform():
    n = 20_000
    pts = synth.uniform_cloud(n, 3)
    roi = Roi((0, 0, 0), (1, 1, 1), (64, 64, 64), bw="mbe", set="in_roi")
    ell, flags = oracle.mbe_initial_ell(pts, roi)
    # P80 - P20 -> 0.6 for uniform data, so l -> 1.2 / ln N = 0.1212
    assert flags == 0
    np.testing.assert_allclose(ell, 1.2 / math.log(n), rtol=0.02)


def test_eq1_degenerate_uses_cap():
    pts = np.array([[0.5, 0.5, 0.5]], dtype=np.float32)
    roi = Roi((0, 0, 0), (1, 1, 1), (11, 21, 41), bw="mbe", set="in_roi")
    ell, flags = oracle.mbe_initial_ell(pts, roi)
    assert flags == 7
    np.testing.assert_array_equal(ell, np.array([0.5, 0.25, 0.125], dtype=np.float32))


def test_trilinear_affine_exact():
    roi = Roi((0.1, 0.2, 0.0), (0.9, 0.7, 1.0), (9, 7, 11))
    ax = [np.linspace(roi.lo[k], roi.hi[k], roi.res[k]) for k in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    f = lambda x, y, z: 1.5 - 2.0 * x + 0.75 * y + 3.25 * z  # noqa: E731
    grid = f(x, y, z).ravel()
    g = np.random.default_rng(2)
    for _ in range(50):
        p = np.array([g.uniform(roi.lo[k], roi.hi[k]) for k in range(3)], dtype=np.float32)
        val = oracle.trilinear(grid, roi, p)
        assert val == pytest.approx(f(*p.astype(np.float64)), abs=1e-12)
    # at nodes it returns the node value, including the upper faces
    for (i, j, k) in [(0, 0, 0), (8, 6, 10), (3, 2, 5)]:
        p = np.array([ax[0][i], ax[1][j], ax[2][k]], dtype=np.float32)
        assert oracle.trilinear(grid, roi, p) == pytest.approx(f(*p.astype(np.float64)), abs=1e-12)


def test_asl_mean_and_constant_ratio():
    # a constant pilot field gives pden = aveDen everywhere, so l_kj = min(l_k, 5 s_k)
    pts = synth.uniform_cloud(2000, 4)
    roi = Roi((0, 0, 0), (1, 1, 1), (9, 9, 9), bw="mbe", set="in_roi")
    pilot = np.full(9 ** 3, 3.0)
    ell0 = np.array([0.05, 0.2, 0.9], dtype=np.float32)
    pden, ave, ell_j = oracle.mbe_asl(pts, roi, pilot, ell0)
    assert np.allclose(pden, 3.0) and ave == pytest.approx(3.0)
    expect = np.minimum(ell0.astype(np.float64), 5.0 / 8.0).astype(np.float32)
    assert np.all(ell_j == expect)
    # the mean is the arithmetic mean over the particles (numpy)
    pilot = np.random.default_rng(9).uniform(0.5, 2.0, 9 ** 3)
    pden, ave, ell_j = oracle.mbe_asl(pts, roi, pilot, ell0)
    assert ave == pytest.approx(pden.mean(), rel=1e-13)
    # zero pilot density takes the cap
    pden, ave, ell_j = oracle.mbe_asl(pts, roi, np.zeros(9 ** 3), ell0)
    assert np.all(ell_j == np.float32(5.0 / 8.0))
    # Eq. 6 on a varying field: ratio^(1/3) scaling, capped
    pilot = np.random.default_rng(9).uniform(0.5, 2.0, 9 ** 3)
    pden, ave, ell_j = oracle.mbe_asl(pts, roi, pilot, ell0)
    ref = np.minimum(ell0[None, :].astype(np.float64) * np.cbrt(ave / pden)[:, None], 5.0 / 8.0)
    np.testing.assert_allclose(ell_j, ref.astype(np.float32), rtol=0, atol=0)


def test_asl_eq6_golden():
    # hand-worked Eq. 6 (tests/golden/asl_eq6.txt): a pilot ratio of 8 doubles
    # every length (capped at 5 s), 1/8 halves it, 1 keeps it
    rows, extra = _golden("asl_eq6.txt")
    roi = Roi((0, 0, 0), (1, 1, 1), (9, 9, 9), bw="mbe", set="in_roi")
    pilot = np.ones(9 ** 3)
    pts = []
    for i, j, k, v, *_ in rows:
        pilot[int(i) + 9 * (int(j) + 9 * int(k))] = v
        pts.append([i / 8.0, j / 8.0, k / 8.0])
    pts = np.array(pts, dtype=np.float32)
    ell0 = np.array(extra["lengths"], dtype=np.float32)
    pden, ave, ell_j = oracle.mbe_asl(pts, roi, pilot, ell0)
    assert ave == extra["mean"][0]
    np.testing.assert_array_equal(pden, [r[3] for r in rows])
    np.testing.assert_allclose(ell_j, np.array([r[4:7] for r in rows]), rtol=1e-7, atol=0)


def test_mbe_all_capped_equals_fixed():
    # uniform data at 64^3: l = 1.2/ln N > 5 s, so every l_kj is the cap and the
    # final field is the fixed-bandwidth field with h = 5 s over the box particles
    n = 3000
    pts = synth.uniform_cloud(n, 8)
    roi = Roi((0, 0, 0), (1, 1, 1), (64, 64, 64), kernel="epanechnikov", bw="mbe",
              set="in_roi")
    nodes = np.arange(0, 64 ** 3, 97)
    r = oracle.mbe(pts, roi, nodes=nodes)
    cap = np.float32(5.0 / 63.0)
    assert np.all(r["ell_j"] == cap)
    fixed = roi.replace(bw="fixed", h=(cap, cap, cap))
    ref = oracle.density(pts, fixed, nodes=nodes)
    np.testing.assert_allclose(r["final"], ref, rtol=1e-13, atol=0)


def test_mbe_final_mass():
    # a compact clumpy cloud well inside the box: the adaptive field has unit mass
    g = np.random.default_rng(4)
    pts = np.concatenate([g.normal(0.5, 0.05, size=(1500, 3)),
                          g.normal(0.42, 0.03, size=(500, 3))]).astype(np.float32)
    # grid fine enough that the adaptive lengths span >= 1 node spacing
    roi = Roi((0, 0, 0), (1, 1, 1), (61, 61, 61), kernel="epanechnikov", bw="mbe",
              set="in_roi")
    r = oracle.mbe(pts, roi)
    assert r["n_b"] == 2000
    mass = r["final"].sum() / 60.0 ** 3
    assert mass == pytest.approx(1.0, rel=3e-3)
    pmass = r["pilot"].sum() / 60.0 ** 3
    assert pmass == pytest.approx(1.0, rel=3e-3)
    # adaptive lengths shrink where the pilot density is high
    hi = r["pden"] > np.median(r["pden"])
    assert r["ell_j"][hi, 0].mean() < r["ell_j"][~hi, 0].mean()


def test_roi_scaled_bandwidth():
    roi = Roi((0.25, 0.5, 0.0), (0.75, 0.625, 1.0), (8, 8, 8), bw="roi_scaled",
              h=(0.01, 0.01, 0.01))
    h = oracle.roi_h(roi)
    np.testing.assert_array_equal(
        h, np.array([np.float64(np.float32(0.01)) * s for s in (0.5, 0.125, 1.0)]).astype(np.float32))


def test_c1_oracle_full_grid_runs():
    pts = synth.c1_cloud(1)
    rho = oracle.density(pts, synth.c1_roi())
    assert rho.shape == (32 ** 3,) and np.all(rho >= 0)
    # boundary loss of the uniform half is a few percent; clusters are inside
    mass = rho.sum() / 31.0 ** 3
    assert 0.97 < mass < 1.01


def test_zero_bandwidth_has_empty_support():
    # 40 coincident particles: their 32nd-neighbour distance is 0, so their
    # bandwidth is zero and they belong to no support, not even a node at
    # their exact position; the other particles are unaffected
    pts = np.concatenate([np.full((40, 3), 0.5, np.float32), synth.uniform_cloud(200, 1)])
    h2 = oracle.knn_h2(pts, 32)
    assert np.all(h2[:40] == 0.0) and np.all(h2[40:] > 0.0)
    roi = Roi((0, 0, 0), (1, 1, 1), (5, 5, 5), kernel="gauss_trunc3", bw="per_point",
              norm="count")
    centre = np.array([2 + 5 * (2 + 5 * 2)])  # (0.5, 0.5, 0.5)
    offs, idx = oracle.candidates(pts, roi, centre, h2=h2)
    assert not np.any(idx < 40)
    assert len(idx) > 0
    assert np.isfinite(oracle.density(pts, roi, nodes=centre, h2=h2)[0])


# ---------------------------------------------------------------------------
# consumers of a density grid: trilinear density at points, selection by a
# density threshold, Marching Cubes cell classification
# ---------------------------------------------------------------------------

def _field(res, seed):
    g = np.random.default_rng(seed)
    return g.random(int(np.prod(res))).astype(np.float32) * 3.0


def test_sample_matches_scipy_trilinear():
    from scipy.interpolate import RegularGridInterpolator
    res = (7, 5, 6)
    roi = Roi((0.1, -0.3, 0.2), (0.9, 0.5, 1.4), res)
    grid = _field(res, 11)
    g = np.random.default_rng(12)
    pts = np.column_stack([g.uniform(roi.lo[k], roi.hi[k], 500) for k in range(3)]).astype(np.float32)
    pts = np.vstack([pts, np.array([roi.hi, roi.lo], np.float32)])
    axes = [np.linspace(roi.lo[k], roi.hi[k], res[k]) for k in range(3)]
    # grid is x fastest: index [z, y, x]
    f = RegularGridInterpolator(axes[::-1], grid.reshape(res[2], res[1], res[0]).astype(np.float64),
                                method="linear")
    inside = np.all((pts.astype(np.float64) >= roi.lo) & (pts.astype(np.float64) <= roi.hi), axis=1)
    ref = np.zeros(len(pts))
    ref[inside] = f(pts[inside][:, ::-1].astype(np.float64))
    got = oracle.sample_density(grid, roi, pts)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_sample_exact_at_nodes_outside_zero():
    res = (4, 3, 5)
    roi = Roi((0.0, 0.0, 0.0), (3.0, 2.0, 4.0), res)  # spacing 1: node coordinates are integers
    grid = _field(res, 13)
    nodes = np.array([[i, j, k] for k in range(5) for j in range(3) for i in range(4)], np.float32)
    assert np.array_equal(oracle.sample_density(grid, roi, nodes), grid.astype(np.float64))
    out = np.array([[-1e-3, 1, 1], [3.001, 1, 1], [1, 2.5, 1], [1, 1, -0.5]], np.float32)
    assert np.array_equal(oracle.sample_density(grid, roi, out), np.zeros(4))
    # midpoint of an edge: the mean of its two nodes
    v = oracle.sample_density(grid, roi, np.array([[1.5, 1, 2]], np.float32))[0]
    assert v == pytest.approx(0.5 * (float(grid[1 + 4 * (1 + 3 * 2)]) + float(grid[2 + 4 * (1 + 3 * 2)])), rel=1e-15)


def test_select_matches_scipy_mask_and_is_inclusive():
    from scipy.interpolate import RegularGridInterpolator
    res = (9, 8, 7)
    roi = Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), res)
    grid = _field(res, 14)
    g = np.random.default_rng(15)
    pts = g.uniform(-0.1, 1.1, size=(4000, 3)).astype(np.float32)
    axes = [np.linspace(0, 1, r) for r in res]
    f = RegularGridInterpolator(axes[::-1], grid.reshape(res[2], res[1], res[0]).astype(np.float64))
    inside = np.all((pts >= 0) & (pts <= 1), axis=1)
    vals = np.full(len(pts), -1.0)
    vals[inside] = f(pts[inside][:, ::-1].astype(np.float64))
    iso = float(np.median(vals[inside]))
    clear = np.abs(vals - iso) > 1e-9
    got = oracle.select_points(grid, roi, iso, pts)
    assert np.all(np.diff(got) > 0)
    want = np.nonzero(inside & (vals >= iso))[0]
    assert np.array_equal(np.intersect1d(got, np.nonzero(clear)[0]), np.intersect1d(want, np.nonzero(clear)[0]))
    # a point exactly at a node whose value equals the threshold is selected (>=)
    roi1 = Roi((0.0, 0.0, 0.0), (8.0, 7.0, 6.0), res)
    node = np.array([[3, 4, 2]], np.float32)
    v = float(grid[3 + 9 * (4 + 8 * 2)])
    assert list(oracle.select_points(grid, roi1, v, node)) == [0]
    assert list(oracle.select_points(grid, roi1, np.nextafter(v, 10.0), node)) == []


def test_iso_cells_closed_forms():
    res = (6, 5, 4)
    roi = Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), res)
    n = int(np.prod(res))
    # one node above the threshold: the (up to) 8 cells around it, each with
    # the bit of the corner that node is
    hot = (2, 3, 1)
    grid = np.zeros(n, np.float32)
    grid[hot[0] + 6 * (hot[1] + 5 * hot[2])] = 1.0
    cells, cases = oracle.iso_cells(grid, roi, 0.5)
    want = {}
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                ci, cj, ck = hot[0] - dx, hot[1] - dy, hot[2] - dz
                if 0 <= ci < 5 and 0 <= cj < 4 and 0 <= ck < 3:
                    want[ci + 5 * (cj + 4 * ck)] = 1 << (dx + 2 * dy + 4 * dz)
    assert list(cells) == sorted(want) and [want[c] for c in cells] == list(cases)
    # a ramp along x: only the cells whose x-edge straddles the threshold,
    # with the four dx = 1 corners set
    ramp = np.tile(np.arange(6, dtype=np.float32), 5 * 4)
    cells, cases = oracle.iso_cells(ramp, roi, 2.5)
    assert len(cells) == 4 * 3 and np.all(cells % 5 == 2) and np.all(cases == 0b10101010)
    # a constant field, and thresholds outside the range: nothing active
    assert len(oracle.iso_cells(np.full(n, 2.0, np.float32), roi, 1.0)[0]) == 0
    assert len(oracle.iso_cells(grid, roi, -1.0)[0]) == 0
    assert len(oracle.iso_cells(grid, roi, 2.0)[0]) == 0
    # the threshold itself counts as inside (>=)
    cells, cases = oracle.iso_cells(grid, roi, 1.0)
    assert len(cells) == len(want)


# ---------------------------------------------------------------------------
# Marching Cubes iso-surface (Section 4.1): closed forms on a sphere, a closed
# and consistently oriented mesh on random fields, a hand-worked cell
# ---------------------------------------------------------------------------

def _sphere_grid(res, centre, scale=1.0):
    ax = np.arange(res) / (res - 1)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return (-scale * r2).astype(np.float32).ravel()


def _area_volume(tris):
    t = tris.astype(np.float64)
    a, b, c = t[:, 0], t[:, 1], t[:, 2]
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0  # outward normals: > 0
    return area, vol


def test_iso_surface_single_cell_golden():
    # one cell, corner 0 at +1 (inside), the others at -1, iso 0: the three
    # edges at corner 0 are cut at their midpoints; the triangle is
    # (x-edge, y-edge, z-edge) = ((.5,0,0), (0,.5,0), (0,0,.5)), its normal
    # (b - a) x (c - a) = (1,1,1)/4 pointing away from the inside corner
    roi = Roi((0, 0, 0), (1, 1, 1), (2, 2, 2))
    g = -np.ones(8, dtype=np.float32)
    g[0] = 1.0
    tris = oracle.iso_surface(g, roi, 0.0)
    assert tris.shape == (1, 3, 3)
    np.testing.assert_array_equal(tris[0], [[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
    assert np.array_equal(oracle.mc_case(1), [[0, 4, 8]])
    # no surface in a cell whose corners are all inside or all outside
    assert len(oracle.mc_case(0)) == 0 and len(oracle.mc_case(255)) == 0


@pytest.mark.parametrize("res", [33, 65])
def test_iso_surface_sphere_area_volume(res):
    # f = -|x - c|^2, iso = -R^2: a sphere of radius R; the mesh's area and
    # enclosed volume (divergence theorem) converge to 4 pi R^2 and
    # 4/3 pi R^3 with the square of the spacing
    R = 0.3
    c = (0.5, 0.47, 0.52)
    roi = Roi((0, 0, 0), (1, 1, 1), (res, res, res))
    tris = oracle.iso_surface(_sphere_grid(res, c), roi, -R * R)
    area, vol = _area_volume(tris)
    s = 1.0 / (res - 1)
    ea = abs(area / (4 * math.pi * R * R) - 1)
    ev = abs(vol / (4 / 3 * math.pi * R ** 3) - 1)
    bound = 2.0 * (s / R) ** 2
    assert ea < bound and ev < bound, (ea, ev, bound)


def _directed_edges(tris):
    v = tris.reshape(-1, 3, 3)
    keys = {}
    for t in v:
        pts = [tuple(p) for p in t]
        for i in range(3):
            e = (pts[i], pts[(i + 1) % 3])
            keys[e] = keys.get(e, 0) + 1
    return keys


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_iso_surface_closed_and_oriented(seed):
    # a random smooth field that is below iso on the grid's faces: every
    # mesh edge is shared by exactly two triangles traversing it in opposite
    # directions (closed, consistently oriented; ambiguous faces are
    # resolved alike by the two cells that share them); Euler
    # characteristic V - E + F = 2 per closed component without handles
    res = 21
    g = np.random.default_rng(seed)
    f = g.standard_normal((res, res, res))
    for _ in range(2):  # smooth a little
        f = (f + np.roll(f, 1, 0) + np.roll(f, 1, 1) + np.roll(f, 1, 2)) / 4
    f[0, :, :] = f[-1, :, :] = f[:, 0, :] = f[:, -1, :] = f[:, :, 0] = f[:, :, -1] = -10.0
    roi = Roi((0, 0, 0), (1, 1, 1), (res, res, res))
    tris = oracle.iso_surface(f.astype(np.float32).ravel(), roi, 0.05)
    assert len(tris) > 100
    d = _directed_edges(tris)
    for (a, b), k in d.items():
        assert k == 1, "directed edge used %d times" % k
        assert d.get((b, a), 0) == 1, "edge without its opposite"
    verts = {p for t in tris for p in map(tuple, t)}
    E = len(d) // 2
    chi = len(verts) - E + len(tris)
    assert chi % 2 == 0
    # volume enclosed is positive with outward normals
    assert _area_volume(tris)[1] > 0


def test_iso_surface_two_spheres_euler():
    res = 41
    roi = Roi((0, 0, 0), (1, 1, 1), (res, res, res))
    # centres and radius off the lattice, so no node value equals iso
    a = _sphere_grid(res, (0.3103, 0.4971, 0.5033))
    b = _sphere_grid(res, (0.7211, 0.5087, 0.4923))
    f = np.maximum(a, b)
    tris = oracle.iso_surface(f, roi, -0.1487 ** 2)
    d = _directed_edges(tris)
    assert all(k == 1 and d.get((b_, a_), 0) == 1 for (a_, b_), k in d.items())
    verts = {p for t in tris for p in map(tuple, t)}
    assert len(verts) - len(d) // 2 + len(tris) == 4  # two spheres
