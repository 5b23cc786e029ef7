"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Densities: max relative error 1e-5 at nodes with rho >= 1e-3 of the peak,
absolute error <= 1e-8 of the peak elsewhere. Support sets and counts:
bit-exact. k-NN bandwidths and Eq. 1 lengths: bit-exact. ASL stages:
1e-6 relative given the GPU's verified upstream arrays.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import Roi

pytestmark = pytest.mark.gpu

from gpu_common import (ABS_TOL, REL_TOL, check_density, check_sampled, ctx, dev,  # noqa: F401
                        sample_nodes, say, sfk, torch)


# ---------------------------------------------------------------------------
# C1: 20k points, 32^3, Epanechnikov, fixed h = 0.02 (full grid)
# ---------------------------------------------------------------------------

def test_c1_full_grid(ctx, torch):
    pts = synth.c1_cloud(1)
    roi = synth.c1_roi()
    tree = ctx.build_tree(dev(torch, pts))
    out = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.density(pts, roi)
    err = check_density(got, ref, "c1")
    say("c1 max rel err", err)
    # support counts of every node, from the evaluation kernel itself
    cnt = ctx.debug_support_counts(tree, roi)
    torch.cuda.synchronize()
    ref_cnt = oracle.support_counts(pts, roi)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), ref_cnt)
    # support sets of sampled nodes, bit-exact
    nodes = sample_nodes(None, roi.n_nodes, 200, 5, extra=[0, roi.n_nodes - 1, int(np.argmax(ref))])
    for a, b in [(int(n), int(n) + 1) for n in nodes[:60]] + [(1000, 1100)]:
        offs, idx = ctx.debug_candidates(tree, roi, a, b)
        ro, ri = oracle.candidates(pts, roi, np.arange(a, b))
        assert np.array_equal(offs, ro) and np.array_equal(idx, ri), (a, b)
    # useful pairs = sum of support sizes
    useful, tested = ctx.debug_eval_count(tree, roi)
    assert useful == int(ref_cnt.sum()) and tested >= useful


@pytest.mark.parametrize("kernel,h,norm", [
    ("gauss_trunc3", (0.01, 0.01, 0.01), "count"),
    ("epanechnikov", (0.05, 0.03, 0.04), "paper"),
    ("gauss_trunc3", (0.004, 0.006, 0.005), "paper"),
])
def test_c1_kernels_and_norms(ctx, torch, kernel, h, norm):
    pts = synth.c1_cloud(1)
    roi = Roi((0, 0, 0), (1, 1, 1), (29, 31, 33), kernel=kernel, bw="fixed", h=h, norm=norm)
    tree = ctx.build_tree(dev(torch, pts))
    got = ctx.eval_roi(tree, roi).cpu().numpy()
    check_density(got, oracle.density(pts, roi), "%s %s" % (kernel, h))
    cnt = ctx.debug_support_counts(tree, roi).cpu().numpy().astype(np.int64)
    assert np.array_equal(cnt, oracle.support_counts(pts, roi))


def test_ragged_subbox_roi_scaled(ctx, torch):
    pts = synth.c1_cloud(3)
    for roi in [
        Roi((0.1, 0.2, 0.3), (0.45, 0.9, 0.5), (13, 7, 9), bw="roi_scaled", h=(0.1, 0, 0)),
        Roi((0.3, 0.3, 0.3), (0.31, 0.32, 0.305), (5, 6, 7), bw="roi_scaled", h=(0.5, 0, 0)),
        Roi((-0.2, 0.5, 0.9), (0.3, 1.3, 1.4), (17, 2, 3), bw="fixed", h=(0.05, 0.05, 0.05)),
    ]:
        tree = ctx.build_tree(dev(torch, pts))
        got = ctx.eval_roi(tree, roi).cpu().numpy()
        check_density(got, oracle.density(pts, roi), str(roi.res))
        cnt = ctx.debug_support_counts(tree, roi).cpu().numpy().astype(np.int64)
        assert np.array_equal(cnt, oracle.support_counts(pts, roi))


def test_support_boundary_golden(ctx, torch):
    import os
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "support_boundary.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    pts = np.array([r[:3] for r in rows], dtype=np.float32)
    member = np.array([int(r[3]) for r in rows])
    roi = Roi((0, 0, 0), (1, 1, 1), (5, 5, 5), bw="fixed", h=(0.25, 0.25, 0.25), norm="count")
    tree = ctx.build_tree(dev(torch, pts))
    node = 2 + 5 * (2 + 5 * 2)
    offs, idx = ctx.debug_candidates(tree, roi, node, node + 1)
    assert np.array_equal(np.sort(idx), np.nonzero(member)[0])
    cnt = ctx.debug_support_counts(tree, roi).cpu().numpy()
    assert int(cnt[node]) == int(member.sum())


def test_empty_single_and_degenerate_clouds(ctx, torch):
    roi = Roi((0, 0, 0), (1, 1, 1), (9, 10, 11), bw="fixed", h=(0.3, 0.2, 0.25))
    # empty cloud: every node zero
    tree = ctx.build_tree(torch.zeros((0, 3), dtype=torch.float32, device="cuda"))
    got = ctx.eval_roi(tree, roi).cpu().numpy()
    assert np.all(got == 0)
    # one particle: the kernel profile
    p = np.array([[0.37, 0.52, 0.61]], dtype=np.float32)
    tree = ctx.build_tree(dev(torch, p))
    check_density(ctx.eval_roi(tree, roi).cpu().numpy(), oracle.density(p, roi), "single")
    # all particles coincident, some on grid nodes and on faces
    p = np.concatenate([np.full((300, 3), 0.5, np.float32),
                        np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.125, 0.5, 1.0]], np.float32)])
    tree = ctx.build_tree(dev(torch, p))
    for r in [roi, roi.replace(res=(9, 9, 9), h=(0.125, 0.125, 0.125))]:
        check_density(ctx.eval_roi(tree, r).cpu().numpy(), oracle.density(p, r), "coincident")
        cnt = ctx.debug_support_counts(tree, r).cpu().numpy().astype(np.int64)
        assert np.array_equal(cnt, oracle.support_counts(p, r))
    # a ROI far from every particle
    far = roi.replace(lo=(5, 5, 5), hi=(6, 6, 6))
    assert np.all(ctx.eval_roi(tree, far).cpu().numpy() == 0)


def test_determinism_and_permutation(ctx, torch):
    pts = synth.c1_cloud(4)
    roi = Roi((0, 0, 0), (1, 1, 1), (24, 24, 24), bw="fixed", h=(0.04, 0.04, 0.04))
    tree = ctx.build_tree(dev(torch, pts))
    a = ctx.eval_roi(tree, roi).cpu().numpy()
    b = ctx.eval_roi(tree, roi).cpu().numpy()
    assert np.array_equal(a, b)
    perm = np.random.default_rng(1).permutation(len(pts))
    tree2 = ctx.build_tree(dev(torch, pts[perm]))
    c = ctx.eval_roi(tree2, roi).cpu().numpy()
    check_density(c, oracle.density(pts, roi), "permuted")
    node = 12 + 24 * (12 + 24 * 12)
    o1, i1 = ctx.debug_candidates(tree, roi, node, node + 1)
    o2, i2 = ctx.debug_candidates(tree2, roi, node, node + 1)
    assert np.array_equal(np.sort(perm[i2]), i1)


@pytest.mark.parametrize("curve", ["hilbert", "morton"])
def test_tree_order_follows_curve_keys(ctx, sfk, torch, curve):
    # one particle at the centre of each cell of a 16^3 lattice, shuffled:
    # with 4 key bits every particle quantises to its own cell, so the
    # device sort must give the order of the host-side keys
    c = 16
    g = np.stack(np.meshgrid(np.arange(c), np.arange(c), np.arange(c), indexing="ij"),
                 -1).reshape(-1, 3)
    perm = np.random.default_rng(5).permutation(len(g))
    cells = g[perm]
    pts = ((cells + 0.5) / c).astype(np.float32)
    tree = ctx.build_tree(dev(torch, pts), key_bits=4, curve=curve)
    order = ctx.debug_tree_order(tree)
    keys = sfk.curve_keys(curve, 4, cells)
    assert np.array_equal(order, np.argsort(keys))
    if curve == "hilbert":
        assert np.all(np.abs(np.diff(cells[order], axis=0)).sum(1) == 1)
    tree.close()


def quantise_like_device(pts, bbox, bits):
    """The build's float32 cell of every particle: (x - lo) * (2^bits / extent),
    each operation rounded to float32, truncated and clamped to the lattice."""
    lo = np.array(bbox[:3], dtype=np.float32)
    ext = np.array(bbox[3:], dtype=np.float32) - lo
    cells = np.float32(1 << bits)
    sc = np.where(ext > 0, cells / np.where(ext > 0, ext, np.float32(1)), np.float32(0))
    f = (pts.astype(np.float32) - lo) * sc.astype(np.float32)
    qmax = (1 << bits) - 1
    q = np.where(f <= 0, 0, np.where(f >= np.float32(qmax), qmax,
                                     np.floor(np.maximum(f, 0)).astype(np.int64)))
    return q.astype(np.uint32)


@pytest.mark.parametrize("curve", ["hilbert", "morton"])
def test_tree_order_exact_at_every_key_width(ctx, sfk, torch, curve):
    # ragged cloud (not a multiple of the sort tile); 1 bit per axis gives
    # 8 cells and massive ties (stable: input order), 21 bits 63-bit keys
    # (eight passes, the 64-bit path), the automatic width 10 bits (four
    # passes, the 32-bit path)
    pts = synth.clumpy_cloud(50_003, 31)
    for bits in (1, 0, 21):
        tree = ctx.build_tree(dev(torch, pts), key_bits=bits, curve=curve)
        n, bbox, _ = tree.info()
        b = bits or 10
        keys = sfk.curve_keys(curve, b, quantise_like_device(pts, bbox, b))
        order = ctx.debug_tree_order(tree)
        assert np.array_equal(order, np.argsort(keys, kind="stable")), (curve, bits)
        tree.close()


def test_morton_curve_parity(ctx, sfk, torch):
    pts = synth.clumpy_cloud(30_000, 5)
    tree = ctx.build_tree(dev(torch, pts), knn_k=16, curve="morton")
    h2 = ctx.debug_point_h2(tree)
    assert np.array_equal(h2, oracle.knn_h2(pts, 16))
    roi = Roi((0.1, 0, 0.05), (0.9, 1, 0.95), (29, 31, 26), kernel="gauss_trunc3",
              bw="per_point")
    check_density(ctx.eval_roi(tree, roi).cpu().numpy(), oracle.density(pts, roi, h2=h2),
                  "morton per-point")
    fixed = Roi((0, 0, 0), (1, 1, 1), (30, 30, 30), bw="fixed", h=(0.04, 0.04, 0.04))
    check_density(ctx.eval_roi(tree, fixed).cpu().numpy(), oracle.density(pts, fixed),
                  "morton fixed")
    tree.close()
    for kw in (dict(curve=2), dict(key_bits=22), dict(key_bits=-1)):
        with pytest.raises(sfk.SfkError) as e:
            ctx.build_tree(dev(torch, pts[:1000]), **kw)
        assert e.value.status == 1, kw


# ---------------------------------------------------------------------------
# chunk splitting and the in-kernel tree walk (lists that do not fit)
# ---------------------------------------------------------------------------

def test_split_chunks_and_walk_fallback_bitwise(ctx, torch):
    pts = synth.clumpy_cloud(60_000, 7)
    roi = Roi((0.2, 0.2, 0.2), (0.8, 0.8, 0.8), (40, 40, 40), bw="fixed", h=(0.05, 0.05, 0.05))
    tree = ctx.build_tree(dev(torch, pts))
    ref = oracle.density(pts, roi)
    outs = {}
    for label, kw in [("default", {}), ("chunks4", {"chunk_leaves": 4}),
                      ("walk4", {"chunk_leaves": 4, "list_capacity": 1}),
                      ("walk64", {"list_capacity": 1}),
                      ("chunkwalk4", {"chunk_leaves": 4, "list_capacity": 1,
                                      "partial_capacity": 1 << 20}),
                      ("mixed4", {"chunk_leaves": 4, "list_capacity": 3000,
                                  "partial_capacity": 1500})]:
        ctx.set_eval_opts(**kw)
        outs[label] = ctx.eval_roi(tree, roi).cpu().numpy()
        check_density(outs[label], ref, label)
    ctx.set_eval_opts()
    # the tree walks (per tile, per chunk, and a mix of lists and both
    # walks) reproduce the stored-list results bit for bit
    assert np.array_equal(outs["chunks4"], outs["walk4"])
    assert np.array_equal(outs["chunks4"], outs["chunkwalk4"])
    assert np.array_equal(outs["chunks4"], outs["mixed4"])
    assert np.array_equal(outs["default"], outs["walk64"])


def test_roi_lists_and_tile_slots_match_walks_bitwise(ctx, torch):
    # small boxes reach few leaves: every tile takes its candidates from the
    # ROI's leaf list and the fill pass copies the count pass's slots; the
    # in-kernel walk (no stored lists at all) must give the same bits
    pts = synth.clumpy_cloud(200_000, 11)
    tree = ctx.build_tree(dev(torch, pts))
    c = pts[np.argmax(np.linalg.norm(pts - pts.mean(0), axis=1) < 0.3)]
    rois = [Roi(*synth.box_around(c, side), (res, res, res), kernel=k, bw="fixed",
                h=(0.2 * side,) * 3)
            for side, res, k in ((0.02, 33, "epanechnikov"), (0.05, 40, "gauss_trunc3"),
                                 (0.1, 24, "epanechnikov"))]
    for r in rois:
        ctx.set_eval_opts()
        a = ctx.eval_roi(tree, r).cpu().numpy()
        ctx.set_eval_opts(list_capacity=1)
        b = ctx.eval_roi(tree, r).cpu().numpy()
        ctx.set_eval_opts()
        assert np.array_equal(a, b), r
        nodes = sample_nodes(a, r.n_nodes, 24, 1)
        check_sampled(a, nodes, oracle.density(pts, r, nodes=nodes), "small box")
    tree.close()
    # wide supports: tiles overlap more leaves than the count pass keeps, so
    # the fill pass walks again for them (a node whose support holds more
    # than 256 leaves' worth of particles proves that its tile does)
    wpts = synth.uniform_cloud(40_000, 12)
    wide = ctx.build_tree(dev(torch, wpts))
    r = Roi((0, 0, 0), (1, 1, 1), (21, 22, 23), kernel="epanechnikov", bw="fixed",
            h=(0.5,) * 3)
    cnt = ctx.debug_support_counts(wide, r).cpu().numpy().astype(np.int64)
    assert cnt.max() > 256 * 64
    a = ctx.eval_roi(wide, r).cpu().numpy()
    ctx.set_eval_opts(list_capacity=1)
    b = ctx.eval_roi(wide, r).cpu().numpy()
    ctx.set_eval_opts()
    assert np.array_equal(a, b)
    nodes = sample_nodes(a, r.n_nodes, 24, 2)
    check_sampled(a, nodes, oracle.density(wpts, r, nodes=nodes), "wide supports")
    wide.close()


# ---------------------------------------------------------------------------
# per-point bandwidth (k-NN), Gaussian truncated at 3h
# ---------------------------------------------------------------------------

def test_knn_h2_bit_exact_and_lattice(ctx, torch):
    pts = synth.clumpy_cloud(30_000, 2)
    tree = ctx.build_tree(dev(torch, pts), knn_k=32)
    h2 = ctx.debug_point_h2(tree)
    ref = oracle.knn_h2(pts, 32)
    assert np.array_equal(h2, ref), np.nonzero(h2 != ref)[0][:10]
    lat = synth.lattice_cloud(9, 0.0625, 0.25)
    tree = ctx.build_tree(dev(torch, lat), knn_k=32)
    h2 = ctx.debug_point_h2(tree)
    assert h2[4 + 9 * (4 + 9 * 4)] == np.float32(0.015625)
    assert np.array_equal(h2, oracle.knn_h2(lat, 32))
    # k = 8, 16 (below), 32 and 64 fill the query leaf by sorting networks,
    # k = 1 and 7 by insertion
    for k in (1, 7, 8, 64):
        tree = ctx.build_tree(dev(torch, pts[:5000]), knn_k=k)
        assert np.array_equal(ctx.debug_point_h2(tree), oracle.knn_h2(pts[:5000], k)), k


def test_per_point_gauss_density(ctx, torch):
    pts = synth.clumpy_cloud(40_000, 3)
    roi = Roi((0, 0, 0), (1, 1, 1), (33, 30, 27), kernel="gauss_trunc3", bw="per_point")
    tree = ctx.build_tree(dev(torch, pts), knn_k=32)
    h2 = ctx.debug_point_h2(tree)
    got = ctx.eval_roi(tree, roi).cpu().numpy()
    ref = oracle.density(pts, roi, h2=h2)
    check_density(got, ref, "per-point gauss")
    cnt = ctx.debug_support_counts(tree, roi).cpu().numpy().astype(np.int64)
    assert np.array_equal(cnt, oracle.support_counts(pts, roi, h2=h2))
    nodes = [int(np.argmax(ref)), 0, 5000, 12345]
    for n in nodes:
        o, i = ctx.debug_candidates(tree, roi, n, n + 1)
        ro, ri = oracle.candidates(pts, roi, np.array([n]), h2=h2)
        assert np.array_equal(i, ri)
    # Epanechnikov with the same per-point bandwidths
    r2 = roi.replace(kernel="epanechnikov")
    check_density(ctx.eval_roi(tree, r2).cpu().numpy(), oracle.density(pts, r2, h2=h2), "pp epan")


def test_zero_bandwidth_particles(ctx, torch):
    pts = np.concatenate([np.full((40, 3), 0.5, np.float32), synth.uniform_cloud(3000, 1)])
    roi = Roi((0, 0, 0), (1, 1, 1), (9, 9, 9), kernel="gauss_trunc3", bw="per_point")
    tree = ctx.build_tree(dev(torch, pts), knn_k=32)
    h2 = ctx.debug_point_h2(tree)
    assert np.array_equal(h2, oracle.knn_h2(pts, 32))
    check_density(ctx.eval_roi(tree, roi).cpu().numpy(), oracle.density(pts, roi, h2=h2), "zero-h")
    centre = 4 + 9 * (4 + 9 * 4)
    _, idx = ctx.debug_candidates(tree, roi, centre, centre + 1)
    _, ridx = oracle.candidates(pts, roi, np.array([centre]), h2=h2)
    assert np.array_equal(idx, ridx) and not np.any(idx < 40)


def test_user_given_bandwidth(ctx, torch):
    pts = synth.c1_cloud(5)[:8000].copy()
    h = np.random.default_rng(2).uniform(0.01, 0.05, size=len(pts)).astype(np.float32)
    roi = Roi((0, 0, 0), (1, 1, 1), (21, 21, 21), kernel="epanechnikov", bw="per_point")
    tree = ctx.build_tree(dev(torch, pts), h=dev(torch, h))
    got = ctx.eval_roi(tree, roi).cpu().numpy()
    ih, w = oracle.params_from_h(h)
    ref = oracle.density_raw(pts, roi, "epanechnikov", oracle.kernel_ck("epanechnikov") / len(pts),
                             ih_pp=ih, w_pp=w)
    check_density(got, ref, "user h")


# ---------------------------------------------------------------------------
# particles inside B only, and the MBE chain
# ---------------------------------------------------------------------------

def test_in_roi_set(ctx, torch):
    pts = synth.c1_cloud(6)
    roi = Roi((0.25, 0.3, 0.2), (0.7, 0.8, 0.6), (19, 21, 17), bw="fixed", h=(0.04, 0.04, 0.04),
              set="in_roi")
    tree = ctx.build_tree(dev(torch, pts))
    check_density(ctx.eval_roi(tree, roi).cpu().numpy(), oracle.density(pts, roi), "in_roi")
    tree = ctx.build_tree(dev(torch, pts), knn_k=16)
    h2 = ctx.debug_point_h2(tree)
    r2 = roi.replace(bw="per_point", kernel="gauss_trunc3")
    check_density(ctx.eval_roi(tree, r2).cpu().numpy(), oracle.density(pts, r2, h2=h2), "in_roi pp")


def test_in_roi_edge_boxes(ctx, torch):
    # the in-box set is taken from the leaves whose box meets B: a box that
    # meets none, and a box around a single particle
    pts = synth.c1_cloud(7)
    tree = ctx.build_tree(dev(torch, pts))
    far = Roi((2, 2, 2), (3, 3, 3), (9, 9, 9), bw="fixed", h=(0.1, 0.1, 0.1), set="in_roi")
    assert float(ctx.eval_roi(tree, far).abs().max()) == 0.0
    d = ctx.debug_mbe(tree, far.replace(bw="mbe"), per_particle=False)
    assert d["n_b"] == 0 and float(d["final"].abs().max()) == 0.0
    p = pts[1234].astype(np.float64)
    one = Roi(tuple(p - 1e-6), tuple(p + 1e-6), (5, 5, 5), bw="fixed", h=(1e-5,) * 3,
              set="in_roi")
    inside = np.all((pts.astype(np.float64) >= np.array(one.lo)) &
                    (pts.astype(np.float64) <= np.array(one.hi)), axis=1)
    assert inside.sum() >= 1
    check_density(ctx.eval_roi(tree, one).cpu().numpy(), oracle.density(pts, one), "one particle")
    d = ctx.debug_mbe(tree, one.replace(bw="mbe"))
    assert d["n_b"] == int(inside.sum())
    assert np.array_equal(d["idx_b"], np.nonzero(inside)[0])
    tree.close()


@pytest.mark.parametrize("case", ["full", "sub", "tiny"])
def test_mbe_stagewise(ctx, torch, case):
    pts = synth.clumpy_cloud(50_000, 11)
    if case == "full":
        roi = Roi((0, 0, 0), (1, 1, 1), (32, 32, 32), bw="mbe", set="in_roi")
    elif case == "sub":
        roi = Roi((0.2, 0.25, 0.3), (0.7, 0.75, 0.9), (24, 20, 28), bw="mbe", set="in_roi")
    else:
        roi = Roi((0.5, 0.5, 0.5), (0.52, 0.52, 0.52), (8, 8, 8), bw="mbe", set="in_roi")
    tree = ctx.build_tree(dev(torch, pts))
    d = ctx.debug_mbe(tree, roi)
    torch.cuda.synchronize()
    inc = oracle.in_box_mask(pts, roi.lo, roi.hi)
    idx_b = np.nonzero(inc)[0]
    assert d["n_b"] == len(idx_b) and np.array_equal(d["idx_b"], idx_b)
    if len(idx_b) == 0:
        assert np.all(d["final"].cpu().numpy() == 0)
        return
    pts_b = pts[idx_b]
    # Eq. 1: bit-exact
    ell0, _ = oracle.mbe_initial_ell(pts_b, roi)
    assert np.array_equal(d["ell0"], ell0)
    # pilot grid against the oracle's own pilot
    full = oracle.mbe(pts, roi)
    check_density(d["pilot"], full["pilot"], "pilot")
    # ASL given the GPU pilot
    pden, ave, ell_j = oracle.mbe_asl(pts_b, roi, d["pilot"].astype(np.float64), ell0)
    np.testing.assert_allclose(d["pden"], pden, rtol=1e-6, atol=1e-12 * max(pden.max(), 1e-30))
    assert d["aveden"] == pytest.approx(ave, rel=1e-6)
    np.testing.assert_allclose(d["ell_j"], ell_j, rtol=1e-6)
    # final density given the GPU's adaptive lengths
    ref = oracle.mbe(pts, roi, ell_j_in=d["ell_j"])["final"]
    check_density(d["final"].cpu().numpy(), ref, "final")
    # and the plain evaluation entry point gives the same grid
    again = ctx.eval_roi(tree, roi).cpu().numpy()
    assert np.array_equal(again, d["final"].cpu().numpy())


@pytest.mark.parametrize("side,res", [(0.03, 64), (0.06, 96)])
def test_mbe_at_scale_sampled(ctx, torch, side, res):
    # the MBE chain on a 10M-point cloud, in a box around its most massive
    # clump (8e4-3e5 particles in B): every stage against the oracle, the
    # grids on sampled nodes (a full oracle grid would take hours)
    pts, info = synth.clumpy_cloud(10_000_000, 3, with_info=True)
    c = info.centres[int(np.argmax(info.counts))]
    roi = Roi(tuple(c - side / 2), tuple(c + side / 2), (res,) * 3, bw="mbe", set="in_roi")
    tree = ctx.build_tree(dev(torch, pts))
    d = ctx.debug_mbe(tree, roi, cap_b=4_000_000)
    torch.cuda.synchronize()
    idx_b = np.nonzero(oracle.in_box_mask(pts, roi.lo, roi.hi))[0]
    say("mbe at scale: N_B =", len(idx_b))
    assert d["n_b"] == len(idx_b) > 50_000 and np.array_equal(d["idx_b"], idx_b)
    pts_b = pts[idx_b]
    ell0, _ = oracle.mbe_initial_ell(pts_b, roi)
    assert np.array_equal(d["ell0"], ell0)  # Eq. 1, bit-exact
    scale = oracle.kernel_ck("epanechnikov") * oracle._nu(roi, len(idx_b))
    ih, w = oracle.uniform_params(ell0)
    pilot = d["pilot"].astype(np.float64)
    nodes = sample_nodes(None, roi.n_nodes, 64, 7, extra=[int(np.argmax(pilot))])
    want = oracle.density_raw(pts_b, roi, "epanechnikov", scale, ih_u=ih, w_u=w, nodes=nodes)
    check_sampled(pilot, nodes, want, "pilot at scale")
    # Eqs. 5-6 given the GPU pilot, every particle of B
    pden, ave, ell_j = oracle.mbe_asl(pts_b, roi, pilot, ell0)
    np.testing.assert_allclose(d["pden"], pden, rtol=1e-6, atol=1e-12 * max(pden.max(), 1e-30))
    assert d["aveden"] == pytest.approx(ave, rel=1e-6)
    np.testing.assert_allclose(d["ell_j"], ell_j, rtol=1e-6)
    # Eq. 7 given the GPU's adaptive lengths, on sampled nodes
    final = d["final"].cpu().numpy()
    nodes = sample_nodes(None, roi.n_nodes, 64, 8, extra=[int(np.argmax(final))])
    ref = oracle.mbe(pts, roi, nodes=nodes, pilot_in=pilot, ell_j_in=d["ell_j"])["final"]
    check_sampled(final, nodes, ref, "final at scale")
    tree.close()


# ---------------------------------------------------------------------------
# batches: each grid is the same alone and in the mix
# ---------------------------------------------------------------------------

def test_batch_alone_vs_mix(ctx, torch):
    pts = synth.clumpy_cloud(200_000, 4)
    tree = ctx.build_tree(dev(torch, pts))
    rois = synth.random_batch_rois(24, seed=9, side_lo=0.02, res_lo=8, res_hi=40, h0=0.03)
    outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in rois]
    t = ctx.submit(tree, rois, outs)
    ctx.wait(t)
    for i, r in enumerate(rois):
        alone = ctx.eval_roi(tree, r).cpu().numpy()
        mixed = outs[i].cpu().numpy()
        assert np.array_equal(alone, mixed), i
    # sampled nodes of every ROI against the oracle
    for i, r in enumerate(rois[:8]):
        nodes = sample_nodes(None, r.n_nodes, 24, i)
        check_sampled(outs[i].cpu().numpy(), nodes, oracle.density(pts, r, nodes=nodes), "batch")
    # a batch mixing kernels and bandwidth modes, and polling
    tree2 = ctx.build_tree(dev(torch, pts[:50_000]), knn_k=32)
    mix = [rois[0], rois[1].replace(kernel="gauss_trunc3"),
           rois[2].replace(bw="per_point", kernel="gauss_trunc3"),
           rois[3].replace(set="in_roi", bw="fixed", h=(0.02, 0.02, 0.02))]
    outs2 = [torch.zeros((r.n_nodes,), device="cuda") for r in mix]
    t2 = ctx.submit(tree2, mix, outs2)
    while not ctx.poll(t2):
        pass
    ctx.wait(t2)
    for r, o in zip(mix, outs2):
        assert np.array_equal(o.cpu().numpy(), ctx.eval_roi(tree2, r).cpu().numpy())


def test_errors(ctx, torch, sfk):
    pts = synth.c1_cloud(1)[:1000].copy()
    tree = ctx.build_tree(dev(torch, pts))
    bad = [synth.c1_roi().replace(res=(1, 4, 4)), synth.c1_roi().replace(lo=(1, 0, 0)),
           synth.c1_roi().replace(h=(0.0, 0.1, 0.1)), synth.c1_roi().replace(bw="per_point"),
           synth.c1_roi().replace(bw="mbe")]
    for r in bad:
        out = torch.zeros(max(1, r.n_nodes), device="cuda")
        with pytest.raises(sfk.SfkError) as e:
            ctx._check(ctx._lib.sfk_eval_roi(ctx._h, tree._h,
                                             __import__("ctypes").byref(sfk.roi_struct(r, out.data_ptr())),
                                             None))
        assert e.value.name == "SFK_E_INVAL"
    with pytest.raises(sfk.SfkError) as e:
        ctx.eval_roi(tree, synth.c1_roi().replace(bw="mbe", set="in_roi", kernel="gauss_trunc3"))
    assert e.value.name == "SFK_E_UNSUPPORTED"
    nanpts = pts.copy()
    nanpts[5, 1] = np.nan
    with pytest.raises(sfk.SfkError):
        ctx.build_tree(dev(torch, nanpts))
    with pytest.raises(sfk.SfkError):
        ctx.build_tree(dev(torch, pts[:10]), knn_k=32)
    r = synth.c1_roi()
    shared = torch.zeros(r.n_nodes + 10, device="cuda")
    with pytest.raises(sfk.SfkError):
        ctx.submit(tree, [r, r], [shared[:r.n_nodes], shared[10:]])
    # the context stays usable after errors
    check_density(ctx.eval_roi(tree, r).cpu().numpy(), oracle.density(pts, r), "after errors")


@pytest.mark.gpu
def test_non_finite_coordinates_fail_every_build_path(ctx, torch, sfk):
    """A non-finite coordinate fails the build with SFK_E_INVAL on every
    bandwidth path (found at the build's end; the k-NN returns at once on
    such a cloud), and the next build on the same context is correct."""
    pts = synth.uniform_cloud(5000, 7)
    h = torch.full((len(pts),), 0.02, device="cuda")
    for bad in (np.nan, np.inf, -np.inf):
        for where in (0, 2500, 4999):
            cloud = pts.copy()
            cloud[where, where % 3] = bad
            for kw in (dict(), dict(knn_k=32), dict(knn_k=8, curve="morton"), dict(h=h)):
                with pytest.raises(sfk.SfkError) as e:
                    ctx.build_tree(dev(torch, cloud), **kw)
                assert e.value.name == "SFK_E_INVAL", (bad, where, kw)
                assert "non-finite" in str(e.value), (bad, where, kw)
    tree = ctx.build_tree(dev(torch, pts), knn_k=32)
    h2 = ctx.debug_point_h2(tree)
    assert np.array_equal(h2, oracle.knn_h2(pts, 32))
    roi = Roi((0, 0, 0), (1, 1, 1), (17, 19, 21), kernel="gauss_trunc3", bw="per_point")
    check_density(ctx.eval_roi(tree, roi).cpu().numpy(), oracle.density(pts, roi, h2=h2),
                  "after non-finite clouds")


# ---------------------------------------------------------------------------
# the benchmarked workload at full size: 10M clumpy points, 128^3, Gaussian
# truncated at 3h, per-point h from the 32nd neighbour (sampled checks)
# ---------------------------------------------------------------------------

def test_full_size_per_point_workload(ctx, torch):
    pts = synth.clumpy_cloud(10_000_000, 2)
    say("generated 10M")
    roi = synth.c2_roi(128)
    tree = ctx.build_tree(dev(torch, pts), knn_k=32)
    torch.cuda.synchronize()
    say("tree + kNN built")
    h2 = ctx.debug_point_h2(tree)
    q = np.random.default_rng(3).choice(len(pts), size=48, replace=False)
    assert np.array_equal(h2[q], oracle.knn_h2(pts, 32, queries=q))
    say("kNN sample exact")
    out = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    am = int(np.argmax(got))
    above = np.nonzero(got >= 1e-3 * got.max())[0]
    g = np.random.default_rng(4)
    nodes = np.unique(np.concatenate([[am], g.choice(roi.n_nodes, 24, replace=False),
                                      g.choice(above, 24, replace=False)]))
    ref = oracle.density(pts, roi, nodes=nodes, h2=h2)
    peak = max(ref.max(), got.max())
    big = ref >= 1e-3 * peak
    rel = np.abs(got[nodes][big] - ref[big]) / ref[big]
    assert rel.max() <= REL_TOL, rel.max()
    assert np.max(np.abs(got[nodes][~big] - ref[~big]), initial=0) <= ABS_TOL * peak
    say("density sample max rel err", rel.max())
    for n in nodes[:6]:
        o, i = ctx.debug_candidates(tree, roi, int(n), int(n) + 1)
        ro, ri = oracle.candidates(pts, roi, np.array([n]), h2=h2)
        assert np.array_equal(i, ri)
    say("candidate sample exact")


# ---------------------------------------------------------------------------
# serving: continuous batching over streams; every result equals its alone run
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [0, 1])
def test_serve_alone_vs_mix(ctx, torch, mode):
    pts = synth.clumpy_cloud(300_000, 5)
    tree = ctx.build_tree(dev(torch, pts))
    arr, streams, rois = synth.serving_trace(seed=3, duration_s=0.25, res_choices=(16, 24, 32, 48))
    outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in rois]
    res, summ = ctx.serve(tree, arr, rois, outs, mode=mode, n_slots=4, max_batch=32,
                          budget_bytes=64 << 20)
    torch.cuda.synchronize()
    say("serve mode", mode, "requests", len(rois), "batches", summ.n_batches, "p50",
        summ.p50_ms, "p99", summ.p99_ms, "mean batch", summ.mean_batch)
    assert summ.n_batches >= 1 and summ.p99_ms >= summ.p50_ms > 0
    for i in range(len(rois)):
        assert res[i].status == 0 and res[i].done_s >= res[i].admit_s >= res[i].arrival_s - 1e-9
    for i, r in enumerate(rois):
        alone = ctx.eval_roi(tree, r).cpu().numpy()
        assert np.array_equal(alone, outs[i].cpu().numpy()), i
    # a few requests against the oracle on sampled nodes
    for i in range(0, len(rois), max(1, len(rois) // 5)):
        r = rois[i]
        nodes = sample_nodes(None, r.n_nodes, 16, i)
        check_sampled(outs[i].cpu().numpy(), nodes, oracle.density(pts, r, nodes=nodes), "serve")


def test_serve_binding_budget_and_heavy_requests(ctx, torch):
    # an admission budget that binds (requests wait for memory), a work cap
    # that splits heavy requests into batches of their own, saturating
    # arrivals: every grid still equals the request evaluated alone
    pts = synth.clumpy_cloud(400_000, 15)
    tree = ctx.build_tree(dev(torch, pts))
    arr, _, rois = synth.serving_trace(seed=8, duration_s=0.3, res_choices=(32, 48, 64))
    arr = [0.0] * len(rois)  # everything waiting at the start
    outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in rois]
    res, summ = ctx.serve(tree, arr, rois, outs, mode=0, n_slots=4, max_batch=16,
                          budget_bytes=6 << 20, max_batch_work=2e6)
    torch.cuda.synchronize()
    say("binding budget: requests", len(rois), "batches", summ.n_batches, "waits",
        summ.budget_waits, "mean batch", summ.mean_batch)
    assert summ.budget_waits > 0
    assert summ.n_batches > len(rois) / 16
    for i, r in enumerate(rois):
        assert res[i].status == 0
        alone = ctx.eval_roi(tree, r).cpu().numpy()
        assert np.array_equal(alone, outs[i].cpu().numpy()), i
    tree.close()


# ---------------------------------------------------------------------------
# every tile shape, and the autotuner that picks among them
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [1, 2, 3, 4, 5, 6, 7])
def test_every_tile_shape(ctx, torch, shape):
    pts = synth.clumpy_cloud(80_000, 8)
    ctx.set_eval_opts(tile_shape=shape)
    tree = ctx.build_tree(dev(torch, pts), knn_k=16)
    h2 = ctx.debug_point_h2(tree)
    for roi in [Roi((0, 0, 0), (1, 1, 1), (23, 19, 17), bw="fixed", h=(0.05, 0.04, 0.06)),
                Roi((0.1, 0.1, 0.1), (0.9, 0.8, 0.7), (21, 22, 13), kernel="gauss_trunc3",
                    bw="per_point")]:
        got = ctx.eval_roi(tree, roi).cpu().numpy()
        check_density(got, oracle.density(pts, roi, h2=h2), "shape %d" % shape)
        cnt = ctx.debug_support_counts(tree, roi).cpu().numpy().astype(np.int64)
        assert np.array_equal(cnt, oracle.support_counts(pts, roi, h2=h2))
        n = roi.n_nodes // 2
        _, idx = ctx.debug_candidates(tree, roi, n, n + 1)
        _, ridx = oracle.candidates(pts, roi, np.array([n]), h2=h2)
        assert np.array_equal(idx, ridx)
    ctx.set_eval_opts()


def test_autotune(ctx, torch, sfk):
    pts = synth.clumpy_cloud(200_000, 9)
    tree = ctx.build_tree(dev(torch, pts))
    rois = synth.random_batch_rois(6, seed=2, res_lo=16, res_hi=40)
    outs = [torch.empty(r.n_nodes, device="cuda") for r in rois]
    ctx.autotune(tree, rois, outs)
    table = ctx.autotune_table()
    costs = ctx.autotune_costs()
    assert len(table) >= 1 and set(table) == set(costs)
    for key, shape in table.items():
        assert 1 <= shape <= sfk.NUM_TILE_SHAPES
        # the pick is the fastest shape measured for that key
        assert costs[key][shape - 1] == min(costs[key]), (key, shape, costs[key])
    # persisted with the device architecture, reloaded into a fresh context
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = d + "/tune.txt"
        ctx.autotune_save(path)
        head = open(path).read().split("\n")[0].split()
        assert head[0] == "sfkde-autotune" and head[2].startswith("gfx")
        c2 = type(ctx)(0)
        c2.autotune_load(path)
        assert c2.autotune_table() == table
        # another architecture is refused
        lines = open(path).read().split("\n")
        lines[0] = "sfkde-autotune 2 gfx000 %d" % sfk.NUM_TILE_SHAPES
        open(path, "w").write("\n".join(lines))
        with pytest.raises(Exception):
            c2.autotune_load(path)
        c2.close()
    for r in rois:
        nodes = sample_nodes(None, r.n_nodes, 16, 1)
        check_sampled(ctx.eval_roi(tree, r).cpu().numpy(), nodes,
                      oracle.density(pts, r, nodes=nodes), "autotuned")


# ---------------------------------------------------------------------------
# captured-graph submit path: replays (and recaptures as batches grow) give
# the same grids as direct launches and as one-ROI evaluation
# ---------------------------------------------------------------------------

def test_graph_replays_match_direct(ctx, torch):
    pts = synth.clumpy_cloud(150_000, 12)
    tree = ctx.build_tree(dev(torch, pts))
    batches = [synth.random_batch_rois(k, seed=20 + i, side_lo=0.05, res_lo=8, res_hi=36, h0=0.02)
               for i, k in enumerate([5, 5, 9, 3, 17, 5])]
    for rep in range(2):  # the second pass replays graphs captured in the first
        for rois in batches:
            outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in rois]
            ctx.wait(ctx.submit(tree, rois, outs))
            # eager work between replays
            alone = [ctx.eval_roi(tree, r).cpu().numpy() for r in rois]
            for a, o in zip(alone, outs):
                assert np.array_equal(a, o.cpu().numpy())
    ctx.set_eval_opts(disable_graphs=True)
    rois = batches[4]
    outs = [torch.zeros((r.n_nodes,), device="cuda") for r in rois]
    ctx.wait(ctx.submit(tree, rois, outs))
    ctx.set_eval_opts()
    outs2 = [torch.zeros((r.n_nodes,), device="cuda") for r in rois]
    ctx.wait(ctx.submit(tree, rois, outs2))
    for a, b in zip(outs, outs2):
        assert torch.equal(a, b)


def test_graph_cache_survives_tree_replacement(ctx, torch):
    # a new tree (possibly at a recycled address) must not replay a graph
    # captured for a destroyed one
    rois = synth.random_batch_rois(4, seed=31, side_lo=0.1, res_lo=8, res_hi=20, h0=0.03)
    for seed in (1, 2, 3):
        pts = synth.clumpy_cloud(40_000, seed)
        tree = ctx.build_tree(dev(torch, pts))
        outs = [torch.zeros((r.n_nodes,), device="cuda") for r in rois]
        ctx.wait(ctx.submit(tree, rois, outs))
        for r, o in zip(rois, outs):
            assert np.array_equal(o.cpu().numpy(), ctx.eval_roi(tree, r).cpu().numpy())
        nodes = sample_nodes(None, rois[0].n_nodes, 12, seed)
        check_sampled(outs[0].cpu().numpy(), nodes, oracle.density(pts, rois[0], nodes=nodes),
                      "replaced tree")
        tree.close()
