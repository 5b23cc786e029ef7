"""Particle sweep (uniform bandwidths, tile shape 7): parity with the oracle,
exact support counts, bit-for-bit equality with the bricks (both sum the
same fixed-point terms exactly), and bitwise independence of the batch, the
captured-graph replay and the blocking of wide windows."""
import numpy as np
import pytest

import oracle
import synth
from synth import Roi

pytestmark = pytest.mark.gpu

from gpu_common import (check_density, check_sampled, ctx, dev, sample_nodes, say,  # noqa: F401
                        sfk, torch)

SWEEP, BRICK = 7, 6


def _eval(ctx, torch, tree, roi, shape):
    ctx.set_eval_opts(tile_shape=shape)
    got = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    cnt = ctx.debug_support_counts(tree, roi)
    torch.cuda.synchronize()
    ctx.set_eval_opts()
    return got.cpu().numpy(), cnt.cpu().numpy().astype(np.int64)


def test_sweep_c1_full_grid_counts_and_bricks(ctx, torch):
    pts = synth.c1_cloud(1)
    tree = ctx.build_tree(dev(torch, pts))
    roi = synth.c1_roi()
    got, cnt = _eval(ctx, torch, tree, roi, SWEEP)
    say("sweep c1 max rel err", check_density(got, oracle.density(pts, roi), "sweep c1"))
    assert np.array_equal(cnt, oracle.support_counts(pts, roi))
    brk, bcnt = _eval(ctx, torch, tree, roi, BRICK)
    assert np.array_equal(got, brk) and np.array_equal(cnt, bcnt)
    tree.close()


@pytest.mark.parametrize("roi", [
    # ragged grids, anisotropic bandwidths, both kernels and norms
    Roi((0, 0, 0), (1, 1, 1), (29, 31, 33), kernel="epanechnikov", bw="fixed",
        h=(0.05, 0.03, 0.04), norm="paper"),
    Roi((0.1, 0.2, 0.05), (0.8, 0.7, 0.95), (40, 17, 23), kernel="gauss_trunc3", bw="fixed",
        h=(0.006, 0.004, 0.005), norm="count"),
    Roi((0.3, 0.3, 0.3), (0.6, 0.55, 0.62), (64, 50, 37), kernel="epanechnikov",
        bw="roi_scaled", h=(0.02,) * 3),
    # supports under half a spacing (one node per axis at most) ...
    Roi((0, 0, 0), (1, 1, 1), (41, 41, 41), kernel="epanechnikov", bw="fixed", h=(0.01,) * 3),
    # ... and spanning 5, 6, 7 and 8 nodes per axis (8 is the widest the
    # sweep takes) ...
    Roi((0, 0, 0), (1, 1, 1), (21, 21, 21), kernel="epanechnikov", bw="fixed", h=(0.12,) * 3),
    Roi((0.05, 0.05, 0.05), (0.95, 0.95, 0.95), (19, 19, 19), kernel="gauss_trunc3",
        bw="fixed", h=(0.039,) * 3),
    Roi((0, 0, 0), (1, 1, 1), (21, 21, 21), kernel="epanechnikov", bw="fixed", h=(0.13,) * 3),
    Roi((0.05, 0.05, 0.05), (0.95, 0.95, 0.95), (25, 23, 21), kernel="gauss_trunc3",
        bw="fixed", h=(0.04, 0.035, 0.045)),
    Roi((0.1, 0.0, 0.05), (0.9, 1.0, 0.95), (18, 22, 20), kernel="epanechnikov",
        bw="roi_scaled", h=(0.16,) * 3),
    Roi((0, 0, 0), (1, 1, 1), (21, 21, 21), kernel="epanechnikov", bw="fixed", h=(0.18,) * 3),
    # a box smaller than one spacing of the cloud's structure, 2 nodes on an axis
    Roi((0.45, 0.45, 0.45), (0.47, 0.46, 0.48), (2, 3, 2), kernel="epanechnikov", bw="fixed",
        h=(0.01,) * 3),
])
def test_sweep_vs_oracle_and_bricks(ctx, torch, roi):
    pts = synth.c1_cloud(2)
    tree = ctx.build_tree(dev(torch, pts))
    got, cnt = _eval(ctx, torch, tree, roi, SWEEP)
    check_density(got, oracle.density(pts, roi), "sweep %s" % (roi.res,))
    assert np.array_equal(cnt, oracle.support_counts(pts, roi))
    brk, bcnt = _eval(ctx, torch, tree, roi, BRICK)
    assert np.array_equal(got, brk) and np.array_equal(cnt, bcnt)
    tree.close()


def test_sweep_forced_past_its_widest_takes_the_default(ctx, torch):
    # supports spanning 9 nodes per axis: a forced sweep runs the default
    # shape instead (tiles here), with the default's result bit for bit
    pts = synth.c1_cloud(2)
    tree = ctx.build_tree(dev(torch, pts))
    roi = Roi((0, 0, 0), (1, 1, 1), (21, 21, 21), kernel="epanechnikov", bw="fixed",
              h=(0.2,) * 3)
    got, cnt = _eval(ctx, torch, tree, roi, SWEEP)
    check_density(got, oracle.density(pts, roi), "forced sweep, 9 nodes")
    assert np.array_equal(cnt, oracle.support_counts(pts, roi))
    ref, _ = _eval(ctx, torch, tree, roi, 0)
    assert np.array_equal(got, ref)
    ctx.set_eval_opts(tile_shape=SWEEP)
    shape, _, _ = ctx.debug_tile_leaves(tree, roi)
    ctx.set_eval_opts()
    assert tuple(shape) != (8, 8, 8)
    tree.close()


def test_sweep_tree_of_few_leaves(ctx, torch):
    # at most 64 leaves: the hierarchy has no interior level, items are leaves
    g = np.random.default_rng(3)
    pts = (0.5 + 0.1 * g.standard_normal((3000, 3))).astype(np.float32)
    tree = ctx.build_tree(dev(torch, pts))
    roi = Roi((0.2, 0.25, 0.3), (0.8, 0.75, 0.7), (36, 30, 24), kernel="epanechnikov",
              bw="fixed", h=(0.04,) * 3)
    got, cnt = _eval(ctx, torch, tree, roi, SWEEP)
    check_density(got, oracle.density(pts, roi), "sweep few leaves")
    assert np.array_equal(cnt, oracle.support_counts(pts, roi))
    brk, _ = _eval(ctx, torch, tree, roi, BRICK)
    assert np.array_equal(got, brk)
    tree.close()


@pytest.mark.parametrize("roi", [
    # 2-node supports: windows blocked at 16^3 nodes
    Roi((0, 0, 0), (1, 1, 1), (160, 150, 140), kernel="epanechnikov", bw="fixed",
        h=(0.004, 0.004, 0.0045)),
    # 1-node supports: windows blocked at 8^3 nodes
    Roi((0, 0, 0), (1, 1, 1), (200, 190, 180), kernel="epanechnikov", bw="fixed",
        h=(0.002, 0.002, 0.0022)),
])
def test_sweep_wide_windows_in_blocks(ctx, torch, roi):
    # fine grids over sparse regions: the 4096-particle boxes of the uniform
    # background span tens of nodes per axis, so their windows are swept in
    # blocks, each reading the box again
    pts = synth.clumpy_cloud(400_000, 6)
    tree = ctx.build_tree(dev(torch, pts))
    got, cnt = _eval(ctx, torch, tree, roi, SWEEP)
    brk, bcnt = _eval(ctx, torch, tree, roi, BRICK)
    assert np.array_equal(got, brk) and np.array_equal(cnt, bcnt)
    nodes = sample_nodes(None, roi.n_nodes, 96, 4, extra=[int(np.argmax(got))])
    check_sampled(got, nodes, oracle.density(pts, roi, nodes=nodes), "sweep wide windows")
    assert np.array_equal(cnt[nodes], oracle.support_counts(pts, roi, nodes=nodes))
    tree.close()


def test_sweep_items_not_a_prefix_of_the_boxes(ctx, torch):
    # a box of part of the cloud lists boxes that are not 0..n-1: each
    # claimed position must be read through the item list (a kernel that
    # took the position for the box evaluated the wrong particles)
    pts = synth.clumpy_cloud(400_000, 7)
    tree = ctx.build_tree(dev(torch, pts))
    for roi in (Roi((0.2, 0.3, 0.25), (0.7, 0.6, 0.8), (16, 12, 14), kernel="epanechnikov",
                    bw="roi_scaled", h=(0.03,) * 3),
                Roi((0.55, 0.1, 0.2), (0.9, 0.5, 0.6), (20, 24, 18), kernel="gauss_trunc3",
                    bw="fixed", h=(0.004,) * 3)):
        ctx.set_eval_opts(tile_shape=SWEEP)
        _, _, boxes = ctx.debug_tile_leaves(tree, roi)
        ctx.set_eval_opts()
        assert len(boxes) > 0 and not np.array_equal(boxes, np.arange(len(boxes)))
        got, cnt = _eval(ctx, torch, tree, roi, SWEEP)
        check_density(got, oracle.density(pts, roi), "sweep items %s" % (roi.res,))
        assert np.array_equal(cnt, oracle.support_counts(pts, roi))
        brk, _ = _eval(ctx, torch, tree, roi, BRICK)
        assert np.array_equal(got, brk)
    tree.close()


def test_sweep_default_batch_and_graph_bitwise(ctx, torch):
    pts = synth.clumpy_cloud(400_000, 7)
    tree = ctx.build_tree(dev(torch, pts), knn_k=8)
    dense = [Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (40, 44, 36), kernel="epanechnikov",
                 bw="roi_scaled", h=(0.02,) * 3),
             Roi((0.2, 0.3, 0.25), (0.7, 0.6, 0.8), (16, 12, 14), kernel="epanechnikov",
                 bw="roi_scaled", h=(0.03,) * 3),
             Roi((0.1, 0.1, 0.1), (0.9, 0.9, 0.9), (30, 30, 30), kernel="gauss_trunc3",
                 bw="fixed", h=(0.01,) * 3)]
    # the default picks the sweep for these dense uniform-bandwidth ROIs
    for r in dense:
        shape, _, boxes = ctx.debug_tile_leaves(tree, r)
        torch.cuda.synchronize()
        assert shape == (8, 8, 8), (r.res, shape)
        assert len(boxes) > 0 and np.all(np.diff(boxes) > 0)
    alone = []
    for i, r in enumerate(dense):
        o = ctx.eval_roi(tree, r)
        torch.cuda.synchronize()
        alone.append(o.cpu().numpy())
        nodes = sample_nodes(None, r.n_nodes, 48, 30 + i, extra=[int(np.argmax(alone[-1]))])
        check_sampled(alone[-1], nodes, oracle.density(pts, r, nodes=nodes), "sweep %d" % i)
        brk, _ = _eval(ctx, torch, tree, r, BRICK)
        assert np.array_equal(alone[-1], brk)
    # one batch (captured graph, replayed with eager work in between), with a
    # per-point ROI evaluated by tiles beside the sweep's group
    pp = Roi((0.3, 0.3, 0.3), (0.7, 0.7, 0.7), (20, 20, 20), kernel="epanechnikov",
             bw="per_point")
    pp_alone = ctx.eval_roi(tree, pp).cpu().numpy()
    # one group (same kernel, bandwidth mode and node span): a captured graph
    twin = Roi((0.05, 0.0, 0.0), (1.0, 0.95, 1.0), (40, 44, 36), kernel="epanechnikov",
               bw="roi_scaled", h=(0.02,) * 3)
    twin_alone = ctx.eval_roi(tree, twin).cpu().numpy()
    for rep in range(3):
        outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in (dense[0], twin)]
        ctx.wait(ctx.submit(tree, [dense[0], twin], outs))
        for o, a in zip(outs, (alone[0], twin_alone)):
            assert np.array_equal(o.cpu().numpy(), a), rep
        _ = ctx.eval_roi(tree, dense[rep % 3]).cpu().numpy()
    # several groups in one batch (direct launches)
    mix = dense + [pp]
    outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in mix]
    ctx.wait(ctx.submit(tree, mix, outs))
    for o, a in zip(outs, alone + [pp_alone]):
        assert np.array_equal(o.cpu().numpy(), a)
    tree.close()


@pytest.mark.parametrize("shape", [7, 6, 1])
def test_sub_roi_window_consistency(ctx, torch, shape):
    # a sub-box whose nodes coincide with the full box's (dyadic spacing
    # 1/64 on both) has the full grid's values there: bit for bit where the
    # terms are summed as integers (sweep, bricks), within the bar for tiles
    pts = synth.clumpy_cloud(300_000, 9)
    tree = ctx.build_tree(dev(torch, pts))
    full = Roi((0, 0, 0), (1, 1, 1), (65, 65, 65), kernel="epanechnikov", bw="fixed",
               h=(0.03, 0.03, 0.03))
    sub = Roi((0.25, 0.125, 0.5), (0.75, 0.5, 1.0), (33, 25, 33), kernel="epanechnikov",
              bw="fixed", h=(0.03, 0.03, 0.03))
    ctx.set_eval_opts(tile_shape=shape)
    g_full = ctx.eval_roi(tree, full).cpu().numpy().reshape(65, 65, 65)  # z, y, x
    g_sub = ctx.eval_roi(tree, sub).cpu().numpy().reshape(33, 25, 33)
    torch.cuda.synchronize()
    ctx.set_eval_opts()
    window = g_full[32:65, 8:33, 16:49]
    if shape in (6, 7):
        assert np.array_equal(g_sub, window)
    else:
        check_density(g_sub.ravel(), window.ravel().astype(np.float64), "sub-ROI window")
    tree.close()
