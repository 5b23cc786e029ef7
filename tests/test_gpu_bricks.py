"""Brick evaluation by scattering (uniform bandwidths, tile shape 6): parity
with the oracle, exact support counts, and bitwise independence of the
evaluation mode, the chunking and the batch (integer node sums)."""
import numpy as np
import pytest

import oracle
import synth
from synth import Roi

pytestmark = pytest.mark.gpu

from gpu_common import (check_density, check_sampled, ctx, dev, sample_nodes, say,  # noqa: F401
                        sfk, torch)

BRICK = 6


def test_bricks_c1_full_grid_and_counts(ctx, torch):
    pts = synth.c1_cloud(1)
    tree = ctx.build_tree(dev(torch, pts))
    ctx.set_eval_opts(tile_shape=BRICK)
    roi = synth.c1_roi()
    got = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    ref = oracle.density(pts, roi)
    say("bricks c1 max rel err", check_density(got.cpu().numpy(), ref, "bricks c1"))
    cnt = ctx.debug_support_counts(tree, roi)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), oracle.support_counts(pts, roi))
    tree.close()


@pytest.mark.parametrize("roi", [
    Roi((0, 0, 0), (1, 1, 1), (29, 31, 33), kernel="epanechnikov", bw="fixed",
        h=(0.05, 0.03, 0.04), norm="paper"),
    Roi((0.1, 0.2, 0.05), (0.8, 0.7, 0.95), (40, 17, 23), kernel="gauss_trunc3", bw="fixed",
        h=(0.006, 0.004, 0.005), norm="count"),
    Roi((0.3, 0.3, 0.3), (0.6, 0.55, 0.62), (64, 50, 37), kernel="epanechnikov",
        bw="roi_scaled", h=(0.02,) * 3),
    Roi((0.45, 0.45, 0.45), (0.47, 0.46, 0.48), (2, 3, 2), kernel="epanechnikov", bw="fixed",
        h=(0.01,) * 3),
])
def test_bricks_vs_oracle(ctx, torch, roi):
    pts = synth.c1_cloud(2)
    tree = ctx.build_tree(dev(torch, pts))
    ctx.set_eval_opts(tile_shape=BRICK)
    got = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    check_density(got.cpu().numpy(), oracle.density(pts, roi), "bricks %s" % (roi.res,))
    cnt = ctx.debug_support_counts(tree, roi)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), oracle.support_counts(pts, roi))
    tree.close()


def test_bricks_modes_chunks_and_batch_bitwise(ctx, torch):
    pts = synth.clumpy_cloud(400_000, 6)
    tree = ctx.build_tree(dev(torch, pts))
    rois = [Roi((0.05, 0.1, 0.0), (0.95, 0.9, 1.0), (70, 66, 72), kernel="epanechnikov",
                bw="roi_scaled", h=(0.012,) * 3),
            Roi((0.4, 0.35, 0.45), (0.6, 0.55, 0.65), (48, 48, 48), kernel="epanechnikov",
                bw="fixed", h=(0.003,) * 3),
            Roi((0.2, 0.6, 0.3), (0.35, 0.75, 0.45), (33, 17, 25), kernel="gauss_trunc3",
                bw="fixed", h=(0.002,) * 3)]
    ctx.set_eval_opts(tile_shape=BRICK)
    ref = []
    for r in rois:
        o = ctx.eval_roi(tree, r)
        torch.cuda.synchronize()
        ref.append(o.cpu().numpy())
    # oracle on sampled nodes
    for i, (r, g) in enumerate(zip(rois, ref)):
        nodes = sample_nodes(None, r.n_nodes, 64, 20 + i, extra=[int(np.argmax(g))])
        check_sampled(g, nodes, oracle.density(pts, r, nodes=nodes), "bricks sampled %d" % i)
    # many small chunks (split bricks, integer sums combined across items)
    ctx.set_eval_opts(tile_shape=BRICK, chunk_leaves=3)
    for r, g in zip(rois, ref):
        o = ctx.eval_roi(tree, r)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), g)
    # lists that do not fit: every brick walks the tree in one item
    ctx.set_eval_opts(tile_shape=BRICK, list_capacity=5)
    for r, g in zip(rois, ref):
        o = ctx.eval_roi(tree, r)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), g)
    # one batch with all of them (and a tile-evaluated per-point ROI beside)
    ctx.set_eval_opts(tile_shape=0)
    ctx.set_eval_opts(tile_shape=BRICK)
    outs = [torch.empty(r.n_nodes, device="cuda") for r in rois]
    ctx.wait(ctx.submit(tree, rois, outs))
    for o, g in zip(outs, ref):
        assert np.array_equal(o.cpu().numpy(), g)
    tree.close()
