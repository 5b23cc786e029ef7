"""The tree's particle-count estimate (the summed-volume table built with
the tree), against exact counts: it chooses tile shapes and caps serving
batches, so gross errors (a swapped axis, a shifted cell) would silently
change those choices."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

from gpu_common import ctx, dev, sfk, torch  # noqa: F401


def _exact(pts, lo, hi):
    p = pts.astype(np.float64)
    return int(np.count_nonzero(np.all((p >= lo) & (p <= hi), axis=1)))


def test_estimate_whole_cloud_outside_and_boxes(ctx, torch):
    pts = synth.clumpy_cloud(400_000, 6)
    tree = ctx.build_tree(dev(torch, pts))
    n = len(pts)
    lo, hi = pts.min(axis=0).astype(np.float64), pts.max(axis=0).astype(np.float64)
    # every particle: exact up to rounding
    assert abs(ctx.debug_particle_estimate(tree, lo - 0.1, hi + 0.1) - n) <= 1e-6 * n
    # a box beside the cloud holds nothing
    assert ctx.debug_particle_estimate(tree, hi + 0.01, hi + 0.2) == 0.0
    # half spaces along each axis, and random boxes of at least 1/8 of the
    # unit cube: within 8% of the exact count plus 1% of the cloud
    for k in range(3):
        b_lo, b_hi = lo - 0.1, hi + 0.1
        b_hi = b_hi.copy()
        b_hi[k] = 0.5
        est, ex = ctx.debug_particle_estimate(tree, b_lo, b_hi), _exact(pts, b_lo, b_hi)
        assert abs(est - ex) <= 0.08 * ex + 0.01 * n, (k, est, ex)
    g = np.random.default_rng(11)
    for i in range(12):
        side = g.uniform(0.5, 0.9, size=3)
        b_lo = g.uniform(0.0, 1.0 - side)
        b_hi = b_lo + side
        est, ex = ctx.debug_particle_estimate(tree, b_lo, b_hi), _exact(pts, b_lo, b_hi)
        assert abs(est - ex) <= 0.08 * ex + 0.01 * n, (i, b_lo, b_hi, est, ex)
    tree.close()


def test_estimate_flat_cloud(ctx, torch):
    # a flat axis of the bounding box: boxes holding the plane count their
    # xy part, boxes beside it nothing
    g = np.random.default_rng(12)
    pts = np.empty((50_000, 3), dtype=np.float32)
    pts[:, :2] = g.random((50_000, 2), dtype=np.float32)
    pts[:, 2] = 0.5
    tree = ctx.build_tree(dev(torch, pts))
    n = len(pts)
    est = ctx.debug_particle_estimate(tree, np.array([0.0, 0.0, 0.4]), np.array([1.0, 0.5, 0.6]))
    ex = _exact(pts, np.array([0.0, 0.0, 0.4]), np.array([1.0, 0.5, 0.6]))
    assert abs(est - ex) <= 0.05 * ex + 0.01 * n, (est, ex)
    assert ctx.debug_particle_estimate(tree, np.array([0.0, 0.0, 0.6]),
                                       np.array([1.0, 1.0, 0.7])) == 0.0
    tree.close()


def test_estimate_rejects_bad_boxes(ctx, torch, sfk):
    pts = synth.c1_cloud(1)
    tree = ctx.build_tree(dev(torch, pts))
    with pytest.raises(sfk.SfkError):
        ctx.debug_particle_estimate(tree, np.array([0.5, 0.0, 0.0]), np.array([0.4, 1.0, 1.0]))
    with pytest.raises(sfk.SfkError):
        ctx.debug_particle_estimate(tree, np.array([np.nan, 0.0, 0.0]), np.ones(3))
    tree.close()
