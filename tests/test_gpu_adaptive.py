"""Adaptive resolution: which bricks are refined is re-derived here from the
GPU's own grids with the documented float32 rule (the decision is taken in
the same precision on both sides); every refined brick's values must equal,
bitwise, sfk_eval_roi of the documented brick ROI, and sampled nodes of the
base grid and of the bricks must match the oracle."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Roi

from gpu_common import check_density, check_sampled, ctx, dev, say, sfk, torch  # noqa: F401

pytestmark = pytest.mark.gpu


def node(lo, hi, res, i):
    return lo + (i * (hi - lo)) / (res - 1)


def expected_bricks(base, roi, vals, brick, max_level, threshold, listed):
    """The brick list the documented rule gives, level by level, reading
    each level's grids from the GPU's output (base and listed bricks)."""
    parents = [(base.reshape(roi.res[2], roi.res[1], roi.res[0]), tuple(roi.lo), tuple(roi.hi),
                tuple(roi.res), -1)]
    out = []
    peak = np.float32(base.max())
    thr = np.float32(float(np.float32(threshold)) * float(peak))
    for level in range(1, max_level + 1):
        lvl = []
        for grid, lo, hi, res, idx in parents:
            nb = [math.ceil((res[k] - 1) / brick) for k in range(3)]
            for bz in range(nb[2]):
                for by in range(nb[1]):
                    for bx in range(nb[0]):
                        n0 = (bx * brick, by * brick, bz * brick)
                        cells = [min(brick, res[k] - 1 - n0[k]) for k in range(3)]
                        sub = grid[n0[2]:n0[2] + cells[2] + 1, n0[1]:n0[1] + cells[1] + 1,
                                   n0[0]:n0[0] + cells[0] + 1]
                        rng = np.float32(sub.max() - sub.min())
                        if not rng > thr:
                            continue
                        lvl.append({
                            "level": level, "parent": idx, "cell0": n0,
                            "res": tuple(2 * cells[k] + 1 for k in range(3)),
                            "lo": tuple(node(lo[k], hi[k], res[k], n0[k]) for k in range(3)),
                            "hi": tuple(node(lo[k], hi[k], res[k], n0[k] + cells[k])
                                        for k in range(3))})
        if not lvl or len(out) + len(lvl) > len(listed):
            break
        nxt = []
        for i, b in enumerate(lvl):
            got = listed[len(out) + i]
            n = b["res"][0] * b["res"][1] * b["res"][2]
            g = vals[got["offset"]:got["offset"] + n].reshape(b["res"][2], b["res"][1], b["res"][0])
            nxt.append((g, b["lo"], b["hi"], b["res"], len(out) + i))
        out += lvl
        parents = nxt
    return out


def brick_roi(roi, b, h_base):
    bw = "per_point" if roi.bw == "per_point" else "fixed"
    return Roi(b["lo"], b["hi"], b["res"], kernel=roi.kernel, bw=bw, norm=roi.norm, h=h_base)


def run_case(ctx, torch, pts, tree, roi, h_base, brick, max_level, threshold, h2=None,
             n_oracle_bricks=2, seed=0):
    base, vals, listed, info = ctx.eval_adaptive(tree, roi, brick=brick, max_level=max_level,
                                                 threshold=threshold)
    base = base.cpu().numpy()
    vals = vals.cpu().numpy()
    assert np.array_equal(base, ctx.eval_roi(tree, roi).cpu().numpy())
    assert info["complete"] and info["peak"] == base.max()
    exp = expected_bricks(base, roi, vals, brick, max_level, threshold, listed)
    assert len(exp) == len(listed) == info["n_bricks"]
    for e, g in zip(exp, listed):
        for key in ("level", "parent", "cell0", "res", "lo", "hi"):
            assert tuple(np.atleast_1d(e[key])) == tuple(np.atleast_1d(g[key])), (key, e, g)
    say("bricks per level:", [sum(1 for b in listed if b["level"] == l)
                              for l in range(1, max_level + 1)])
    g = np.random.default_rng(seed)
    for i, b in enumerate(listed):
        r = brick_roi(roi, b, h_base)
        n = r.n_nodes
        got = vals[b["offset"]:b["offset"] + n]
        assert np.array_equal(got, ctx.eval_roi(tree, r).cpu().numpy()), "brick %d" % i
        if i < n_oracle_bricks or i == len(listed) - 1:
            nodes = np.unique(np.concatenate([g.choice(n, min(n, 20), replace=False),
                                              [int(np.argmax(got))]])).astype(np.int64)
            check_sampled(got, nodes, oracle.density(pts, r, nodes=nodes, h2=h2), "brick %d" % i)
    nodes = np.unique(np.concatenate([g.choice(base.size, 30, replace=False),
                                      [int(np.argmax(base))]])).astype(np.int64)
    check_sampled(base, nodes, oracle.density(pts, roi, nodes=nodes, h2=h2), "base")
    return listed, info


def test_adaptive_two_levels(ctx, torch):
    pts = synth.clumpy_cloud(200_000, 21)
    tree = ctx.build_tree(dev(torch, pts))
    roi = Roi((0, 0, 0), (1, 1, 1), (33, 33, 33), kernel="epanechnikov", bw="roi_scaled",
              h=(0.02,) * 3)
    h = float(np.float32(float(np.float32(0.02)) * 1.0))
    listed, info = run_case(ctx, torch, pts, tree, roi, (h, h, h), 8, 2, 0.05)
    assert info["levels"] == 2 and 0 < sum(b["level"] == 1 for b in listed) < 64
    tree.close()


def test_adaptive_ragged_per_point(ctx, torch):
    pts = synth.clumpy_cloud(80_000, 22)
    tree = ctx.build_tree(dev(torch, pts), knn_k=16)
    h2 = ctx.debug_point_h2(tree)
    roi = Roi((0.1, 0.05, 0.2), (0.9, 0.8, 0.85), (30, 27, 21), kernel="gauss_trunc3",
              bw="per_point")
    listed, _ = run_case(ctx, torch, pts, tree, roi, (1.0, 1.0, 1.0), 6, 3, 0.1, h2=h2, seed=3)
    assert any(b["res"] != (13, 13, 13) for b in listed)  # partial bricks at the edges
    tree.close()


def test_adaptive_capacity_and_errors(ctx, sfk, torch):
    pts = synth.clumpy_cloud(50_000, 23)
    tree = ctx.build_tree(dev(torch, pts))
    roi = Roi((0, 0, 0), (1, 1, 1), (25, 25, 25), kernel="epanechnikov", bw="fixed",
              h=(0.03,) * 3)
    _, _, full, finfo = ctx.eval_adaptive(tree, roi, brick=4, max_level=2, threshold=0.05)
    n1 = [b for b in full if b["level"] == 1]
    assert finfo["complete"] and len(n1) > 0 and len(full) > len(n1)
    # room for level 1 only: refinement stops before level 2
    _, vals, part, pinfo = ctx.eval_adaptive(tree, roi, brick=4, max_level=2, threshold=0.05,
                                             cap_bricks=len(n1))
    assert not pinfo["complete"] and pinfo["levels"] == 1 and len(part) == len(n1)
    assert [b["lo"] for b in part] == [b["lo"] for b in n1]
    for kw in (dict(brick=1), dict(brick=65), dict(max_level=0), dict(max_level=5),
               dict(threshold=0.0), dict(threshold=float("nan"))):
        with pytest.raises(sfk.SfkError) as e:
            ctx.eval_adaptive(tree, roi, **kw)
        assert e.value.status == 1, kw
    with pytest.raises(sfk.SfkError) as e:
        ctx.eval_adaptive(tree, roi.replace(set="in_roi"))
    assert e.value.status == 7  # SFK_E_UNSUPPORTED
    # an empty field refines nothing
    far = Roi((5, 5, 5), (6, 6, 6), (9, 9, 9), kernel="epanechnikov", bw="fixed", h=(0.01,) * 3)
    base, _, none, einfo = ctx.eval_adaptive(tree, far)
    assert float(base.abs().max()) == 0.0 and none == [] and einfo["levels"] == 0
    tree.close()
