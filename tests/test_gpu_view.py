"""View cache (recomputation policy with reuse across frames): every frame's
grid must equal, bitwise, the lattice nodes of freshly evaluated block ROIs
(sfk_eval_roi on the documented block boxes), and sampled block nodes must
match the oracle. The frame geometry (which lattice, which nodes, which
blocks) is re-derived here from the documented rules, independently of the
library."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Roi

from gpu_common import check_sampled, ctx, dev, say, sfk, torch  # noqa: F401

pytestmark = pytest.mark.gpu


# ---- the documented geometry, written out independently -------------------

def lattice_nodes(o, s, lo, hi):
    """Largest node index at or below lo, smallest at or above hi (per axis)."""
    gl, gh = [], []
    for k in range(3):
        g = math.floor((lo[k] - o[k]) / s)
        while o[k] + (g + 1) * s <= lo[k]:
            g += 1
        while o[k] + g * s > lo[k]:
            g -= 1
        h = math.ceil((hi[k] - o[k]) / s)
        while o[k] + (h - 1) * s >= hi[k]:
            h -= 1
        while o[k] + h * s < hi[k]:
            h += 1
        gl.append(g)
        gh.append(h)
    return gl, gh


def block_roi(o, s, b, B, kernel, bw, h):
    lo = tuple(o[k] + float(b[k] * B) * s for k in range(3))
    hi = tuple(o[k] + float(b[k] * B + B - 1) * s for k in range(3))
    return Roi(lo, hi, (B, B, B), kernel=kernel, bw=bw, h=h)


class Fresh:
    """Fresh sfk_eval_roi of block ROIs (memoised per block)."""

    def __init__(self, ctx, tree, kernel, bw, B):
        self.ctx, self.tree, self.kernel, self.bw, self.B = ctx, tree, kernel, bw, B
        self.cache = {}

    def block(self, o, s, h, b):
        key = (s, h, tuple(b))
        if key not in self.cache:
            r = block_roi(o, s, b, self.B, self.kernel, self.bw, h)
            self.cache[key] = (r, self.ctx.eval_roi(self.tree, r).cpu().numpy())
        return self.cache[key]

    def assemble(self, o, s, h, g0, res):
        B = self.B
        out = np.empty(res[0] * res[1] * res[2], np.float32)
        gx = np.arange(g0[0], g0[0] + res[0])
        gy = np.arange(g0[1], g0[1] + res[1])
        gz = np.arange(g0[2], g0[2] + res[2])
        for bz in range(gz[0] // B, gz[-1] // B + 1):
            for by in range(gy[0] // B, gy[-1] // B + 1):
                for bx in range(gx[0] // B, gx[-1] // B + 1):
                    _, blk = self.block(o, s, h, (bx, by, bz))
                    blk = blk.reshape(B, B, B)  # [z, y, x]
                    sx = gx[(gx // B) == bx]
                    sy = gy[(gy // B) == by]
                    sz = gz[(gz // B) == bz]
                    sub = blk[np.ix_(sz - bz * B, sy - by * B, sx - bx * B)]
                    ix = sx - g0[0]
                    iy = sy - g0[1]
                    iz = sz - g0[2]
                    idx = (ix[None, None, :] + res[0] * (iy[None, :, None] + res[1] * iz[:, None, None]))
                    out[idx.ravel()] = sub.ravel()
        return out


def expect_geometry(info, o, box, res_want, B, margin, spacing):
    lo, hi = box
    side = max(hi[k] - lo[k] for k in range(3))
    gl, gh = lattice_nodes(o, spacing, lo, hi)
    assert list(info["g0"]) == gl
    assert list(info["res"]) == [gh[k] - gl[k] + 1 for k in range(3)]
    m = margin * side
    nb = 1
    for k in range(3):
        ml = min(math.floor((lo[k] - m - o[k]) / spacing), gl[k])
        mh = max(math.ceil((hi[k] + m - o[k]) / spacing), gh[k])
        nb *= mh // B - ml // B + 1
    assert info["blocks_needed"] == nb


def check_frame(fresh, view, box, o, h, pts, label, n_oracle=0, seed=0):
    grid, info = view.frame(*box)
    torch_grid = grid.cpu().numpy()
    s = info["spacing"]
    exp = fresh.assemble(o, s, h, info["g0"], info["res"])
    assert np.array_equal(torch_grid, exp), label + ": frame differs from fresh block evaluations"
    if n_oracle:
        # oracle on sampled nodes of one block of the frame
        B = fresh.B
        b = tuple(info["g0"][k] // B for k in range(3))
        r, blk = fresh.block(o, s, h, b)
        g = np.random.default_rng(seed)
        nodes = np.unique(np.concatenate([g.choice(B ** 3, n_oracle, replace=False),
                                          [int(np.argmax(blk))]])).astype(np.int64)
        ref = oracle.density(pts, r, nodes=nodes, h2=getattr(fresh, "h2", None))
        check_sampled(blk, nodes, ref, label + " oracle")
    return torch_grid, info


# ---- tests -----------------------------------------------------------------

def test_view_reuse_pan_zoom(ctx, torch):
    pts = synth.clumpy_cloud(200_000, 11)
    tree = ctx.build_tree(dev(torch, pts))
    _, bbox, _ = tree.info()
    o = bbox[:3]
    ctx.set_eval_opts(tile_shape=1)
    B, res, margin = 16, 40, 0.25
    h = 0.02
    view = ctx.view(tree, kernel="epanechnikov", bw="fixed", h=(h,) * 3, res=res, block=B,
                    scale_threshold=1.5, margin=margin, max_blocks=4096)
    fresh = Fresh(ctx, tree, "epanechnikov", "fixed", B)
    hh = (h, h, h)
    box0 = ((0.30, 0.32, 0.34), (0.60, 0.62, 0.64))
    say("frame 0: new lattice")
    plan0 = view.plan(*box0)
    assert plan0["new_lattice"] and plan0["blocks_evaluated"] == plan0["blocks_needed"]
    g0, i0 = check_frame(fresh, view, box0, o, hh, pts, "f0", n_oracle=24, seed=1)
    assert i0["new_lattice"] and i0["lattice_id"] == 0
    assert i0["spacing"] == 0.30 / (res - 1) or abs(i0["spacing"] - 0.3 / 39) < 1e-15
    expect_geometry(i0, o, box0, res, B, margin, i0["spacing"])
    assert i0["blocks_evaluated"] == i0["blocks_needed"]
    say("frame 1: same box, nothing evaluated")
    g1, i1 = check_frame(fresh, view, box0, o, hh, pts, "f1")
    assert i1["blocks_evaluated"] == 0 and not i1["new_lattice"]
    assert np.array_equal(g0, g1)
    say("frame 2: pan by more than a block width")
    box2 = ((0.43, 0.32, 0.34), (0.73, 0.62, 0.64))
    p2 = view.plan(*box2)
    _, i2 = check_frame(fresh, view, box2, o, hh, pts, "f2")
    assert i2["blocks_evaluated"] == p2["blocks_evaluated"]
    assert 0 < i2["blocks_evaluated"] < i2["blocks_needed"]
    expect_geometry(i2, o, box2, res, B, margin, i2["spacing"])
    say("frame 3: zoom out by 1.2, same lattice")
    box3 = ((0.30, 0.32, 0.34), (0.66, 0.68, 0.70))
    _, i3 = check_frame(fresh, view, box3, o, hh, pts, "f3")
    assert not i3["new_lattice"] and i3["lattice_id"] == 0 and i3["spacing"] == i0["spacing"]
    assert i3["res"][0] > res
    say("frame 4: zoom in by 2, new lattice")
    box4 = ((0.40, 0.42, 0.44), (0.55, 0.57, 0.59))
    _, i4 = check_frame(fresh, view, box4, o, hh, pts, "f4", n_oracle=24, seed=2)
    assert i4["new_lattice"] and i4["lattice_id"] == 1
    assert i4["blocks_evaluated"] == i4["blocks_needed"]
    say("frame 5: back to the first scale: lattice 0 reused")
    _, i5 = check_frame(fresh, view, box0, o, hh, pts, "f5")
    assert i5["lattice_id"] == 0 and i5["blocks_evaluated"] == 0
    view.close()
    ctx.set_eval_opts()
    tree.close()


def test_view_eviction_and_threshold_one(ctx, torch):
    pts = synth.clumpy_cloud(100_000, 12)
    tree = ctx.build_tree(dev(torch, pts))
    o = tree.info()[1][:3]
    ctx.set_eval_opts(tile_shape=2)
    B = 8
    view = ctx.view(tree, kernel="gauss_trunc3", bw="roi_scaled", h=(0.02,), res=20, block=B,
                    scale_threshold=1.0, margin=0.0, max_blocks=30)
    boxes = [((0.1, 0.1, 0.1), (0.3, 0.3, 0.3)), ((0.5, 0.5, 0.5), (0.7, 0.7, 0.7)),
             ((0.1, 0.1, 0.1), (0.3, 0.3, 0.3)), ((0.5, 0.5, 0.5), (0.7, 0.7, 0.7))]
    need = [view.plan(*b)["blocks_needed"] for b in boxes[:2]]
    view.close()
    # room for the larger frame only: each frame evicts the other's blocks
    view = ctx.view(tree, kernel="gauss_trunc3", bw="roi_scaled", h=(0.02,), res=20, block=B,
                    scale_threshold=1.0, margin=0.0, max_blocks=max(need))
    fresh = Fresh(ctx, tree, "gauss_trunc3", "fixed", B)
    # LRU with free slots first, two disjoint block sets: the number of
    # blocks each frame evaluates does not depend on ties
    cap = max(need)
    cached = [0, 0]
    for i, box in enumerate(boxes):
        cur, other = i % 2, 1 - i % 2
        missing = need[cur] - cached[cur]
        free = cap - cached[0] - cached[1]
        cached[other] -= max(0, missing - free)
        cached[cur] = need[cur]
        plan = view.plan(*box)
        s = plan["spacing"]
        hh = float(np.float32(float(np.float32(0.02)) * 19 * s))
        say("frame", i, "blocks", plan["blocks_needed"])
        _, info = check_frame(fresh, view, box, o, (hh, hh, hh), pts, "evict %d" % i,
                              n_oracle=16 if i < 2 else 0, seed=i)
        assert info["blocks_needed"] == need[cur] and info["blocks_evaluated"] == missing
    # threshold 1: any change of spacing starts a new lattice
    box = ((0.1, 0.1, 0.1), (0.3001, 0.3, 0.3))
    assert view.plan(*box)["new_lattice"]
    view.close()
    ctx.set_eval_opts()
    tree.close()


def test_view_per_point_default_shape(ctx, torch):
    pts = synth.clumpy_cloud(60_000, 13)
    tree = ctx.build_tree(dev(torch, pts), knn_k=16)
    h2 = ctx.debug_point_h2(tree)
    o = tree.info()[1][:3]
    B = 16
    view = ctx.view(tree, kernel="gauss_trunc3", bw="per_point", res=24, block=B,
                    scale_threshold=2.0, margin=0.1, max_blocks=512)
    fresh = Fresh(ctx, tree, "gauss_trunc3", "per_point", B)
    fresh.h2 = h2
    for i, box in enumerate([((0.2, 0.25, 0.3), (0.5, 0.55, 0.6)),
                             ((0.22, 0.25, 0.3), (0.52, 0.55, 0.6))]):
        _, info = check_frame(fresh, view, box, o, (1.0, 1.0, 1.0), pts, "pp %d" % i,
                              n_oracle=20, seed=10 + i)
        if i == 1:
            assert info["blocks_evaluated"] < info["blocks_needed"]
    view.close()
    tree.close()


def test_view_errors(ctx, sfk, torch):
    pts = synth.uniform_cloud(5000, 14)
    tree = ctx.build_tree(dev(torch, pts))
    bad = [dict(block=12), dict(scale_threshold=0.5), dict(margin=-1.0), dict(max_blocks=0),
           dict(res=1), dict(bw="mbe"), dict(bw="per_point"), dict(h=(0.0, 0.1, 0.1))]
    for kw in bad:
        args = dict(kernel="epanechnikov", bw="fixed", h=(0.05,) * 3, res=16, block=8,
                    scale_threshold=1.0, margin=0.0, max_blocks=64)
        args.update(kw)
        with pytest.raises(sfk.SfkError) as e:
            ctx.view(tree, **args)
        assert e.value.status == 1, kw  # SFK_E_INVAL
    box = ((0.1, 0.1, 0.1), (0.9, 0.9, 0.9))
    # a margin of one side triples the span: far more than 64 blocks of 8^3
    view = ctx.view(tree, kernel="epanechnikov", bw="fixed", h=(0.05,) * 3, res=16, block=8,
                    scale_threshold=1.0, margin=1.0, max_blocks=64)
    assert view.plan(*box)["blocks_needed"] > 64
    with pytest.raises(sfk.SfkError) as e:
        view.frame(*box)
    assert e.value.status == 3  # SFK_E_BUDGET
    view.close()
    view = ctx.view(tree, kernel="epanechnikov", bw="fixed", h=(0.05,) * 3, res=16, block=8,
                    scale_threshold=1.0, margin=0.0, max_blocks=64)
    out = torch.empty(10, device="cuda")
    with pytest.raises(sfk.SfkError) as e:  # the grid needs at least 16^3 floats
        view.frame(*box, out=out)
    assert e.value.status == 1
    with pytest.raises(sfk.SfkError):
        view.frame((0.2, 0.1, 0.1), (0.1, 0.2, 0.2))
    grid, info = view.frame(*box)
    assert all(r >= 16 for r in info["res"]) and grid.numel() == int(np.prod(info["res"]))
    view.close()
    tree.close()
