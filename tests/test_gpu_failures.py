"""Failure handling through the C ABI, every condition forced from the host:
leaf-id checks (test-only out-of-range ids, reported as SFK_E_INTERNAL with
nothing read out of bounds), an allocator that returns NULL (SFK_E_NOMEM,
the context stays usable), a workspace over the context budget
(SFK_E_BUDGET), cancellation of a pending ticket (SFK_E_CANCELLED); and the
tile range query's leaf lists against a CPU walk of the exported leaf boxes."""
import numpy as np
import pytest

import oracle
import synth
from synth import Roi

pytestmark = pytest.mark.gpu

from gpu_common import check_sampled, ctx, dev, sample_nodes, say, sfk, torch  # noqa: F401


def _cpu_tile_lists(roi, boxes, ih, c2, shape):
    """Per tile (x fastest), the ascending leaves whose box passes the range
    query's test against the tile's node box: per-axis gap between the boxes
    in double on the float32 box, scaled by the float32 inverse bandwidth,
    u2 = (ux^2 + uy^2) + uz^2 < c2."""
    ax = [oracle.axis_coords(roi.lo[k], roi.hi[k], int(roi.res[k])) for k in range(3)]
    nt = [-(-int(roi.res[k]) // shape[k]) for k in range(3)]
    blo = boxes[:, :3].astype(np.float64)
    bhi = boxes[:, 3:].astype(np.float64)
    ihd = np.asarray(ih, dtype=np.float32).astype(np.float64)
    out = []
    for tk in range(nt[2]):
        for tj in range(nt[1]):
            for ti in range(nt[0]):
                t0 = (ti, tj, tk)
                tlo = np.array([ax[k][t0[k] * shape[k]] for k in range(3)])
                thi = np.array([ax[k][min(t0[k] * shape[k] + shape[k], int(roi.res[k])) - 1]
                                for k in range(3)])
                g = np.maximum(np.maximum(blo - thi, tlo - bhi), 0.0)
                u = g * ihd
                u2 = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2]
                out.append(np.nonzero(u2 < c2)[0].astype(np.int32))
    return out


def _cpu_sweep_items(roi, boxes, ih, c2):
    """The particle sweep's work items: the boxes of 64 consecutive leaves
    (each leaf alone for a tree of at most 64 leaves), bounded by their
    leaves' boxes, that pass the same test against the box of all the ROI's
    nodes; ascending."""
    n = boxes.shape[0]
    if n > 64:
        g = [boxes[i:i + 64] for i in range(0, n, 64)]
        boxes = np.array([np.concatenate([b[:, :3].min(0), b[:, 3:].max(0)]) for b in g],
                         dtype=np.float32)
    ax = [oracle.axis_coords(roi.lo[k], roi.hi[k], int(roi.res[k])) for k in range(3)]
    tlo = np.array([ax[k][0] for k in range(3)])
    thi = np.array([ax[k][-1] for k in range(3)])
    gap = np.maximum(np.maximum(boxes[:, :3].astype(np.float64) - thi,
                                tlo - boxes[:, 3:].astype(np.float64)), 0.0)
    u = gap * np.asarray(ih, dtype=np.float32).astype(np.float64)
    u2 = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2]
    return np.nonzero(u2 < c2)[0].astype(np.int32)


@pytest.mark.parametrize("shape_id", [0, 2, 4, 5, 7])
def test_tile_lists_match_cpu_walk(ctx, torch, shape_id):
    pts = synth.clumpy_cloud(200_000, 7)
    tree = ctx.build_tree(dev(torch, pts))
    boxes = ctx.debug_leaf_boxes(tree)
    ctx.set_eval_opts(tile_shape=shape_id)
    rois = [
        # large: every tile walks the hierarchy
        Roi((0.1, 0.15, 0.05), (0.9, 0.8, 0.95), (23, 19, 21), kernel="epanechnikov",
            bw="fixed", h=(0.03, 0.05, 0.04)),
        # small: tiles test the ROI's leaf list
        Roi((0.48, 0.5, 0.47), (0.52, 0.53, 0.51), (13, 11, 9), kernel="gauss_trunc3",
            bw="fixed", h=(0.002, 0.002, 0.002)),
    ]
    for i, roi in enumerate(rois):
        shape, cnt, leaves = ctx.debug_tile_leaves(tree, roi)
        h = oracle.roi_h(roi)
        ih = (1.0 / h.astype(np.float64)).astype(np.float32)
        c2 = 1.0 if roi.kernel == "epanechnikov" else 9.0
        if shape == (8, 8, 8):
            # the sweep (chosen, or by default for the dense ROI): its items
            assert np.all(cnt == 0)
            assert np.array_equal(leaves, _cpu_sweep_items(roi, boxes, ih, c2)), "roi %d" % i
            say("roi", i, "sweep items", len(leaves))
            continue
        want = _cpu_tile_lists(roi, boxes, ih, c2, shape)
        assert len(cnt) == len(want)
        assert np.array_equal(cnt, [len(w) for w in want]), "roi %d counts" % i
        assert np.array_equal(leaves, np.concatenate(want)), "roi %d lists" % i
        say("roi", i, "shape", shape, "tiles", len(cnt), "max leaves per tile", int(cnt.max()))
    tree.close()


def test_poisoned_leaf_ids_are_reported(ctx, torch, sfk):
    pts = synth.clumpy_cloud(200_000, 8)
    tree = ctx.build_tree(dev(torch, pts))
    # wide supports so that tiles hold 65-256 candidate leaves
    roi = Roi((0.2, 0.2, 0.2), (0.8, 0.8, 0.8), (24, 24, 24), kernel="epanechnikov", bw="fixed",
              h=(0.15, 0.15, 0.15))
    ctx.set_eval_opts(tile_shape=1)  # wavefront tiles (the default would sweep this ROI)
    _, cnt, _ = ctx.debug_tile_leaves(tree, roi)
    assert np.any((cnt > 64) & (cnt <= 256)), "no tile exercises the slot copy past 64"
    ref = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    out = torch.empty(roi.n_nodes, device="cuda")
    for bits in (1, 2):
        ctx.debug_poison(bits)
        t = ctx.submit(tree, [roi], [out])
        with pytest.raises(sfk.SfkError) as e:
            ctx.wait(t)
        assert e.value.status == 8, bits  # SFK_E_INTERNAL
        assert "leaf" in ctx.last_error()
        # stream-ordered path: reported by the next call, which does no work
        ctx.eval_roi(tree, roi, out=out)
        torch.cuda.synchronize()
        ctx.debug_poison(0)
        with pytest.raises(sfk.SfkError) as e:
            ctx.eval_roi(tree, roi, out=out)
        assert e.value.status == 8
        # the context is usable again and its results are unchanged
        got = ctx.eval_roi(tree, roi, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref)
        ctx.wait(ctx.submit(tree, [roi], [out]))
        assert np.array_equal(out.cpu().numpy(), ref)
    tree.close()


def test_allocator_null_gives_nomem(ctx, torch, sfk):
    pts = synth.clumpy_cloud(100_000, 9)
    tree = ctx.build_tree(dev(torch, pts))
    small = Roi((0, 0, 0), (1, 1, 1), (16, 16, 16), bw="fixed", h=(0.03,) * 3)
    big = Roi((0, 0, 0), (1, 1, 1), (160, 150, 140), bw="fixed", h=(0.01,) * 3)
    ctx.eval_roi(tree, small)
    torch.cuda.synchronize()
    ctx.fail_allocations = True
    out = torch.empty(big.n_nodes, device="cuda")
    with pytest.raises(sfk.SfkError) as e:
        ctx.eval_roi(tree, big, out=out)  # the workspace must grow
    assert e.value.status == 2  # SFK_E_NOMEM
    with pytest.raises(sfk.SfkError) as e:
        ctx.build_tree(dev(torch, pts[:1000]))
    assert e.value.status == 2
    ctx.fail_allocations = False
    got = ctx.eval_roi(tree, big, out=out)
    torch.cuda.synchronize()
    nodes = sample_nodes(None, big.n_nodes, 48, 3, extra=[int(torch.argmax(got))])
    check_sampled(got.cpu().numpy(), nodes, oracle.density(pts, big, nodes=nodes), "after NOMEM")
    tree.close()


def test_budget_rejects_submit(sfk, torch):
    pts = synth.clumpy_cloud(100_000, 10)
    with sfk.Context(0, budget_bytes=24 << 20) as c:
        tree = c.build_tree(dev(torch, pts))  # trees are not charged to the budget
        big = Roi((0, 0, 0), (1, 1, 1), (200, 200, 200), bw="fixed", h=(0.01,) * 3)
        out = torch.empty(big.n_nodes, device="cuda")
        with pytest.raises(sfk.SfkError) as e:
            c.submit(tree, [big], [out])
        assert e.value.status == 3  # SFK_E_BUDGET
        small = Roi((0.3, 0.3, 0.3), (0.6, 0.6, 0.6), (20, 20, 20), bw="fixed", h=(0.02,) * 3)
        o2 = torch.empty(small.n_nodes, device="cuda")
        c.wait(c.submit(tree, [small], [o2]))
        nodes = sample_nodes(None, small.n_nodes, 32, 4)
        check_sampled(o2.cpu().numpy(), nodes, oracle.density(pts, small, nodes=nodes), "budget")
        tree.close()


def test_cancel_pending_ticket(ctx, torch, sfk):
    pts = synth.uniform_cloud(1_000_000, 11)
    tree = ctx.build_tree(dev(torch, pts))
    # four heavy batches occupy the four slots; the fifth waits
    heavy = Roi((0, 0, 0), (1, 1, 1), (160, 160, 160), bw="fixed", h=(0.08,) * 3)
    outs = [torch.empty(heavy.n_nodes, device="cuda") for _ in range(5)]
    ctx.wait(ctx.submit(tree, [heavy], [outs[0]]))  # warm: buffers and graphs
    ts = [ctx.submit(tree, [heavy], [outs[i]]) for i in range(5)]
    ctx.cancel(ts[4])
    with pytest.raises(sfk.SfkError) as e:
        ctx.wait(ts[4])
    assert e.value.status == 6  # SFK_E_CANCELLED
    with pytest.raises(sfk.SfkError) as e:
        ctx.cancel(ts[0])  # already on the device
    assert e.value.status == 5  # SFK_E_NOT_READY
    for t in ts[:4]:
        ctx.wait(t)
    ref = ctx.eval_roi(tree, heavy)
    torch.cuda.synchronize()
    for o in outs[:4]:
        assert torch.equal(o, ref)
    tree.close()
