"""Parity at the full sizes of the large workloads, on sampled nodes (the
oracle brute-forces every particle for each sampled node):

- 100M clumpy points drawn on the device; 11 nested ROIs (side 1 down to
  1/1024 around one of the 10 most massive clumps) at 64^3, 128^3 and 256^3,
  Epanechnikov, bandwidth 0.01 x ROI side;
- the same cloud; 256 uneven ROIs (side log-uniform in [1e-3, 1], grids
  16^3-128^3) in one persistent submit, bitwise equal to one launch per ROI;
- 1B clumpy points drawn on the device (tree resident); one second of the
  8-stream, 90 Hz request trace served with continuous batching; results
  bitwise equal to their alone evaluation and to the oracle on samples.

Sampled nodes: random ones plus the GPU grid's largest values (only the node
choice comes from the GPU; every expected value is the oracle's).
"""
import numpy as np
import pytest

import oracle
import synth

from gpu_common import check_sampled, ctx, say, sfk, torch  # noqa: F401

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def pick_nodes(grid, k, seed, n_top=4):
    g = np.random.default_rng(seed)
    m = grid.shape[0]
    nodes = set(int(v) for v in g.choice(m, size=min(k, m), replace=False))
    if m > 0 and grid.max() > 0:
        nodes.update(int(v) for v in np.argpartition(-grid, min(n_top, m - 1))[:n_top])
    return np.array(sorted(nodes), dtype=np.int64)


@pytest.fixture(scope="module")
def cloud_100m(torch):
    say("drawing 100M clumpy points on the device (seed 3)")
    xyz, info = synth.clumpy_cloud_device(100_000_000, 3)
    torch.cuda.synchronize()
    host = xyz.cpu().numpy()
    say("cloud ready")
    yield xyz, info, host
    del xyz


def test_nested_zoom_100m(ctx, torch, cloud_100m):
    xyz, info, host = cloud_100m
    tree = ctx.build_tree(xyz)
    rois = synth.nested_zoom_rois(info, seed=3)
    assert len(rois) == 33
    grids = []
    for r in rois:
        say("zoom ROI", r.tag, "side %.6g" % (r.hi[0] - r.lo[0]), "res", r.res[0])
        grids.append(ctx.eval_roi(tree, r).cpu().numpy())
    for r, got in zip(rois, grids):
        nodes = pick_nodes(got, 12, 100 + r.tag)
        check_sampled(got, nodes, oracle.density(host, r, nodes=nodes), "zoom %d" % r.tag)
    tree.close()


def test_batch_256_rois_100m(ctx, torch, cloud_100m):
    xyz, info, host = cloud_100m
    tree = ctx.build_tree(xyz)
    rois = synth.random_batch_rois(256, seed=4)
    outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in rois]
    say("one persistent submit of 256 ROIs,", sum(r.n_nodes for r in rois), "nodes")
    ctx.wait(ctx.submit(tree, rois, outs))
    torch.cuda.synchronize()
    say("one launch per ROI")
    for i, r in enumerate(rois):
        single = ctx.eval_roi(tree, r)
        assert torch.equal(single, outs[i]), "ROI %d differs between batch and single launch" % i
    order = sorted(range(len(rois)), key=lambda i: -rois[i].n_nodes)
    check = order[:8] + list(range(0, len(rois), 16))
    for i in sorted(set(check)):
        got = outs[i].cpu().numpy()
        nodes = pick_nodes(got, 12, 200 + i)
        check_sampled(got, nodes, oracle.density(host, rois[i], nodes=nodes), "batch %d" % i)
    tree.close()


def test_serving_1b(ctx, torch):
    say("drawing 1B clumpy points on the device (seed 5)")
    xyz, info = synth.clumpy_cloud_device(1_000_000_000, 5)
    torch.cuda.synchronize()
    say("building the 1B-point tree")
    tree = ctx.build_tree(xyz)
    n, bbox, nbytes = tree.info()
    assert n == 1_000_000_000
    say("tree resident: %.1f GB" % (nbytes / 1e9))
    arr, streams, rois = synth.serving_trace(seed=5, duration_s=1.0)
    outs = [torch.full((r.n_nodes,), -1.0, device="cuda") for r in rois]
    say("serving", len(rois), "requests")
    res, summ = ctx.serve(tree, arr, rois, outs, mode=0, n_slots=4, max_batch=64,
                          budget_bytes=8 << 30)
    torch.cuda.synchronize()
    say("p50 %.3f ms p99 %.3f ms, batches %d, mean batch %.2f" % (
        summ.p50_ms, summ.p99_ms, summ.n_batches, summ.mean_batch))
    for i in range(len(rois)):
        assert res[i].status == 0, i
    # alone vs in the mix, bitwise, for every 16th request and the largest ones
    order = sorted(range(len(rois)), key=lambda i: -rois[i].n_nodes)
    pick = sorted(set(list(range(0, len(rois), 16)) + order[:6]))
    for i in pick:
        alone = ctx.eval_roi(tree, rois[i])
        assert torch.equal(alone, outs[i]), "request %d differs alone vs in the mix" % i
    say("copying the cloud to the host for the oracle")
    host = xyz.cpu().numpy()
    for i in pick[::4][:6]:
        got = outs[i].cpu().numpy()
        nodes = pick_nodes(got, 10, 300 + i, n_top=2)
        say("oracle on request", i, "side %.3g" % (rois[i].hi[0] - rois[i].lo[0]), len(nodes), "nodes")
        check_sampled(got, nodes, oracle.density(host, rois[i], nodes=nodes), "serve %d" % i)
    tree.close()
