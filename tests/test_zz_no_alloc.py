"""sfk_eval_roi_noalloc (workspace in the library's static scratch array)
against sfk_eval_roi through the C ABI: bitwise equal grids on consecutive
calls of shrinking and growing size, sampled nodes within the oracle bar,
and the documented rejections (over-size ROI, in-box set)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from synth import Roi

pytestmark = pytest.mark.gpu

from gpu_common import check_sampled, ctx, dev, sample_nodes, say, sfk, torch  # noqa: F401


@pytest.fixture(scope="module")
def cloud():
    return synth.clumpy_cloud(300_000, 2)


def _both(ctx, torch, tree, roi, stream=None):
    a = torch.full((roi.n_nodes,), -1.0, device="cuda")
    ctx.eval_roi_noalloc(tree, roi, a, stream=stream)
    b = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_matches_eval_roi(ctx, torch, cloud):
    pts = cloud
    tree = ctx.build_tree(dev(torch, pts), knn_k=32)
    h2 = ctx.debug_point_h2(tree)
    rois = [
        # 112^3 uniform Epanechnikov (4x4x4 tiles, full slot capacity)
        Roi((0.2, 0.15, 0.25), (0.8, 0.85, 0.75), (112, 112, 112), kernel="epanechnikov",
            bw="roi_scaled", h=(0.012,) * 3),
        # a smaller second call: per-point truncated Gaussian, ragged grid
        Roi((0.3, 0.35, 0.2), (0.55, 0.6, 0.5), (40, 36, 44), kernel="gauss_trunc3",
            bw="per_point", norm="count"),
        # 200^3: the per-tile arrays take the slot capacity down to 32
        Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (200, 200, 200), kernel="epanechnikov",
            bw="fixed", h=(0.008, 0.008, 0.008)),
        # small again, fixed anisotropic bandwidth
        Roi((0.4, 0.1, 0.3), (0.6, 0.9, 0.7), (17, 29, 23), kernel="epanechnikov",
            bw="fixed", h=(0.02, 0.05, 0.03)),
        # sparse: 16^3 bricks (scatter evaluation)
        Roi((0.45, 0.45, 0.45), (0.55, 0.55, 0.55), (150, 150, 150), kernel="epanechnikov",
            bw="roi_scaled", h=(0.01,) * 3),
        # dense (several particles per node): the particle sweep
        Roi((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (44, 40, 48), kernel="epanechnikov",
            bw="roi_scaled", h=(0.02,) * 3),
    ]
    for i, roi in enumerate(rois):
        say("noalloc roi", i, roi.res, roi.kernel, roi.bw)
        got, ref = _both(ctx, torch, tree, roi)
        assert np.array_equal(got, ref), "roi %d: %d nodes differ" % (i, int(np.sum(got != ref)))
        nodes = sample_nodes(None, roi.n_nodes, 48, 10 + i, extra=[int(np.argmax(got))])
        want = oracle.density(pts, roi, nodes=nodes, h2=h2 if roi.bw == "per_point" else None)
        check_sampled(got, nodes, want, "noalloc roi %d" % i)
    # the same ROI again after the larger ones (stale scratch contents), on
    # another stream
    s = torch.cuda.Stream()
    got, ref = _both(ctx, torch, tree, rois[1], stream=s)
    assert np.array_equal(got, ref)
    tree.close()


def test_noalloc_rejections(ctx, torch, cloud, sfk):
    from paper_2601_20758_amd import _lib as L
    tree = ctx.build_tree(dev(torch, cloud[:20000]))
    # 600^3 nodes = 3.4M tiles of 4x4x4: the per-tile arrays exceed the array
    # (forced tiles: this sparse ROI would otherwise take 16^3 bricks, 54k of
    # which fit)
    ctx.set_eval_opts(tile_shape=1)
    big = Roi((0, 0, 0), (1, 1, 1), (600, 600, 600), kernel="epanechnikov", bw="fixed",
              h=(0.01,) * 3)
    out = torch.full((big.n_nodes,), 7.0, device="cuda")
    with pytest.raises(sfk.SfkError) as e:
        ctx.eval_roi_noalloc(tree, big, out)
    assert e.value.status == 3  # SFK_E_BUDGET
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))  # nothing was launched
    del out
    ctx.set_eval_opts()
    inbox = Roi((0.2, 0.2, 0.2), (0.6, 0.6, 0.6), (16, 16, 16), bw="fixed", h=(0.02,) * 3,
                set="in_roi")
    with pytest.raises(sfk.SfkError) as e:
        ctx.eval_roi_noalloc(tree, inbox, torch.empty(inbox.n_nodes, device="cuda"))
    assert e.value.status == 7  # SFK_E_UNSUPPORTED
    # a NULL tree through the raw ABI
    r = L.RoiC()
    assert L.lib().sfk_eval_roi_noalloc(ctx._h, None, C.byref(r), None) == 1
    assert L.NOALLOC_SCRATCH_BYTES == 64 << 20
    tree.close()


def test_noalloc_sweep_too_large_takes_the_default_without_it(ctx, torch, cloud):
    # a ROI forced to the particle sweep whose 8^3-node sums (8 B a node)
    # do not fit the array: the entry point takes the shape the ROI would
    # take without the sweep (here sparse: bricks), which sum the same
    # integer terms, so the grid still equals the sweep's bit for bit
    tree = ctx.build_tree(dev(torch, cloud))
    roi = Roi((0, 0, 0), (1, 1, 1), (216, 208, 200), kernel="epanechnikov", bw="fixed",
              h=(0.006,) * 3)
    ctx.set_eval_opts(tile_shape=7)
    a = torch.full((roi.n_nodes,), -1.0, device="cuda")
    ctx.eval_roi_noalloc(tree, roi, a)
    b = ctx.eval_roi(tree, roi)
    torch.cuda.synchronize()
    ctx.set_eval_opts()
    got, ref = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(got, ref)
    nodes = sample_nodes(None, roi.n_nodes, 48, 21, extra=[int(np.argmax(got))])
    check_sampled(got, nodes, oracle.density(cloud, roi, nodes=nodes), "noalloc sweep fallback")
    tree.close()
