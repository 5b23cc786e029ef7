"""Helpers and fixtures shared by the GPU parity tests (numerical bars,
sampled-node checks, a context per test)."""
import sys

import numpy as np
import pytest


REL_TOL = 1e-5
ABS_TOL = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def sfk():
    import paper_2601_20758_amd as m
    return m


@pytest.fixture()
def ctx(sfk, torch):
    c = sfk.Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_density(got, ref, label=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    peak = ref.max() if ref.size else 0.0
    if peak <= 0:
        assert np.all(got == 0), label
        return 0.0
    big = ref >= 1e-3 * peak
    rel = np.abs(got[big] - ref[big]) / ref[big]
    small = np.abs(got[~big] - ref[~big]).max(initial=0.0)
    assert rel.max() <= REL_TOL, "%s: max rel err %.3g at %d" % (label, rel.max(), np.argmax(rel))
    assert small <= ABS_TOL * peak, "%s: small-node abs err %.3g (peak %.3g)" % (label, small, peak)
    return rel.max()


def check_sampled(got_full, nodes, ref, label=""):
    """Sampled-node check: the peak is the larger of the GPU grid's maximum
    and the sampled reference maximum; an empty field must be exactly zero."""
    got_full = np.asarray(got_full, dtype=np.float64)
    got = got_full[nodes]
    peak = max(float(np.max(ref, initial=0.0)), float(got_full.max(initial=0.0)))
    if peak <= 0.0:
        assert np.all(got == 0.0) and np.all(ref == 0.0), label
        return
    big = ref >= 1e-3 * peak
    if big.any():
        rel = np.abs(got[big] - ref[big]) / ref[big]
        assert rel.max() <= REL_TOL, "%s: max rel err %.3g" % (label, rel.max())
    assert np.max(np.abs(got[~big] - ref[~big]), initial=0.0) <= ABS_TOL * peak, label


def sample_nodes(ref_full_or_none, m, k, seed, extra=()):
    g = np.random.default_rng(seed)
    nodes = set(int(v) for v in g.choice(m, size=min(k, m), replace=False))
    nodes.update(int(v) for v in extra)
    return np.array(sorted(nodes), dtype=np.int64)


