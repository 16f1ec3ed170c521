"""Cached-row mode (lmmew_plan_cache_rows): the rows of every subset are
computed once and the iterations read them.  The results must be bitwise
identical to the matrix-free iterations, which the parity tests pin to the
FP64 oracle."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def small():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_17111_amd as lm

    g = np.load(os.path.join(GOLD, "16x16_2k_oracle.npz"))
    p = synth.CONFIGS["16x16_2k"].params
    ctx = lm.Context(p, torch.from_numpy(g["mu"].astype(np.float32)))
    ev = lm.events_to_device({"bin": g["bin"], "angle": g["angle"], "energy": g["energy"]})
    return lm, p, g, ctx, ev


def test_cached_equals_matrix_free_eager_graph_and_stats(small):
    import torch

    lm, p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    a = lam0.clone()
    sk_a, ll_a = plan.osem_iter(10, sens, a, stats=True)
    plan.cache_rows(True)
    b = lam0.clone()
    sk_b, ll_b = plan.osem_iter(10, sens, b, stats=True)
    assert torch.equal(a, b)
    assert sk_a == sk_b and ll_a == ll_b
    c = lam0.clone()
    plan.osem_graph(10, sens, c)
    assert torch.equal(a, c)
    plan.cache_rows(False)
    d = lam0.clone()
    plan.osem_graph(10, sens, d)                  # recaptured without the cache
    assert torch.equal(a, d)


def test_cached_batched_cases(small):
    import torch

    lm, p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    n = ev["bin"].numel()
    offs = [0, 700, 1500, n]
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda().repeat(3, 1).contiguous()
    plan = ctx.plan(ev, 4, case_offsets=offs)
    a = lam0.clone()
    plan.osem_iter(3, sens, a)
    plan.cache_rows(True)
    b = lam0.clone()
    plan.osem_graph(3, sens, b)
    assert torch.equal(a, b)


def test_cached_rows_follow_the_scatter_model(small):
    import torch

    lm, p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    net = ctx.mlp(seed=3)
    net.fit(2000, epochs=1, batch=4096, lr=2e-3, floor_frac=3e-2, seed=1)
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    try:
        ctx.set_scatter_model(net)
        a = lam0.clone()
        plan.osem_iter(2, sens, a)
        plan.cache_rows(True)
        b = lam0.clone()
        plan.osem_iter(2, sens, b)
        assert torch.equal(a, b)
        ctx.set_scatter_model(None)              # the cached rows are now stale
        with pytest.raises(lm.LmmewError):
            plan.osem_iter(1, sens, lam0.clone())
        plan.cache_rows(True)
        c = lam0.clone()
        plan.osem_iter(2, sens, c)
        ref = lam0.clone()
        ctx.plan(ev, 4).osem_iter(2, sens, ref)
        assert torch.equal(c, ref)
    finally:
        ctx.set_scatter_model(None)


def test_cached_full_size_iteration():
    import torch

    import paper_2305_17111_amd as lm

    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True)
    sens = ctx.sensitivity(w.n_subsets)
    plan = ctx.plan(lm.events_to_device(ev), w.n_subsets)
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    a = lam0.clone()
    plan.osem_iter(1, sens, a)
    plan.cache_rows(True)
    b = lam0.clone()
    plan.osem_graph(1, sens, b)
    assert torch.equal(a, b)


def test_cached_rows_match_oracle_every_subiteration(small):
    """The cached-row iterations (Algorithm 1's loop read from stored rows)
    against the FP64 oracle's images after each of the 40 sub-iterations."""
    import torch

    lm, p, g, ctx, ev = small
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    plan.cache_rows(True)
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    for k in range(g["hist"].shape[0]):
        sk, ll = plan.osem_subiter(k % 4, sens, lam, stats=True)
        ref = g["hist"][k]
        d = lam.cpu().numpy().astype(np.float64) - ref
        assert np.abs(d).max() / np.abs(ref).max() < 1e-4, k
        assert np.linalg.norm(d) / np.linalg.norm(ref) < 1e-4, k
        assert sk == int(g["skipped"][k])
        assert ll == pytest.approx(float(g["ll"][k]), rel=1e-4)
