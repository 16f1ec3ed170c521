"""The scatter-path parameter table (lmmew_path_table): rows and OSEM with the
table must match the FP64 oracle like the in-kernel evaluation does, and agree
with it to rounding."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-4


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


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b).max() / np.abs(b).max(), np.linalg.norm(a - b) / np.linalg.norm(b)


def test_table_rows_and_osem_match_oracle(small):
    import torch

    lm, p, g, ctx, ev = small
    rows0 = ctx.rows(ev, part=3).cpu().numpy()
    ctx.path_table(True)
    try:
        assert ctx.path_table_bytes == p.na * 52 * 3 * 2 * 256 * 4   # 52 points, 3 lines, 2 values
        rows1 = ctx.rows(ev, part=3).cpu().numpy()
        mx, l2 = _rel(rows1, rows0)
        assert mx < 1e-6 and l2 < 1e-6, (mx, l2)
        sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
        lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
        plan = ctx.plan(ev, 4)
        for k in range(g["hist"].shape[0]):
            plan.osem_subiter(k % 4, sens, lam)
            mx, l2 = _rel(lam.cpu().numpy(), g["hist"][k])
            assert mx < TOL and l2 < TOL, (k, mx, l2)
    finally:
        ctx.path_table(False)


def test_table_graph_recaptures_when_the_table_goes(small):
    import torch

    lm, p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    ref = lam0.clone()
    plan.osem_iter(3, sens, ref)
    ctx.path_table(True)
    a = lam0.clone()
    plan.osem_graph(3, sens, a)
    ctx.path_table(False)                      # the captured graph refers to the freed table
    b = lam0.clone()
    plan.osem_graph(3, sens, b)                # must recapture without it
    assert torch.equal(b, ref)
    mx, l2 = _rel(a.cpu().numpy(), ref.cpu().numpy())
    assert mx < 1e-5 and l2 < 1e-5


def test_table_full_size_iteration():
    import torch

    import paper_2305_17111_amd as lm

    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    ev = lm.events_to_device(synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True))
    sens = ctx.sensitivity(w.n_subsets)
    plan = ctx.plan(ev, w.n_subsets)
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    a = lam0.clone()
    plan.osem_iter(1, sens, a)
    ctx.path_table(True)
    b = lam0.clone()
    plan.osem_graph(1, sens, b)
    ctx.path_table(False)
    mx, l2 = _rel(b.cpu().numpy(), a.cpu().numpy())
    assert mx < 1e-5 and l2 < 1e-5, (mx, l2)


def test_table_in_plans_over_several_maps():
    import torch

    import paper_2305_17111_amd as lm

    w = synth.CONFIGS["16x16_2k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    maps = [mu] + list(synth.random_body_maps(p, 2, seed=8))
    ctxs = [lm.Context(p, torch.from_numpy(m.astype(np.float32))) for m in maps]
    counts = [600, 900, 300]
    evs = [synth.generic_events(p, act, n, 40 + c) for c, n in enumerate(counts)]
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("bin", "angle", "energy")}
    offs = np.concatenate([[0], np.cumsum(counts)]).tolist()
    sens = torch.stack([c.sensitivity(4) for c in ctxs]).contiguous()
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda().repeat(3, 1).contiguous()
    plan = lm.plan_maps(ctxs, lm.events_to_device(cat), 4, offs)
    ref = lam0.clone()
    plan.osem_iter(2, sens, ref)
    for c in ctxs[:2]:
        c.path_table(True)
    mixed = lam0.clone()                        # one case without a table: no table is used
    plan.osem_graph(2, sens, mixed)
    assert torch.equal(mixed, ref)
    ctxs[2].path_table(True)
    tab = lam0.clone()
    plan.osem_graph(2, sens, tab)
    for c, e in enumerate(evs):
        own = lam0[c].clone()
        ctxs[c].plan(lm.events_to_device(e), 4).osem_iter(2, sens[c], own)
        assert torch.equal(own, tab[c]), c
    mx, l2 = _rel(tab.cpu().numpy(), ref.cpu().numpy())
    assert mx < 1e-5 and l2 < 1e-5
    for c in ctxs:
        c.path_table(False)
