"""GPU parity of events that carry a continuous lateral position (mm) instead
of a detector bin: the collimator response becomes the Gaussian density at
the position.  Expected values come from tests/golden/make_oracle_golden.py
(small_pos, pos64), which calls only the FP64 oracle and the seeded generators.
The bar is the parity tests' 1e-4 relative error in max-norm and L2."""
import hashlib
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-4


def _rel(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = got - ref
    return (np.abs(d).max() / np.abs(ref).max(), np.linalg.norm(d) / np.linalg.norm(ref))


@pytest.fixture(scope="module")
def small_pos():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_17111_amd as lm

    g = np.load(os.path.join(GOLD, "16x16_2k_pos_oracle.npz"))
    mu = np.load(os.path.join(GOLD, "16x16_2k_oracle.npz"))["mu"]
    p = synth.CONFIGS["16x16_2k"].params
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    ev = lm.events_to_device({"position": g["position"], "angle": g["angle"],
                              "energy": g["energy"]})
    assert "bin" not in ev
    return lm, p, g, ctx, ev


def test_position_rows_and_forward_match_oracle(small_pos):
    import torch

    lm, p, g, ctx, ev = small_pos
    rows = ctx.rows(ev, part=3).cpu().numpy()
    for k, j in enumerate(g["idx"]):
        mx, l2 = _rel(rows[j], g["rows"][k])
        assert mx < TOL and l2 < TOL, (j, mx, l2)
    # the context's model without a surrogate is the exact one
    assert np.array_equal(ctx.rows(ev, part=0).cpu().numpy(), rows)
    act = np.load(os.path.join(GOLD, "16x16_2k_oracle.npz"))["act"]
    pj = ctx.forward(ev, torch.from_numpy(act.astype(np.float32)).cuda()).cpu().numpy()
    rel = np.abs(pj - g["p_act"]) / g["p_act"]
    assert rel.max() < TOL, rel.max()


def test_position_osem_every_subiteration(small_pos):
    import torch

    lm, p, g, ctx, ev = small_pos
    nsub = g["sens"].shape[0]
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, nsub)
    for k in range(g["hist"].shape[0]):
        sk, ll = plan.osem_subiter(k % nsub, sens, lam, stats=True)
        assert sk == int(g["skipped"][k])
        assert ll == pytest.approx(float(g["ll"][k]), rel=1e-5, abs=1e-3)
        mx, l2 = _rel(lam.cpu().numpy(), g["hist"][k])
        assert mx < TOL and l2 < TOL, (k, mx, l2)
    niter = g["hist"].shape[0] // nsub
    graphed = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan.osem_graph(niter, sens, graphed)
    assert torch.equal(graphed, lam)


def test_position_event_tiles_table_and_cached_rows(small_pos):
    import torch

    lm, p, g, ctx, ev = small_pos
    nsub = g["sens"].shape[0]
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    ref = g["hist"][-1]
    niter = g["hist"].shape[0] // nsub
    plan = ctx.plan(ev, nsub)
    outs = {}
    for jt in (16, 32, 64):
        plan.set_event_tile(jt)
        lam = lam0.clone()
        plan.osem_iter(niter, sens, lam)
        mx, l2 = _rel(lam.cpu().numpy(), ref)
        assert mx < TOL and l2 < TOL, (jt, mx, l2)
        outs[jt] = lam
    ctx.path_table(True)
    try:
        tab = lam0.clone()
        plan.osem_iter(niter, sens, tab)
        mx, l2 = _rel(tab.cpu().numpy(), outs[64].cpu().numpy())
        assert mx < 1e-5 and l2 < 1e-5, (mx, l2)
    finally:
        ctx.path_table(False)
    plan.cache_rows(True)
    cached = lam0.clone()
    plan.osem_graph(niter, sens, cached)
    assert torch.equal(cached, outs[64])
    plan.cache_rows(False)


def test_position_batched_cases_equal_independent_runs(small_pos):
    import torch

    lm, p, g, ctx, ev = small_pos
    n = ev["angle"].numel()
    offs = [0, 400, 1100, n]
    sens = ctx.sensitivity(4)
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    batched = lam0.repeat(3, 1).contiguous()
    ctx.plan(ev, 4, case_offsets=offs).osem_iter(2, sens, batched)
    for c in range(3):
        one = {k: v[offs[c]:offs[c + 1]].contiguous() for k, v in ev.items()}
        lam = lam0.clone()
        ctx.plan(one, 4).osem_iter(2, sens, lam)
        assert torch.equal(lam, batched[c]), c


def test_position_rejections(small_pos):
    import torch

    lm, p, g, ctx, ev = small_pos
    for val in (p.R, -p.R - 0.01, float("nan"), float("inf")):
        bad = {k: v.clone() for k, v in ev.items()}
        bad["position"][5] = val
        with pytest.raises(lm.LmmewError) as e:
            ctx.plan(bad, 4)
        assert "event 5" in str(e.value)
    edge = {k: v.clone() for k, v in ev.items()}
    edge["position"][5] = -p.R
    ctx.plan(edge, 4)
    # the scatter surrogate models binned events
    net = ctx.mlp(seed=3)
    net.fit(2000, epochs=1, batch=4096, lr=2e-3, floor_frac=3e-2, seed=1)
    sens = ctx.sensitivity(4)
    plan = ctx.plan(ev, 4)
    try:
        ctx.set_scatter_model(net)
        with pytest.raises(lm.LmmewError):
            plan.osem_iter(1, sens, torch.from_numpy(g["lam0"].astype(np.float32)).cuda())
        with pytest.raises(lm.LmmewError):
            plan.osem_graph(1, sens, torch.from_numpy(g["lam0"].astype(np.float32)).cuda())
        with pytest.raises(lm.LmmewError):
            ctx.forward(ev, sens[0])
        exact = ctx.rows(ev, part=3)               # the exact model stays available
        assert bool(torch.isfinite(exact).all())
    finally:
        ctx.set_scatter_model(None)
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan.osem_iter(1, sens, lam)                   # usable again without the surrogate
    assert bool(torch.isfinite(lam).all())


def test_64x64_position_rows_elementwise_and_conservation_full_size():
    import torch

    import paper_2305_17111_amd as lm

    g = np.load(os.path.join(GOLD, "64x64_50k_pos_oracle.npz"))
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True)
    h = hashlib.sha256()
    for k in ("position", "angle", "energy"):
        h.update(np.ascontiguousarray(ev[k]).tobytes())
    assert h.hexdigest() == str(g["digest"])
    evd = lm.events_to_device({k: ev[k] for k in ("position", "angle", "energy")})
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    pj = ctx.forward(evd, torch.from_numpy(act.astype(np.float32)).cuda()).cpu().numpy()
    rel = np.abs(pj[g["idx"]] - g["p_act"]) / g["p_act"]
    assert rel.max() < TOL, rel.max()
    # whole rows of the sampled events from the plan's sub-iteration launches,
    # with and without the path table, at every event tile: element by element,
    # |gpu - oracle| <= 1e-4 |oracle| + 1e-7 max_q oracle on the support (the
    # density is cut beyond 7 standard deviations, R20/R24), 0 off it
    sens = ctx.sensitivity(w.n_subsets)
    plan = ctx.plan(evd, w.n_subsets)
    support = synth.fov_support(p).ravel()
    ref = g["rows"]
    for table in (False, True):
        ctx.path_table(table)
        for jt in (16, 32, 64):
            plan.set_event_tile(jt)
            rows = {}
            for s in range(w.n_subsets):
                sel = [int(j) for j in g["idx"] if int(ev["angle"][j]) % w.n_subsets == s]
                if sel:
                    for j, r in zip(sel, plan.rows(s, sel).cpu().numpy()):
                        rows[j] = r
            for k, j in enumerate(g["idx"]):
                x, r = rows[int(j)].astype(np.float64), ref[k]
                assert np.all(x[~support] == 0), (table, jt, k)
                m = np.abs(r[support]).max()
                err = np.abs(x[support] - r[support])
                assert np.all(err <= TOL * np.abs(r[support]) + 1e-7 * m), (
                    table, jt, k, float((err / (np.abs(r[support]) + 1e-7 * m)).max()))
    ctx.path_table(False)
    plan.set_event_tile(16)
    # count conservation of every sub-iteration (holds for any row scale)
    lam = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    for s in range(w.n_subsets):
        sk, _ = plan.osem_subiter(s, sens, lam, stats=True)
        Js = int(np.sum(ev["angle"] % w.n_subsets == s))
        tot = float((sens[s].double() * lam.double()).sum())
        assert tot == pytest.approx(Js - sk, rel=TOL)
        assert bool(torch.all(lam >= 0))
