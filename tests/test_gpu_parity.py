"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Expected values come from tests/golden/make_oracle_golden.py, which calls only
the oracle and the seeded input generators.  The bar (relative error of images
and rows, in max-norm and L2) is 1e-4, the tolerance the method's FP32 images
are held to against the FP64 oracle.
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-4


@pytest.fixture(scope="module")
def lm():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_17111_amd as lm

    return lm


def _rel(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = got - ref
    return (np.abs(d).max() / np.abs(ref).max(), np.linalg.norm(d) / np.linalg.norm(ref))


def _dev(ev):
    from paper_2305_17111_amd import events_to_device

    return events_to_device(ev)


def _digest(ev):
    import hashlib

    h = hashlib.sha256()
    for k in ("bin", "angle", "energy"):
        h.update(np.ascontiguousarray(ev[k]).tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def small(lm):
    import torch

    g = np.load(os.path.join(GOLD, "16x16_2k_oracle.npz"))
    p = synth.CONFIGS["16x16_2k"].params
    ctx = lm.Context(p, torch.from_numpy(g["mu"].astype(np.float32)))
    ev = {"bin": g["bin"], "angle": g["angle"], "energy": g["energy"]}
    return p, g, ctx, _dev(ev)


def test_small_sensitivity(small):
    p, g, ctx, ev = small
    sens = ctx.sensitivity(4).cpu().numpy()
    mx, l2 = _rel(sens, g["sens"])
    assert mx < TOL and l2 < TOL, (mx, l2)


def test_small_forward_every_event(small):
    import torch

    p, g, ctx, ev = small
    pj = ctx.forward(ev, torch.from_numpy(g["act"].astype(np.float32)).cuda()).cpu().numpy()
    rel = np.abs(pj - g["p_act"]) / g["p_act"]
    assert rel.max() < TOL, rel.max()


def test_small_backproject(small):
    import torch

    p, g, ctx, ev = small
    out = ctx.backproject(ev, torch.from_numpy(g["bp_w"].astype(np.float32)).cuda()).cpu().numpy()
    mx, l2 = _rel(out, g["bp"])
    assert mx < TOL and l2 < TOL, (mx, l2)
    assert np.all(out[~g["support"]] == 0)


def test_small_osem_every_subiteration(small):
    import torch

    p, g, ctx, ev = small
    nsub = 4
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, nsub)
    worst = 0.0
    for k in range(g["hist"].shape[0]):
        sk, ll = plan.osem_subiter(k % nsub, sens, lam, stats=True)
        mx, l2 = _rel(lam.cpu().numpy(), g["hist"][k])
        worst = max(worst, mx, l2)
        assert mx < TOL and l2 < TOL, (k, mx, l2)
        assert sk == g["skipped"][k]
        assert ll == pytest.approx(g["ll"][k], rel=1e-5)
    print("small worst relative error over 40 sub-iterations", worst)


def test_small_end_to_end_with_gpu_sensitivity(small):
    import torch

    p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    plan.osem_iter(10, sens, lam)
    mx, l2 = _rel(lam.cpu().numpy(), g["hist"][-1])
    assert mx < TOL and l2 < TOL, (mx, l2)


def test_small_resume_is_bitwise_identical(small):
    import torch

    p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    plan = ctx.plan(ev, 4)
    a = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    b = a.clone()
    plan.osem_iter(3, sens, a)
    plan.osem_iter(1, sens, b)
    for s in range(4):                 # stop after iteration 1, resume subset by subset
        plan.osem_subiter(s, sens, b)
    plan.osem_iter(1, sens, b)
    assert torch.equal(a, b)


def test_small_event_tiles_agree_and_runs_are_deterministic(small):
    import torch

    p, g, ctx, ev = small
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    outs = {}
    for jt in (16, 32, 64, 64):
        plan.set_event_tile(jt)
        lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
        plan.osem_iter(2, sens, lam)
        if jt in outs:
            assert torch.equal(outs[jt], lam)          # run-to-run bitwise
        outs[jt] = lam
    ref = g["hist"][7]
    for jt, lam in outs.items():
        mx, l2 = _rel(lam.cpu().numpy(), ref)
        assert mx < TOL and l2 < TOL, (jt, mx, l2)
    a, b = outs[16].cpu().numpy(), outs[64].cpu().numpy()
    assert np.abs(a - b).max() / np.abs(a).max() < 1e-5


def test_batched_cases_equal_independent_runs(small, lm):
    import torch

    p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    rng = np.random.default_rng(3)
    n = ev["bin"].numel()
    cuts = np.sort(rng.choice(np.arange(1, n), 2, replace=False))
    offs = [0, int(cuts[0]), int(cuts[1]), n]
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    batched = lam0.repeat(3, 1).contiguous()
    ctx.plan(ev, 4, case_offsets=offs).osem_iter(2, sens, batched)
    for c in range(3):
        sub = {k: v[offs[c]:offs[c + 1]].contiguous() for k, v in ev.items()}
        lam = lam0.clone()
        ctx.plan(sub, 4).osem_iter(2, sens, lam)
        assert torch.equal(lam, batched[c])


def test_64x64_sampled_rows_at_full_size(lm):
    import torch

    g = np.load(os.path.join(GOLD, "64x64_50k_oracle.npz"))
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True)
    assert _digest(ev) == str(g["digest"])
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    pj = ctx.forward(_dev(ev), torch.from_numpy(act.astype(np.float32)).cuda()).cpu().numpy()
    rel = np.abs(pj[g["idx"]] - g["p_act"]) / g["p_act"]
    assert rel.max() < TOL, rel.max()
    sens = ctx.sensitivity(w.n_subsets).cpu().numpy()
    got = sens[:, g["pix"]]
    assert np.abs(got - g["sens"]).max() / np.abs(g["sens"]).max() < TOL


def test_64x64_count_conservation_full_size(lm):
    import torch

    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True)
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    sens = ctx.sensitivity(w.n_subsets)
    plan = ctx.plan(_dev(ev), w.n_subsets)
    lam = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    for s in range(w.n_subsets):
        sk, _ = plan.osem_subiter(s, sens, lam, stats=True)
        Js = int(np.sum(ev["angle"] % w.n_subsets == s))
        tot = float((sens[s].double() * lam.double()).sum())
        assert tot == pytest.approx(Js - sk, rel=TOL)
        assert bool(torch.all(lam >= 0))


def test_64x64_one_full_iteration(lm):
    import torch

    path = os.path.join(GOLD, "64x64_50k_iter_oracle.npz")
    g = np.load(path)
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, 2000, 23)
    assert _digest(ev) == str(g["digest"])
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(_dev(ev), w.n_subsets)
    for k in range(g["hist"].shape[0]):
        plan.osem_subiter(k, sens, lam)
        mx, l2 = _rel(lam.cpu().numpy(), g["hist"][k])
        assert mx < TOL and l2 < TOL, (k, mx, l2)


def test_128x128_sampled_rows_at_128(lm):
    import torch

    g = np.load(os.path.join(GOLD, "128x128_16cases_oracle.npz"))
    w = synth.CONFIGS["128x128_16cases"]
    p = w.params
    mu, act, _ = synth.phantom(w, 0)
    ev = synth.generic_events(p, act, 20000, 5300)
    assert _digest(ev) == str(g["digest"])
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    pj = ctx.forward(_dev(ev), torch.from_numpy(act.astype(np.float32)).cuda()).cpu().numpy()
    rel = np.abs(pj[g["idx"]] - g["p_act"]) / g["p_act"]
    assert rel.max() < TOL, rel.max()


def test_invalid_inputs_are_rejected(small, lm):
    import torch

    p, g, ctx, ev = small
    for key, val in (("bin", 16), ("angle", 32), ("energy", 110.0), ("energy", float("nan"))):
        bad = {k: v.clone() for k, v in ev.items()}
        bad[key][5] = val
        with pytest.raises(lm.LmmewError) as e:
            ctx.plan(bad, 4)
        assert e.value.status == -1 and "event 5" in str(e.value)
    with pytest.raises(lm.LmmewError):
        ctx.plan(ev, 0)
    with pytest.raises(lm.LmmewError):
        ctx.sensitivity(33)
    mu = torch.from_numpy(g["mu"].astype(np.float32)).clone()
    mu[3] = float("nan")
    with pytest.raises(lm.LmmewError):
        lm.Context(p, mu)
    with pytest.raises(lm.LmmewError):
        lm.Context(synth.replace(p, ns=5), torch.from_numpy(g["mu"].astype(np.float32)))


def test_empty_and_single_event_lists(small, lm):
    import torch

    p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    empty = {k: v[:0].contiguous() for k, v in ev.items()}
    assert ctx.forward(empty, sens[0]).numel() == 0
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    ctx.plan(empty, 4).osem_iter(1, sens, lam)
    # no events: every pixel the subsets can see goes to zero (Eq. (18) numerator is 0)
    assert float(lam.abs().max()) == 0.0
    one = {k: v[:1].contiguous() for k, v in ev.items()}
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(one, 1)
    s1 = ctx.sensitivity(1)
    plan.osem_iter(1, s1, lam)
    # count conservation with a single event
    assert float((s1[0].double() * lam.double()).sum()) == pytest.approx(1.0, rel=TOL)


def test_graph_launch_equals_eager_and_replays(small):
    import torch

    p, g, ctx, ev = small
    sens = ctx.sensitivity(4)
    plan = ctx.plan(ev, 4)
    lam0 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    eager = lam0.clone()
    plan.osem_iter(3, sens, eager)
    lam = lam0.clone()
    for rep in range(3):
        lam.copy_(lam0)                    # eager work between replays
        torch.cuda.synchronize()
        plan.osem_graph(3, sens, lam)
        torch.cuda.synchronize()
        assert torch.equal(lam, eager), rep
    mx, l2 = _rel(lam.cpu().numpy(), g["hist"][11])
    assert mx < TOL and l2 < TOL


def test_autotune_keeps_results(small):
    import torch

    p, g, ctx, ev = small
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    jt = plan.autotune(use_cache=False)
    assert jt in (16, 32, 64) and plan.event_tile == jt
    assert plan.autotune(use_cache=True) == jt
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan.osem_graph(2, sens, lam)
    mx, l2 = _rel(lam.cpu().numpy(), g["hist"][7])
    assert mx < TOL and l2 < TOL


def test_batched_uneven_cases_in_one_graph(lm):
    import torch

    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    sens = ctx.sensitivity(w.n_subsets)
    counts = [1500, 9000, 300, 4200]
    evs = [synth.generic_events(p, act, n, 700 + c) for c, n in enumerate(counts)]
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("bin", "angle", "energy")}
    offs = np.concatenate([[0], np.cumsum(counts)]).tolist()
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    batched = lam0.repeat(len(counts), 1).contiguous()
    plan = ctx.plan(_dev(cat), w.n_subsets, case_offsets=offs)
    plan.autotune()
    plan.osem_graph(2, sens, batched)
    for c, e in enumerate(evs):
        lam = lam0.clone()
        single = ctx.plan(_dev(e), w.n_subsets)
        single.set_event_tile(plan.event_tile)
        single.osem_iter(2, sens, lam)
        assert torch.equal(lam, batched[c]), c


def test_small_osem_with_unscattered_probabilities_in_kernel(lm):
    """The per-event kernel forming the unscattered paths' bin probabilities
    itself (the table disabled, as when it would not fit) against the oracle,
    every sub-iteration; and the table re-enabled gives the same images to
    rounding."""
    import torch

    g = np.load(os.path.join(GOLD, "16x16_2k_oracle.npz"))
    p = synth.CONFIGS["16x16_2k"].params
    ctx = lm.Context(p, torch.from_numpy(g["mu"].astype(np.float32)))
    assert ctx.psf_table(False) is False
    ev = _dev({"bin": g["bin"], "angle": g["angle"], "energy": g["energy"]})
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan = ctx.plan(ev, 4)
    for k in range(g["hist"].shape[0]):
        plan.osem_subiter(k % 4, sens, lam)
        mx, l2 = _rel(lam.cpu().numpy(), g["hist"][k])
        assert mx < TOL and l2 < TOL, (k, mx, l2)
    assert ctx.psf_table(True) is True
    lam2 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    ctx.plan(ev, 4).osem_iter(10, sens, lam2)
    d = (lam2 - lam).abs().max().item() / lam.abs().max().item()
    assert d < 1e-5, d


def test_rows_of_events_far_from_every_line(lm, oracle_mod):
    """Events in a window below every line's scattered range (30-34 keV with
    lines at 85/154/270 keV: every line's Gaussian factor is below 2^-40 of
    its peak at every reachable scattered energy) keep the nearest line's
    scattered terms, since the line cut is relative to the event's largest
    line factor; their rows (about 1e-18, still normal FP32 numbers) match the
    oracle's, which keeps every term."""
    import math

    import torch

    from paper_2305_17111_amd import line_mask

    p = synth.SysParams(16, 4.0, 8, 16, 16, windows=((30.0, 34.0), synth.EW1))
    k = (p.eres_frac * p.eres_ref / (2.0 * math.sqrt(2.0 * math.log(2.0)))) ** 2 / p.eres_ref
    emin = p.lines[0] / (1.0 + 2.0 * p.lines[0] / p.me)
    mu, act, _ = synth.phantom_disk2(p)
    mu32 = np.asarray(mu, np.float32)
    o = oracle_mod.Oracle(p, mu32.astype(np.float64))
    ctx = lm.Context(p, torch.from_numpy(mu32))
    ev = {"bin": np.array([5, 8, 10, 7], np.int16), "angle": np.array([0, 3, 9, 14], np.int16),
          "energy": np.array([30.5, 32.0, 33.8, 80.0], np.float32)}
    for E in ev["energy"][:3]:
        assert (emin - E) ** 2 / (2 * k * emin) > 40 * math.log(2.0)   # beyond the absolute cut
        assert line_mask(p, float(E)) == 0b001
    rows = ctx.rows(_dev(ev)).cpu().numpy().astype(np.float64)
    for j in range(4):
        ref = o.row(int(ev["bin"][j]), int(ev["angle"][j]), float(ev["energy"][j]))
        m = np.abs(ref).max()
        assert m > 1e-30
        err = np.abs(rows[j] - ref)
        assert np.all(err <= 1e-4 * np.abs(ref) + 1e-7 * m), (j, (err / (np.abs(ref) + 1e-7 * m)).max())
