"""GPU parity at the benchmarked sizes, element by element, through the C ABI.

- Rows a_jq (Eq. (3)) of sampled events of the 64x64 workload (50k events, 8
  subsets) taken from the sub-iteration launches of the full plan, with and
  without the path-parameter table, at every event tile, against the FP64
  oracle's rows over every support pixel.
- The same at 128x128 (2 mm pixels, 64x64 scatter points, four windows).
- One sub-iteration of Eq. (18) on a plan over two patients of the 128x128
  workload with their own attenuation maps, against the oracle's update of
  each patient (and the GPU sensitivity of that subset against the oracle's).
- One full iteration of the 64x64 workload's 2000-event list with the path
  table (the configuration the bench times).

Row tolerance: |gpu - oracle| <= 1e-4 |oracle| + 1e-7 max_q oracle, per row:
the method's FP32 bar, plus the absolute floor below which an FP32 row may
round single tiny elements (terms dropped beyond 7 standard deviations of a
Gaussian are relatively < 2.3e-11 of their row).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-4
FLOOR = 1e-7


@pytest.fixture(scope="module")
def lm():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_17111_amd as lm

    return lm


def _digest(ev):
    import hashlib

    h = hashlib.sha256()
    for k in ("bin", "angle", "energy"):
        h.update(np.ascontiguousarray(ev[k]).tobytes())
    return h.hexdigest()


def _rel(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = got - ref
    return (np.abs(d).max() / np.abs(ref).max(), np.linalg.norm(d) / np.linalg.norm(ref))


def _check_rows(got, ref, support, what):
    """Element-wise bar on every support pixel; zero off the support."""
    got = np.asarray(got, np.float64)
    worst = 0.0
    for k in range(ref.shape[0]):
        r, g_ = ref[k], got[k]
        assert np.all(g_[~support] == 0), (what, k)
        m = np.abs(r[support]).max()
        err = np.abs(g_[support] - r[support])
        bound = TOL * np.abs(r[support]) + FLOOR * m
        assert np.all(err <= bound), (what, k, float((err / (np.abs(r[support]) + FLOOR * m)).max()))
        worst = max(worst, float((err / (np.abs(r[support]) + FLOOR * m)).max()))
    return worst


def _plan_rows(plan, ev, idx, nsub):
    """Rows of input events idx from the sub-iteration launches of the plan."""
    rows = {}
    for s in range(nsub):
        sel = [int(j) for j in idx if int(ev["angle"][j]) % nsub == s]
        if sel:
            r = plan.rows(s, sel).cpu().numpy()
            for j, row in zip(sel, r):
                rows[j] = row
    return np.stack([rows[int(j)] for j in idx])


def test_64x64_rows_elementwise_full_plan(lm):
    import torch

    g = np.load(os.path.join(GOLD, "64x64_50k_oracle.npz"))
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True)
    assert _digest(ev) == str(g["digest"])
    support = synth.fov_support(p)
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    plan = ctx.plan(lm.events_to_device(ev), w.n_subsets)
    ref = g["rows"]
    assert np.allclose(ref @ act.astype(np.float32).astype(np.float64), g["p_act"], rtol=1e-12)
    worst = {}
    for table in (False, True):
        ctx.path_table(table)
        for jt in (16, 32, 64):
            plan.set_event_tile(jt)
            print(f"64x64 rows: table={table} event_tile={jt}", flush=True)
            got = _plan_rows(plan, ev, g["idx"], w.n_subsets)
            worst[(table, jt)] = _check_rows(got, ref, support, (table, jt))
    ctx.path_table(False)
    print("64x64 worst relative element error", worst)


def test_64x64_one_full_iteration_with_path_table(lm):
    import torch

    g = np.load(os.path.join(GOLD, "64x64_50k_iter_oracle.npz"))
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, 2000, 23)
    assert _digest(ev) == str(g["digest"])
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    ctx.path_table(True)
    sens = torch.from_numpy(g["sens"].astype(np.float32)).cuda()
    plan = ctx.plan(lm.events_to_device(ev), w.n_subsets)
    plan.autotune(use_cache=False)
    lam = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    for k in range(g["hist"].shape[0]):
        sk, ll = plan.osem_subiter(k, sens, lam, stats=True)
        mx, l2 = _rel(lam.cpu().numpy(), g["hist"][k])
        assert mx < TOL and l2 < TOL, (k, mx, l2)
        assert sk == int(g["skipped"][k])
        assert ll == pytest.approx(float(g["ll"][k]), rel=TOL)
    # and the same iteration as one graph launch from the start
    lam2 = torch.from_numpy(g["lam0"].astype(np.float32)).cuda()
    plan.osem_graph(1, sens, lam2)
    assert torch.equal(lam2, lam)


def test_128x128_rows_elementwise_full_plan(lm):
    import torch

    g = np.load(os.path.join(GOLD, "128x128_16cases_oracle.npz"))
    w = synth.CONFIGS["128x128_16cases"]
    p = w.params
    mu, act, _ = synth.phantom(w, 0)
    ev = synth.generic_events(p, act, 20000, 5300)
    assert _digest(ev) == str(g["digest"])
    support = synth.fov_support(p)
    ctx = lm.Context(p, torch.from_numpy(mu.astype(np.float32)))
    plan = ctx.plan(lm.events_to_device(ev), w.n_subsets)
    worst = {}
    for jt in (16, 32, 64):
        plan.set_event_tile(jt)
        print(f"128x128 rows: event_tile={jt}", flush=True)
        got = _plan_rows(plan, ev, g["idx"], w.n_subsets)
        worst[jt] = _check_rows(got, g["rows"], support, jt)
    print("128x128 worst relative element error", worst)


def test_128x128_two_patient_maps_one_subiteration(lm):
    import torch

    g = np.load(os.path.join(GOLD, "128x128_maps_subiter_oracle.npz"))
    w = synth.CONFIGS["128x128_16cases"]
    p = w.params
    nsub = w.n_subsets
    ctxs, evs, sens_ref = [], [], []
    for c in (0, 1):
        _, mu, act, _, ev = synth.workload_inputs(w.name, c)
        assert _digest(ev) == str(g[f"digest{c}"])
        sel = g[f"sel{c}"]
        evs.append({k: ev[k][sel] for k in ("bin", "angle", "energy")})
        ctxs.append(lm.Context(p, torch.from_numpy(mu.astype(np.float32))))
        sens_ref.append(g[f"sens{c}"])
    # the GPU sensitivity of subset 0 against the oracle's
    for c in (0, 1):
        s_gpu = ctxs[c].sensitivity(nsub)[0].cpu().numpy()
        mx, l2 = _rel(s_gpu, sens_ref[c])
        assert mx < TOL and l2 < TOL, (c, mx, l2)
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("bin", "angle", "energy")}
    offs = [0, evs[0]["bin"].size, evs[0]["bin"].size + evs[1]["bin"].size]
    plan = lm.plan_maps(ctxs, lm.events_to_device(cat), nsub, offs)
    Q = p.n * p.n
    sens = np.zeros((2, nsub, Q), np.float32)
    for c in (0, 1):
        sens[c, 0] = sens_ref[c].astype(np.float32)
    sens = torch.from_numpy(sens).cuda()
    lam = torch.from_numpy(np.stack([g["lam0_0"], g["lam0_1"]]).astype(np.float32)).cuda()
    for jt in (16, 32, 64):
        plan.set_event_tile(jt)
        lam_j = lam.clone()
        sk, ll = plan.osem_subiter(0, sens, lam_j, stats=True)
        assert sk == int(g["skipped0"]) + int(g["skipped1"])
        assert ll == pytest.approx(float(g["ll0"]) + float(g["ll1"]), rel=TOL)
        for c in (0, 1):
            mx, l2 = _rel(lam_j[c].cpu().numpy(), g[f"lam1_{c}"])
            assert mx < TOL and l2 < TOL, (jt, c, mx, l2)
    # the same sub-iteration from cached rows (every subset's rows computed
    # once): equal to the matrix-free one bitwise, so to the oracle as above
    lam_mf = lam.clone()
    plan.osem_subiter(0, sens, lam_mf)
    plan.cache_rows(True)
    try:
        lam_c = lam.clone()
        sk, ll = plan.osem_subiter(0, sens, lam_c, stats=True)
        assert sk == int(g["skipped0"]) + int(g["skipped1"])
        assert bool((lam_c == lam_mf).all())
    finally:
        plan.cache_rows(False)
