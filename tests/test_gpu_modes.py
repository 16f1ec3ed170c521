"""The single-window special cases of the method (Sec. 3.2.2) and the regional
figures of merit (Sec. 3.1.4), on the GPU through the C ABI.

LM-MEW uses every window of the 16x16 workload (68-102 and 123-184 keV);
LM-SEW uses the model and the events of the 68-102 keV window only;
Binned-SEW is LM-SEW with every event assigned 85 keV.  Each method
reconstructs S object realisations x N noise realisations of exact-model
events as ONE batched plan (one captured graph for all cases).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
S, N, J = 3, 8, 2000


@pytest.fixture(scope="module")
def study():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import oracle

    w = synth.CONFIGS["16x16_2k"]
    p = w.params
    mu, acts, rois = synth.disk2_objects(p, S, seed=101)
    mu32 = mu.astype(np.float32)
    orc = oracle.Oracle(p, mu32.astype(np.float64))
    evs, truth = [], np.zeros((S, len(rois)))
    for s in range(S):
        ev = orc.sample_events(acts[s], J * N, seed=500 + s)
        # the expected counts are lambda_q x sensitivity_q: the true image in the
        # reconstruction's units is activity x J / (total detected mass)
        lam_true = acts[s] * J / ev["total_mass"]
        truth[s] = [lam_true[r].sum() for r in rois]
        for n in range(N):
            sl = slice(n * J, (n + 1) * J)
            evs.append({"bin": ev["bin"][sl], "angle": ev["angle"][sl],
                        "energy": ev["energy"][sl].astype(np.float32)})
    return p, mu32, rois, orc, evs, truth


def _reconstruct(lm, ctx, evs, p, n_iters=10, nsub=4):
    import torch

    counts = [len(e["bin"]) for e in evs]
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("bin", "angle", "energy")}
    offs = np.concatenate([[0], np.cumsum(counts)]).tolist()
    plan = ctx.plan(lm.events_to_device(cat), nsub, case_offsets=offs)
    lam = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    lam = lam.repeat(len(evs), 1).contiguous()
    plan.osem_graph(n_iters, ctx.sensitivity(nsub), lam)
    return lam


def test_single_window_model_matches_oracle(study):
    import torch

    import oracle
    import paper_2305_17111_amd as lm

    p, mu32, rois, orc, evs, truth = study
    p1 = synth.replace(p, windows=(synth.EW1,))
    ev = synth.sew_events(evs[0], synth.EW1)
    o1 = oracle.Oracle(p1, mu32.astype(np.float64))
    lam0 = o1.support.astype(np.float64)
    ref, _, _, _ = o1.osem({**ev, "energy": ev["energy"].astype(np.float64)}, 4, 1, lam0)
    ctx = lm.Context(p1, torch.from_numpy(mu32))
    lam = torch.from_numpy(lam0.astype(np.float32)).cuda()
    ctx.plan(lm.events_to_device(ev), 4).osem_iter(1, ctx.sensitivity(4), lam)
    d = lam.cpu().numpy() - ref
    assert np.abs(d).max() / np.abs(ref).max() < 1e-4
    assert np.linalg.norm(d) / np.linalg.norm(ref) < 1e-4


def test_mew_sew_binned_figures_of_merit(study):
    import torch

    import paper_2305_17111_amd as lm
    from oracle import fom

    p, mu32, rois, orc, evs, truth = study
    masks = np.stack(rois).astype(np.uint8)
    p1 = synth.replace(p, windows=(synth.EW1,))
    methods = {
        "LM-MEW": (p, evs),
        "LM-SEW": (p1, [synth.sew_events(e, synth.EW1) for e in evs]),
        "Binned-SEW": (p1, [synth.sew_events(e, synth.EW1, energy_keV=85.0) for e in evs]),
    }
    res = {}
    for name, (pp, ee) in methods.items():
        ctx = lm.Context(pp, torch.from_numpy(mu32))
        lam = _reconstruct(lm, ctx, ee, pp)
        up = ctx.roi_uptake(lam, masks)
        ref_up = fom.roi_uptake(lam.cpu().numpy(), masks)
        assert np.allclose(up, ref_up, rtol=1e-12, atol=0)
        est = up.reshape(S, N, len(rois))
        got = lm.roi_metrics(est, truth)
        ref = (fom.enrmse(est, truth), fom.ens_bias(est, truth), fom.ens_std(est, truth))
        for g, r in zip(got, ref):
            assert np.allclose(g, r, rtol=1e-12, atol=1e-15)
        res[name] = got
        print(f"{name:11s} counts/case {np.mean([len(e['bin']) for e in ee]):7.1f}  "
              f"ENRMSE {got[0]}  bias {got[1]}  std {got[2]}")
    # more windows, more counts: lower noise than either single-window method
    for k in range(len(rois)):
        assert res["LM-MEW"][2][k] < res["LM-SEW"][2][k]
        assert res["LM-MEW"][2][k] < res["Binned-SEW"][2][k]
