"""GPU tests of plans whose cases have their own attenuation maps
(lmmew_plan_create_maps): every case must reconstruct exactly as it would in
a plan of its own context, and match the FP64 oracle run on its own map."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def small_maps():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_17111_amd as lm

    w = synth.CONFIGS["16x16_2k"]
    p = w.params
    mu_disk, act, _ = synth.phantom(w)
    maps = [mu_disk] + list(synth.random_body_maps(p, 2, seed=5))
    ctxs = [lm.Context(p, torch.from_numpy(m.astype(np.float32))) for m in maps]
    return lm, p, act, maps, ctxs


def _cat(evs):
    return {k: np.concatenate([np.asarray(e[k]) for e in evs]) for k in ("bin", "angle", "energy")}


def _sens_stack(ctxs, nsub):
    import torch

    return torch.stack([c.sensitivity(nsub) for c in ctxs]).contiguous()


def test_maps_plan_equals_independent_plans(small_maps):
    import torch

    lm, p, act, maps, ctxs = small_maps
    counts = [700, 1900, 260]
    evs = [synth.generic_events(p, act, n, 900 + c) for c, n in enumerate(counts)]
    offs = np.concatenate([[0], np.cumsum(counts)]).tolist()
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    sens = _sens_stack(ctxs, 4)
    batched = lam0.repeat(3, 1).contiguous()
    plan = lm.plan_maps(ctxs, lm.events_to_device(_cat(evs)), 4, offs)
    plan.osem_iter(2, sens, batched)
    graphed = lam0.repeat(3, 1).contiguous()
    plan.osem_graph(2, sens, graphed)
    assert torch.equal(batched, graphed)
    for c, e in enumerate(evs):
        lam = lam0.clone()
        ctxs[c].plan(lm.events_to_device(e), 4).osem_iter(2, sens[c], lam)
        assert torch.equal(lam, batched[c]), c
    # the maps differ, so the cases' images do too
    assert not torch.equal(batched[1], batched[2])


def test_maps_plan_matches_oracle_per_case(small_maps):
    import torch

    import oracle

    lm, p, act, maps, ctxs = small_maps
    evs, refs = [], []
    for c, m in enumerate(maps[:2]):
        orc = oracle.Oracle(p, m.astype(np.float32).astype(np.float64))
        ev = orc.sample_events(act, 500 + 300 * c, seed=60 + c)
        ev = {"bin": ev["bin"], "angle": ev["angle"], "energy": ev["energy"].astype(np.float32)}
        lam0 = orc.support.astype(np.float64)
        lam, _, _, _ = orc.osem({**ev, "energy": ev["energy"].astype(np.float64)}, 4, 1, lam0)
        evs.append(ev)
        refs.append(lam)
    offs = [0, len(evs[0]["bin"]), len(evs[0]["bin"]) + len(evs[1]["bin"])]
    sens = _sens_stack(ctxs[:2], 4)
    lam = torch.from_numpy(np.stack([synth.fov_support(p)] * 2).astype(np.float32)).cuda()
    lm.plan_maps(ctxs[:2], lm.events_to_device(_cat(evs)), 4, offs).osem_iter(1, sens, lam)
    got = lam.cpu().numpy()
    for c in range(2):
        d = got[c] - refs[c]
        assert np.abs(d).max() / np.abs(refs[c]).max() < TOL, c
        assert np.linalg.norm(d) / np.linalg.norm(refs[c]) < TOL, c


def test_maps_plan_with_surrogate_equals_independent(small_maps):
    import torch

    lm, p, act, maps, ctxs = small_maps
    net = ctxs[0].mlp(seed=4)
    net.fit(3000, epochs=1, batch=4096, lr=2e-3, floor_frac=3e-2, seed=1)
    theta, c0, fl = net.get_params()
    counts = [400, 900]
    evs = [synth.generic_events(p, act, n, 950 + c) for c, n in enumerate(counts)]
    offs = [0, counts[0], sum(counts)]
    sens = _sens_stack(ctxs[:2], 4)
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    batched = lam0.repeat(2, 1).contiguous()
    ctxs[0].set_scatter_model(net)
    try:
        lm.plan_maps(ctxs[:2], lm.events_to_device(_cat(evs)), 4, offs).osem_graph(2, sens, batched)
        for c, e in enumerate(evs):
            own = ctxs[c].mlp(seed=0)
            own.set_params(theta, c0, fl)
            ctxs[c].set_scatter_model(own)
            lam = lam0.clone()
            ctxs[c].plan(lm.events_to_device(e), 4).osem_iter(2, sens[c], lam)
            if c:
                ctxs[c].set_scatter_model(None)
            assert torch.equal(lam, batched[c]), c
    finally:
        for c in ctxs:
            c.set_scatter_model(None)


def test_maps_plan_with_coarse_grid_networks_equals_independent(small_maps):
    """Cases whose networks are evaluated on different coarse grids (2 and 3
    pixels, R28) in one graph-captured plan: each case reconstructs bitwise
    as in a plan of its own context."""
    import torch

    lm, p, act, maps, ctxs = small_maps
    net = ctxs[0].mlp(seed=4)
    net.fit(3000, epochs=1, batch=4096, lr=2e-3, floor_frac=3e-2, seed=1)
    theta, c0, fl = net.get_params()
    own = ctxs[1].mlp(seed=0)
    own.set_params(theta, c0, fl)
    net.set_grid(2)
    own.set_grid(3)
    counts = [500, 700]
    evs = [synth.generic_events(p, act, n, 970 + c) for c, n in enumerate(counts)]
    offs = [0, counts[0], sum(counts)]
    sens = _sens_stack(ctxs[:2], 4)
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    batched = lam0.repeat(2, 1).contiguous()
    ctxs[0].set_scatter_model(net)
    ctxs[1].set_scatter_model(own)
    try:
        lm.plan_maps(ctxs[:2], lm.events_to_device(_cat(evs)), 4, offs).osem_graph(2, sens, batched)
        for c, e in enumerate(evs):
            lam = lam0.clone()
            ctxs[c].plan(lm.events_to_device(e), 4).osem_iter(2, sens[c], lam)
            assert torch.equal(lam, batched[c]), c
    finally:
        for c in ctxs:
            c.set_scatter_model(None)


def test_maps_plan_rejects_other_systems(small_maps):
    import torch

    lm, p, act, maps, ctxs = small_maps
    other = lm.Context(synth.replace(p, fwhm0=3.0), torch.from_numpy(maps[0].astype(np.float32)))
    ev = lm.events_to_device(synth.generic_events(p, act, 50, 1))
    with pytest.raises(lm.LmmewError):
        lm.plan_maps([ctxs[0], other], ev, 4, [0, 20, 50])
    with pytest.raises(ValueError):
        lm.plan_maps([ctxs[0], ctxs[1]], ev, 4, [0, 50])
