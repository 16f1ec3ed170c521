"""GPU tests of the exact model's scatter at a coarser pixel resolution
(lmmew_set_scatter_pixel_grid): the scattered part of the rows evaluated at
node pixels and interpolated to the support.

- the scattered part equals the interpolation, with nodes and weights derived
  here from the header's definition, of the full-resolution GPU rows at the
  node pixels (1e-6 of the row maximum: the node values are the same
  computation) and of the FP64 oracle's rows (the 1e-4 bar);
- the unscattered part is untouched; grid 1 restores the rows bitwise;
- eager, captured-graph and cached-row iterations agree bitwise, and a plan
  over two maps equals the two independent plans;
- invalid grids, 3-D contexts and plans whose contexts disagree are rejected.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import oracle
    import paper_2305_17111_amd as lm

    w = synth.CONFIGS["16x16_2k"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32 = mu.astype(np.float32)
    ctx = lm.Context(p, torch.from_numpy(mu32))
    orc = oracle.Oracle(p, mu32.astype(np.float64))
    return lm, p, act, ctx, orc


def _dev(lm, ev):
    return lm.events_to_device({"bin": ev["bin"], "angle": ev["angle"],
                                "energy": np.asarray(ev["energy"], np.float32)})


def _stencil(support, n, g):
    """Per support pixel: [(full-grid node pixel, weight)], the header's rule."""
    out = []
    for q in np.flatnonzero(support):
        ix, iy = q % n, q // n
        u0, v0 = ix // g, iy // g
        fx, fy = (ix % g) / g, (iy % g) / g
        cand = [((g * u0, g * v0), (1 - fx) * (1 - fy)), ((g * u0 + g, g * v0), fx * (1 - fy)),
                ((g * u0, g * v0 + g), (1 - fx) * fy), ((g * u0 + g, g * v0 + g), fx * fy)]
        keep = [(cy * n + cx, wk) for (cx, cy), wk in cand
                if wk > 0 and cx < n and cy < n and support[cy * n + cx]]
        s = sum(wk for _, wk in keep)
        out.append([(k, wk / s) for k, wk in keep] if s > 0 else [(q, 1.0)])
    return out


def _interp(rows, st):
    return np.stack([[sum(wk * r[k] for k, wk in s) for s in st] for r in rows])


@pytest.mark.parametrize("grid", [2, 3])
def test_scattered_part_interpolates_node_pixels(env, grid):
    lm, p, act, ctx, orc = env
    ev = orc.sample_events(act, 12, seed=21)
    ev["energy"] = ev["energy"].astype(np.float32)
    d = _dev(lm, ev)
    full_sc = ctx.rows(d, part=1).cpu().numpy().astype(np.float64)
    full = ctx.rows(d, part=3).cpu().numpy()
    ctx.set_scatter_pixel_grid(grid)
    try:
        sc = ctx.rows(d, part=1).cpu().numpy().astype(np.float64)
        tot = ctx.rows(d, part=3).cpu().numpy().astype(np.float64)
        un = ctx.rows(d, part=2).cpu().numpy().astype(np.float64)
        nodes = ctx.scatter_pixel_grid_nodes()
    finally:
        ctx.set_scatter_pixel_grid(1)
    assert np.array_equal(ctx.rows(d, part=3).cpu().numpy(), full)
    sup = orc.support.astype(bool)
    qs = np.flatnonzero(sup)
    st = _stencil(sup, p.n, grid)
    assert nodes == len({k for s in st for k, _ in s})
    # against the full-resolution GPU rows at the node pixels
    want = _interp(full_sc, st)
    got = sc[:, qs]
    assert np.abs(got - want).max() <= 1e-6 * want.max()
    # the unscattered part is the full-resolution one
    assert np.abs(tot[:, qs] - un[:, qs] - got).max() <= 1e-6 * tot.max()
    # against the FP64 oracle's scattered rows at the node pixels
    ref = np.stack([orc.row_scatter(int(b), int(a), float(E))
                    for b, a, E in zip(ev["bin"], ev["angle"], ev["energy"])])
    want_o = _interp(ref, st)
    mx = max(np.abs(g_ - w_).max() / w_.max() for g_, w_ in zip(got, want_o))
    l2 = np.linalg.norm(got - want_o) / np.linalg.norm(want_o)
    print(f"grid {grid}: {nodes} node pixels of {qs.size}; vs oracle: max {mx:.2e} of the row "
          f"maximum, L2 {l2:.2e}; interpolation vs full resolution: max "
          f"{np.abs(got - full_sc[:, qs]).max() / full_sc.max():.3e} of the row maximum")
    assert mx <= TOL


def test_iterations_graph_cached_and_maps(env):
    import torch

    lm, p, act, ctx, orc = env
    ev = orc.sample_events(act, 900, seed=22)
    d = _dev(lm, ev)
    sens = ctx.sensitivity(4)
    plan = ctx.plan(d, 4)
    lam0 = torch.from_numpy(orc.support.astype(np.float32)).cuda()
    ref = lam0.clone()
    plan.osem_iter(2, sens, ref)
    ctx.set_scatter_pixel_grid(2)
    try:
        a, b, c = lam0.clone(), lam0.clone(), lam0.clone()
        plan.osem_iter(2, sens, a)
        plan.osem_graph(2, sens, b)
        plan.cache_rows(True)
        plan.osem_iter(2, sens, c)
        plan.cache_rows(False)
        assert torch.equal(a, b) and torch.equal(a, c)
        assert not torch.equal(a, ref)
        rel = (a - ref).abs().max().item() / ref.abs().max().item()
        # the interpolation smooths the near-field peaks of the scattered part
        # (the 1/r factor next to each scatter point): a percent-level change
        print(f"two iterations, grid 2 against every pixel: max {rel:.2e} of the image maximum")
        assert rel < 0.2
        # two maps in one plan equal their independent plans
        mu2 = synth.random_body_maps(p, 1, seed=7)[0].astype(np.float32)
        ctx2 = lm.Context(p, torch.from_numpy(mu2))
        evs = [synth.generic_events(p, act, n, 990 + k) for k, n in enumerate((500, 700))]
        cat = {k: np.concatenate([np.asarray(e[k]) for e in evs]) for k in ("bin", "angle", "energy")}
        with pytest.raises(lm.LmmewError):
            lm.plan_maps([ctx, ctx2], lm.events_to_device(cat), 4, [0, 500, 1200])
        ctx2.set_scatter_pixel_grid(2)
        sens2 = torch.stack([ctx.sensitivity(4), ctx2.sensitivity(4)]).contiguous()
        batched = lam0.repeat(2, 1).contiguous()
        lm.plan_maps([ctx, ctx2], lm.events_to_device(cat), 4, [0, 500, 1200]).osem_graph(
            2, sens2, batched)
        for k, (cx, e) in enumerate(zip((ctx, ctx2), evs)):
            lam = lam0.clone()
            cx.plan(lm.events_to_device(e), 4).osem_iter(2, sens2[k], lam)
            assert torch.equal(lam, batched[k]), k
    finally:
        ctx.set_scatter_pixel_grid(1)


def test_fused_and_two_pass_rows_agree(env):
    """With the unscattered table the node modes write each row in one pass
    (unscattered part plus interpolation); without it the per-event kernel's
    unscattered pass and a separate interpolation.  Both give the same rows
    (the unscattered arithmetic is the same; the table holds what the kernel
    otherwise forms with erfc, so within float rounding)."""
    lm, p, act, ctx, orc = env
    ev = orc.sample_events(act, 20, seed=24)
    d = _dev(lm, ev)
    ctx.set_scatter_pixel_grid(2)
    try:
        fused = ctx.rows(d, part=3).cpu().numpy().astype(np.float64)
        ctx.lmmew_psf_table(False)
        two = ctx.rows(d, part=3).cpu().numpy().astype(np.float64)
    finally:
        ctx.lmmew_psf_table(True)
        ctx.set_scatter_pixel_grid(1)
    err = np.abs(fused - two).max() / np.abs(two).max()
    print(f"fused against two passes: max {err:.2e} of the largest row element")
    assert err <= 1e-5


def test_continuous_positions(env):
    """Events with continuous positions: the scattered part at node pixels
    interpolates the full-resolution rows the same way (the response factors
    do not depend on the pixel)."""
    lm, p, act, ctx, orc = env
    ev = orc.sample_events(act, 10, seed=23)
    u = np.random.default_rng(23).uniform(0.0, 1.0, 10)
    pos = (-p.R + (np.asarray(ev["bin"]) + u) * (p.fov / p.nb)).astype(np.float32)
    d = lm.events_to_device({"position": pos, "angle": ev["angle"],
                             "energy": np.asarray(ev["energy"], np.float32)})
    full = ctx.rows(d, part=1).cpu().numpy().astype(np.float64)
    ctx.set_scatter_pixel_grid(2)
    try:
        sc = ctx.rows(d, part=1).cpu().numpy().astype(np.float64)
    finally:
        ctx.set_scatter_pixel_grid(1)
    sup = orc.support.astype(bool)
    want = _interp(full, _stencil(sup, p.n, 2))
    got = sc[:, np.flatnonzero(sup)]
    assert np.abs(got - want).max() <= 1e-6 * want.max()


def test_rejections(env):
    import torch

    lm, p, act, ctx, orc = env
    for g in (0, 9, -2):
        with pytest.raises(lm.LmmewError):
            ctx.set_scatter_pixel_grid(g)
    assert ctx.scatter_pixel_grid_nodes() == ctx.support_size
    w3 = synth.CONFIGS["16x16x8_600"]
    mu3 = synth.phantom(w3)[0].astype(np.float32)
    ctx3 = lm.Context(w3.params, torch.from_numpy(mu3))
    with pytest.raises(lm.LmmewError):
        ctx3.set_scatter_pixel_grid(2)
    ctx3.set_scatter_pixel_grid(1)
