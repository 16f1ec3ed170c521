#!/usr/bin/env python
"""Benchmark of list-mode multi-energy-window OSEM on one MI355X.

One step = one OSEM iteration (all angle subsets: per-event system model,
forward projection, compensated backprojection, EM update) over the workload's
whole event list, inputs resident in HBM.  Setup (attenuation tables,
sensitivity, the scatter-path parameter table when it fits in device memory,
event plan, tile autotuning) is timed separately and reported in `setup_ms`;
the same iterations without the path table are reported beside the headline.

Default workload: 64x64 object at 4 mm, 32x32 scatter grid, 64 bins x 120
angles, lines 85/154/270 keV, windows 68-102/123-184/243-297 keV, ~50k events,
8 subsets (the 20-iteration schedule runs as 20 steps).

Beside it: 64 batched cases of that workload in one graph launch ("batched"),
the exact model against the MLP scatter surrogate ("surrogate") on 16
patients with their own maps at 128x128 (1M events) and on the 16x16 workload,
and the cached-row mode ("cached_rows": rows computed once, iterations bound
by HBM bandwidth; a different mode, never the headline value).

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X unit counts: 256 CUs x 128 FP32 lane-operations per cycle (the 157.3
# TFLOP/s vector rate, which needs packed FP32) x 2.4 GHz; v_exp_f32 at a
# quarter of that rate.  One algorithmic term is one energy-Gaussian factor
# exp(-(s E - F)^2 + A): two FMAs to form the exponent, one exp, one add to
# accumulate, i.e. 3 + 4 = 7 issue slots.
LANES_PER_S = 256 * 128 * 2.4e9
SLOTS_PER_TERM = 7.0
PEAK_TERMS_PER_S = LANES_PER_S / SLOTS_PER_TERM
# Without packed FP32 (not used anywhere in this library) a CU issues 64 FP32
# lane-operations per cycle and the exp takes two of those slots: 3 + 2 = 5.
NONPACKED_PEAK_TERMS_PER_S = 256 * 64 * 2.4e9 / 5.0

# HBM bytes per launch of the per-event kernel on the 64x64 workload at event
# tile 16, without and with the path-parameter table (rocprofv3 FETCH_SIZE and
# WRITE_SIZE of these kernel versions, scaled by a 256 MiB copy kernel: fetch
# x2.000, write x1.000)
MEASURED_TRAFFIC = {("64x64_50k", 16, False): {"fetch": 458.9e6, "write": 81.5e6},
                    ("64x64_50k", 16, True): {"fetch": 3449.8e6, "write": 81.5e6}}

# iterations after which the 16-patient images of the exact model, the
# surrogate and no scatter model are compared region by region
ROI_ITERS = 10

# scatter surrogate 6 -> 128 -> 128 -> 128 -> 1: multiply-adds per (event, pixel)
# pair, and MI355X's dense BF16 MFMA peak
MLP_MAC_PER_PAIR = 6 * 128 + 2 * 128 * 128 + 128
MLP_GELU_PER_PAIR = 3 * 128
PEAK_BF16_FLOPS = 2.5e15


def workload_desc(name, p, J, nsub):
    return (f"{name}: {p.n}x{p.n} at {p.pix:g} mm, scatter {p.ns}x{p.ns}, {p.nb} bins x {p.na} "
            f"angles, lines {'/'.join(f'{e:g}' for e in p.lines)} keV, {len(p.windows)} windows, "
            f"{J} events, {nsub} subsets")


def cpu_baseline(p, mu, ev, seconds):
    """The FP64 oracle as it stands, on a bounded sample of the same events: one
    OSEM iteration evaluates each event's system row once, so rows/s is the
    oracle's events*iterations/s."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    o = oracle.Oracle(p, np.asarray(mu, np.float32).astype(np.float64))
    thr = oracle.threads()
    J = ev["bin"].size
    stride = max(1, J // 4096)
    order = np.arange(0, J, stride)
    lam = np.ones(p.n * p.n)
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < order.size:
        idx = order[done:done + thr]
        sub = {"bin": ev["bin"][idx], "angle": ev["angle"][idx],
               "energy": ev["energy"][idx].astype(np.float64)}
        o.forward(sub, lam)
        done += idx.size
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "events*iterations/s", "cores": thr, "kind": "oracle",
            "sample": f"{done} events (every {stride}th of the workload) x 1 iteration, "
                      f"FP64 system rows, {dt:.1f} s"}


def batched(ctx, sens, args):
    """64 independent cases (noise realisations of the 64x64 phantom, per-case means
    uniform in 20k-200k events) packed in one plan; each iteration of all cases is one
    captured hipGraph launch."""
    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import events_to_device

    w = synth.CONFIGS["64x64_64cases"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    counts = synth.case_counts(w)
    t = time.perf_counter()
    evs = [synth.generic_events(p, act, int(n), w.seed_events + c) for c, n in enumerate(counts)]
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("bin", "angle", "energy")}
    offs = np.concatenate([[0], np.cumsum(counts)]).tolist()
    gen_s = time.perf_counter() - t
    t = time.perf_counter()
    plan = ctx.plan(events_to_device(cat), w.n_subsets, case_offsets=offs)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t
    t = time.perf_counter()
    jt = plan.autotune(use_cache=False)
    tune_s = time.perf_counter() - t
    lam = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    lam = lam.repeat(len(counts), 1).contiguous()
    plan.osem_graph(1, sens, lam)                      # capture + first iteration (warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batched_steps):
        plan.osem_graph(1, sens, lam)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    J = int(counts.sum())
    terms, _ = plan.terms()
    assert bool(torch.isfinite(lam).all())
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    lam0 = lam0.repeat(len(counts), 1).contiguous()
    Qp = (int(synth.fov_support(p).sum()) + 63) // 64 * 64
    cached = None if args.no_cached else cached_rows(plan, sens, lam0, J, Qp, args.batched_steps)
    return {"workload": f"{len(counts)} cases of the 64x64 workload, {J} events "
                        f"({int(counts.min())}..{int(counts.max())} per case), {w.n_subsets} subsets",
            "value": J * args.batched_steps / el, "unit": "events*iterations/s",
            "s_per_iteration": el / args.batched_steps, "steps": args.batched_steps,
            "event_tile": jt, "terms_per_s": terms * args.batched_steps / el,
            "frac_of_term_peak": terms * args.batched_steps / el / PEAK_TERMS_PER_S,
            "setup_s": {"events": gen_s, "plan": plan_s, "autotune": tune_s},
            "cached_rows": cached}


PEAK_HBM_BYTES_PER_S = 8.0e12


def cached_rows(plan, sens, lam0, J, Qp, steps):
    """Cached-row mode: the rows of every subset computed once, the iterations
    (forward projection, backprojection, update) read them.  Each iteration
    reads every row twice (forward and backprojection): 2 x J x Qp x 4 bytes."""
    import torch

    from paper_2305_17111_amd import LmmewError

    t = time.perf_counter()
    try:
        plan.cache_rows(True)
    except LmmewError as e:
        return {"skipped": str(e)}
    torch.cuda.synchronize()
    cache_s = time.perf_counter() - t
    lam = lam0.clone()
    s_it = _time_graph(plan, sens, lam, steps)
    plan.cache_rows(False)
    bytes_it = 2.0 * J * Qp * 4
    return {"value": J / s_it, "unit": "events*iterations/s", "s_per_iteration": s_it,
            "steps": steps, "cache_s": cache_s, "cached_bytes": J * Qp * 4.0,
            "roofline": {"bound": "hbm", "kernel": "k_forward + k_back on cached rows",
                         "achieved": bytes_it / s_it / 1e9, "peak": PEAK_HBM_BYTES_PER_S / 1e9,
                         "unit": "GB/s", "frac": bytes_it / s_it / PEAK_HBM_BYTES_PER_S,
                         "traffic": None, "bytes_per_iteration": bytes_it}}


def positions(ctx, ev, nsub, sens, lam0, J, steps):
    """The headline iterations on the same events handed over with their
    continuous lateral positions instead of bins (density response)."""
    import torch

    from paper_2305_17111_amd import events_to_device

    plan = ctx.plan(events_to_device({k: ev[k] for k in ("position", "angle", "energy")}), nsub)
    plan.autotune(use_cache=False)
    lam = lam0.clone()
    plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n_launch = plan.profile_read()
    plan.profile(False)
    terms, _ = plan.terms()
    ach = terms * steps / (ms * 1e-3)
    assert bool(torch.isfinite(lam).all())
    return {"ms_per_step": 1e3 * el / steps, "value": J * steps / el,
            "unit": "events*iterations/s", "event_tile": plan.event_tile,
            "k_row_avg_launch_ms": ms / n_launch, "terms_per_iteration": terms,
            "frac": ach / PEAK_TERMS_PER_S, "frac_of_nonpacked_peak": ach / NONPACKED_PEAK_TERMS_PER_S}


def three_d(steps):
    """The 3-D single-scatter model on the 64x64 workload's slice geometry over
    16 slices (64x64x16 voxels of 4 mm, 32x32x8 scatter grid, 64x16 bins,
    120 angles, ~50k events, 8 subsets), matrix-free with the parameters
    evaluated in the kernel (its path table would need 680 GB)."""
    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import Context, events_to_device

    w = synth.CONFIGS["64x64x16_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events3(p, act, w.n_events, w.seed_events, poisson=w.poisson)
    J = int(ev["angle"].size)
    setup = {}
    t = time.perf_counter()
    ctx = Context(p, torch.from_numpy(np.asarray(mu, np.float32)))
    torch.cuda.synchronize()
    setup["tables_ms"] = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    sens = ctx.sensitivity(w.n_subsets)
    torch.cuda.synchronize()
    setup["sensitivity_ms"] = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    plan = ctx.plan(events_to_device(ev), w.n_subsets)
    torch.cuda.synchronize()
    setup["plan_ms"] = 1e3 * (time.perf_counter() - t)
    plan.autotune(use_cache=False)
    lam = torch.from_numpy(synth.fov_support3(p).astype(np.float32)).cuda()
    plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n_launch = plan.profile_read()
    plan.profile(False)
    assert bool(torch.isfinite(lam).all())
    terms, full = plan.terms()
    ach = terms * steps / (ms * 1e-3)
    return {"workload": "3-D single scatter: 64x64x16 voxels at 4 mm, 32x32x8 scatter grid "
                        "(3048 points), 64x16 bins, 120 angles, EW1-3, %d events, %d subsets"
                        % (J, w.n_subsets),
            "value": J * steps / el, "unit": "events*iterations/s",
            "s_per_iteration": el / steps, "steps": steps, "event_tile": plan.event_tile,
            "k_row_avg_launch_ms": ms / n_launch, "k_row_share_of_step": ms / (1e3 * el),
            "terms_per_iteration": {"evaluated": terms, "unpruned": full},
            "frac": ach / PEAK_TERMS_PER_S,
            "frac_of_nonpacked_peak": ach / NONPACKED_PEAK_TERMS_PER_S,
            "setup_ms": setup}


def scatter_resolution(ev, steps):
    """The headline workload with the scatter modelled on coarser grids (the
    lower-resolution scatter the paper's appendix on 3-D requirements
    proposes): per scatter grid the iteration time and the hot-region
    uptakes after ROI_ITERS iterations relative to the finest grid."""
    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import Context, LmmewError, events_to_device

    w = synth.CONFIGS["64x64_50k"]
    mu, act, rois = synth.phantom(w)
    dev = events_to_device(ev)
    res, ups = {}, {}
    for ns in (8, 16, 32):
        p = synth.replace(w.params, ns=ns)
        ctx = Context(p, torch.from_numpy(mu.astype(np.float32)))
        try:
            ctx.path_table(True)
        except LmmewError:
            pass
        sens = ctx.sensitivity(w.n_subsets)
        plan = ctx.plan(dev, w.n_subsets)
        plan.autotune(use_cache=False)
        lam = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
        s_it = _time_graph(plan, sens, lam, steps)
        plan.osem_graph(ROI_ITERS - steps - 1, sens, lam)
        x = lam.cpu().numpy().astype(np.float64)
        ups[ns] = np.array([x[r].sum() for r in rois])
        terms, _ = plan.terms()
        res[ns] = {"scatter_cell_mm": 2 * p.R / ns, "s_per_iteration": s_it,
                   "terms_per_iteration": terms}
        del plan, ctx
    for ns in res:
        rel = ups[ns] / ups[32] - 1.0
        res[ns]["roi_uptake_vs_finest"] = [float(v) for v in rel]
    return {"workload": "64x64 workload with scatter grids 8x8, 16x16, 32x32 (cells 32, 16, "
                        f"8 mm); uptakes of the hot regions after {ROI_ITERS} iterations",
            "grids": {f"{ns}x{ns}": v for ns, v in res.items()}}


def _time_graph(plan, sens, lam, steps):
    """Seconds per launch of a one-iteration graph (after one warmup launch)."""
    import torch

    plan.osem_graph(1, sens, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.osem_graph(1, sens, lam)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def surrogate(args):
    """Exact model vs the MLP scatter surrogate.

    128x128: 16 patients (own phantom and attenuation map each, uneven counts,
    1M events in total) in one plan, 16 subsets, each iteration one graph launch;
    the network is trained on the GPU on 10M samples of the exact scatter model
    drawn over 16 random water bodies (it has no attenuation-map input).
    16x16: the workload the surrogate's accuracy is tested on (10 iterations
    as one graph launch)."""
    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import Context, events_to_device, plan_maps

    out = {}
    w = synth.CONFIGS["128x128_16cases"]
    p = w.params
    counts = synth.case_counts(w)
    t = time.perf_counter()
    ctxs, evs, rois = [], [], []
    for c in range(w.n_cases):
        mu, act, roi = synth.phantom(w, c)
        rois.append(roi)
        ctxs.append(Context(p, torch.from_numpy(mu.astype(np.float32))))
        evs.append(synth.generic_events(p, act, int(counts[c]), w.seed_events + c))
    sens = torch.stack([c.sensitivity(w.n_subsets) for c in ctxs]).contiguous()
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("bin", "angle", "energy")}
    offs = np.concatenate([[0], np.cumsum(counts)]).tolist()
    plan = plan_maps(ctxs, events_to_device(cat), w.n_subsets, offs)
    jt = plan.autotune(use_cache=False)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    J = int(counts.sum())
    Qm = ctxs[0].support_size
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    lam0 = lam0.repeat(w.n_cases, 1).contiguous()

    lam = lam0.clone()
    exact_s = _time_graph(plan, sens, lam, args.surrogate_steps)
    # the exact model's per-event kernel on its own: one profiled eager iteration
    plan.profile(True)
    plan.osem_iter(1, sens, lam)
    k_ex = plan.profile_read_kernels()
    plan.profile(False)
    ex_ms, ex_n = k_ex["k_row"]
    ex_terms, _ = plan.terms()
    ex_ach = ex_terms / (ex_ms * 1e-3)
    # accuracy reference: the exact model's images after ROI_ITERS iterations
    done = args.surrogate_steps + 2
    roi_iters = max(ROI_ITERS, done)
    if roi_iters > done:
        plan.osem_graph(roi_iters - done, sens, lam)
    lam_exact = lam.cpu().numpy().astype(np.float64)

    net = ctxs[0].mlp(seed=2)
    maps = synth.random_body_maps(p, 16, seed=41).astype(np.float32)
    n_lab = -(-10_000_000 // (16 * Qm))
    t = time.perf_counter()
    losses = net.fit_maps([torch.from_numpy(m) for m in maps], n_lab, epochs=args.surrogate_epochs,
                          batch=8192, lr=2e-3, floor_frac=3e-2, seed=3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    ctxs[0].set_scatter_model(net)
    lam = lam0.clone()
    sur_s = _time_graph(plan, sens, lam, args.surrogate_steps)
    assert bool(torch.isfinite(lam).all())
    plan.profile(True)
    plan.osem_iter(1, sens, lam)
    k = plan.profile_read_kernels()
    plan.profile(False)
    if roi_iters > done:
        plan.osem_graph(roi_iters - done, sens, lam)
    lam_sur = lam.cpu().numpy().astype(np.float64)
    # the same iterations with the scatter term switched off (the network's
    # output shifted by -100 in log space: a density below 1e-40), the method
    # without a scatter model
    theta, c0, _ = net.get_params()
    off = ctxs[0].mlp(seed=0)
    off.set_params(theta, c0 - 100.0, 0.0)
    ctxs[0].set_scatter_model(off)
    lam = lam0.clone()
    plan.osem_graph(roi_iters, sens, lam)
    lam_none = lam.cpu().numpy().astype(np.float64)
    ctxs[0].set_scatter_model(None)
    # every patient's hot-region uptakes (FP64 sums on the host), each image
    # after roi_iters iterations from the same start
    def uptakes(x):
        return np.array([[x[c][r].sum() for r in rois[c]] for c in range(w.n_cases)])
    up_ex = uptakes(lam_exact)
    rel = uptakes(lam_sur) / up_ex - 1.0
    rel0 = uptakes(lam_none) / up_ex - 1.0
    mlp_ms, mlp_n = k["k_mlp_rows"]
    row_ms, row_n = k["k_row"]
    pairs = float(J) * Qm                            # (event, support pixel) pairs per iteration
    flops = pairs * 2 * MLP_MAC_PER_PAIR / (mlp_ms * 1e-3)
    out["128x128_16cases"] = {
        "workload": f"{w.n_cases} patients (own phantom and map) at {p.n}x{p.n}, "
                    f"{p.pix:g} mm, scatter {p.ns}x{p.ns}, {p.nb} bins x {p.na} angles, "
                    f"{len(p.windows)} windows, {J} events ({int(counts.min())}..{int(counts.max())}"
                    f" per case), {w.n_subsets} subsets",
        "unit": "events*iterations/s",
        "exact": {"value": J / exact_s, "s_per_iteration": exact_s, "event_tile": jt,
                  "roofline": {"bound": "alu", "kernel": "k_row (path parameters in the kernel)",
                               "achieved": ex_ach / 1e12, "peak": PEAK_TERMS_PER_S / 1e12,
                               "unit": "Tterm/s", "frac": ex_ach / PEAK_TERMS_PER_S,
                               "frac_of_nonpacked_peak": ex_ach / NONPACKED_PEAK_TERMS_PER_S,
                               "avg_launch_ms": ex_ms / ex_n,
                               "kernel_share_of_iteration": ex_ms * 1e-3 / exact_s}},
        "surrogate": {"value": J / sur_s, "s_per_iteration": sur_s,
                      "unscattered_kernel_ms_per_iteration": row_ms},
        "speedup": exact_s / sur_s,
        "roi_uptake_vs_exact": {"iterations": roi_iters, "regions": int(rel.size),
                                "surrogate": {"mean_rel": float(rel.mean()),
                                              "mean_abs_rel": float(np.abs(rel).mean()),
                                              "max_abs_rel": float(np.abs(rel).max())},
                                "no_scatter_model": {"mean_rel": float(rel0.mean()),
                                                     "mean_abs_rel": float(np.abs(rel0).mean()),
                                                     "max_abs_rel": float(np.abs(rel0).max())}},
        "steps": args.surrogate_steps,
        "training": {"samples": int(16 * n_lab * Qm), "epochs": args.surrogate_epochs,
                     "batch": 8192, "seconds": train_s, "first_loss": losses[0],
                     "last_loss": losses[-1], "maps": "16 random water bodies"},
        "roofline": {"bound": "mfma", "kernel": "k_mlp_rows (surrogate inference)",
                     "achieved": flops / 1e12, "peak": PEAK_BF16_FLOPS / 1e12,
                     "unit": "TFLOP/s", "frac": flops / PEAK_BF16_FLOPS, "traffic": None,
                     "flop_per_pair": 2 * MLP_MAC_PER_PAIR, "gelu_per_pair": MLP_GELU_PER_PAIR,
                     "pairs_per_s": pairs / (mlp_ms * 1e-3), "avg_launch_ms": mlp_ms / mlp_n},
        "setup_s": setup_s,
    }
    del plan, ctxs, sens

    w = synth.CONFIGS["16x16_2k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ctx = Context(p, torch.from_numpy(mu.astype(np.float32)))
    sens = ctx.sensitivity(w.n_subsets)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events)
    plan = ctx.plan(events_to_device(ev), w.n_subsets)
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    maps = synth.random_body_maps(p, 16, seed=41).astype(np.float32)
    net = ctx.mlp(seed=2)
    t = time.perf_counter()
    net.fit_maps([torch.from_numpy(m) for m in maps], 3000, epochs=16, batch=8192, lr=2e-3,
                 floor_frac=3e-2, seed=3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    res = {}
    for key, model in (("exact", None), ("surrogate", net)):
        ctx.set_scatter_model(model)
        lam = lam0.clone()
        plan.osem_graph(w.n_iters, sens, lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.osem_graph(w.n_iters, sens, lam)
        torch.cuda.synchronize()
        s_it = (time.perf_counter() - t0) / w.n_iters
        res[key] = {"value": w.n_events / s_it, "s_per_iteration": s_it}
    ctx.set_scatter_model(None)
    out["16x16_2k"] = {"workload": workload_desc("16x16_2k", p, w.n_events, w.n_subsets),
                       "unit": "events*iterations/s", **res,
                       "training": {"samples": int(16 * 3000 * ctx.support_size), "epochs": 16,
                                    "seconds": train_s, "maps": "16 random water bodies"}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="64x64_50k")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-cached", action="store_true")
    ap.add_argument("--no-position", action="store_true",
                    help="skip the continuous-position variant of the headline iterations")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3-D single-scatter workload")
    ap.add_argument("--no-scatter-grids", action="store_true",
                    help="skip the headline workload on coarser scatter grids")
    ap.add_argument("--steps-3d", type=int, default=2)
    ap.add_argument("--no-path-table", action="store_true",
                    help="evaluate the scatter-path parameters inside the per-event kernel")
    ap.add_argument("--surrogate-steps", type=int, default=1)
    ap.add_argument("--surrogate-epochs", type=int, default=8)
    ap.add_argument("--event-tile", type=int, default=0,
                    help="0 = autotune over 16, 32, 64")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device with a plain copy kernel (a known "
                         "byte count for scaling hardware traffic counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs the whole reconstruction on "
              "a single MI355X (the design notes describe how it would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import Context, events_to_device

    w = synth.CONFIGS[args.workload]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=w.poisson)
    J = int(ev["bin"].size)
    nsub = w.n_subsets
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # one elementwise kernel (a multiply by 1) that reads and writes exactly
        # MIB MiB each
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    setup = {}
    t = time.perf_counter()
    ctx = Context(p, torch.from_numpy(np.asarray(mu, np.float32)))
    torch.cuda.synchronize()
    setup["tables_ms"] = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    sens = ctx.sensitivity(nsub)
    torch.cuda.synchronize()
    setup["sensitivity_ms"] = 1e3 * (time.perf_counter() - t)
    path_table = None
    if not args.no_path_table:
        # event-independent scatter-path parameters, evaluated once per map
        from paper_2305_17111_amd import LmmewError

        t = time.perf_counter()
        try:
            ctx.path_table(True)
            path_table = ctx.path_table_bytes
        except LmmewError as e:
            print(f"path table not used: {e}", file=sys.stderr)
        torch.cuda.synchronize()
        setup["path_table_ms"] = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    plan = ctx.plan(events_to_device(ev), nsub)
    torch.cuda.synchronize()
    setup["plan_ms"] = 1e3 * (time.perf_counter() - t)
    lam = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()

    t = time.perf_counter()
    if args.event_tile:
        plan.set_event_tile(args.event_tile)
    else:                                   # the library's autotuner (times k_row per tile size)
        plan.autotune(use_cache=False)
    setup["autotune_ms"] = 1e3 * (time.perf_counter() - t)

    for _ in range(args.warmup):
        plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()

    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    row_ms, launches = plan.profile_read()
    plan.profile(False)
    assert bool(torch.isfinite(lam).all())

    # the same iterations as one captured hipGraph launch per step
    plan.osem_graph(1, sens, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.osem_graph(1, sens, lam)
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - t0) / args.steps

    terms, full_terms = plan.terms()
    achieved = terms * args.steps / (row_ms * 1e-3)          # terms/s in the per-event kernel
    mt = MEASURED_TRAFFIC.get((w.name, plan.event_tile, bool(path_table)))
    rows_per_launch = J / nsub
    out_bytes = rows_per_launch * ((int(synth.fov_support(p).sum()) + 63) // 64 * 64) * 4
    out = {
        "metric": "LM-MEW OSEM events*iterations/s (exact model), 1 GPU",
        "value": J * args.steps / elapsed,
        "unit": "events*iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "s_per_iteration": elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantom and generic list-mode events)",
        "config": {
            "workload": workload_desc(w.name, p, J, nsub),
            "events": J, "subsets": nsub, "iterations_per_step": 1,
            "event_tile": plan.event_tile, "pixels_in_support": int(synth.fov_support(p).sum()),
            "path_table_bytes": path_table,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_row (per-event system model%s)" % (", path-parameter table" if path_table else ""),
            "achieved": achieved / 1e12,
            "peak": PEAK_TERMS_PER_S / 1e12,
            "unit": "Tterm/s",
            "frac": achieved / PEAK_TERMS_PER_S,
            "nonpacked_peak": NONPACKED_PEAK_TERMS_PER_S / 1e12,
            "frac_of_nonpacked_peak": achieved / NONPACKED_PEAK_TERMS_PER_S,
            "traffic": (mt["fetch"] + mt["write"]) if mt else None,
            "traffic_unit": "bytes per launch",
            "traffic_detail": ({**mt, "algorithmic_write": out_bytes} if mt else None),
            "terms_per_launch": terms * args.steps / launches,
            "avg_launch_ms": row_ms / launches,
            "kernel_share_of_step": row_ms / (1e3 * elapsed),
        },
        "graph_ms_per_step": graph_ms,
        "model_terms_per_iteration": {"evaluated": terms, "unpruned": full_terms},
        "setup_ms": setup,
    }
    if not args.no_cached:
        lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
        Qp = (int(synth.fov_support(p).sum()) + 63) // 64 * 64
        out["cached_rows"] = cached_rows(plan, sens, lam0, J, Qp, args.steps)
    if not args.no_position:
        lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
        out["continuous_positions"] = positions(ctx, ev, nsub, sens, lam0, J, args.steps)
    if not args.no_batched:
        out["batched"] = batched(ctx, sens, args)
    if path_table:
        # the same iterations evaluating the path parameters inside the kernel
        ctx.path_table(False)
        plan.osem_iter(1, sens, lam)
        torch.cuda.synchronize()
        plan.profile(True)
        t0 = time.perf_counter()
        n_nt = min(args.steps, 5)
        for _ in range(n_nt):
            plan.osem_iter(1, sens, lam)
        torch.cuda.synchronize()
        el_nt = time.perf_counter() - t0
        ms_nt, n_launch = plan.profile_read()
        plan.profile(False)
        ach_nt = terms * n_nt / (ms_nt * 1e-3)
        out["without_path_table"] = {"ms_per_step": 1e3 * el_nt / n_nt,
                                     "value": J * n_nt / el_nt,
                                     "k_row_avg_launch_ms": ms_nt / n_launch,
                                     "frac": ach_nt / PEAK_TERMS_PER_S,
                                     "frac_of_nonpacked_peak": ach_nt / NONPACKED_PEAK_TERMS_PER_S}
    del plan
    if not args.no_scatter_grids:
        out["scatter_resolution"] = scatter_resolution(ev, 2)
    if not args.no_3d:
        out["three_d"] = three_d(args.steps_3d)
    if not args.no_surrogate:
        out["surrogate"] = surrogate(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, mu, ev, args.cpu_seconds)
    print(json.dumps(out))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
