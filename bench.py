#!/usr/bin/env python
"""Benchmark of list-mode multi-energy-window OSEM on one MI355X.

Headline (the metric's configuration): 16 patients at 128x128 (2 mm pixels,
64x64 scatter grid, 128 bins x 120 angles, lines 85/154/270 keV, four windows),
each with its own phantom and attenuation map and an uneven share of 1M
events, in one plan with 16 angle subsets.  One step = one OSEM iteration of
all 16 patients (all subsets: per-event system model, forward projection,
compensated backprojection, EM update), inputs resident in HBM.  `value` is
the exact model's events*iterations/s; beside it, in the same line, the MLP
scatter surrogate's (network trained on random water bodies, its density
scaled per patient to the exact model's total over a sample of the patient's
events) with its region-uptake bias against the exact model.  Setup (attenuation tables, sensitivities, event
plan, autotuning, surrogate training) is timed separately in `setup_s`.

The surrogate is also reported with the network evaluated at nodes every 2 and
every 4 pixels, the support pixels interpolated bilinearly (`surrogate_grid2`,
`surrogate_grid4`; each refitted per patient and window, with its own timing and
region bias).

Also beside them: the exact model with its scattered part evaluated at node
pixels every 2 pixels and interpolated (`exact_pixel_grid2`, an approximation
with its own region bias against the exact model).

Beside them (`extras`): the 64x64 workload (50k events, 8 subsets) with the
path-parameter table, 64 batched cases of it, continuous positions, the
cached-row mode (a different mode, never the headline), coarser scatter grids,
the 3-D single-scatter model and the 16x16 surrogate workload.

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X unit counts: 256 CUs x 128 FP32 lane-operations per cycle (the 157.3
# TFLOP/s vector rate) x 2.4 GHz, the transcendental unit at a quarter of it.
# One algorithmic term is one energy-Gaussian factor exp(-(s E - F)^2 + A): two
# FMAs to form the exponent, one exp, one FMA/add to accumulate: 3/128 + 1/32
# CU-cycles per term.
PEAK_TERMS_PER_S = 256 * 2.4e9 / (3.0 / 128.0 + 1.0 / 32.0)

# iterations after which the patients' images of the exact model, the
# surrogate and no scatter model are compared region by region
ROI_ITERS = 10

# scatter surrogate 6 -> 128 -> 128 -> 128 -> 1: multiply-adds per (event, pixel)
# pair, and MI355X's dense BF16/FP16 MFMA peak
MLP_MAC_PER_PAIR = 6 * 128 + 2 * 128 * 128 + 128
MLP_GELU_PER_PAIR = 3 * 128
PEAK_BF16_FLOPS = 2.5e15
PEAK_HBM_BYTES_PER_S = 8.0e12

SECTIONS = ("exact", "surrogate", "cpu", "calib", "64x64", "batched", "positions", "cached",
            "scatter_grids", "three_d", "small_surrogate", "pixel_grid")


def workload_desc(name, p, J, nsub):
    return (f"{name}: {p.n}x{p.n} at {p.pix:g} mm, scatter {p.ns}x{p.ns}, {p.nb} bins x {p.na} "
            f"angles, lines {'/'.join(f'{e:g}' for e in p.lines)} keV, {len(p.windows)} windows, "
            f"{J} events, {nsub} subsets")


def _sha256(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(profile, source):
    """HBM bytes per launch from a committed rocprofv3 counter summary, used only
    while the kernel source is the one the counters were taken on (else null)."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None, f"{profile} missing"
    kv = {}
    for line in open(path):
        m = re.match(r"^\s*([a-z0-9_]+):\s*(\S+)\s*$", line)
        if m:
            kv[m.group(1)] = m.group(2)
    want = _sha256(os.path.join(ROOT, "paper_2305_17111_amd", "csrc", source))
    if kv.get("source_sha256") != want:
        return None, f"{source} changed since the counters in {profile} were taken"
    try:
        return {"fetch": float(kv["fetch_bytes_per_launch"]),
                "write": float(kv["write_bytes_per_launch"])}, profile
    except KeyError:
        return None, f"{profile} has no per-launch byte counts"


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, mu, ev):
    """The FP64 oracle as it stands, on the first events of the headline's first
    patient: one OSEM iteration evaluates each event's system row once, so rows
    per second is the oracle's events*iterations/s.  All host threads on one
    event per thread, then one thread on one event."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    t = time.perf_counter()
    o = oracle.Oracle(p, np.asarray(mu, np.float32).astype(np.float64))
    setup_s = time.perf_counter() - t
    thr = oracle.threads()
    lam = np.ones(p.n * p.n)

    def run(n):
        sub = {"bin": ev["bin"][:n], "angle": ev["angle"][:n],
               "energy": ev["energy"][:n].astype(np.float64)}
        t0 = time.perf_counter()
        o.forward(sub, lam)
        return time.perf_counter() - t0

    dt = run(thr)
    oracle.set_threads(1)
    dt1 = run(1)
    oracle.set_threads(thr)
    return {"value": thr / dt, "unit": "events*iterations/s", "cores": thr, "kind": "oracle",
            "sample": f"first {thr} events of patient 0 of the headline workload x 1 iteration "
                      f"(FP64 system rows, one event per thread), {dt:.1f} s; tables "
                      f"{setup_s:.1f} s not timed",
            "one_thread": {"value": 1.0 / dt1, "sample": f"first event, {dt1:.1f} s"},
            "cpu_model": cpu_model(), "host_threads": os.cpu_count()}


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


def _timed_iterations(plan, sens, lam, warmup, steps):
    """warmup + steps eager iterations; the steps are timed on the host clock
    between two device synchronisations, with HIP events around every launch of
    the per-event kernel and of the surrogate's kernel."""
    import torch

    for _ in range(warmup):
        plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read_kernels()              # start a clean measurement
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.osem_iter(1, sens, lam)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    k = plan.profile_read_kernels()
    plan.profile(False)
    return el, k


def _bias(rel):
    import numpy as np

    return {"mean_rel": float(rel.mean()), "mean_abs_rel": float(np.abs(rel).mean()),
            "max_abs_rel": float(np.abs(rel).max())}


def headline(args, sections, out):
    """The metric's configuration: exact model and MLP surrogate on 16 patients
    at 128x128 with their own maps (1M events, 16 subsets)."""
    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import Context, calibrate, events_to_device, plan_maps

    w = synth.CONFIGS["128x128_16cases"]
    p = w.params
    counts = synth.case_counts(w)
    setup = {}
    t = time.perf_counter()
    ctxs, evs, rois, mus = [], [], [], []
    for c in range(w.n_cases):
        mu, act, roi = synth.phantom(w, c)
        rois.append(roi)
        mus.append(mu)
        evs.append(synth.generic_events(p, act, int(counts[c]), w.seed_events + c))
    setup["events"] = time.perf_counter() - t
    t = time.perf_counter()
    for c in range(w.n_cases):
        ctxs.append(Context(p, torch.from_numpy(mus[c].astype(np.float32))))
    torch.cuda.synchronize()
    setup["tables"] = time.perf_counter() - t
    t = time.perf_counter()
    sens = torch.stack([c.sensitivity(w.n_subsets) for c in ctxs]).contiguous()
    torch.cuda.synchronize()
    setup["sensitivity"] = time.perf_counter() - t
    t = time.perf_counter()
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("bin", "angle", "energy")}
    offs = np.concatenate([[0], np.cumsum(counts)]).tolist()
    plan = plan_maps(ctxs, events_to_device(cat), w.n_subsets, offs)
    torch.cuda.synchronize()
    setup["plan"] = time.perf_counter() - t
    t = time.perf_counter()
    if args.event_tile:
        plan.set_event_tile(args.event_tile)
        jt = args.event_tile
    else:                                   # the library's autotuner (times k_row per tile)
        jt = plan.autotune(use_cache=False)
    setup["autotune"] = time.perf_counter() - t
    J = int(counts.sum())
    Qm = ctxs[0].support_size
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    lam0 = lam0.repeat(w.n_cases, 1).contiguous()
    W, K = args.warmup, args.steps
    roi_iters = max(ROI_ITERS, W + K)
    terms, full_terms = plan.terms()

    def uptakes(x):
        return np.array([[x[c][r].sum() for r in rois[c]] for c in range(w.n_cases)])

    desc = (f"{w.n_cases} patients (own phantom and attenuation map) at {p.n}x{p.n}, "
            f"{p.pix:g} mm pixels, scatter {p.ns}x{p.ns}, {p.nb} bins x {p.na} angles, lines "
            f"{'/'.join(f'{e:g}' for e in p.lines)} keV, {len(p.windows)} windows, {J} events "
            f"({int(counts.min())}..{int(counts.max())} per patient), {w.n_subsets} subsets")

    lam = lam0.clone()
    el, k = _timed_iterations(plan, sens, lam, W, K)
    assert bool(torch.isfinite(lam).all())
    row_ms, row_n = k["k_row"]
    achieved = terms * K / (row_ms * 1e-3)
    compare = ("surrogate" in sections and not args.surrogate_untrained) or "pixel_grid" in sections
    if compare and roi_iters > W + K:
        plan.osem_graph(roi_iters - W - K, sens, lam)
    up_ex = uptakes(lam.cpu().numpy().astype(np.float64))
    mt, mt_src = measured_traffic("k_row_128x128_16cases_hbm_traffic.md", "kernels.hip")
    rows_per_launch = J / w.n_subsets
    Qp = (Qm + 63) // 64 * 64
    meas_peak = calibrate(0) if "calib" in sections else None
    out.update({
        "metric": "LM-MEW OSEM events*iterations/s and s/iteration, exact vs MLP surrogate, 1 GPU",
        "value": J * K / el,
        "unit": "events*iterations/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * el / K,
        "s_per_iteration": el / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantoms and generic list-mode events; random-init "
                "surrogate trained on the exact model's labels)",
        "system_model": "exact (the surrogate's figures are under \"surrogate\")",
        "config": {"workload": desc, "events": J, "patients": w.n_cases,
                   "subsets": w.n_subsets, "iterations_per_step": 1, "event_tile": jt,
                   "pixels_in_support": Qm},
        "roofline": {
            "bound": "alu",
            "kernel": "k_row (per-event system model)",
            "achieved": achieved / 1e12,
            "peak": PEAK_TERMS_PER_S / 1e12,
            "unit": "Tterm/s",
            "frac": achieved / PEAK_TERMS_PER_S,
            "measured_peak": meas_peak / 1e12 if meas_peak else None,
            "frac_of_measured_peak": achieved / meas_peak if meas_peak else None,
            "traffic": (mt["fetch"] + mt["write"]) if mt else None,
            "traffic_unit": "bytes per launch",
            "traffic_source": mt_src,
            "algorithmic_bytes_per_launch": rows_per_launch * Qp * 4,
            "terms_per_launch": terms / w.n_subsets,
            "avg_launch_ms": row_ms / row_n,
            "launches": row_n,
            "kernel_share_of_step": row_ms / (1e3 * el),
        },
        "model_terms_per_iteration": {"evaluated": terms, "unpruned": full_terms},
    })
    setup_total = dict(setup)
    if "pixel_grid" in sections:
        # the exact model with its scattered part at node pixels every 2
        # pixels, interpolated (an approximation; not the headline)
        for c in ctxs:
            c.set_scatter_pixel_grid(2)
        lam = lam0.clone()
        el_g, _ = _timed_iterations(plan, sens, lam, W, K)
        if roi_iters > W + K:
            plan.osem_graph(roi_iters - W - K, sens, lam)
        rel_g = uptakes(lam.cpu().numpy().astype(np.float64)) / up_ex - 1.0
        out["exact_pixel_grid2"] = {
            "value": J * K / el_g, "unit": "events*iterations/s", "s_per_iteration": el_g / K,
            "speedup_vs_exact": el / el_g,
            "what": "exact model, scattered part at node pixels every 2 pixels, interpolated",
            "roi_uptake_vs_exact": {"iterations": roi_iters, **_bias(rel_g)}}
        for c in ctxs:
            c.set_scatter_pixel_grid(1)
    if "cached" in sections:
        # not the headline: the rows of every subset computed once (52 GB at
        # this size), the iterations then read them (HBM-bound)
        out["cached_rows"] = cached_rows(plan, sens, lam0, J, Qp, K)

    if "surrogate" in sections and args.surrogate_untrained:
        # inference cost only (a random-init network on the first of the
        # evaluation grids; for profiling runs)
        net = ctxs[0].mlp(seed=2)
        net.set_grid(args.surrogate_grids[0])
        ctxs[0].set_scatter_model(net)
        lam = lam0.clone()
        el_s, ks = _timed_iterations(plan, sens, lam, W, K)
        mlp_ms, mlp_n = ks["k_mlp_rows"]
        out["surrogate"] = {"untrained": True, "value": J * K / el_s,
                            "evaluation_grid": args.surrogate_grids[0],
                            "s_per_iteration": el_s / K, "avg_ms_per_subset": mlp_ms / mlp_n}
        ctxs[0].set_scatter_model(None)
    elif "surrogate" in sections:
        net = ctxs[0].mlp(seed=2)
        maps = synth.random_body_maps(p, 16, seed=41).astype(np.float32)
        n_lab = -(-10_000_000 // (16 * Qm))
        t = time.perf_counter()
        losses = net.fit_maps([torch.from_numpy(m) for m in maps], n_lab,
                              epochs=args.surrogate_epochs, batch=8192, lr=2e-3,
                              floor_frac=3e-2, seed=3)
        torch.cuda.synchronize()
        pretrain_s = time.perf_counter() - t
        theta, c0, fl = net.get_params()
        # the pre-trained network alone (no map input): every patient uses it
        ctxs[0].set_scatter_model(net)
        lam = lam0.clone()
        plan.osem_graph(roi_iters, sens, lam)
        up_shared = uptakes(lam.cpu().numpy().astype(np.float64))
        # the same iterations with the scatter term switched off (the network's
        # output shifted by -100 in log space: a density below 1e-40): the
        # method without a scatter model
        off = ctxs[0].mlp(seed=0)
        off.set_params(theta, c0 - 100.0, 0.0)
        ctxs[0].set_scatter_model(off)
        lam = lam0.clone()
        plan.osem_graph(roi_iters, sens, lam)
        up_none = uptakes(lam.cpu().numpy().astype(np.float64))
        ctxs[0].set_scatter_model(net)
        mm, mm_src = measured_traffic("k_mlp_rows_128x128_16cases_hbm_traffic.md", "mlp.hip")
        calib_total = 0.0
        for gi, grid in enumerate(args.surrogate_grids):
            net.set_grid(grid)
            nodes = net.grid_nodes()
            # per patient and energy window: the factor that matches the
            # network's total scattered density to the exact model's over a
            # sample of the patient's own events (the network has no
            # attenuation-map input); fitted on the network as evaluated
            t = time.perf_counter()
            kappa = []
            for c in range(w.n_cases):
                e = evs[c]
                idx = np.linspace(0, e["bin"].size - 1, args.calib_events).astype(np.int64)
                sub = events_to_device({k: e[k][idx] for k in ("bin", "angle", "energy")})
                kappa.append(ctxs[c].scatter_scale_fit_windows(net, sub))
                ctxs[c].set_scatter_scale_windows(kappa[-1])
            torch.cuda.synchronize()
            calib_s = time.perf_counter() - t
            calib_total += calib_s
            lam = lam0.clone()
            el_s, ks = _timed_iterations(plan, sens, lam, W, K)
            assert bool(torch.isfinite(lam).all())
            if roi_iters > W + K:
                plan.osem_graph(roi_iters - W - K, sens, lam)
            up_sur = uptakes(lam.cpu().numpy().astype(np.float64))
            for c in range(w.n_cases):
                ctxs[c].set_scatter_scale(1.0)
            rel = up_sur / up_ex - 1.0
            mlp_ms, mlp_n = ks["k_mlp_rows"]
            prim_ms, _ = ks["k_row"]
            pairs = float(J) * nodes
            flops = pairs * 2 * MLP_MAC_PER_PAIR * K / (mlp_ms * 1e-3)
            mt_g, mt_g_src = (mm, mm_src) if grid == 1 else measured_traffic(
                f"k_mlp_rows_grid{grid}_128x128_16cases_hbm_traffic.md", "mlp.hip")
            entry = {
                "value": J * K / el_s, "unit": "events*iterations/s",
                "ms_per_step": 1e3 * el_s / K, "s_per_iteration": el_s / K,
                "speedup_vs_exact": el / el_s,
                "evaluation_grid": {
                    "spacing_pixels": grid, "positions_per_row": nodes,
                    "what": "network at every support pixel" if grid == 1 else
                            f"network at nodes every {grid} pixels ({grid * p.pix:g} mm), "
                            "support pixels interpolated bilinearly"},
                "roi_uptake_vs_exact": {
                    "iterations": roi_iters, "regions": int(rel.size),
                    "calibrated_per_patient_window": _bias(rel),
                    "bias_within_1pct": bool(abs(rel.mean()) <= 0.01),
                    "per_patient_mean_rel": [float(v) for v in rel.mean(1)]},
                "roofline": {
                    "bound": "mfma",
                    "kernel": "k_mlp_rows (surrogate inference, all patients' launches of a "
                              "subset" + (")" if grid == 1 else ", at the nodes)"),
                    "achieved": flops / 1e12, "peak": PEAK_BF16_FLOPS / 1e12,
                    "unit": "TFLOP/s", "frac": flops / PEAK_BF16_FLOPS,
                    "traffic": (mt_g["fetch"] + mt_g["write"]) if mt_g else None,
                    "traffic_source": mt_g_src,
                    "flop_per_pair": 2 * MLP_MAC_PER_PAIR, "gelu_per_pair": MLP_GELU_PER_PAIR,
                    "pairs_per_s": pairs * K / (mlp_ms * 1e-3),
                    "avg_ms_per_subset": mlp_ms / mlp_n, "subsets_timed": mlp_n},
                "unscattered_kernel_ms_per_iteration": prim_ms / K,
                "unscattered_kernel": "k_row, unscattered part" if grid == 1 else
                                      "k_prim_interp: unscattered part and the interpolated "
                                      "node values in one pass",
                "calibration": {"events_per_patient": args.calib_events, "seconds": calib_s,
                                "scales_per_window": [[float(v) for v in k] for k in kappa],
                                "what": "exact / network scattered density summed over the "
                                        "rows of the sampled events of each energy window"},
            }
            if gi == 0:
                entry["roi_uptake_vs_exact"]["uncalibrated"] = _bias(up_shared / up_ex - 1.0)
                entry["roi_uptake_vs_exact"]["no_scatter_model"] = _bias(up_none / up_ex - 1.0)
                entry["training"] = {"pretrain": {
                    "samples": int(16 * n_lab * Qm), "epochs": args.surrogate_epochs,
                    "batch": 8192, "seconds": pretrain_s, "first_loss": losses[0],
                    "last_loss": losses[-1], "maps": "16 random water bodies"}}
                out["surrogate"] = entry
            else:
                entry["training"] = "the network of \"surrogate\""
                out[f"surrogate_grid{grid}"] = entry
        net.set_grid(1)
        ctxs[0].set_scatter_model(None)
        setup_total["surrogate_training"] = pretrain_s + calib_total
    out["setup_s"] = setup_total
    if "cpu" in sections:
        out["cpu_baseline"] = cpu_baseline(p, mus[0], evs[0])
    if "calib" in sections:
        out["calibration"] = {
            "term_chain_per_s": meas_peak,
            "fma_lane_ops_per_s": calibrate(1),
            "exp2_lane_ops_per_s": calibrate(2),
            "note": "lmmew_calibrate: 16 independent chains per lane, 8 waves per SIMD"}
    del plan, ctxs, sens


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
    """The 64x64 iterations on the same events handed over with their
    continuous lateral positions instead of bins (density response)."""
    import torch

    from paper_2305_17111_amd import events_to_device

    plan = ctx.plan(events_to_device({k: ev[k] for k in ("position", "angle", "energy")}), nsub)
    plan.autotune(use_cache=False)
    lam = lam0.clone()
    el, k = _timed_iterations(plan, sens, lam, 1, steps)
    ms, n_launch = k["k_row"]
    terms, _ = plan.terms()
    ach = terms * steps / (ms * 1e-3)
    assert bool(torch.isfinite(lam).all())
    return {"ms_per_step": 1e3 * el / steps, "value": J * steps / el,
            "unit": "events*iterations/s", "event_tile": plan.event_tile,
            "k_row_avg_launch_ms": ms / n_launch, "terms_per_iteration": terms,
            "frac": ach / PEAK_TERMS_PER_S}


def batched(ctx, sens, steps, no_cached):
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
    s_it = _time_graph(plan, sens, lam, steps)
    J = int(counts.sum())
    terms, _ = plan.terms()
    assert bool(torch.isfinite(lam).all())
    lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    lam0 = lam0.repeat(len(counts), 1).contiguous()
    Qp = (int(synth.fov_support(p).sum()) + 63) // 64 * 64
    cached = None if no_cached else cached_rows(plan, sens, lam0, J, Qp, steps)
    return {"workload": f"{len(counts)} cases of the 64x64 workload, {J} events "
                        f"({int(counts.min())}..{int(counts.max())} per case), {w.n_subsets} subsets",
            "value": J / s_it, "unit": "events*iterations/s",
            "s_per_iteration": s_it, "steps": steps,
            "event_tile": jt, "terms_per_s": terms / s_it,
            "frac_of_term_peak": terms / s_it / PEAK_TERMS_PER_S,
            "setup_s": {"events": gen_s, "plan": plan_s, "autotune": tune_s},
            "cached_rows": cached}


def workload_64(args, sections):
    """The 64x64 workload (50k events, 8 subsets) with the path-parameter table,
    and what runs on it."""
    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import Context, LmmewError, events_to_device

    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, _ = synth.phantom(w)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=w.poisson)
    J = int(ev["bin"].size)
    nsub = w.n_subsets
    steps = args.steps_64
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
    t = time.perf_counter()
    plan.autotune(use_cache=False)
    setup["autotune_ms"] = 1e3 * (time.perf_counter() - t)
    lam = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
    el, k = _timed_iterations(plan, sens, lam, 2, steps)
    row_ms, launches = k["k_row"]
    assert bool(torch.isfinite(lam).all())
    graph_s = _time_graph(plan, sens, lam, steps)
    terms, full_terms = plan.terms()
    achieved = terms * steps / (row_ms * 1e-3)
    mt, mt_src = measured_traffic("k_row_64x64_50k_hbm_traffic.md", "kernels.hip")
    Qp = (int(synth.fov_support(p).sum()) + 63) // 64 * 64
    res = {
        "workload": workload_desc(w.name, p, J, nsub),
        "value": J * steps / el, "unit": "events*iterations/s", "steps": steps,
        "ms_per_step": 1e3 * el / steps, "graph_ms_per_step": 1e3 * graph_s,
        "event_tile": plan.event_tile, "path_table_bytes": path_table,
        "roofline": {"bound": "alu",
                     "kernel": "k_row (per-event system model%s)"
                               % (", path-parameter table" if path_table else ""),
                     "achieved": achieved / 1e12, "peak": PEAK_TERMS_PER_S / 1e12,
                     "unit": "Tterm/s", "frac": achieved / PEAK_TERMS_PER_S,
                     "traffic": (mt["fetch"] + mt["write"]) if mt else None,
                     "traffic_unit": "bytes per launch", "traffic_source": mt_src,
                     "algorithmic_bytes_per_launch": J / nsub * Qp * 4,
                     "terms_per_launch": terms / nsub, "avg_launch_ms": row_ms / launches,
                     "kernel_share_of_step": row_ms / (1e3 * el)},
        "model_terms_per_iteration": {"evaluated": terms, "unpruned": full_terms},
        "setup_ms": setup,
    }
    if "cached" in sections:
        lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
        res["cached_rows"] = cached_rows(plan, sens, lam0, J, Qp, steps)
    if "positions" in sections:
        lam0 = torch.from_numpy(synth.fov_support(p).astype(np.float32)).cuda()
        res["continuous_positions"] = positions(ctx, ev, nsub, sens, lam0, J, steps)
    if path_table:
        ctx.path_table(False)
        el_nt, k_nt = _timed_iterations(plan, sens, lam, 1, min(steps, 5))
        ms_nt, n_nt = k_nt["k_row"]
        n = min(steps, 5)
        res["without_path_table"] = {"ms_per_step": 1e3 * el_nt / n, "value": J * n / el_nt,
                                     "k_row_avg_launch_ms": ms_nt / n_nt,
                                     "frac": terms * n / (ms_nt * 1e-3) / PEAK_TERMS_PER_S}
    extra = {}
    if "batched" in sections:
        extra["batched_64x64_64cases"] = batched(ctx, sens, 2, "cached" not in sections)
    del plan
    if "scatter_grids" in sections:
        extra["scatter_resolution"] = scatter_resolution(ev, 2)
    return res, extra


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
    ctx = Context(p, torch.from_numpy(np.asarray(mu, np.float32)))
    sens = ctx.sensitivity(w.n_subsets)
    plan = ctx.plan(events_to_device(ev), w.n_subsets)
    plan.autotune(use_cache=False)
    lam = torch.from_numpy(synth.fov_support3(p).astype(np.float32)).cuda()
    el, k = _timed_iterations(plan, sens, lam, 1, steps)
    ms, n_launch = k["k_row"]
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
            "frac": ach / PEAK_TERMS_PER_S}


def scatter_resolution(ev, steps):
    """The 64x64 workload with the scatter modelled on coarser grids (the
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


def small_surrogate():
    """The 16x16 workload the surrogate's accuracy tests use: exact model against
    the surrogate (10 iterations as one graph launch)."""
    import numpy as np
    import torch

    import synth
    from paper_2305_17111_amd import Context, events_to_device

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
    return {"workload": workload_desc("16x16_2k", p, w.n_events, w.n_subsets),
            "unit": "events*iterations/s", **res,
            "training": {"samples": int(16 * 3000 * ctx.support_size), "epochs": 16,
                         "seconds": train_s, "maps": "16 random water bodies"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5,
                    help="timed iterations of the headline (exact and surrogate each)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--only", default="all",
                    help="comma-separated sections to run: " + ",".join(SECTIONS))
    ap.add_argument("--skip", default="", help="comma-separated sections to leave out")
    ap.add_argument("--steps-64", type=int, default=10)
    ap.add_argument("--steps-3d", type=int, default=2)
    ap.add_argument("--surrogate-epochs", type=int, default=8)
    ap.add_argument("--surrogate-grids", default="1,2,4",
                    help="evaluation grids of the surrogate (node spacing in pixels), the "
                         "first reported as \"surrogate\", the others beside it")
    ap.add_argument("--calib-events", type=int, default=256,
                    help="events per patient for the surrogate's per-patient scale")
    ap.add_argument("--surrogate-untrained", action="store_true",
                    help="time the surrogate's inference with a random-init network (no "
                         "training, no accuracy figures; for profiling runs)")
    ap.add_argument("--event-tile", type=int, default=0, help="0 = autotune over 16, 32, 64")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device with a plain copy kernel (a known "
                         "byte count for scaling hardware traffic counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs the whole reconstruction on "
              "a single MI355X (the design notes describe how it would shard)", file=sys.stderr)
        sys.exit(2)
    sections = set(SECTIONS) if args.only == "all" else set(args.only.split(","))
    sections -= set(s for s in args.skip.split(",") if s)
    unknown = sections - set(SECTIONS)
    if unknown:
        print(f"unknown sections: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    args.surrogate_grids = [int(g) for g in args.surrogate_grids.split(",") if g]
    if not args.surrogate_grids or not all(1 <= g <= 8 for g in args.surrogate_grids):
        print("--surrogate-grids: node spacings of 1 to 8 pixels", file=sys.stderr)
        sys.exit(2)

    import torch

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

    out = {}
    if "exact" in sections:
        headline(args, sections, out)
    extras = {}
    if "64x64" in sections:
        res, extra = workload_64(args, sections)
        extras["64x64_50k"] = res
        extras.update(extra)
    if "three_d" in sections:
        extras["three_d"] = three_d(args.steps_3d)
    if "small_surrogate" in sections:
        extras["surrogate_16x16"] = small_surrogate()
    out["extras"] = extras
    print(json.dumps(out))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
