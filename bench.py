#!/usr/bin/env python
"""Benchmark of list-mode multi-energy-window OSEM on one MI355X.

One step = one OSEM iteration (all angle subsets: per-event system model,
forward projection, compensated backprojection, EM update) over the workload's
whole event list, inputs resident in HBM.  Setup (attenuation tables,
sensitivity, event plan, tile autotuning) is timed separately and reported in
`setup_ms`.

Default workload: 64x64 object at 4 mm, 32x32 scatter grid, 64 bins x 120
angles, lines 85/154/270 keV, windows 68-102/123-184/243-297 keV, ~50k events,
8 subsets (the 20-iteration schedule runs as 20 steps).

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X unit counts: 256 CUs x 128 FP32 lanes per cycle x 2.4 GHz; a
# transcendental (v_exp_f32) issues at a quarter of the FP32 rate.  One
# algorithmic term needs one exp and at least two FP32 operations (forming the
# exponent, accumulating), i.e. 4 + 2 = 6 issue slots.
LANES_PER_S = 256 * 128 * 2.4e9
SLOTS_PER_TERM = 6.0
PEAK_TERMS_PER_S = LANES_PER_S / SLOTS_PER_TERM


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

    w = synth.CONFIGS["c3"]
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
    return {"workload": f"c3: {len(counts)} cases of the 64x64 workload, {J} events "
                        f"({int(counts.min())}..{int(counts.max())} per case), {w.n_subsets} subsets",
            "value": J * args.batched_steps / el, "unit": "events*iterations/s",
            "s_per_iteration": el / args.batched_steps, "steps": args.batched_steps,
            "event_tile": jt, "terms_per_s": terms * args.batched_steps / el,
            "frac_of_term_peak": terms * args.batched_steps / el / PEAK_TERMS_PER_S,
            "setup_s": {"events": gen_s, "plan": plan_s, "autotune": tune_s}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--event-tile", type=int, default=0,
                    help="0 = autotune over 16, 32, 64")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device with a plain copy kernel (a known "
                         "byte count for scaling hardware traffic counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build runs the whole reconstruction on a "
              "single MI355X (see the design notes for how it would shard)", file=sys.stderr)
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
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_row (per-event system model)",
            "achieved": achieved / 1e12,
            "peak": PEAK_TERMS_PER_S / 1e12,
            "unit": "Tterm/s",
            "frac": achieved / PEAK_TERMS_PER_S,
            "traffic": None,
            "terms_per_launch": terms * args.steps / launches,
            "avg_launch_ms": row_ms / launches,
            "kernel_share_of_step": row_ms / (1e3 * elapsed),
        },
        "graph_ms_per_step": graph_ms,
        "model_terms_per_iteration": {"evaluated": terms, "unpruned": full_terms},
        "setup_ms": setup,
    }
    del plan
    if not args.no_batched:
        out["batched"] = batched(ctx, sens, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, mu, ev, args.cpu_seconds)
    print(json.dumps(out))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
