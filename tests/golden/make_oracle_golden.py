"""Writes the oracle's expected values used by the GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators (synth/).
Every floating-point input is rounded to float32 first, exactly as the GPU path
receives it, and the oracle then works in double precision on those values.

    python tests/golden/make_oracle_golden.py small     # ~1 min on 8 cores
    python tests/golden/make_oracle_golden.py rows64    # sampled rows + sensitivity
    python tests/golden/make_oracle_golden.py iter64    # one full iteration, 2000 events
    python tests/golden/make_oracle_golden.py rows128   # sampled rows at 128x128
    python tests/golden/make_oracle_golden.py maps128   # one sub-iteration, two patients' maps
    python tests/golden/make_oracle_golden.py small_pos # continuous positions, 16x16
    python tests/golden/make_oracle_golden.py pos64     # continuous positions, sampled rows
    python tests/golden/make_oracle_golden.py small_3d  # 3-D model, 16x16x8
    python tests/golden/make_oracle_golden.py rows64_3d # 3-D model, sampled rows at 64x64x16
                                                         # (~10 min on 8 cores)
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def digest(ev):
    h = hashlib.sha256()
    for k in ("bin", "angle", "energy"):
        h.update(np.ascontiguousarray(ev[k]).tobytes())
    return h.hexdigest()


def small():
    w = synth.CONFIGS["16x16_2k"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32 = f32(mu)
    o = oracle.Oracle(p, mu32)
    ev = o.sample_events(act, w.n_events, seed=w.seed_events)
    ev = {"bin": ev["bin"].astype(np.int16), "angle": ev["angle"].astype(np.int16),
          "energy": ev["energy"].astype(np.float32)}
    evd = {"bin": ev["bin"], "angle": ev["angle"], "energy": ev["energy"].astype(np.float64)}
    sens = o.sensitivity(w.n_subsets)
    lam0 = o.support.astype(np.float64)
    sens32 = f32(sens)          # the GPU run is checked against the oracle fed the same sens
    t = time.time()
    lam, hist, ll, sk = o.osem(evd, w.n_subsets, w.n_iters, lam0, sens32)
    print("small osem", time.time() - t, "s")
    act32 = f32(act)
    p_act = o.forward(evd, act32)
    rng = np.random.default_rng(1234)
    wts = f32(rng.uniform(0.5, 1.5, ev["bin"].size))
    bp = o.backproject(evd, wts)
    np.savez_compressed(os.path.join(OUT, "16x16_2k_oracle.npz"), mu=mu32, act=act32,
                        support=o.support, bin=ev["bin"], angle=ev["angle"],
                        energy=ev["energy"], sens=sens, lam0=lam0, hist=hist, ll=ll,
                        skipped=sk, p_act=p_act, bp_w=wts, bp=bp)


def rows64():
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32, act32 = f32(mu), f32(act)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True)
    o = oracle.Oracle(p, mu32)
    rng = np.random.default_rng(2222)
    J = ev["bin"].size
    idx = np.sort(rng.choice(J, 12, replace=False))
    sub = {"bin": ev["bin"][idx], "angle": ev["angle"][idx],
           "energy": ev["energy"][idx].astype(np.float64)}
    t = time.time()
    p_act = o.forward(sub, act32)
    rows = np.stack([o.row(int(b), int(a), float(E))
                     for b, a, E in zip(sub["bin"], sub["angle"], sub["energy"])])
    print("rows64 rows", time.time() - t, "s")
    qs = np.flatnonzero(o.support)
    pix = np.sort(rng.choice(qs, 16, replace=False))
    nsub = w.n_subsets
    sens = np.zeros((nsub, pix.size))
    t = time.time()
    for k, q in enumerate(pix):
        for a in range(p.na):
            sens[a % nsub, k] += p.T * o.sens_qa(int(q), a)
    print("rows64 sens", time.time() - t, "s")
    np.savez_compressed(os.path.join(OUT, "64x64_50k_oracle.npz"), digest=digest(ev), J=J, idx=idx,
                        p_act=p_act, rows=rows, pix=pix, sens=sens)


def iter64():
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32 = f32(mu)
    ev = synth.generic_events(p, act, 2000, 23)
    evd = {"bin": ev["bin"], "angle": ev["angle"], "energy": ev["energy"].astype(np.float64)}
    o = oracle.Oracle(p, mu32)
    sens = o.sensitivity(w.n_subsets)
    lam0 = o.support.astype(np.float64)
    t = time.time()
    lam, hist, ll, sk = o.osem(evd, w.n_subsets, 1, lam0, f32(sens))
    print("iter64 iteration", time.time() - t, "s")
    np.savez_compressed(os.path.join(OUT, "64x64_50k_iter_oracle.npz"), digest=digest(ev), sens=sens,
                        lam0=lam0, hist=hist, ll=ll, skipped=sk)


def rows128():
    w = synth.CONFIGS["128x128_16cases"]
    p = w.params
    mu, act, rois = synth.phantom(w, 0)
    mu32, act32 = f32(mu), f32(act)
    ev = synth.generic_events(p, act, 20000, 5300)
    o = oracle.Oracle(p, mu32)
    rng = np.random.default_rng(5555)
    idx = np.sort(rng.choice(ev["bin"].size, 4, replace=False))
    sub = {"bin": ev["bin"][idx], "angle": ev["angle"][idx],
           "energy": ev["energy"][idx].astype(np.float64)}
    t = time.time()
    p_act = o.forward(sub, act32)
    rows = np.stack([o.row(int(b), int(a), float(E))
                     for b, a, E in zip(sub["bin"], sub["angle"], sub["energy"])])
    print("rows128 rows", time.time() - t, "s")
    np.savez_compressed(os.path.join(OUT, "128x128_16cases_oracle.npz"), digest=digest(ev), idx=idx,
                        p_act=p_act, rows=rows)


def maps128():
    """One sub-iteration (subset 0 of 16) of a plan over two patients of the
    128x128 workload, each with its own attenuation map: the first 150 events
    of subset 0 in each patient's event list."""
    w = synth.CONFIGS["128x128_16cases"]
    p = w.params
    nsub, per = w.n_subsets, 150
    out = {}
    for c in (0, 1):
        _, mu, act, _, ev = synth.workload_inputs(w.name, c)
        sel = np.flatnonzero(ev["angle"] % nsub == 0)[:per]
        sub = {"bin": ev["bin"][sel], "angle": ev["angle"][sel], "energy": ev["energy"][sel]}
        evd = {"bin": sub["bin"], "angle": sub["angle"], "energy": sub["energy"].astype(np.float64)}
        t = time.time()
        o = oracle.Oracle(p, f32(mu))
        sens = np.zeros((nsub, o.Q))
        sens[0] = o.sensitivity_subset(nsub, 0)
        print("maps128 case", c, "tables + sensitivity", time.time() - t, "s")
        lam0 = o.support.astype(np.float64)
        lam, hist, ll, sk = o.osem(evd, nsub, 1, lam0, f32(sens))
        print("maps128 case", c, "sub-iteration", time.time() - t, "s")
        out.update({f"sel{c}": sel, f"digest{c}": digest(ev), f"sens{c}": sens[0],
                    f"lam0_{c}": lam0, f"lam1_{c}": hist[0], f"ll{c}": ll[0], f"skipped{c}": sk[0]})
    np.savez_compressed(os.path.join(OUT, "128x128_maps_subiter_oracle.npz"), **out)


def below_R(u, p):
    """Positions as the GPU receives them: float32, kept inside [-R, R)."""
    return np.minimum(np.asarray(u, dtype=np.float32), np.nextafter(np.float32(p.R), np.float32(0)))


def small_pos():
    w = synth.CONFIGS["16x16_2k"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32 = f32(mu)
    o = oracle.Oracle(p, mu32)
    ev = o.sample_events(act, 1500, seed=77)
    ev = {"position": below_R(ev["position"], p), "angle": ev["angle"].astype(np.int16),
          "energy": ev["energy"].astype(np.float32)}
    evd = {"position": ev["position"].astype(np.float64), "angle": ev["angle"],
           "energy": ev["energy"].astype(np.float64)}
    assert o.check_events(evd) == -1
    sens = o.sensitivity(w.n_subsets)
    lam0 = o.support.astype(np.float64)
    t = time.time()
    lam, hist, ll, sk = o.osem(evd, w.n_subsets, 2, lam0, f32(sens))
    print("small_pos osem", time.time() - t, "s")
    p_act = o.forward(evd, f32(act))
    idx = np.arange(0, ev["angle"].size, 97)
    rows = np.stack([o.row_pos(evd["position"][j], evd["angle"][j], evd["energy"][j])
                     for j in idx])
    np.savez_compressed(os.path.join(OUT, "16x16_2k_pos_oracle.npz"), position=ev["position"],
                        angle=ev["angle"], energy=ev["energy"], sens=sens, lam0=lam0,
                        hist=hist, ll=ll, skipped=sk, p_act=p_act, idx=idx, rows=rows)


def pos64():
    w = synth.CONFIGS["64x64_50k"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32, act32 = f32(mu), f32(act)
    ev = synth.generic_events(p, act, w.n_events, w.seed_events, poisson=True)
    o = oracle.Oracle(p, mu32)
    rng = np.random.default_rng(3333)
    J = ev["angle"].size
    idx = np.sort(rng.choice(J, 12, replace=False))
    sub = {"position": ev["position"][idx].astype(np.float64), "angle": ev["angle"][idx],
           "energy": ev["energy"][idx].astype(np.float64)}
    t = time.time()
    p_act = o.forward(sub, act32)
    rows = np.stack([o.row_pos(sub["position"][j], sub["angle"][j], sub["energy"][j])
                     for j in range(idx.size)])
    assert np.allclose(rows @ act32.astype(np.float64), p_act, rtol=1e-12)
    print("pos64 rows", time.time() - t, "s")
    h = hashlib.sha256()
    for k in ("position", "angle", "energy"):
        h.update(np.ascontiguousarray(ev[k]).tobytes())
    np.savez_compressed(os.path.join(OUT, "64x64_50k_pos_oracle.npz"), digest=h.hexdigest(), J=J,
                        idx=idx, p_act=p_act, rows=rows)


def digest3(ev):
    h = hashlib.sha256()
    for k in ("bin", "bin_z", "angle", "energy"):
        h.update(np.ascontiguousarray(ev[k]).tobytes())
    return h.hexdigest()


def small_3d():
    w = synth.CONFIGS["16x16x8_600"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32, act32 = f32(mu), f32(act)
    o = oracle.Oracle3(p, mu32)
    ev = synth.generic_events3(p, act, w.n_events, w.seed_events)
    evd = {"bin": ev["bin"], "bin_z": ev["bin_z"], "angle": ev["angle"],
           "energy": ev["energy"].astype(np.float64)}
    assert o.check_events(evd) == -1
    t = time.time()
    sens = o.sensitivity(w.n_subsets)
    lam0 = o.support.astype(np.float64)
    lam, hist, ll, sk = o.osem(evd, w.n_subsets, w.n_iters, lam0, f32(sens))
    p_act = o.forward(evd, act32)
    idx = np.arange(0, ev["angle"].size, 50)
    rows = np.stack([o.row(evd["bin"][j], evd["bin_z"][j], evd["angle"][j], evd["energy"][j])
                     for j in idx])
    print("small_3d", time.time() - t, "s")
    np.savez_compressed(os.path.join(OUT, "16x16x8_600_oracle.npz"), digest=digest3(ev), mu=mu32,
                        act=act32, support=o.support, sens=sens, lam0=lam0, hist=hist, ll=ll,
                        skipped=sk, p_act=p_act, idx=idx, rows=rows)


def rows64_3d():
    w = synth.CONFIGS["64x64x16_50k"]
    p = w.params
    mu, act, rois = synth.phantom(w)
    mu32, act32 = f32(mu), f32(act)
    ev = synth.generic_events3(p, act, w.n_events, w.seed_events, poisson=True)
    rng = np.random.default_rng(4444)
    J = ev["angle"].size
    idx = np.sort(rng.choice(J, 8, replace=False))
    t = time.time()
    o = oracle.Oracle3(p, mu32)
    print("rows64_3d tables", time.time() - t, "s")
    sub = {"bin": ev["bin"][idx], "bin_z": ev["bin_z"][idx], "angle": ev["angle"][idx],
           "energy": ev["energy"][idx].astype(np.float64)}
    p_act = o.forward(sub, act32)
    qs = np.flatnonzero(o.support)
    pix = np.sort(rng.choice(qs, 8, replace=False))
    nsub = w.n_subsets
    sens = np.zeros((nsub, pix.size))
    for k, q in enumerate(pix):
        for a in range(p.na):
            sens[a % nsub, k] += p.T * o.sens_qa(int(q), a)
    print("rows64_3d p_j and sensitivity", time.time() - t, "s")
    # the sampled events' whole rows (every voxel), two minutes each: one
    # process per row, forked after the tables are built (they are shared)
    global _ROW3
    _ROW3 = (o, sub)
    import multiprocessing as mp
    with mp.get_context("fork").Pool(4) as pool:
        rows = np.stack(pool.map(_row3, range(idx.size)))
    assert np.allclose(rows @ act32.ravel().astype(np.float64), p_act, rtol=1e-12)
    print("rows64_3d rows", time.time() - t, "s")
    np.savez_compressed(os.path.join(OUT, "64x64x16_50k_oracle.npz"), digest=digest3(ev), J=J,
                        idx=idx, p_act=p_act, pix=pix, sens=sens, rows=rows.astype(np.float32))


_ROW3 = None


def _row3(k):
    o, sub = _ROW3
    return o.row(int(sub["bin"][k]), int(sub["bin_z"][k]), int(sub["angle"][k]),
                 float(sub["energy"][k]))


if __name__ == "__main__":
    oracle.build(force=False)
    for name in sys.argv[1:]:
        globals()[name]()
