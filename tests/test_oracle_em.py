"""Pins of the oracle's list-mode OSEM (Sec. 2.3-2.4, Eq. (16)-(20)).

- counts are conserved by every sub-iteration: sum_q sens_s[q] lambda_q^new
  equals the number of the subset's events with p_j > 0 (exact identity);
- images stay non-negative;
- the first update does not depend on the scale of the initial image;
- with one subset the log-likelihood of Eq. (8) never decreases;
- with every energy equal, list-mode OSEM equals an independently written
  binned OSEM on the counts per (bin, angle);
- the maximum-likelihood image found by a generic bounded optimiser is a fixed
  point of the EM update;
- events the image cannot explain (p_j = 0) are skipped and counted;
- the exact-model sampler reproduces the model's distribution over angle and
  bin (chi-square).
"""
import numpy as np
import pytest
from scipy import optimize, stats

import synth


def _setup(oracle_mod, J=300, seed=1, n=8, ns=4, nb=8, na=8, mu_val=0.018):
    p = synth.SysParams(n=n, pix=4.0, ns=ns, nb=nb, na=na)
    x, y = synth.pixel_centres(p)
    body = x * x + y * y <= (0.85 * p.R) ** 2
    mu = np.where(body, mu_val, 0.0)
    act = np.where(body, 1.0, 0.0) + np.where((x - 4) ** 2 + y ** 2 <= 36, 3.0, 0.0)
    o = oracle_mod.Oracle(p, mu)
    ev = o.sample_events(act, J, seed)
    return p, o, act, ev


def test_count_conservation_and_nonnegativity(oracle_mod):
    p, o, act, ev = _setup(oracle_mod)
    nsub, niter = 2, 3
    sens = o.sensitivity(nsub)
    lam0 = o.support.astype(float)
    lam, hist, ll, sk = o.osem(ev, nsub, niter, lam0, sens)
    for k in range(nsub * niter):
        s = k % nsub
        Js = int(np.sum(ev["angle"] % nsub == s))
        assert np.all(hist[k] >= 0)
        assert np.sum(sens[s] * hist[k]) == pytest.approx(Js - sk[k], rel=1e-11)


def test_first_update_invariant_to_initial_scale(oracle_mod):
    p, o, act, ev = _setup(oracle_mod, seed=2)
    sens = o.sensitivity(4)
    lam0 = o.support.astype(float) * (1 + 0.1 * np.arange(p.n * p.n) % 3)
    a = o.osem(ev, 4, 1, lam0, sens)[1][0]
    b = o.osem(ev, 4, 1, 7.5 * lam0, sens)[1][0]
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_loglikelihood_monotone_with_one_subset(oracle_mod):
    p, o, act, ev = _setup(oracle_mod, seed=3)
    sens = o.sensitivity(1)
    lam, hist, ll, sk = o.osem(ev, 1, 25, o.support.astype(float), sens)
    assert np.all(np.diff(ll) >= -1e-10 * np.abs(ll[1:]))
    assert ll[-1] > ll[0]


def test_binned_equivalence_when_energies_coincide(oracle_mod):
    p, o, act, ev = _setup(oracle_mod, J=400, seed=4)
    ev = dict(ev)
    ev["energy"] = np.full(ev["bin"].size, 85.0)
    nsub, niter = 4, 3
    sens = o.sensitivity(nsub)
    lam0 = o.support.astype(float)
    lam_lm = o.osem(ev, nsub, niter, lam0, sens)[0]
    # independent binned OSEM on counts y[b, a] with H[(b,a), q] = density at 85 keV
    y = np.zeros((p.nb, p.na))
    np.add.at(y, (ev["bin"], ev["angle"]), 1.0)
    H = {(b, a): o.row(b, a, 85.0) for b in range(p.nb) for a in range(p.na) if y[b, a] > 0}
    lam = lam0.copy()
    for _ in range(niter):
        for s in range(nsub):
            back = np.zeros_like(lam)
            for (b, a), h in H.items():
                if a % nsub != s:
                    continue
                pb = h @ lam
                if pb > 0:
                    back += y[b, a] * h / pb
            upd = sens[s] > 0
            lam = np.where(upd, lam * back / np.where(upd, sens[s], 1.0), lam)
    np.testing.assert_allclose(lam_lm, lam, rtol=1e-10, atol=1e-14 * lam.max())


def test_mle_is_fixed_point_of_em(oracle_mod):
    p, o, act, ev = _setup(oracle_mod, J=250, seed=5, n=4, ns=2, nb=4, na=4)
    sup = o.support
    qs = np.flatnonzero(sup)
    sens = o.sensitivity(1)[0]
    A = np.stack([o.row(b, a, e) for b, a, e in zip(ev["bin"], ev["angle"], ev["energy"])])[:, qs]
    S = sens[qs]

    def negll(x):
        pj = A @ x
        return -(np.sum(np.log(pj)) - S @ x)

    def grad(x):
        pj = A @ x
        return -(A.T @ (1.0 / pj) - S)

    x0 = np.full(qs.size, ev["bin"].size / S.sum())
    res = optimize.minimize(negll, x0, jac=grad, method="L-BFGS-B",
                            bounds=[(1e-12, None)] * qs.size,
                            options=dict(ftol=1e-15, gtol=1e-12, maxiter=20000))
    lam_star = np.zeros(p.n * p.n)
    lam_star[qs] = res.x
    upd = o.osem(ev, 1, 1, lam_star, sens[None, :])[0]
    big = res.x > 1e-6 * res.x.max()
    np.testing.assert_allclose(upd[qs][big], res.x[big], rtol=2e-5)
    # and EM started elsewhere climbs to the same likelihood
    lls = [-negll(np.maximum(o.osem(ev, 1, k, sup.astype(float), sens[None, :])[0][qs], 1e-300))
           for k in (100, 3000)]
    assert lls[0] < lls[1] <= -res.fun + 1e-9
    assert -res.fun - lls[1] < 0.1 * (-res.fun - lls[0])


def test_unexplained_events_are_skipped(oracle_mod):
    # narrow collimator response so that the far tail underflows to exactly 0
    p = synth.SysParams(n=16, pix=4.0, ns=8, nb=16, na=8, fwhm0=0.5, fwhm_slope=0.0)
    o = oracle_mod.Oracle(p, np.zeros(p.n * p.n))     # no attenuation, no scatter
    lam = np.zeros(p.n * p.n)
    q = 8 * 16 + 1          # pixel centre (-26, 2) mm: projects into bin 8 at angle 0
    lam[q] = 1.0
    ev = {"bin": np.array([15, 8], np.int32), "angle": np.array([0, 0], np.int32),
          "energy": np.array([85.0, 85.0])}
    pj = o.forward(ev, lam)
    assert pj[0] == 0.0 and pj[1] > 0.0
    sens = o.sensitivity(1)
    lam1, hist, ll, sk = o.osem(ev, 1, 1, lam, sens)
    assert sk[0] == 1
    assert np.sum(sens[0] * lam1) == pytest.approx(1.0, rel=1e-12)


def test_invalid_events_are_reported(oracle_mod):
    p = synth.SysParams(n=8, pix=4.0, ns=4, nb=8, na=8)
    o = oracle_mod.Oracle(p, np.zeros(p.n * p.n))
    good = {"bin": np.array([1, 2]), "angle": np.array([0, 7]), "energy": np.array([80.0, 150.0])}
    assert o.check_events(good) == -1
    for key, val in [("bin", 8), ("angle", -1), ("energy", 110.0), ("energy", np.nan)]:
        bad = {k: v.copy() for k, v in good.items()}
        bad[key] = bad[key].astype(float if key == "energy" else int)
        bad[key][1] = val
        assert o.check_events(bad) == 1


def test_sampler_matches_model_distribution(oracle_mod):
    p = synth.SysParams(n=8, pix=4.0, ns=4, nb=8, na=8)
    x, y = synth.pixel_centres(p)
    mu = np.where(x * x + y * y <= 196, 0.02, 0.0)
    act = np.where(x * x + y * y <= 196, 1.0, 0.0) + np.where((x + 4) ** 2 + (y - 2) ** 2 <= 20, 4.0, 0.0)
    o = oracle_mod.Oracle(p, mu)
    J = 20000
    ev = o.sample_events(act, J, seed=9)
    # expected probability of each (angle, bin): sum over the categories of
    # mass x P(bin | point, angle) / P(detector | point, angle)
    m = o.sample_masses(act).reshape(-1, p.na, len(p.lines), 1 + o.nsc)
    qs = np.flatnonzero(o.support)
    sxy, _ = o.scatter_points()
    expct = np.zeros((p.na, p.nb))
    for a in range(p.na):
        for qi, q in enumerate(qs):
            pts = [o.pixel_centre(q)] + [tuple(s) for s in sxy]
            for c, (px, py) in enumerate(pts):
                mass = m[qi, a, :, c].sum()
                if mass == 0:
                    continue
                D = o.psf_total(px, py, a)
                for b in range(p.nb):
                    expct[a, b] += mass * o.psf_bin(b, px, py, a) / D
    expct *= J / expct.sum()
    obs = np.zeros_like(expct)
    np.add.at(obs, (ev["angle"], ev["bin"]), 1.0)
    keep = expct > 5
    chi2 = np.sum((obs[keep] - expct[keep]) ** 2 / expct[keep])
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi2, dof) > 1e-3
