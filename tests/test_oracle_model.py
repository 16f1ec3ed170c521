"""Pins of the oracle's system model (the per-event density and the sensitivity).

- mu = 0: the model reduces to the blurred parallel projection of each line,
  checked against scipy's normal CDF/PDF;
- a uniform square map: the unscattered path's attenuation is exp(-mu * chord),
  the chord from analytic clipping;
- the per-event density integrates (over bins and window energies) to the
  sensitivity, for every pixel;
- rotating object and detector together by 90 degrees leaves the model
  unchanged (catches sign, index and transposition mistakes);
- an independent Monte Carlo of photon histories (continuous transport through
  the uniform square, isotropic emission, 2-D Klein-Nishina scattering, forced
  detection) agrees with the scatter-point sum, and the disagreement shrinks
  as the scatter grid is refined.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import synth

ME = 510.99895
FWHM = 2 * math.sqrt(2 * math.log(2))


def _p(**kw):
    base = dict(n=8, pix=4.0, ns=4, nb=8, na=8)
    base.update(kw)
    return synth.SysParams(**base)


def test_primary_closed_form_without_attenuation(oracle_mod):
    p = _p(n=16, ns=8, nb=16, na=12)
    o = oracle_mod.Oracle(p, np.zeros(p.n * p.n))
    assert o.nsc == 0                      # no scatter points where mu = 0
    rng = np.random.default_rng(5)
    db = p.fov / p.nb
    for _ in range(6):
        b, a = int(rng.integers(0, p.nb)), int(rng.integers(0, p.na))
        E = float(rng.uniform(*p.windows[int(rng.integers(0, 2))]))
        row = o.row(b, a, E)
        th = 2 * math.pi * a / p.na
        for q in np.flatnonzero(o.support)[::7]:
            x, y = o.pixel_centre(q)
            u, depth = -x * math.sin(th) + y * math.cos(th), p.R - (x * math.cos(th) + y * math.sin(th))
            sig = (p.fwhm0 + p.fwhm_slope * depth) / FWHM
            lo = -p.R + b * db
            if lo > u:      # evaluate on the side of the tail that does not cancel
                psf = stats.norm.sf(lo, u, sig) - stats.norm.sf(lo + db, u, sig)
            else:
                psf = stats.norm.cdf(lo + db, u, sig) - stats.norm.cdf(lo, u, sig)
            ref = sum(al * p.dtheta / (2 * math.pi) * psf *
                      stats.norm.pdf(E, Ew, p.eres_frac * p.eres_ref * math.sqrt(Ew / p.eres_ref) / FWHM)
                      for Ew, al in zip(p.lines, p.yields))
            assert row[q] == pytest.approx(ref, rel=1e-9, abs=1e-300)


def _chord_square(x0, y0, dx, dy, half):
    """Distance from (x0,y0) (inside the square [-half,half]^2) to its boundary
    along the unit direction (dx,dy)."""
    ts = []
    for p_, o_ in ((dx, x0), (dy, y0)):
        if p_ > 0:
            ts.append((half - o_) / p_)
        elif p_ < 0:
            ts.append((-half - o_) / p_)
    return min(ts)


def test_attenuated_primary_uniform_square(oracle_mod):
    p = _p(n=16, ns=8, nb=16, na=16)
    mu = np.zeros((p.n, p.n))
    mu[4:12, 4:12] = 0.02
    o = oracle_mod.Oracle(p, mu.ravel())
    for q in [4 * 16 + 4, 7 * 16 + 9, 11 * 16 + 11, 8 * 16 + 5]:
        x, y = o.pixel_centre(q)
        for a in range(p.na):
            th = 2 * math.pi * a / p.na
            L = _chord_square(x, y, math.cos(th), math.sin(th), 16.0)
            for w, (Ew, al) in enumerate(zip(p.lines, p.yields)):
                ref = al * p.dtheta / (2 * math.pi) * math.exp(-0.02 * (Ew / 85.0) ** (-1 / 3) * L)
                assert o.Pp(q, a, w) == pytest.approx(ref, rel=1e-12)


def test_row_integrates_to_sensitivity(oracle_mod):
    p = _p(n=8, ns=4, nb=8, na=8)
    rng = np.random.default_rng(6)
    mu = rng.uniform(0.01, 0.03, p.n * p.n) * synth.fov_support(p)
    o = oracle_mod.Oracle(p, mu)
    assert o.nsc > 0
    xg, wg = np.polynomial.legendre.leggauss(96)
    for a in (0, 3):
        total = np.zeros(p.n * p.n)
        for lo, hi in p.windows:
            Es = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
            ws = 0.5 * (hi - lo) * wg
            for b in range(p.nb):
                for E, wt in zip(Es, ws):
                    total += wt * o.row(b, a, E)
        for q in np.flatnonzero(o.support):
            assert total[q] == pytest.approx(o.sens_qa(q, a), rel=1e-9)


def test_rotation_by_90_degrees(oracle_mod):
    p = _p(n=8, ns=4, nb=8, na=8)
    rng = np.random.default_rng(7)
    mu = (rng.uniform(0.0, 0.04, p.n * p.n) * synth.fov_support(p)).reshape(p.n, p.n)
    n = p.n
    # rotation (x, y) -> (-y, x): pixel (ix, iy) moves to (n-1-iy, ix)
    rot = np.zeros_like(mu)
    qmap = np.zeros(n * n, dtype=int)
    for iy in range(n):
        for ix in range(n):
            rot[ix, n - 1 - iy] = mu[iy, ix]
            qmap[iy * n + ix] = ix * n + (n - 1 - iy)
    o1 = oracle_mod.Oracle(p, mu.ravel())
    o2 = oracle_mod.Oracle(p, rot.ravel())
    for b, a, E in [(3, 1, 80.0), (5, 2, 150.0), (2, 5, 270.0), (4, 0, 95.0)]:
        r1 = o1.row(b, a, E)
        r2 = o2.row(b, (a + p.na // 4) % p.na, E)
        np.testing.assert_allclose(r2[qmap], r1, rtol=1e-10, atol=1e-300)
    for q in np.flatnonzero(o1.support)[::5]:
        assert o2.sens_qa(qmap[q], 2 + p.na // 4) == pytest.approx(o1.sens_qa(q, 2), rel=1e-10)


# ---- Monte Carlo of photon histories ---------------------------------------

def _kn(cosphi, E):
    P = 1.0 / (1.0 + E / ME * (1.0 - cosphi))
    return P * P * (P + 1.0 / P - (1.0 - cosphi ** 2))


def _mc_scatter(p, mu0, half, x0, y0, a, n_photons, seed):
    """Expected detected once-scattered photons per emitted decay from (x0,y0)
    at angle a, by simulating photon histories: isotropic emission, free path
    drawn from the exponential law in a uniform square of attenuation mu0 (at
    85 keV) scaled to each energy, Compton scattering into the collimator's
    acceptance with the planar Klein-Nishina density (forced detection),
    attenuation on the way out, then detector extent and energy windows."""
    rng = np.random.default_rng(seed)
    th = 2 * math.pi * a / p.na
    na_ = np.array([math.cos(th), math.sin(th)])
    if (4 * a) % p.na == 0:
        na_ = np.round(na_)
    total = 0.0
    for Ew, al in zip(p.lines, p.yields):
        Z = integrate.quad(lambda f: _kn(math.cos(f), Ew), 0, 2 * math.pi, epsabs=1e-12)[0]
        muw = mu0 * (Ew / 85.0) ** (-1 / 3)
        phi0 = rng.uniform(0, 2 * math.pi, n_photons)
        v = np.stack([np.cos(phi0), np.sin(phi0)], 1)
        tex = np.full(n_photons, np.inf)
        for k, o_ in ((0, x0), (1, y0)):
            pos, neg = v[:, k] > 0, v[:, k] < 0
            tex[pos] = np.minimum(tex[pos], (half - o_) / v[pos, k])
            tex[neg] = np.minimum(tex[neg], (-half - o_) / v[neg, k])
        r = rng.exponential(1.0, n_photons) / muw
        hit = r < tex
        x = x0 + r[hit] * v[hit, 0]
        y = y0 + r[hit] * v[hit, 1]
        cphi = v[hit] @ na_
        Ep = Ew / (1 + Ew / ME * (1 - cphi))
        # path to the detector along n_a inside the square
        tout = np.full(x.size, np.inf)
        for k, o_ in ((0, x), (1, y)):
            if na_[k] > 0:
                tout = np.minimum(tout, (half - o_) / na_[k])
            elif na_[k] < 0:
                tout = np.minimum(tout, (-half - o_) / na_[k])
        att = np.exp(-mu0 * (Ep / 85.0) ** (-1 / 3) * tout)
        u = -x * na_[1] + y * na_[0]
        depth = p.R - (x * na_[0] + y * na_[1])
        sig = (p.fwhm0 + p.fwhm_slope * depth) / FWHM
        D = stats.norm.cdf(p.R, u, sig) - stats.norm.cdf(-p.R, u, sig)
        se = p.eres_frac * p.eres_ref * np.sqrt(Ep / p.eres_ref) / FWHM
        acc = sum(stats.norm.cdf(hi, Ep, se) - stats.norm.cdf(lo, Ep, se) for lo, hi in p.windows)
        wgt = _kn(cphi, Ew) / Z * p.dtheta * att * D * acc
        total += al * wgt.sum() / n_photons
    return total


def test_scatter_model_matches_monte_carlo(oracle_mod):
    half, mu0 = 16.0, 0.02                 # uniform square [-16,16]^2 of water-like mu
    errs = []
    for n, pix, ns in [(16, 4.0, 8), (32, 2.0, 16), (64, 1.0, 32)]:
        p = synth.SysParams(n=n, pix=pix, ns=ns, nb=16, na=8)
        mu = np.zeros((n, n))
        k = int(round((p.R - half) / pix))
        mu[k:n - k, k:n - k] = mu0
        o = oracle_mod.Oracle(p, mu.ravel())
        # source pixel: the one whose centre is nearest (-6, 3) mm
        ix = int(np.floor((-6.0 + p.R) / pix))
        iy = int(np.floor((3.0 + p.R) / pix))
        q = iy * n + ix
        x0, y0 = o.pixel_centre(q)
        for a in (1, 4):
            prim = sum(o.Pp(q, a, w) * o.psf_total(x0, y0, a) * o.acc(Ew)
                       for w, Ew in enumerate(p.lines))
            model = o.sens_qa(q, a) - prim
            mc = _mc_scatter(p, mu0, half, x0, y0, a, 400000, seed=100 + n + a)
            errs.append((n, a, model / mc - 1.0))
    by_n = {}
    for n, a, e in errs:
        by_n.setdefault(n, []).append(abs(e))
    coarse, mid, fine = (np.mean(by_n[k]) for k in (16, 32, 64))
    # grid quadrature of a 1/r-weighted integrand converges to the histories
    assert fine < mid < coarse
    assert coarse > 2 * fine
    assert fine < 0.05, errs
