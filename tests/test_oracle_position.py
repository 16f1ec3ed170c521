"""Pins of the oracle's continuous position attribute (events that carry the
lateral position u in mm instead of a detector bin).

- the density row integrated over a bin is the bin row, for bins at the
  centre and at both edges of the detector (composite Gauss-Legendre
  quadrature in u, so the density is pinned to the bin probabilities that
  the model tests pin to scipy);
- without attenuation the density's unscattered part is the parallel
  projection blurred by the depth-dependent Gaussian, from scipy's pdf;
- one OSEM pass over position events equals the update of Eq. (18) written
  out in numpy from the oracle's density rows (pins the event indexing of the
  list calls);
- positions outside [-R, R) and non-finite ones are rejected.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth

FWHM = 2 * math.sqrt(2 * math.log(2))


def _p(**kw):
    base = dict(n=8, pix=4.0, ns=4, nb=8, na=8)
    base.update(kw)
    return synth.SysParams(**base)


def _disk(p, mu=0.015):
    c = (np.arange(p.n) + 0.5) * p.pix - p.R
    x, y = np.meshgrid(c, c)
    return np.where(x * x + y * y <= (0.8 * p.R) ** 2, mu, 0.0).ravel()


def _bin_integral(o, lo, hi, a, E, pieces=16, nodes=10):
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    acc = np.zeros(o.Q)
    edges = np.linspace(lo, hi, pieces + 1)
    for u0, u1 in zip(edges[:-1], edges[1:]):
        h = 0.5 * (u1 - u0)
        for xk, wk in zip(xg, wg):
            acc += wk * h * o.row_pos(u0 + h * (xk + 1.0), a, E)
    return acc


@pytest.mark.parametrize("b,a,E", [(3, 1, 84.0), (0, 5, 150.0), (7, 2, 95.5), (4, 7, 130.0)])
def test_density_integrates_to_bin_row(oracle_mod, b, a, E):
    p = _p()
    o = oracle_mod.Oracle(p, _disk(p))
    assert o.nsc > 0
    db = p.fov / p.nb
    lo = -p.R + b * db
    got = _bin_integral(o, lo, lo + db, a, E)
    ref = o.row(b, a, E)
    assert np.abs(ref).max() > 0
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_density_closed_form_without_attenuation(oracle_mod):
    p = _p(n=16, ns=8, nb=16, na=12)
    o = oracle_mod.Oracle(p, np.zeros(p.n * p.n))
    assert o.nsc == 0
    rng = np.random.default_rng(7)
    for _ in range(6):
        a = int(rng.integers(0, p.na))
        u = float(rng.uniform(-p.R, p.R))
        E = float(rng.uniform(*p.windows[int(rng.integers(0, 2))]))
        row = o.row_pos(u, a, E)
        th = 2 * math.pi * a / p.na
        for q in np.flatnonzero(o.support)[::5]:
            x, y = o.pixel_centre(q)
            u0 = -x * math.sin(th) + y * math.cos(th)
            depth = p.R - (x * math.cos(th) + y * math.sin(th))
            sig = (p.fwhm0 + p.fwhm_slope * depth) / FWHM
            ref = sum(al * p.dtheta / (2 * math.pi) * stats.norm.pdf(u, u0, sig) *
                      stats.norm.pdf(E, Ew, p.eres_frac * p.eres_ref * math.sqrt(Ew / p.eres_ref) / FWHM)
                      for Ew, al in zip(p.lines, p.yields))
            assert row[q] == pytest.approx(ref, rel=1e-9, abs=1e-300)


def test_position_osem_is_eq18_on_density_rows(oracle_mod):
    p = _p()
    o = oracle_mod.Oracle(p, _disk(p))
    lam_true = o.support * (1.0 + np.arange(o.Q) % 3)
    ev = o.sample_events(lam_true, 40, seed=3)
    pe = {"position": ev["position"], "angle": ev["angle"], "energy": ev["energy"]}
    nsub = 2
    sens = o.sensitivity(nsub)
    lam0 = o.support.astype(np.float64)
    got, _, _, _ = o.osem(pe, nsub, 1, lam0, sens)
    lam = lam0.copy()
    for s in range(nsub):
        js = [j for j in range(len(pe["angle"])) if pe["angle"][j] % nsub == s]
        B = np.zeros(o.Q)
        for j in js:
            r = o.row_pos(pe["position"][j], pe["angle"][j], pe["energy"][j])
            pj = r @ lam
            if pj > 0:
                B += r / pj
        d = sens[s]
        lam = np.where(d > 0, lam * B / np.where(d > 0, d, 1.0), lam)
    assert np.allclose(got, lam, rtol=1e-12, atol=0)
    # the binned events of the same photons give a different image
    binned, _, _, _ = o.osem({k: ev[k] for k in ("bin", "angle", "energy")}, nsub, 1, lam0, sens)
    assert not np.allclose(binned, got, rtol=1e-6)
    fwd = o.forward(pe, lam0)
    for j in (0, 7, 39):
        assert fwd[j] == pytest.approx(o.row_pos(pe["position"][j], pe["angle"][j],
                                                 pe["energy"][j]) @ lam0, rel=1e-13)


def test_position_checks_and_sampler(oracle_mod):
    p = _p()
    o = oracle_mod.Oracle(p, _disk(p))
    ev = o.sample_events(o.support.astype(float), 200, seed=11)
    u = ev["position"]
    assert np.all((u >= -p.R) & (u < p.R))
    db = p.fov / p.nb
    assert np.array_equal(np.minimum(np.floor((u + p.R) / db), p.nb - 1).astype(int), ev["bin"])
    pe = {"position": u.copy(), "angle": ev["angle"], "energy": ev["energy"]}
    assert o.check_events(pe) == -1
    for bad in (p.R, -p.R - 1e-9, np.nan, np.inf):
        q = dict(pe, position=u.copy())
        q["position"][5] = bad
        assert o.check_events(q) == 5, bad
    q = dict(pe, position=u.copy())
    q["position"][9] = -p.R
    assert o.check_events(q) == -1
