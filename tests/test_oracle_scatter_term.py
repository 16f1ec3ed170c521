"""Pins of the oracle's once-scattered path term (Eq. (5) read in the plane), of
its scattered row part and of its backprojection, each against arithmetic
written out here independently of the oracle's C code.

- One (pixel, scatter point, angle, line) term of Eq. (5) against a
  transcription in Python's math module: emission into the cell's planar solid
  angle h_s^2/(2 pi r), interaction with mu(E_w), attenuation to the point at
  E_w, the planar Klein-Nishina density normalised by adaptive quadrature
  (scipy), the collimator acceptance, and attenuation from the point to the
  detector at the scattered energy E' = E_w P(phi).  On a uniform square the
  two attenuation integrals are analytic chords, so the pin does not lean on
  the oracle's line integrals at all; on a random map it takes them from the
  oracle's tables, which the line-integral pins fix.  Slips this catches: the
  exit leg attenuated at E_w instead of E' (1-2 % of the scattered flux), a
  missing or squared f_w, a Klein-Nishina density unnormalised or taken at E',
  the wrong cell's mu_s, 1/r^2 for 1/r, the angle's sign.
- The scattered part of a row (or_event_row_scatter) against the sum of the
  hand terms times the collimator response of the scatter point and the
  energy Gaussian at E' (scipy's normal CDF and PDF); the full row minus that
  part against the unscattered closed form (Eq. (3)-(5) with n = 0).
- The backprojection (the sum over events that Algorithm 1 accumulates for
  the numerator of Eq. (18)) against the explicit sum of weighted rows, and
  the adjoint identity <A lambda, w> = <lambda, A^T w>.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import synth

ME = 510.99895
FWHM = 2 * math.sqrt(2 * math.log(2))


def _f(p, E):
    """mu(E) / mu(85 keV) (the power law of the system parameters)."""
    return (E / p.mu_ref) ** (-p.mu_pow)


def _dir(a, na):
    if (4 * a) % na == 0:
        return [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][(4 * a // na) % 4]
    th = 2 * math.pi * a / na
    return math.cos(th), math.sin(th)


def _kn(cosphi, E):
    P = 1.0 / (1.0 + E / ME * (1.0 - cosphi))
    return P * P * (P + 1.0 / P - (1.0 - cosphi * cosphi))


_ZCACHE = {}


def _Z(E):
    if E not in _ZCACHE:
        _ZCACHE[E] = integrate.quad(lambda f: _kn(math.cos(f), E), 0.0, 2 * math.pi,
                                    epsabs=0, epsrel=1e-13, limit=200)[0]
    return _ZCACHE[E]


def _hand_Ps(p, xq, yq, xs, ys, mu_s, a, w, g_qs, g_sa):
    """The once-scattered path weight pixel -> point -> detector (planar Eq. (5))."""
    c, s = _dir(a, p.na)
    hs = p.fov / p.ns
    dx, dy = xs - xq, ys - yq
    r = math.hypot(dx, dy)
    reff = max(r, hs / (2 * math.sqrt(math.pi)))
    cosphi = (dx * c + dy * s) / r
    Ew, al = p.lines[w], p.yields[w]
    Ep = Ew / (1.0 + Ew / ME * (1.0 - cosphi))
    pkn = _kn(cosphi, Ew) / _Z(Ew)
    fw, fp = _f(p, Ew), _f(p, Ep)
    v = (al * hs * hs / (2 * math.pi * reff) * mu_s * fw * math.exp(-fw * g_qs)
         * pkn * p.dtheta * math.exp(-fp * g_sa))
    return v, Ep


def _chord_square(x0, y0, dx, dy, half):
    ts = []
    for d, o in ((dx, x0), (dy, y0)):
        if d > 0:
            ts.append((half - o) / d)
        elif d < 0:
            ts.append((-half - o) / d)
    return min(ts)


def _cells(p, mu):
    """Scatter cells in the oracle's order (row-major over the coarse grid,
    kept when inside the field of view with positive mean attenuation):
    centre and mean attenuation of the covered pixels."""
    n, m = p.n, p.n // p.ns
    hs = p.fov / p.ns
    mu = np.asarray(mu, float).reshape(n, n)
    out = []
    for ky in range(p.ns):
        for kx in range(p.ns):
            x, y = (kx + 0.5) * hs - p.R, (ky + 0.5) * hs - p.R
            ms = mu[ky * m:(ky + 1) * m, kx * m:(kx + 1) * m].mean()
            if x * x + y * y <= p.R * p.R and ms > 0:
                out.append((x, y, ms))
    return out


def _centre(p, q):
    return ((q % p.n) + 0.5) * p.pix - p.R, ((q // p.n) + 0.5) * p.pix - p.R


def _psf_bin(p, b, x, y, a):
    c, s = _dir(a, p.na)
    u, depth = -x * s + y * c, p.R - (x * c + y * s)
    sig = (p.fwhm0 + p.fwhm_slope * depth) / FWHM
    db = p.fov / p.nb
    lo = -p.R + b * db
    if lo > u:       # the tail side that does not cancel
        return stats.norm.sf(lo, u, sig) - stats.norm.sf(lo + db, u, sig)
    return stats.norm.cdf(lo + db, u, sig) - stats.norm.cdf(lo, u, sig)


def _gE(p, Ehat, E):
    return stats.norm.pdf(Ehat, E, p.eres_frac * p.eres_ref * math.sqrt(E / p.eres_ref) / FWHM)


def test_scatter_term_uniform_square_analytic_chords(oracle_mod):
    p = synth.SysParams(n=16, pix=4.0, ns=8, nb=16, na=16)
    half, mu0 = 16.0, 0.02
    mu = np.zeros((p.n, p.n))
    k = int(round((p.R - half) / p.pix))
    mu[k:p.n - k, k:p.n - k] = mu0
    o = oracle_mod.Oracle(p, mu.ravel())
    cells = _cells(p, mu)
    pts, smu = o.scatter_points()
    assert o.nsc == len(cells) == 16
    np.testing.assert_array_equal(pts, np.array([(x, y) for x, y, _ in cells]))
    np.testing.assert_array_equal(smu, np.array([m for _, _, m in cells]))
    rng = np.random.default_rng(71)
    inside = [q for q in range(p.n * p.n)
              if abs(_centre(p, q)[0]) < half and abs(_centre(p, q)[1]) < half]
    checked = 0
    for _ in range(120):
        q = int(rng.choice(inside))
        si = int(rng.integers(0, o.nsc))
        a = int(rng.integers(0, p.na))
        w = int(rng.integers(0, len(p.lines)))
        xq, yq = _centre(p, q)
        xs, ys, ms = cells[si]
        c, s = _dir(a, p.na)
        g_qs = mu0 * math.hypot(xs - xq, ys - yq)            # both inside the square
        g_sa = mu0 * _chord_square(xs, ys, c, s, half)
        ref, Ep_ref = _hand_Ps(p, xq, yq, xs, ys, ms, a, w, g_qs, g_sa)
        got, Ep = o.Ps(q, si, a, w)
        assert Ep == pytest.approx(Ep_ref, rel=1e-14)
        assert got == pytest.approx(ref, rel=1e-11), (q, si, a, w)
        checked += 1
    assert checked == 120


def test_scatter_term_random_map_every_line(oracle_mod):
    p = synth.SysParams(n=16, pix=4.0, ns=8, nb=16, na=12)
    rng = np.random.default_rng(72)
    mu = rng.uniform(0.005, 0.03, p.n * p.n) * synth.fov_support(p)
    o = oracle_mod.Oracle(p, mu)
    cells = _cells(p, mu)
    assert o.nsc == len(cells)
    _, g_qs_t, g_sa_t = o.tables()
    sup = np.flatnonzero(o.support)
    for _ in range(60):
        q = int(rng.choice(sup))
        si = int(rng.integers(0, o.nsc))
        a = int(rng.integers(0, p.na))
        xq, yq = _centre(p, q)
        xs, ys, ms = cells[si]
        for w in range(len(p.lines)):
            ref, Ep_ref = _hand_Ps(p, xq, yq, xs, ys, ms, a, w, g_qs_t[q, si], g_sa_t[a, si])
            got, Ep = o.Ps(q, si, a, w)
            assert Ep == pytest.approx(Ep_ref, rel=1e-14)
            assert got == pytest.approx(ref, rel=1e-11), (q, si, a, w)


def test_scattered_row_and_unscattered_remainder(oracle_mod):
    p = synth.SysParams(n=8, pix=4.0, ns=4, nb=8, na=8, windows=(synth.EW1, synth.EW2, synth.EW3))
    rng = np.random.default_rng(73)
    mu = rng.uniform(0.01, 0.03, p.n * p.n) * synth.fov_support(p)
    o = oracle_mod.Oracle(p, mu)
    cells = _cells(p, mu)
    g_qa_t, g_qs_t, g_sa_t = o.tables()
    sup = np.flatnonzero(o.support)
    for b, a, Eh in [(3, 1, 80.0), (5, 2, 150.0), (2, 5, 270.0), (4, 0, 95.0), (0, 6, 130.0)]:
        rs = o.row_scatter(b, a, Eh)
        rf = o.row(b, a, Eh)
        for q in sup:
            xq, yq = _centre(p, q)
            acc = 0.0
            for w in range(len(p.lines)):
                for si, (xs, ys, ms) in enumerate(cells):
                    v, Ep = _hand_Ps(p, xq, yq, xs, ys, ms, a, w, g_qs_t[q, si], g_sa_t[a, si])
                    acc += v * _psf_bin(p, b, xs, ys, a) * _gE(p, Eh, Ep)
            assert rs[q] == pytest.approx(acc, rel=1e-9, abs=1e-300), (b, a, Eh, q)
            prim = sum(al * p.dtheta / (2 * math.pi) * math.exp(-_f(p, Ew) * g_qa_t[a, q])
                       * _psf_bin(p, b, xq, yq, a) * _gE(p, Eh, Ew)
                       for Ew, al in zip(p.lines, p.yields))
            assert rf[q] - rs[q] == pytest.approx(prim, rel=1e-9, abs=1e-12 * rf[q]), q
        off = np.flatnonzero(~o.support)
        assert np.all(rs[off] == 0) and np.all(rf[off] == 0)


def _events(p, rng, n):
    return {"bin": rng.integers(0, p.nb, n).astype(np.int32),
            "angle": rng.integers(0, p.na, n).astype(np.int32),
            "energy": np.concatenate([rng.uniform(*p.windows[k % len(p.windows)], 1)
                                      for k in range(n)])}


def test_backprojection_is_weighted_row_sum_and_adjoint(oracle_mod):
    p = synth.SysParams(n=8, pix=4.0, ns=4, nb=8, na=8)
    rng = np.random.default_rng(74)
    mu = rng.uniform(0.01, 0.03, p.n * p.n) * synth.fov_support(p)
    o = oracle_mod.Oracle(p, mu)
    ev = _events(p, rng, 40)
    wj = rng.normal(0.0, 1.0, 40)
    wj[::7] = 0.0                      # events with zero weight contribute nothing
    lam = rng.uniform(0.2, 2.0, p.n * p.n) * o.support
    bp = o.backproject(ev, wj)
    rows = np.array([o.row(b, a, E) for b, a, E in zip(ev["bin"], ev["angle"], ev["energy"])])
    ref = (rows * wj[:, None]).sum(0)
    np.testing.assert_allclose(bp, ref, rtol=1e-12, atol=1e-15 * np.abs(ref).max())
    fwd = o.forward(ev, lam)
    np.testing.assert_allclose(fwd, rows @ lam, rtol=1e-12)
    lhs, rhs = float(fwd @ wj), float(lam @ bp)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # a single event: the backprojection is that event's row times its weight
    one = {k: v[3:4] for k, v in ev.items()}
    np.testing.assert_allclose(o.backproject(one, np.array([2.5])), 2.5 * rows[3], rtol=1e-13)
