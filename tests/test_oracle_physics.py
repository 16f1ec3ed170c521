"""Pins of the oracle's physics and geometry primitives.

Each check compares the oracle with something other than itself: a closed form,
a textbook limit, an independent library routine (scipy) or brute force.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import synth

ME = 510.99895


def test_kn_thomson_limit(oracle_mod):
    # As E -> 0 the Klein-Nishina weight tends to 1 + cos^2(phi), whose
    # integral over the full circle is 3 pi.
    assert oracle_mod.kn_Z(1e-6) == pytest.approx(3 * math.pi, rel=1e-8)
    for phi in np.linspace(0, 2 * np.pi, 17):
        assert oracle_mod.kn_K(np.cos(phi), 1e-9) == pytest.approx(1 + np.cos(phi) ** 2, rel=1e-9)


@pytest.mark.parametrize("E", [85.0, 154.0, 270.0])
def test_kn_normalised_by_adaptive_quadrature(oracle_mod, E):
    Z = oracle_mod.kn_Z(E)
    val, err = integrate.quad(lambda p: oracle_mod.kn_K(np.cos(p), E), 0, 2 * np.pi,
                              epsabs=1e-13, epsrel=1e-13, limit=200)
    assert Z == pytest.approx(val, rel=1e-11)


@pytest.mark.parametrize("E", [85.0, 154.0, 270.0, 1000.0])
def test_kn_forward_and_backward_limits(oracle_mod, E):
    # Forward scattering keeps the energy (P = 1) and K = P^2 (P + 1/P) = 2;
    # backscatter at the Compton edge P = 1/(1 + 2E/mc^2).
    assert oracle_mod.kn_K(1.0, E) == pytest.approx(2.0, rel=1e-14)
    P = 1.0 / (1.0 + 2.0 * E / ME)
    assert oracle_mod.kn_K(-1.0, E) == pytest.approx(P * P * (P + 1 / P), rel=1e-13)


def test_kn_regression_values(oracle_mod):
    # Values of the 2-D normaliser at the three lines, computed once by
    # adaptive quadrature (test above) and kept to catch regressions.
    for E, Z in [(85.0, 7.308724), (154.0, 6.389732), (270.0, 5.466138)]:
        assert oracle_mod.kn_Z(E) == pytest.approx(Z, abs=2e-6)


def _sysp(**kw):
    base = dict(n=16, pix=4.0, ns=8, nb=16, na=32)
    base.update(kw)
    return synth.SysParams(**base)


def test_energy_resolution_and_acceptance(oracle_mod):
    p = _sysp()
    o = oracle_mod.Oracle(p, np.zeros(p.n * p.n))
    # 10% FWHM at 140 keV (Sec. 3.1.2); FWHM / sigma = 2 sqrt(2 ln 2).
    assert o.sigmaE(140.0) * 2 * math.sqrt(2 * math.log(2)) == pytest.approx(14.0, rel=1e-14)
    assert o.sigmaE(140.0) == pytest.approx(5.945, abs=1e-3)
    # absolute FWHM grows as sqrt(E): relative FWHM falls as 1/sqrt(E)
    assert o.sigmaE(4 * 85.0) / o.sigmaE(85.0) == pytest.approx(2.0, rel=1e-14)
    # window acceptance = sum of normal CDF differences (scipy)
    for E in [70.0, 85.0, 110.0, 154.0, 200.0, 270.0]:
        s = o.sigmaE(E)
        ref = sum(stats.norm.cdf(hi, E, s) - stats.norm.cdf(lo, E, s) for lo, hi in p.windows)
        assert o.acc(E) == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_attenuation_power_law(oracle_mod):
    p = _sysp()
    o = oracle_mod.Oracle(p, np.zeros(p.n * p.n))
    assert o.mu_scale(85.0) == 1.0
    assert o.mu_scale(170.0) == pytest.approx(2 ** (-1 / 3), rel=1e-14)


def test_phi_diff_matches_scipy(oracle_mod):
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b = sorted(rng.normal(0, 6, 2))
        ref = special.ndtr(b) - special.ndtr(a)
        if a > 0:
            ref = special.ndtr(-a) - special.ndtr(-b)
        assert oracle_mod.Phi_diff(b, a) == pytest.approx(ref, rel=1e-12, abs=1e-300)


def _clip_chord(x0, y0, x1, y1, lo, hi):
    """Length of the part of a segment inside the square [lo,hi]^2
    (Liang-Barsky parametric clipping)."""
    dx, dy = x1 - x0, y1 - y0
    t0, t1 = 0.0, 1.0
    for p_, q_ in ((-dx, x0 - lo), (dx, hi - x0), (-dy, y0 - lo), (dy, hi - y0)):
        if p_ == 0:
            if q_ < 0:
                return 0.0
            continue
        t = q_ / p_
        if p_ < 0:
            t0 = max(t0, t)
        else:
            t1 = min(t1, t)
    return max(0.0, t1 - t0) * math.hypot(dx, dy)


def test_segment_integral_uniform_square_closed_form(oracle_mod):
    n, pix = 16, 4.0
    R = n * pix / 2
    mu = np.zeros((n, n))
    mu[4:12, 4:12] = 0.02                      # square [-16, 16]^2
    rng = np.random.default_rng(1)
    for _ in range(300):
        x0, y0, x1, y1 = rng.uniform(-R * 1.2, R * 1.2, 4)
        v = oracle_mod.segment_integral(mu, n, pix, x0, y0, x1, y1)
        assert v == pytest.approx(0.02 * _clip_chord(x0, y0, x1, y1, -16, 16), rel=1e-11, abs=1e-13)


def test_segment_integral_brute_force(oracle_mod):
    n, pix = 8, 3.0
    R = n * pix / 2
    rng = np.random.default_rng(2)
    mu = rng.uniform(0, 0.05, (n, n))

    def mu_at(x, y):
        ix = np.floor((x + R) / pix).astype(int)
        iy = np.floor((y + R) / pix).astype(int)
        ok = (ix >= 0) & (iy >= 0) & (ix < n) & (iy < n)
        out = np.zeros_like(x)
        out[ok] = mu[iy[ok], ix[ok]]
        return out

    for _ in range(40):
        x0, y0, x1, y1 = rng.uniform(-R * 1.1, R * 1.1, 4)
        L = math.hypot(x1 - x0, y1 - y0)
        N = 200000
        t = (np.arange(N) + 0.5) / N
        brute = mu_at(x0 + t * (x1 - x0), y0 + t * (y1 - y0)).sum() * L / N
        v = oracle_mod.segment_integral(mu, n, pix, x0, y0, x1, y1)
        # midpoint sampling misplaces at most one sample per grid crossing
        bound = 2 * (2 * n + 2) * mu.max() * L / N
        assert abs(v - brute) <= bound


def test_segment_on_grid_line_takes_mean_of_neighbours(oracle_mod):
    n, pix = 8, 2.0
    R = n * pix / 2
    rng = np.random.default_rng(3)
    mu = rng.uniform(0, 0.05, (n, n))
    # vertical segment on the grid line between columns 2 and 3
    x = -R + 3 * pix
    v = oracle_mod.segment_integral(mu, n, pix, x, -R - 1, x, R + 1)
    assert v == pytest.approx(0.5 * pix * (mu[:, 2].sum() + mu[:, 3].sum()), rel=1e-12)
    # the same value is the limit of segments displaced to either side
    d = 1e-7
    lim = 0.5 * (oracle_mod.segment_integral(mu, n, pix, x - d, -R - 1, x - d, R + 1)
                 + oracle_mod.segment_integral(mu, n, pix, x + d, -R - 1, x + d, R + 1))
    assert v == pytest.approx(lim, rel=1e-10)
    # horizontal
    y = -R + 5 * pix
    v = oracle_mod.segment_integral(mu, n, pix, R + 1, y, -R - 1, y)
    assert v == pytest.approx(0.5 * pix * (mu[4, :].sum() + mu[5, :].sum()), rel=1e-12)


def test_angle_directions_exact_on_axes(oracle_mod):
    for na in (4, 32, 120):
        for a in range(na):
            c, s = oracle_mod.angle_dir(a, na)
            th = 2 * math.pi * a / na
            assert c == pytest.approx(math.cos(th), abs=1e-15)
            assert s == pytest.approx(math.sin(th), abs=1e-15)
            if (4 * a) % na == 0:
                assert {abs(c), abs(s)} == {0.0, 1.0}


def test_psf_bins_sum_to_detector_probability(oracle_mod):
    p = _sysp()
    o = oracle_mod.Oracle(p, np.zeros(p.n * p.n))
    rng = np.random.default_rng(4)
    for _ in range(50):
        x, y = rng.uniform(-20, 20, 2)
        a = int(rng.integers(0, p.na))
        tot = sum(o.psf_bin(b, x, y, a) for b in range(p.nb))
        assert tot == pytest.approx(o.psf_total(x, y, a), rel=1e-12)
        # against scipy for the depth-dependent Gaussian
        c, s = oracle_mod.angle_dir(a, p.na)
        u, depth = -x * s + y * c, p.R - (x * c + y * s)
        sig = (p.fwhm0 + p.fwhm_slope * depth) / (2 * math.sqrt(2 * math.log(2)))
        b = int(np.floor((u + p.R) / (p.fov / p.nb)))
        lo = -p.R + b * p.fov / p.nb
        ref = stats.norm.cdf(lo + p.fov / p.nb, u, sig) - stats.norm.cdf(lo, u, sig)
        assert o.psf_bin(b, x, y, a) == pytest.approx(ref, rel=1e-10)
    # deep inside a wide detector almost every photon lands on it
    assert o.psf_total(0.0, 0.0, 0) == pytest.approx(1.0, abs=1e-12)
