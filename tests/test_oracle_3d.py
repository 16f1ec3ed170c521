"""Pins of the oracle's 3-D single-scatter model.

- the Klein-Nishina normaliser over the sphere equals the closed-form total
  cross-section (textbook formula), with the Thomson limit 16 pi / 3;
- 3-D line integrals: exact chords through a uniform box (slab clipping),
  brute-force midpoint quadrature within its error bound on a random map,
  the grid-plane tie rule as the limit of displaced segments, and a segment
  inside one slice equal to the planar oracle's integral on that slice;
- mu = 0: the unscattered row is the parallel projection blurred by the
  depth-dependent Gaussian in u and v (scipy);
- a uniform box: the unscattered path's attenuation is exp(-mu chord);
- the per-event density integrates over both bin indices and the window
  energies to the sensitivity, for every voxel;
- rotating the object by 90 degrees about z with the angle, and mirroring it
  in z with the axial bin, leave the model unchanged;
- a photon-history Monte Carlo (isotropic emission in 3-D, free paths in a
  uniform cube, Klein-Nishina scattering into the collimator's solid angle,
  forced detection) agrees with the scatter-point sum, the disagreement
  shrinking as the scatter grid is refined;
- OSEM on 3-D rows conserves counts per subset.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth

ME = 510.99895
FWHM = 2 * math.sqrt(2 * math.log(2))


def _p(**kw):
    base = dict(n=8, pix=4.0, ns=4, nb=8, na=8, nz=4, nsz=2, nbz=4)
    base.update(kw)
    return synth.SysParams(**base)


def _vox(p):
    return synth.voxel_centres(p)


def _box_map(p, half, mu0, halfz=None):
    x, y, z = _vox(p)
    hz = half if halfz is None else halfz
    inside = (np.abs(x) < half) & (np.abs(y) < half) & (np.abs(z) < hz)
    return np.where(inside, mu0, 0.0)


def _chord(o, d, lo, hi):
    """Length of the part of segment o + t d, t in [0, 1], inside the box [lo, hi]."""
    t0, t1 = 0.0, 1.0
    for k in range(3):
        if d[k] == 0.0:
            if not (lo[k] < o[k] < hi[k]):
                return 0.0
            continue
        a, b = (lo[k] - o[k]) / d[k], (hi[k] - o[k]) / d[k]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return max(0.0, t1 - t0) * float(np.linalg.norm(d))


def test_kn_normaliser_matches_total_cross_section(oracle_mod):
    for E in (1e-6, 85.0, 154.0, 270.0, 511.0):
        k = E / ME
        lg = math.log1p(2 * k)
        sig = ((1 + k) / k ** 2 * (2 * (1 + k) / (1 + 2 * k) - lg / k) + lg / (2 * k)
               - (1 + 3 * k) / (1 + 2 * k) ** 2)
        ref = 4 * math.pi * sig          # integral of K over the sphere = 2 sigma / r_e^2
        if E < 1.0:                       # the closed form cancels at tiny k: Thomson limit
            ref = 16 * math.pi / 3
        assert oracle_mod.kn_Z3(E) == pytest.approx(ref, rel=1e-6 if E < 1.0 else 1e-12)


def test_segment_integral_3d(oracle_mod):
    rng = np.random.default_rng(3)
    n, nz, pix = 8, 6, 3.0
    R, Zh = n * pix / 2, nz * pix / 2
    p = synth.SysParams(n=n, pix=pix, ns=4, nb=8, na=8, nz=nz, nsz=2, nbz=4)
    # exact chords through a uniform box aligned with the grid
    mu = _box_map(p, 6.0, 0.02, halfz=6.0)           # box edges on voxel boundaries
    for _ in range(40):
        a = rng.uniform([-R, -R, -Zh], [R, R, Zh])
        b = rng.uniform([-R, -R, -Zh], [R, R, Zh])
        got = oracle_mod.segment_integral3(mu, n, nz, pix, *a, *b)
        ref = 0.02 * _chord(a, b - a, [-6, -6, -6], [6, 6, 6])
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-13)
    # random map: midpoint quadrature with its error bound
    mu = rng.uniform(0, 0.03, n * n * nz)
    for _ in range(6):
        a = rng.uniform([-R, -R, -Zh], [R, R, Zh])
        b = rng.uniform([-R, -R, -Zh], [R, R, Zh])
        got = oracle_mod.segment_integral3(mu, n, nz, pix, *a, *b)
        m = 200000
        t = (np.arange(m) + 0.5) / m
        pts = a[None, :] + t[:, None] * (b - a)[None, :]
        ix = np.clip(np.floor((pts[:, 0] + R) / pix).astype(int), 0, n - 1)
        iy = np.clip(np.floor((pts[:, 1] + R) / pix).astype(int), 0, n - 1)
        iz = np.clip(np.floor((pts[:, 2] + Zh) / pix).astype(int), 0, nz - 1)
        L = float(np.linalg.norm(b - a))
        ref = mu[(iz * n + iy) * n + ix].mean() * L
        crossings = 2 * n + nz + 3
        assert abs(got - ref) <= crossings * 0.03 * L / m * 2 + 1e-12
    # a segment in a grid plane sees the mean of the two sides
    zb = -Zh + 2 * pix
    for _ in range(5):
        a = rng.uniform([-R, -R], [R, R])
        b = rng.uniform([-R, -R], [R, R])
        tie = oracle_mod.segment_integral3(mu, n, nz, pix, a[0], a[1], zb, b[0], b[1], zb)
        lo = oracle_mod.segment_integral3(mu, n, nz, pix, a[0], a[1], zb - 1e-7, b[0], b[1],
                                          zb - 1e-7)
        hi = oracle_mod.segment_integral3(mu, n, nz, pix, a[0], a[1], zb + 1e-7, b[0], b[1],
                                          zb + 1e-7)
        assert tie == pytest.approx(0.5 * (lo + hi), rel=1e-12)
    # inside one slice: the planar oracle on that slice's map
    for k in (0, 3, 5):
        zk = -Zh + (k + 0.5) * pix
        sl = mu.reshape(nz, n * n)[k]
        for _ in range(4):
            a = rng.uniform([-R, -R], [R, R])
            b = rng.uniform([-R, -R], [R, R])
            got = oracle_mod.segment_integral3(mu, n, nz, pix, a[0], a[1], zk, b[0], b[1], zk)
            ref = oracle_mod.segment_integral(sl, n, pix, a[0], a[1], b[0], b[1])
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-15)


def _bin_prob(lo, hi, mean, sig):
    """Normal probability of [lo, hi), on the side of the tail that does not cancel."""
    if lo > mean:
        return stats.norm.sf(lo, mean, sig) - stats.norm.sf(hi, mean, sig)
    return stats.norm.cdf(hi, mean, sig) - stats.norm.cdf(lo, mean, sig)


def test_primary_closed_form_without_attenuation_3d(oracle_mod):
    p = _p(n=12, ns=6, nb=12, na=12, nz=6, nsz=3, nbz=6)
    o = oracle_mod.Oracle3(p, np.zeros(p.n * p.n * p.nz))
    assert o.nsc == 0
    rng = np.random.default_rng(5)
    db, dbz = p.fov / p.nb, 2 * p.Zh / p.nbz
    for _ in range(5):
        b, bz, a = int(rng.integers(0, p.nb)), int(rng.integers(0, p.nbz)), int(rng.integers(0, p.na))
        E = float(rng.uniform(*p.windows[int(rng.integers(0, 2))]))
        row = o.row(b, bz, a, E)
        th = 2 * math.pi * a / p.na
        for q in np.flatnonzero(o.support)[::11]:
            x, y, z = o.voxel_centre(q)
            u = -x * math.sin(th) + y * math.cos(th)
            depth = p.R - (x * math.cos(th) + y * math.sin(th))
            sig = (p.fwhm0 + p.fwhm_slope * depth) / FWHM
            lo, lz = -p.R + b * db, -p.Zh + bz * dbz
            pu = _bin_prob(lo, lo + db, u, sig)
            pv = _bin_prob(lz, lz + dbz, z, sig)
            ref = sum(al * p.domega / (4 * math.pi) * pu * pv *
                      stats.norm.pdf(E, Ew, p.eres_frac * p.eres_ref * math.sqrt(Ew / p.eres_ref) / FWHM)
                      for Ew, al in zip(p.lines, p.yields))
            assert row[q] == pytest.approx(ref, rel=1e-8, abs=1e-300)


def test_attenuated_primary_uniform_box_3d(oracle_mod):
    p = _p(n=10, ns=5, nb=10, na=12, nz=6, nsz=3, nbz=6)
    mu0 = 0.015
    o = oracle_mod.Oracle3(p, _box_map(p, 12.0, mu0, halfz=8.0))
    for q in np.flatnonzero(o.support)[::13]:
        x, y, z = o.voxel_centre(q)
        for a in (0, 1, 5, 9):
            th = 2 * math.pi * a / p.na
            c, s = math.cos(th), math.sin(th)
            if (4 * a) % p.na == 0:
                c, s = round(c), round(s)
            d = p.R - (x * c + y * s)
            L = _chord(np.array([x, y, z]), np.array([d * c, d * s, 0.0]), [-12, -12, -8],
                       [12, 12, 8])
            for w, Ew in enumerate(p.lines):
                f = (Ew / p.mu_ref) ** (-p.mu_pow)
                ref = p.yields[w] * p.domega / (4 * math.pi) * math.exp(-f * mu0 * L)
                assert o.Pp(q, a, w) == pytest.approx(ref, rel=1e-12)


def test_row_integrates_to_sensitivity_3d(oracle_mod):
    p = _p()
    x, y, z = _vox(p)
    mu = np.where(x * x + y * y <= 12.0 ** 2, 0.015, 0.0) * (np.abs(z) < 6.0)
    o = oracle_mod.Oracle3(p, mu)
    assert o.nsc > 0
    xg, wg = np.polynomial.legendre.leggauss(48)
    for a in (1,):
        tot = np.zeros(o.Q)
        for lo, hi in p.windows:
            Es = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
            ws = 0.5 * (hi - lo) * wg
            for E, wE in zip(Es, ws):
                for b in range(p.nb):
                    for bz in range(p.nbz):
                        tot += wE * o.row(b, bz, a, E)
        for q in np.flatnonzero(o.support):
            assert tot[q] == pytest.approx(o.sens_qa(q, a), rel=1e-9)


def test_rotation_and_z_mirror_3d(oracle_mod):
    p = _p(na=8)
    rng = np.random.default_rng(9)
    x, y, z = _vox(p)
    n, nz = p.n, p.nz
    mu = np.where(x * x + y * y <= 14.0 ** 2, rng.uniform(0.005, 0.02, x.size), 0.0)
    o = oracle_mod.Oracle3(p, mu)
    # rotation by +90 degrees about z: voxel (ix, iy) -> (n-1-iy, ix)
    g = mu.reshape(nz, n, n)
    rot = np.zeros_like(g)
    for iy in range(n):
        for ix in range(n):
            rot[:, ix, n - 1 - iy] = g[:, iy, ix]
    o_rot = oracle_mod.Oracle3(p, rot.ravel())
    # z mirror
    o_mir = oracle_mod.Oracle3(p, g[::-1].ravel())
    perm_rot = np.zeros(o.Q, int)
    perm_mir = np.zeros(o.Q, int)
    for iz in range(nz):
        for iy in range(n):
            for ix in range(n):
                q = (iz * n + iy) * n + ix
                perm_rot[q] = (iz * n + ix) * n + (n - 1 - iy)
                perm_mir[q] = ((nz - 1 - iz) * n + iy) * n + ix
    for b, bz, a, E in ((3, 1, 1, 90.0), (5, 2, 2, 140.0), (2, 0, 7, 170.0)):
        r0 = o.row(b, bz, a, E)
        r1 = o_rot.row(b, bz, (a + p.na // 4) % p.na, E)
        assert np.allclose(r1[perm_rot], r0, rtol=1e-10, atol=1e-14 * np.abs(r0).max())
        r2 = o_mir.row(b, p.nbz - 1 - bz, a, E)
        assert np.allclose(r2[perm_mir], r0, rtol=1e-10, atol=1e-14 * np.abs(r0).max())


# ---- Monte Carlo of photon histories in 3-D ---------------------------------

def _kn(cosphi, E):
    P = 1.0 / (1.0 + E / ME * (1.0 - cosphi))
    return P * P * (P + 1.0 / P - (1.0 - cosphi ** 2))


def _mc_scatter3(p, mu0, half, x0, y0, z0, a, n_photons, seed):
    """Expected detected once-scattered photons per decay from (x0,y0,z0) at
    angle a: isotropic emission, exponential free path in the uniform cube
    [-half, half]^3 (attenuation mu0 at 85 keV scaled to each energy), Compton
    scattering into the collimator's solid angle with the Klein-Nishina
    density per steradian (forced detection), attenuation on the way out,
    detector extent in u and v and the energy windows."""
    rng = np.random.default_rng(seed)
    th = 2 * math.pi * a / p.na
    na_ = np.array([math.cos(th), math.sin(th), 0.0])
    total = 0.0
    for Ew, al in zip(p.lines, p.yields):
        k = Ew / ME
        lg = math.log1p(2 * k)
        Z3 = 4 * math.pi * ((1 + k) / k ** 2 * (2 * (1 + k) / (1 + 2 * k) - lg / k)
                            + lg / (2 * k) - (1 + 3 * k) / (1 + 2 * k) ** 2)
        muw = mu0 * (Ew / 85.0) ** (-1 / 3)
        w = rng.uniform(-1, 1, n_photons)
        ph = rng.uniform(0, 2 * math.pi, n_photons)
        st = np.sqrt(1 - w * w)
        v = np.stack([st * np.cos(ph), st * np.sin(ph), w], 1)
        o = np.array([x0, y0, z0])
        tex = np.full(n_photons, np.inf)
        for kk in range(3):
            pos, neg = v[:, kk] > 0, v[:, kk] < 0
            tex[pos] = np.minimum(tex[pos], (half - o[kk]) / v[pos, kk])
            tex[neg] = np.minimum(tex[neg], (-half - o[kk]) / v[neg, kk])
        r = rng.exponential(1.0, n_photons) / muw
        hit = r < tex
        P = o[None, :] + r[hit, None] * v[hit]
        cphi = v[hit] @ na_
        Ep = Ew / (1 + Ew / ME * (1 - cphi))
        tout = np.full(P.shape[0], np.inf)
        for kk in range(2):
            if na_[kk] > 0:
                tout = np.minimum(tout, (half - P[:, kk]) / na_[kk])
            elif na_[kk] < 0:
                tout = np.minimum(tout, (-half - P[:, kk]) / na_[kk])
        att = np.exp(-mu0 * (Ep / 85.0) ** (-1 / 3) * tout)
        u = -P[:, 0] * na_[1] + P[:, 1] * na_[0]
        depth = p.R - (P[:, 0] * na_[0] + P[:, 1] * na_[1])
        sig = (p.fwhm0 + p.fwhm_slope * depth) / FWHM
        D = ((stats.norm.cdf(p.R, u, sig) - stats.norm.cdf(-p.R, u, sig)) *
             (stats.norm.cdf(p.Zh, P[:, 2], sig) - stats.norm.cdf(-p.Zh, P[:, 2], sig)))
        se = p.eres_frac * p.eres_ref * np.sqrt(Ep / p.eres_ref) / FWHM
        acc = sum(stats.norm.cdf(hi, Ep, se) - stats.norm.cdf(lo, Ep, se) for lo, hi in p.windows)
        wgt = _kn(cphi, Ew) / Z3 * p.domega * att * D * acc
        total += al * wgt.sum() / n_photons
    return total


def test_scatter_model_matches_monte_carlo_3d(oracle_mod):
    half, mu0 = 12.0, 0.02                 # uniform cube [-12, 12]^3
    errs = []
    for n, pix, ns in [(12, 4.0, 6), (24, 2.0, 12), (48, 1.0, 24)]:
        nz = int(round(32.0 / pix))        # axial length 32 mm
        p = synth.SysParams(n=n, pix=pix, ns=ns, nb=16, na=8, nz=nz, nsz=nz // 2, nbz=8)
        x, y, z = synth.voxel_centres(p)
        mu = np.where((np.abs(x) < half) & (np.abs(y) < half) & (np.abs(z) < half), mu0, 0.0)
        # source voxel: the one whose centre is nearest (-5, 3, 2) mm; only it is modelled
        q = int(np.argmin((x + 5.0) ** 2 + (y - 3.0) ** 2 + (z - 2.0) ** 2))
        mask = np.zeros(x.size, np.uint8)
        mask[q] = 1
        o = oracle_mod.Oracle3(p, mu, mask)
        x0, y0, z0 = o.voxel_centre(q)
        for a in (1, 4):
            prim = sum(o.Pp(q, a, w) * o.psf_total(x0, y0, z0, a) * synth_acc(o, p, Ew)
                       for w, Ew in enumerate(p.lines))
            model = o.sens_qa(q, a) - prim
            mc = _mc_scatter3(p, mu0, half, x0, y0, z0, a, 400000, seed=300 + n + a)
            errs.append((n, a, model / mc - 1.0))
    by_n = {}
    for n, a, e in errs:
        by_n.setdefault(n, []).append(abs(e))
    coarse, mid, fine = (np.mean(by_n[k]) for k in (12, 24, 48))
    print("3-D scatter model vs Monte Carlo (n, angle, relative error):", errs)
    assert fine < mid < coarse, errs
    assert fine < 0.05, errs


def synth_acc(o, p, E):
    """Window acceptance at true energy E (scipy), for the primary term."""
    se = p.eres_frac * p.eres_ref * math.sqrt(E / p.eres_ref) / FWHM
    return sum(stats.norm.cdf(hi, E, se) - stats.norm.cdf(lo, E, se) for lo, hi in p.windows)


def test_osem_count_conservation_3d(oracle_mod):
    p = _p()
    x, y, z = _vox(p)
    mu = np.where(x * x + y * y <= 12.0 ** 2, 0.015, 0.0)
    act = np.where(x * x + y * y <= 12.0 ** 2, 1.0, 0.0) + (np.abs(x - 4) < 3)
    o = oracle_mod.Oracle3(p, mu)
    ev = synth.generic_events3(p, act, 120, seed=4)
    ev = {k: np.asarray(v) for k, v in ev.items()}
    ev["energy"] = ev["energy"].astype(np.float64)
    assert o.check_events(ev) == -1
    nsub = 2
    sens = o.sensitivity(nsub)
    lam0 = o.support.astype(np.float64)
    lam, hist, ll, sk = o.osem(ev, nsub, 2, lam0, sens)
    for k in range(hist.shape[0]):
        s = k % nsub
        Js = int(np.sum(ev["angle"] % nsub == s))
        assert float(sens[s] @ hist[k]) == pytest.approx(Js - sk[k], rel=1e-10)
        assert np.all(hist[k] >= 0)
    fwd = o.forward(ev, lam0)
    j = 17
    assert fwd[j] == pytest.approx(o.row(ev["bin"][j], ev["bin_z"][j], ev["angle"][j],
                                         ev["energy"][j]) @ lam0, rel=1e-13)
    bad = dict(ev, bin_z=ev["bin_z"].copy())
    bad["bin_z"][7] = p.nbz
    assert o.check_events(bad) == 7
