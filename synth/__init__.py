"""Seeded synthetic inputs shared by the GPU path, the oracle and the tests.

This module holds only inputs: system parameters, phantoms (activity and
attenuation maps) and a generic list-mode event generator.  It contains none of
the reconstruction method's arithmetic (no attenuation line integrals, no
Klein-Nishina weights, no collimator or energy-acceptance model): the events it
makes have the structure of the paper's workloads (angles over 360 degrees,
bins concentrated on the object's projection, energies clustered on the
emission lines inside the windows) and serve as inputs whose exact values do
not matter.  Events drawn from the exact model itself come from the oracle's
sampler, which only the tests use.

Workloads follow the paper's simulation (Sec. 3.1): a 2-D phantom with an
elliptical water body and circular or elliptical hot regions, 120 angles over
360 degrees, the Ra-223-like lines at 85/154/270 keV and the windows
68-102, 123-184 and 243-297 keV.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

EW1 = (68.0, 102.0)
EW2 = (123.0, 184.0)
EW3 = (243.0, 297.0)
SW = (184.0, 243.0)
# collimator acceptance solid angle of the 3-D model: a cone whose full
# opening angle is the planar model's acceptance angle (0.03 rad)
DOMEGA = float(2.0 * np.pi * (1.0 - np.cos(0.015)))


@dataclass(frozen=True)
class SysParams:
    n: int                 # pixels per side
    pix: float             # pixel size, mm
    ns: int                # scatter points per side
    nb: int                # detector bins
    na: int                # angles over 360 degrees
    fwhm0: float = 2.0     # collimator-detector FWHM at depth 0, mm
    fwhm_slope: float = 0.03
    dtheta: float = 0.03   # collimator angular acceptance, rad
    lines: tuple = (85.0, 154.0, 270.0)
    yields: tuple = (0.25, 0.06, 0.14)
    windows: tuple = (EW1, EW2)
    eres_frac: float = 0.10
    eres_ref: float = 140.0
    mu_ref: float = 85.0
    mu_pow: float = 1.0 / 3.0
    T: float = 1.0
    me: float = 510.99895  # electron rest energy, keV
    nz: int = 0            # slices (0: the planar model of the paper's evaluation)
    nsz: int = 0           # scatter points along z (3-D)
    nbz: int = 0           # axial detector bins (3-D)
    domega: float = DOMEGA # collimator acceptance solid angle, sr (3-D)

    @property
    def fov(self):
        return self.n * self.pix

    @property
    def R(self):
        return 0.5 * self.n * self.pix

    @property
    def Zh(self):
        return 0.5 * self.nz * self.pix


@dataclass(frozen=True)
class Workload:
    name: str
    params: SysParams
    n_events: int
    n_subsets: int
    n_iters: int
    phantom: str
    seed_phantom: int
    seed_events: int
    poisson: bool = False
    n_cases: int = 1
    case_min: int = 0
    case_max: int = 0
    seed_cases: int = 0
    own_phantom_per_case: bool = False


CONFIGS = {
    # 16x16 at 4 mm, 8x8 scatter grid, 16 bins x 32 angles, EW1+EW2, 2000 events.
    "16x16_2k": Workload("16x16_2k", SysParams(16, 4.0, 8, 16, 32, windows=(EW1, EW2)),
                         2000, 4, 10, "disk2", 11, 12),
    # 64x64 at 4 mm, 32x32 scatter grid, 64 bins x 120 angles, EW1-3, ~50k events.
    "64x64_50k": Workload("64x64_50k", SysParams(64, 4.0, 32, 64, 120,
                                                 windows=(EW1, EW2, EW3)),
                          50000, 8, 20, "ellipse3", 21, 22, poisson=True),
    # 64 cases of the 64x64 geometry, per-case means uniform in [20k, 200k].
    "64x64_64cases": Workload("64x64_64cases", SysParams(64, 4.0, 32, 64, 120,
                                                         windows=(EW1, EW2, EW3)),
                              0, 8, 20, "ellipse3", 21, 3100, poisson=True, n_cases=64,
                              case_min=20000, case_max=200000, seed_cases=31),
    # 128x128 at 2 mm, 64x64 scatter grid, 128 bins x 120 angles, EW1-3 + SW,
    # 1M events over 16 uneven cases, each with a phantom and attenuation map
    # of its own.
    "128x128_16cases": Workload("128x128_16cases", SysParams(128, 2.0, 64, 128, 120,
                                                             windows=(EW1, EW2, SW, EW3)),
                                1000000, 16, 20, "ellipse3", 5200, 5300, poisson=False,
                                n_cases=16, case_min=20000, case_max=200000, seed_cases=51,
                                own_phantom_per_case=True),
    # 3-D single scatter: 16x16x8 voxels of 4 mm, 8x8x4 scatter grid, 16x8 bins,
    # 16 angles, EW1+EW2, 600 events.
    "16x16x8_600": Workload("16x16x8_600", SysParams(16, 4.0, 8, 16, 16, windows=(EW1, EW2),
                                                     nz=8, nsz=4, nbz=8),
                            600, 4, 2, "disk2_3d", 11, 13),
    # 3-D: the 64x64 workload's slice geometry over 16 slices (256x256x64 mm),
    # 32x32x8 scatter grid, 64x16 bins, 120 angles, EW1-3, ~50k events.
    "64x64x16_50k": Workload("64x64x16_50k", SysParams(64, 4.0, 32, 64, 120,
                                                       windows=(EW1, EW2, EW3), nz=16, nsz=8,
                                                       nbz=16),
                             50000, 8, 20, "ellipse3_3d", 21, 23, poisson=True),
}


def pixel_centres(p: SysParams):
    c = (np.arange(p.n) + 0.5) * p.pix - p.R
    x, y = np.meshgrid(c, c)          # x varies along columns (ix), y along rows (iy)
    return x.ravel(), y.ravel()


def fov_support(p: SysParams):
    x, y = pixel_centres(p)
    return (x * x + y * y <= p.R * p.R)


def phantom_disk2(p: SysParams, mu85=0.018, body_r=28.0, hot_r=6.0, hot_x=14.0,
                  ratio=4.0):
    """Water disk with two hot disks on the x axis (activity ratio `ratio`:1)."""
    x, y = pixel_centres(p)
    body = x * x + y * y <= body_r * body_r
    mu = np.where(body, mu85, 0.0)
    act = np.where(body, 1.0, 0.0)
    rois = []
    for cx in (-hot_x, hot_x):
        roi = (x - cx) ** 2 + y ** 2 <= hot_r * hot_r
        act = np.where(roi, ratio, act)
        rois.append(roi)
    return mu, act, rois


def disk2_objects(p: SysParams, n_objects: int, seed: int, n_lumps=8, amp=(0.0, 0.6),
                  width=6.0, ratio=4.0, **disk):
    """Object realisations of phantom_disk2 with a lumpy background (Sec. 3.1.1
    draws a new background sample per object realisation; its lumpy-model
    parameters are not given, these are ours): background 1 + sum of n_lumps
    Gaussian lumps (amplitude U[amp], standard deviation `width` mm, centres
    uniform in the body), scaled to mean 1 in the body; the two hot disks hold
    `ratio` times that mean.  Returns (mu [Q], activities [n_objects, Q], rois)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu, act0, rois = phantom_disk2(p, ratio=ratio, **disk)
    x, y = pixel_centres(p)
    body = act0 > 0
    r_body = np.sqrt((x[body] ** 2 + y[body] ** 2).max())
    acts = np.zeros((n_objects, x.size))
    for o in range(n_objects):
        b = np.ones(x.size)
        for _ in range(n_lumps):
            rr, th = r_body * np.sqrt(rng.random()), 2 * np.pi * rng.random()
            cx, cy = rr * np.cos(th), rr * np.sin(th)
            b += rng.uniform(*amp) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * width ** 2))
        b = np.where(body, b / b[body].mean(), 0.0)
        for roi in rois:
            b = np.where(roi, ratio, b)
        acts[o] = b
    return mu, acts, rois


def sew_events(ev, window, energy_keV=None):
    """The events of one energy window (the single-window methods of Sec. 3.2.2);
    with energy_keV, every kept event is assigned that energy (the binned-energy
    variant)."""
    e = np.asarray(ev["energy"])
    keep = (e >= window[0]) & (e <= window[1])
    out = {k: np.asarray(ev[k])[keep] for k in ("bin", "angle", "energy")}
    if energy_keV is not None:
        out["energy"] = np.full(int(keep.sum()), energy_keV, dtype=out["energy"].dtype)
    return out


def _in_ellipse(x, y, cx, cy, a, b, th):
    c, s = np.cos(th), np.sin(th)
    u = (x - cx) * c + (y - cy) * s
    v = -(x - cx) * s + (y - cy) * c
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def phantom_ellipse3(p: SysParams, seed: int, body=(110.0, 90.0), rim=8.0,
                     mu_rim=0.021, mu_inner=0.018):
    """Elliptical water body (rim and inner attenuation of Sec. 3.1.1, given
    there in 1/cm) with three random non-overlapping elliptical hot regions
    (semi-axes U[7,20] mm, random orientation, ratios drawn from {2,4,6}:1)
    on a uniform background."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = pixel_centres(p)
    A, B = body
    scale = min(1.0, 0.9 * p.R / A)       # keep the body inside smaller fields of view
    A, B, rim = A * scale, B * scale, rim * scale
    outer = _in_ellipse(x, y, 0, 0, A, B, 0.0)
    inner = _in_ellipse(x, y, 0, 0, A - rim, B - rim, 0.0)
    mu = np.where(inner, mu_inner, np.where(outer, mu_rim, 0.0))
    act = np.where(outer, 1.0, 0.0)
    rois, placed = [], []
    tries = 0
    while len(rois) < 3 and tries < 10000:
        tries += 1
        a_ = rng.uniform(7.0, 20.0) * scale
        b_ = rng.uniform(7.0, 20.0) * scale
        th = rng.uniform(0, np.pi)
        r = max(a_, b_)
        cx = rng.uniform(-(A - rim - r), A - rim - r)
        cy = rng.uniform(-(B - rim - r), B - rim - r)
        if not _in_ellipse(np.array([cx]), np.array([cy]), 0, 0, A - rim - r, B - rim - r, 0)[0]:
            continue
        if any(np.hypot(cx - px, cy - py) < r + pr + 2 * p.pix for px, py, pr in placed):
            continue
        roi = _in_ellipse(x, y, cx, cy, a_, b_, th)
        if roi.sum() == 0:
            continue
        ratio = float(rng.choice([2.0, 4.0, 6.0]))
        act = np.where(roi, ratio, act)
        rois.append(roi)
        placed.append((cx, cy, r))
    return mu, act, rois


def random_body_maps(p: SysParams, n_maps: int, seed: int, axes=(0.7, 0.95), shift=0.05,
                     rim=8.0, mu_rim=0.021, mu_inner=0.018):
    """Attenuation maps of random elliptical water bodies for one geometry:
    semi-axes U[axes]*R, orientation U[0, pi), centre offset U[-shift, shift]*R
    per coordinate, with the rim of phantom_ellipse3 (scaled like its body).
    Returns [n_maps, n*n] float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = pixel_centres(p)
    rim = rim * min(1.0, 0.9 * p.R / 110.0)
    out = np.zeros((n_maps, p.n * p.n))
    for k in range(n_maps):
        A, B = rng.uniform(axes[0], axes[1], 2) * p.R
        th = rng.uniform(0, np.pi)
        cx, cy = rng.uniform(-shift, shift, 2) * p.R
        outer = _in_ellipse(x, y, cx, cy, A, B, th)
        inner = _in_ellipse(x, y, cx, cy, A - rim, B - rim, th)
        out[k] = np.where(inner, mu_inner, np.where(outer, mu_rim, 0.0))
    return out


def voxel_centres(p: SysParams):
    """Voxel centres of a 3-D grid, flat index (iz*n + iy)*n + ix."""
    c = (np.arange(p.n) + 0.5) * p.pix - p.R
    cz = (np.arange(p.nz) + 0.5) * p.pix - p.Zh
    z, y, x = np.meshgrid(cz, c, c, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def fov_support3(p: SysParams):
    x, y, _ = voxel_centres(p)
    return x * x + y * y <= p.R * p.R


def phantom_disk2_3d(p: SysParams, mu85=0.018, body_r=28.0, half_z=None, hot_r=6.0,
                     hot=((-14.0, 0.0, -4.0), (14.0, 0.0, 4.0)), ratio=4.0):
    """Water cylinder (radius body_r, |z| <= half_z, default 3/4 of the axial
    half-length) with two hot spheres (activity ratio `ratio`:1)."""
    x, y, z = voxel_centres(p)
    hz = 0.75 * p.Zh if half_z is None else half_z
    body = (x * x + y * y <= body_r * body_r) & (np.abs(z) <= hz)
    mu = np.where(body, mu85, 0.0)
    act = np.where(body, 1.0, 0.0)
    rois = []
    for cx, cy, cz in hot:
        roi = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= hot_r * hot_r
        act = np.where(roi, ratio, act)
        rois.append(roi)
    return mu, act, rois


def phantom_ellipse3_3d(p: SysParams, seed: int, half_z_frac=0.8):
    """phantom_ellipse3's elliptical body extruded over |z| <= half_z_frac * Zh;
    each of its three hot regions becomes an elliptic cylinder of axial
    half-length U[7,20] mm centred at z uniform in the middle half of the
    body."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    p2 = replace(p, nz=0, nsz=0, nbz=0)
    mu2, act2, rois2 = phantom_ellipse3(p2, seed)
    zc = (np.arange(p.nz) + 0.5) * p.pix - p.Zh
    hz = half_z_frac * p.Zh
    inside = (np.abs(zc) <= hz)[:, None]
    mu = np.where(inside, mu2[None, :], 0.0)
    act = np.where(inside, (act2 > 0).astype(np.float64)[None, :], 0.0)
    rois = []
    for roi2 in rois2:
        ratio = float(act2[roi2].max())
        cz = rng.uniform(-0.5 * hz, 0.5 * hz)
        c = rng.uniform(7.0, 20.0)
        roi = roi2[None, :] & ((np.abs(zc - cz) <= c) & (np.abs(zc) <= hz))[:, None]
        act = np.where(roi, ratio, act)
        rois.append(roi.ravel())
    return mu.ravel(), act.ravel(), rois


def generic_events3(p: SysParams, activity, n_events: int, seed: int, poisson=False,
                    blur_mm=3.0, peak_frac=0.7, peak_sigma=5.0):
    """generic_events for the 3-D geometry: emission voxel drawn in
    proportion to `activity`, angle uniform, detector position = projection
    of the voxel centre (u) and its z (v) plus a fixed Gaussian blur, energy as
    in generic_events.  Returns bin, bin_z, angle, energy."""
    rng = np.random.Generator(np.random.PCG64(seed))
    J = int(rng.poisson(n_events)) if poisson else int(n_events)
    act = np.asarray(activity, dtype=np.float64).ravel()
    cdf = np.cumsum(act)
    cdf /= cdf[-1]
    x, y, z = voxel_centres(p)
    lines = np.asarray(p.lines)
    yields = np.asarray(p.yields) / np.sum(p.yields)
    wins = np.asarray(p.windows)
    out = {"bin": np.empty(J, np.int16), "bin_z": np.empty(J, np.int16),
           "angle": np.empty(J, np.int16), "energy": np.empty(J, np.float32)}
    db, dbz = p.fov / p.nb, 2 * p.Zh / p.nbz
    filled = 0
    while filled < J:
        m = max(1024, 2 * (J - filled))
        q = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), act.size - 1)
        a = rng.integers(0, p.na, m)
        th = 2 * np.pi * a / p.na
        u = -x[q] * np.sin(th) + y[q] * np.cos(th) + rng.normal(0, blur_mm, m)
        v = z[q] + rng.normal(0, blur_mm, m)
        b = np.floor((u + p.R) / db).astype(np.int64)
        bz = np.floor((v + p.Zh) / dbz).astype(np.int64)
        w = rng.choice(len(lines), size=m, p=yields)
        peak = rng.random(m) < peak_frac
        e = np.where(peak, rng.normal(lines[w], peak_sigma), rng.uniform(0.4 * lines[w], lines[w]))
        inwin = np.zeros(m, bool)
        for lo, hi in wins:
            inwin |= (e >= lo) & (e <= hi)
        ok = (b >= 0) & (b < p.nb) & (bz >= 0) & (bz < p.nbz) & inwin
        k = min(int(ok.sum()), J - filled)
        idx = np.flatnonzero(ok)[:k]
        out["bin"][filled:filled + k] = b[idx]
        out["bin_z"][filled:filled + k] = bz[idx]
        out["angle"][filled:filled + k] = a[idx]
        out["energy"][filled:filled + k] = e[idx]
        filled += k
    return out


def phantom(w: Workload, case: int = 0):
    if w.phantom == "disk2":
        return phantom_disk2(w.params)
    if w.phantom == "disk2_3d":
        return phantom_disk2_3d(w.params)
    if w.phantom == "ellipse3_3d":
        return phantom_ellipse3_3d(w.params, w.seed_phantom)
    seed = w.seed_phantom + (case if w.own_phantom_per_case else 0)
    return phantom_ellipse3(w.params, seed)


def case_counts(w: Workload):
    """Per-case event counts for batched workloads."""
    rng = np.random.Generator(np.random.PCG64(w.seed_cases))
    means = rng.uniform(w.case_min, w.case_max, size=w.n_cases)
    if w.n_events > 0:                       # fixed total split in proportion
        cnt = np.floor(means / means.sum() * w.n_events).astype(np.int64)
        cnt[: w.n_events - cnt.sum()] += 1
        return cnt
    return np.array([np.random.Generator(np.random.PCG64(w.seed_events + 1000 + c)).poisson(m)
                     for c, m in enumerate(means)], dtype=np.int64)


def generic_events(p: SysParams, activity, n_events: int, seed: int, poisson=False,
                   blur_mm=3.0, peak_frac=0.7, peak_sigma=5.0):
    """List-mode events with the structure of a SPECT acquisition.

    Emission pixel drawn in proportion to `activity`, angle uniform over the
    `na` angles, lateral detector position = projection of the pixel centre
    plus a fixed Gaussian blur (`blur_mm`), energy either near an emission line
    (line chosen by yield, fixed Gaussian spread `peak_sigma`) or uniform below
    it (a stand-in for the scatter continuum), kept only inside the windows.
    None of these draws uses the reconstruction model.  "position" holds the
    continuous lateral position (mm, float32, in [-R, R)) that "bin" quantises;
    drop "bin" to hand the events over as continuous."""
    rng = np.random.Generator(np.random.PCG64(seed))
    J = int(rng.poisson(n_events)) if poisson else int(n_events)
    act = np.asarray(activity, dtype=np.float64).ravel()
    cdf = np.cumsum(act)
    cdf /= cdf[-1]
    x, y = pixel_centres(p)
    lines = np.asarray(p.lines)
    yields = np.asarray(p.yields) / np.sum(p.yields)
    wins = np.asarray(p.windows)
    bins = np.empty(J, np.int16)
    pos = np.empty(J, np.float32)
    angs = np.empty(J, np.int16)
    ener = np.empty(J, np.float32)
    db = p.fov / p.nb
    below_R = np.nextafter(np.float32(p.R), np.float32(0))
    filled = 0
    while filled < J:
        m = max(1024, 2 * (J - filled))
        q = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), act.size - 1)
        a = rng.integers(0, p.na, m)
        th = 2 * np.pi * a / p.na
        u = -x[q] * np.sin(th) + y[q] * np.cos(th) + rng.normal(0, blur_mm, m)
        b = np.floor((u + p.R) / db).astype(np.int64)
        w = rng.choice(len(lines), size=m, p=yields)
        peak = rng.random(m) < peak_frac
        e = np.where(peak, rng.normal(lines[w], peak_sigma), rng.uniform(0.4 * lines[w], lines[w]))
        inwin = np.zeros(m, bool)
        for lo, hi in wins:
            inwin |= (e >= lo) & (e <= hi)
        ok = (b >= 0) & (b < p.nb) & inwin
        k = min(int(ok.sum()), J - filled)
        idx = np.flatnonzero(ok)[:k]
        bins[filled:filled + k] = b[idx]
        pos[filled:filled + k] = np.minimum(u[idx].astype(np.float32), below_R)
        angs[filled:filled + k] = a[idx]
        ener[filled:filled + k] = e[idx]
        filled += k
    return {"bin": bins, "angle": angs, "energy": ener, "position": pos}


def workload_inputs(name: str, case: int = 0, n_events=None):
    """(params, mu85 [Q], activity [Q], rois, events) for one case of a workload,
    with generic events."""
    w = CONFIGS[name]
    mu, act, rois = phantom(w, case)
    if n_events is None:
        n_events = int(case_counts(w)[case]) if w.n_cases > 1 else w.n_events
    ev = generic_events(w.params, act, n_events, w.seed_events + case,
                        poisson=(w.poisson and w.n_cases == 1))
    return w.params, mu, act, rois, ev


__all__ = ["SysParams", "Workload", "CONFIGS", "EW1", "EW2", "EW3", "SW", "pixel_centres",
           "fov_support", "phantom_disk2", "disk2_objects", "sew_events", "phantom_ellipse3",
           "random_body_maps", "phantom", "case_counts", "DOMEGA", "voxel_centres",
           "fov_support3", "phantom_disk2_3d", "phantom_ellipse3_3d", "generic_events3",
           "generic_events", "workload_inputs", "replace", "field"]
