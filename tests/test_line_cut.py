"""The per-event line cut of the per-event kernel, checked on the host.

An event of measured energy E keeps line w's once-scattered terms unless the
energy-resolution Gaussian exp(-(E - E')^2 / (2 k E')) of its probability
(Eq. (3); variance k E' with k = (eres_frac eres_ref / 2.3548)^2 / eres_ref,
Sec. 3.1.2) is below 2^-40 for every scattered energy E' the line can
produce; Compton kinematics puts the scattered energies of Eq. (5) between
E_w / (1 + 2 E_w / m_e c^2) (backscatter) and E_w.  The
library's mask (lmmew_line_mask, host code) is compared with a brute-force
maximum of the Gaussian over a fine grid of scattering angles, away from the
2^-40 boundary where the grid's own resolution decides."""
import math

import numpy as np
import pytest

import synth

CUT = 40 * math.log(2.0)


@pytest.fixture(autouse=True, scope="module")
def _library():
    import os

    from paper_2305_17111_amd import build as libbuild

    if not os.path.exists(libbuild.LIB):
        libbuild.build()


def _max_exponent_margin(p, E, w):
    """Smallest (E - E')^2 / (2 k E') over scattering angles (brute force)."""
    k = (p.eres_frac * p.eres_ref / (2.0 * math.sqrt(2.0 * math.log(2.0)))) ** 2 / p.eres_ref
    Ew = p.lines[w]
    cos = np.linspace(-1.0, 1.0, 200001)
    Ep = Ew / (1.0 + Ew / p.me * (1.0 - cos))
    return np.min((E - Ep) ** 2 / (2.0 * k * Ep))


def test_line_mask_matches_brute_force_over_scattering_angles():
    """A line is kept when its largest Gaussian factor is within 2^-40 of the
    largest over the event's lines."""
    from paper_2305_17111_amd import line_mask

    p = synth.CONFIGS["64x64_50k"].params
    checked = 0
    for E in np.linspace(20.0, 420.0, 801):
        m = line_mask(p, float(np.float32(E)))
        xs = [_max_exponent_margin(p, float(np.float32(E)), w) for w in range(len(p.lines))]
        for w, x in enumerate(xs):
            rel = x - min(xs)
            if abs(rel - CUT) < 0.05:
                continue                      # the grid decides at the boundary
            assert bool((m >> w) & 1) == (rel <= CUT), (E, w, x, m)
            checked += 1
        assert m != 0, E                      # some line's scattered terms are always kept
    assert checked > 2300


def test_line_mask_far_from_every_line_keeps_the_nearest():
    """An in-window energy far outside every line's reachable scattered range
    (a 10-20 keV window with these lines) keeps the line whose range is nearest
    instead of dropping every scattered term."""
    from paper_2305_17111_amd import line_mask

    p = synth.SysParams(16, 4.0, 8, 16, 16, windows=((10.0, 20.0),))
    for E in (10.0, 15.0, 20.0):
        xs = [_max_exponent_margin(p, E, w) for w in range(3)]
        assert min(xs) > CUT                  # beyond the absolute cut for every line
        m = line_mask(p, E)
        assert m & (1 << int(np.argmin(xs))), (E, m)
    # and above every line
    assert line_mask(p, 400.0) & 0b100


def test_line_mask_on_the_windows():
    """Events in 243-297 keV keep only the 270 keV line, those in 123-184 keV
    the 154 and 270 keV lines; events near 85 keV keep all three lines' or the
    two lower lines' scattered terms."""
    from paper_2305_17111_amd import line_mask

    p = synth.CONFIGS["64x64_50k"].params
    for E in np.linspace(243.0, 297.0, 28):
        assert line_mask(p, float(E)) == 0b100
    for E in np.linspace(123.0, 184.0, 31):
        assert line_mask(p, float(E)) == 0b110
    for E in np.linspace(68.0, 102.0, 35):
        assert line_mask(p, float(E)) in (0b011, 0b111)
    assert line_mask(p, 70.0) == 0b011 and line_mask(p, 102.0) == 0b111


def test_line_mask_keeps_every_line_beyond_three_and_rejects_bad_input():
    from paper_2305_17111_amd import LmmewError, line_mask

    p = synth.SysParams(16, 4.0, 8, 16, 16, lines=(81.1, 83.8, 95.0, 144.0, 154.0, 270.0),
                        yields=(1.0 / 6,) * 6)
    assert line_mask(p, 270.0) == 0b111111
    q = synth.CONFIGS["64x64_50k"].params
    with pytest.raises(LmmewError):
        line_mask(q, float("nan"))
