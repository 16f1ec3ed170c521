"""The synthetic workloads use the acquisition parameters the paper prints."""
import json
import os

import pytest

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def test_windows_follow_the_paper():
    paper = [tuple(float(x) for x in w) for w in GOLD["energy_windows_keV"]["value"]]
    assert (synth.EW1, synth.EW2, synth.EW3) == tuple(paper)
    for name in ("64x64_50k", "64x64_64cases"):
        assert synth.CONFIGS[name].params.windows == tuple(paper)
    assert synth.CONFIGS["16x16_2k"].params.windows == tuple(paper[:2])


def test_resolution_angles_and_attenuation_follow_the_paper():
    r = GOLD["energy_resolution"]["value"]
    for w in synth.CONFIGS.values():
        assert w.params.eres_frac == r["fwhm_fraction"]
        assert w.params.eres_ref == r["at_keV"]
    for name in ("64x64_50k", "64x64_64cases", "128x128_16cases"):
        assert synth.CONFIGS[name].params.na == GOLD["angles"]["value"]["count"]
    mu, act, rois = synth.phantom_ellipse3(synth.CONFIGS["64x64_50k"].params, 21)
    vals = sorted(set(mu[mu > 0].round(6)))
    att = GOLD["attenuation_85keV_per_cm"]["value"]
    assert vals == pytest.approx(sorted([att["rim"] / 10, att["inner"] / 10]))


def test_lines_include_the_papers_high_energy_line():
    assert 270.0 in GOLD["emission_lines_keV"]["value"]
    assert synth.CONFIGS["64x64_50k"].params.lines[-1] == 270.0
