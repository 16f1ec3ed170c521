"""Pins of the regional figures of merit (Sec. 3.1.4) in oracle/fom.py."""
import numpy as np

from oracle import fom


def test_hand_computed_example():
    # one object, two noise realisations 1.1 and 0.9 of a true uptake 1:
    # RMS error 0.1, mean error 0, sample standard deviation sqrt(0.02 / 1)
    yhat = np.array([[[1.1], [0.9]]])
    y = np.array([[1.0]])
    assert abs(fom.enrmse(yhat, y)[0] - 0.1) < 1e-15
    assert abs(fom.ens_bias(yhat, y)[0]) < 1e-15
    assert abs(fom.ens_std(yhat, y)[0] - np.sqrt(0.02)) < 1e-15


def test_perfect_estimates_and_constant_offset():
    rng = np.random.default_rng(0)
    y = rng.uniform(1, 5, (3, 4))
    yhat = np.repeat(y[:, None, :], 6, axis=1)
    assert np.all(fom.enrmse(yhat, y) == 0) and np.all(fom.ens_bias(yhat, y) == 0)
    assert np.allclose(fom.ens_std(yhat, y), 0.0, atol=1e-14)
    # every estimate 10 % high: bias = ENRMSE = 0.1, std = 0
    assert np.allclose(fom.ens_bias(1.1 * yhat, y), 0.1, rtol=0, atol=1e-14)
    assert np.allclose(fom.enrmse(1.1 * yhat, y), 0.1, rtol=0, atol=1e-14)
    assert np.allclose(fom.ens_std(1.1 * yhat, y), 0.0, atol=1e-14)


def test_mse_decomposition_single_object():
    # for one object: ENRMSE^2 = bias^2 + (N - 1)/N std^2 (normalised by y)
    rng = np.random.default_rng(1)
    N, K = 9, 3
    y = rng.uniform(1, 3, (1, K))
    yhat = y[:, None, :] * (1 + rng.normal(0.05, 0.2, (1, N, K)))
    e, b, s = fom.enrmse(yhat, y), fom.ens_bias(yhat, y), fom.ens_std(yhat, y)
    assert np.allclose(e ** 2, b ** 2 + (N - 1) / N * s ** 2, rtol=1e-12)


def test_scale_invariance_and_object_average():
    rng = np.random.default_rng(2)
    y = rng.uniform(1, 3, (4, 2))
    yhat = y[:, None, :] * (1 + rng.normal(0, 0.1, (4, 5, 2)))
    for f in (fom.enrmse, fom.ens_bias, fom.ens_std):
        assert np.allclose(f(7.0 * yhat, 7.0 * y), f(yhat, y), rtol=1e-12)
        # the ensemble value is the mean of the per-object values
        per = np.array([f(yhat[s:s + 1], y[s:s + 1]) for s in range(4)])
        assert np.allclose(per.mean(0), f(yhat, y), rtol=1e-12)


def test_roi_uptake_is_masked_sum():
    lam = np.arange(12.0).reshape(2, 6)
    masks = np.array([[1, 0, 1, 0, 0, 0], [0, 0, 0, 1, 1, 1]], np.uint8)
    assert np.array_equal(fom.roi_uptake(lam, masks), [[2.0, 12.0], [14.0, 30.0]])
