"""Figures of merit for regional uptake, Sec. 3.1.4 (TEST INFRASTRUCTURE ONLY).

Plain numpy in FP64, written from the three ensemble definitions of the
section: S object realisations, N noise realisations, K regions, true uptake
y[s, k], estimates yhat[s, n, k].
"""
import numpy as np


def roi_uptake(lam, masks):
    """Uptake of region k in image c: the sum of lam[c] over the pixels of masks[k]."""
    lam = np.atleast_2d(np.asarray(lam, np.float64))
    masks = np.atleast_2d(np.asarray(masks)).astype(bool)
    return np.array([[lam[c][masks[k]].sum() for k in range(masks.shape[0])]
                     for c in range(lam.shape[0])])


def enrmse(yhat, y):
    """Ensemble normalised RMSE: mean over objects of the RMS error over noise
    realisations, divided by the true uptake."""
    yhat, y = np.asarray(yhat, np.float64), np.asarray(y, np.float64)
    S, N, K = yhat.shape
    out = np.zeros(K)
    for k in range(K):
        for s in range(S):
            out[k] += np.sqrt(np.sum((yhat[s, :, k] - y[s, k]) ** 2) / N) / y[s, k]
    return out / S


def ens_bias(yhat, y):
    """Ensemble normalised bias: mean over objects and noise realisations of
    the error divided by the true uptake."""
    yhat, y = np.asarray(yhat, np.float64), np.asarray(y, np.float64)
    S, N, K = yhat.shape
    out = np.zeros(K)
    for k in range(K):
        for s in range(S):
            out[k] += np.sum(yhat[s, :, k] - y[s, k]) / y[s, k]
    return out / (S * N)


def ens_std(yhat, y):
    """Ensemble normalised standard deviation: mean over objects of the sample
    standard deviation (N - 1 in the denominator) over noise realisations,
    divided by the true uptake."""
    yhat, y = np.asarray(yhat, np.float64), np.asarray(y, np.float64)
    S, N, K = yhat.shape
    out = np.zeros(K)
    for k in range(K):
        for s in range(S):
            m = np.sum(yhat[s, :, k]) / N
            out[k] += np.sqrt(np.sum(np.abs(yhat[s, :, k] - m) ** 2) / (N - 1)) / y[s, k]
    return out / S
