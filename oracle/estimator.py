"""TE-PAI estimator (oracle side, float64).

Per sample l the estimate is o_l = ||g||_1 sign(g_l) Tr[O U_l rho_0] (proof
of Statement 2), with ||g||_1 = exp(log ||g||_1) from the PAI table.  The
estimator is the sample mean; its standard error is s / sqrt(N_s) with s^2
the unbiased (ddof = 1) sample variance of the o_l; the configuration
variance Var[v_l] = s^2 / ||g||_1^2 (eq. config_var).
"""
from __future__ import annotations

import math

import numpy as np


def weights(signs, log_g1: float) -> np.ndarray:
    return np.asarray(signs, dtype=np.float64) * math.exp(log_g1)


def estimate(values: np.ndarray, w: np.ndarray):
    """values[s, o], w[s] -> (mean[o], std_err[o], config_var[o])."""
    x = np.asarray(values, dtype=np.float64) * np.asarray(w, dtype=np.float64)[:, None]
    ns = x.shape[0]
    mean = x.mean(axis=0)
    if ns > 1:
        var = ((x - mean) ** 2).sum(axis=0) / (ns - 1)
        se = np.sqrt(var / ns)
    else:
        var = np.full(x.shape[1], np.nan)
        se = np.full(x.shape[1], np.nan)
    g1 = float(np.abs(w[0])) if ns else 1.0
    return mean, se, var / (g1 * g1)
