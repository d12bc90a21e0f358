"""Prevalence and quantile reductions (TEST INFRASTRUCTURE ONLY).

Population prevalence of section 4.2's prevalence(): cases over the
individuals at risk, here per run and recorded time point from the per-run
compartment sums; then, over the replicates of each parameter set, the
type-7 quantiles (linear interpolation between order statistics at
h = (R - 1) p), computed in binary64 and rounded once to float32.
"""
from __future__ import annotations

import math

import numpy as np


def prevalence(sums: np.ndarray, case_c: int, at_risk) -> np.ndarray:
    """sums: int64 (runs, Ntspan, Nc) -> float64 (runs, Ntspan); 0 where no one is at risk."""
    den = np.zeros(sums.shape[:2], dtype=np.int64)
    for c in at_risk:
        den += sums[:, :, c]
    num = sums[:, :, case_c].astype(np.float64)
    out = np.zeros(sums.shape[:2], dtype=np.float64)
    pos = den > 0
    out[pos] = num[pos] / den[pos].astype(np.float64)
    return out


def type7_quantile(values, p: float) -> float:
    """Quantile of one sample by linear interpolation of the order statistics."""
    x = sorted(float(v) for v in values)
    h = (len(x) - 1) * p
    lo = math.floor(h)
    frac = h - lo
    if lo + 1 < len(x):
        return x[lo] + (x[lo + 1] - x[lo]) * frac
    return x[lo]


def prevalence_quantiles(sums, case_c, at_risk, replicates, k0, nk, probs) -> np.ndarray:
    """float32 (sets, nk, len(probs)) for runs grouped in consecutive sets."""
    P = prevalence(np.asarray(sums), case_c, at_risk)
    sets = P.shape[0] // replicates
    out = np.zeros((sets, nk, len(probs)), dtype=np.float32)
    for s in range(sets):
        for kk in range(nk):
            col = P[s * replicates:(s + 1) * replicates, k0 + kk]
            for q, p in enumerate(probs):
                out[s, kk, q] = np.float32(type7_quantile(col, p))
    return out
