"""FP64 estimator assembly from integer counts (test infrastructure only).

Follows the paper's estimators with the per-visit increments 1/(omega d_u)
summed as integers first and divided once:
  y1(u) = Y1[u] / (omega d_u)      -> (L_v^{-1})_uu             (Alg. 2, walk loop)
  y2(u) = Y2[u] / (omega d_u)      -> (1/n) e_u^T L_v^{-1} 1     (Alg. 2, absorbed loop)
  L^dagger_uu ~ y1(u) - 2 y2(u) + (1/n) ||y2||_1                 (Alg. 2, last loop)
  c(u) = (n-1) / (Tr + n L^dagger_uu)                            (Sec. 2)
  kappa ~ (sum_i y1_i - sum_i y2_i) / omega                      (Alg. 4)
with y1_i the total draws of Wilson sample i and y2_i the length of the
i-th stationary-start absorbed walk.  Standard errors: Kemeny from the
per-sample differences; per-node vectors from batch means over B
contiguous sample blocks.
"""
from __future__ import annotations

import math

import numpy as np


def block_sizes(omega, B):
    """Samples per block when sample i goes to block floor(i*B/omega)."""
    i = np.arange(omega, dtype=np.int64)
    return np.bincount((i * B) // omega, minlength=B)


def diag_ldagger(Y1, Y2, omega, deg, root=None):
    """Y1, Y2: int64 [n] totals over omega samples / omega absorbed walks."""
    deg = np.asarray(deg, np.float64)
    n = len(deg)
    y1 = np.asarray(Y1, np.float64) / (omega * deg)
    y2 = np.asarray(Y2, np.float64) / (omega * deg)
    s = math.fsum(y2.tolist())
    return y1 - 2.0 * y2 + s / n


def closeness(diag):
    n = len(diag)
    tr = math.fsum(np.asarray(diag).tolist())
    return (n - 1) / (tr + n * np.asarray(diag)), tr


def diag_ldagger_blocks(Y1b, Y2b, omega, deg):
    """Batch means: per-block estimates and their standard error."""
    B = Y1b.shape[0]
    sizes = block_sizes(omega, B)
    est = np.stack([diag_ldagger(Y1b[b], Y2b[b], int(sizes[b]), deg) for b in range(B)])
    full = diag_ldagger(Y1b.sum(0), Y2b.sum(0), omega, deg)
    se = est.std(axis=0, ddof=1) / math.sqrt(B) if B > 1 else np.full(len(deg), np.nan)
    return full, se


def kemeny(y1, y2len):
    y1 = np.asarray(y1, np.int64)
    y2 = np.asarray(y2len, np.int64)
    omega = len(y1)
    z = (y1 - y2).astype(np.float64)
    est = float(int(y1.sum() - y2.sum())) / omega
    se = float(z.std(ddof=1) / math.sqrt(omega)) if omega > 1 else float("nan")
    return est, se
