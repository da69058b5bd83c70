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


def kirchhoff(diag):
    """Kirchhoff index n * Tr(L^dagger) (= sum over node pairs of resistance
    distance).  The text at the end of Sec. 5 names Tr(L^dagger); the factor n
    comes from the standard definition as the pair sum of resistances, which
    the library reports beside Tr(L^dagger) itself."""
    return len(diag) * math.fsum(np.asarray(diag).tolist())


def rw_betweenness(diag):
    """1/n + Tr/((n-1)(Tr + n L^dagger_uu)), the formula quoted at the end of
    Sec. 5, as printed.  Pinned by closed forms (complete graphs, stars) and
    by the identity Tr + n L^dagger_uu = sum_v r(u,v) on resistances from the
    other pseudo-inverse route."""
    n = len(diag)
    tr = math.fsum(np.asarray(diag).tolist())
    return 1.0 / n + tr / ((n - 1) * (tr + n * np.asarray(diag)))


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


# ----------------------------------------------------------------- queries
def globals_from_counts(Y1, Y2, omega, deg, root):
    """Cached global terms for single-node queries:
    Tr(L_v^{-1}) ~ sum_u Y1[u]/(omega d_u) and 1^T L_v^{-1} 1 ~ n sum_w Y2[w]/(omega d_w)."""
    deg = np.asarray(deg, np.float64)
    n = len(deg)
    mask = np.arange(n) != root
    tr = math.fsum((np.asarray(Y1, np.float64)[mask] / (omega * deg[mask])).tolist())
    s = n * math.fsum((np.asarray(Y2, np.float64)[mask] / (omega * deg[mask])).tolist())
    return tr, s


def closeness_query(dep_u, norm_len, d_u, n, tr_lv, s_lv):
    """c(u) from walks started at u: (L_v^{-1})_uu ~ mean dep_u / d_u (Lemma 1),
    e_u^T L_v^{-1} 1 ~ mean normalised length (Sec. 4.3 lemma), then the
    element-wise equation for L^dagger_uu, Tr(L^dagger) = Tr(L_v^{-1}) - S/n and
    c(u) = (n-1)/(Tr + n L^dagger_uu).  Returns (c, L^dagger_uu, se of L^dagger_uu)."""
    dep_u = np.asarray(dep_u, np.float64)
    norm_len = np.asarray(norm_len, np.float64)
    b = len(dep_u)
    z = dep_u / d_u - 2.0 * norm_len / n
    ld = float(math.fsum(z.tolist()) / b) + s_lv / n ** 2
    tr = tr_lv - s_lv / n
    c = (n - 1) / (tr + n * ld)
    se = float(z.std(ddof=1) / math.sqrt(b)) if b > 1 else float("nan")
    return c, ld, se


def resistance_query(ss, st, tt, ts, d_s, d_t):
    """r(s,t) = (L_v^{-1})_ss + (L_v^{-1})_tt - 2 (L_v^{-1})_st from walk pairs:
    per pair ss/d_s - st/d_t + tt/d_t - ts/d_s (Lemma 1, both orders of the
    symmetric off-diagonal term).  Returns (r, se)."""
    r = (np.asarray(ss, np.float64) / d_s - np.asarray(st, np.float64) / d_t
         + np.asarray(tt, np.float64) / d_t - np.asarray(ts, np.float64) / d_s)
    b = len(r)
    return float(math.fsum(r.tolist()) / b), (float(r.std(ddof=1) / math.sqrt(b)) if b > 1 else float("nan"))


def spantree_diag(X1, X2, omega, n):
    """SpanTree estimate of diag(L^dagger) (Alg. 1, last loop):
    x1(u) - 2 x2(u) + (1/n) sum_w x2(w), where x1 = X1 / omega and
    x2 = X2 / (n omega) (X2 counts the path support in units of 1/n)."""
    x1 = np.asarray(X1, np.float64) / omega
    x2 = np.asarray(X2, np.float64) / (n * omega)
    return x1 - 2.0 * x2 + math.fsum(x2.tolist()) / n


def spantree_kemeny(s1, s2, two_m):
    """SpanTree estimate of Kemeny's constant (Alg. 3): the mean over
    samples of s1 - s2 / 2m (s2 counts the path support in units of 1/2m),
    and its standard error."""
    z = np.asarray(s1, np.float64) - np.asarray(s2, np.float64) / two_m
    omega = len(z)
    est = math.fsum(z.tolist()) / omega
    se = float(z.std(ddof=1) / math.sqrt(omega)) if omega > 1 else float("nan")
    return est, se


def spantree_diag_blocks(X1b, X2b, omega, n):
    """Alg. 1 estimate from per-block sums ([B][n]) and its batch-means
    standard error (blocks of floor(i*B/omega) samples)."""
    B = X1b.shape[0]
    sizes = block_sizes(omega, B)
    est = np.stack([spantree_diag(X1b[b], X2b[b], int(sizes[b]), n) for b in range(B)])
    full = spantree_diag(X1b.sum(0), X2b.sum(0), omega, n)
    se = est.std(axis=0, ddof=1) / math.sqrt(B) if B > 1 else np.full(n, np.nan)
    return full, se


def pair_entries(V, omega, d_s, d_t):
    """Entries of L_v^{-1} and resistances from loop-included path counts
    (Sec. 3.4; r(s,t) of Sec. 2 through the grounded inverse).

    V: int64 [B][n_pairs][4] per-block departures (s on the path from s, t on
    the path from s, t on the path from t, s on the path from t); d_s, d_t:
    degrees.  Returns a dict of FP64 arrays over pairs:
      lv_ss = sum V0 / (omega d_s), lv_tt = sum V2 / (omega d_t),
      lv_st = (sum V1 / d_t + sum V3 / d_s) / (2 omega)   (both orders of the
              symmetric entry),
      r     = (sum V0 / d_s - sum V1 / d_t + sum V2 / d_t - sum V3 / d_s) / omega,
      r_se  = batch-means standard error of r over the B blocks.
    """
    V = np.asarray(V, np.int64)
    B = V.shape[0]
    d_s = np.asarray(d_s, np.float64)
    d_t = np.asarray(d_t, np.float64)
    tot = V.sum(0).astype(np.float64)

    def r_of(a, m):
        return (a[..., 0] / d_s - a[..., 1] / d_t + a[..., 2] / d_t - a[..., 3] / d_s) / m

    out = dict(lv_ss=tot[:, 0] / (omega * d_s), lv_tt=tot[:, 2] / (omega * d_t),
               lv_st=(tot[:, 1] / d_t + tot[:, 3] / d_s) / (2.0 * omega), r=r_of(tot, omega))
    if B > 1:
        sizes = block_sizes(omega, B).astype(np.float64)
        rb = np.stack([r_of(V[b].astype(np.float64), sizes[b]) for b in range(B)])
        out["r_se"] = rb.std(axis=0, ddof=1) / math.sqrt(B)
    else:
        out["r_se"] = np.full(V.shape[1], np.nan)
    return out


def lv_rows(Y, omega, deg, root):
    """Rows of L_v^{-1} from loop-included path counts (Sec. 3.4):
    (L_v^{-1})_{s u} = sum_b Y[b][j][u] / (omega d_u); column v is zero."""
    tot = np.asarray(Y, np.int64).sum(0).astype(np.float64)
    out = tot / (omega * np.asarray(deg, np.float64)[None, :])
    out[:, root] = 0.0
    return out
