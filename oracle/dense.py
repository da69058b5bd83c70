"""FP64 dense ground truth for small graphs (test infrastructure only).

Plain definitions (Sec. 2):
  L = D - A; L^dagger its Moore-Penrose pseudo-inverse; closeness
  c(u) = (n-1) / (Tr L^dagger + n L^dagger_uu); Kemeny's constant
  kappa = Tr(normalised-Laplacian pseudo-inverse) = sum_{i>=2} 1/sigma_i;
  resistance r(s,t) = L^dagger_ss + L^dagger_tt - 2 L^dagger_st.
L^dagger is computed by two independent routes, eigendecomposition and
(L + 11^T/n)^{-1} - 11^T/n (Sec. 1).  The paper's identities relating
L^dagger to L_v^{-1} (Thm. 1 and the element-wise equations after it), the
normalised counterpart used by the Kemeny lemma (Sec. 5) and the
random-walk matrices (I - P_v)^{-1} used by the sampling lemmas (Lemmas 1,
4, 5) are written out as printed, for tests to check against the plain
definitions.
"""
from __future__ import annotations

import numpy as np


def adjacency(g):
    A = np.zeros((g.n, g.n))
    for u in range(g.n):
        A[u, g.col[g.rp[u]:g.rp[u + 1]]] = 1.0
    return A


def laplacian(g):
    A = adjacency(g)
    return np.diag(A.sum(1)) - A


def pinv_eigh(L):
    """sum over nonzero eigenpairs of (1/lambda) u u^T (connected graph: drop the smallest)."""
    lam, U = np.linalg.eigh(L)
    return (U[:, 1:] / lam[1:]) @ U[:, 1:].T


def pinv_inverse(L):
    n = L.shape[0]
    J = np.full((n, n), 1.0 / n)
    return np.linalg.inv(L + J) - J


def lv_inv(L, v):
    """L_v^{-1} embedded back into n x n with zero row and column v."""
    n = L.shape[0]
    keep = np.array([i for i in range(n) if i != v])
    out = np.zeros((n, n))
    out[np.ix_(keep, keep)] = np.linalg.inv(L[np.ix_(keep, keep)])
    return out


def walk_green(L, v):
    """(I - P_v)^{-1} = L_v^{-1} D_v, embedded with zero row/col v.  Entry
    (s,u) is the expected number of departures from u of a walk started at
    s and absorbed at v (Lemma 1)."""
    d = np.diag(L)
    return lv_inv(L, v) * d[None, :]


def ldagger_thm1(Lvi, v):
    """Thm. 1: L^dagger = [I - 11^T/n; -1^T/n] L_v^{-1} [I - 11^T/n, -1/n],
    with the rows/columns of the block form placed back at index v."""
    n = Lvi.shape[0]
    keep = np.array([i for i in range(n) if i != v])
    M = Lvi[np.ix_(keep, keep)]
    k = n - 1
    left = np.vstack([np.eye(k) - np.ones((k, k)) / n, -np.ones((1, k)) / n])
    right = np.hstack([np.eye(k) - np.ones((k, k)) / n, -np.ones((k, 1)) / n])
    B = left @ M @ right
    perm = np.concatenate([keep, [v]])
    out = np.zeros((n, n))
    out[np.ix_(perm, perm)] = B
    return out


def ldagger_entry(Lvi, v, s, t):
    """The four element-wise cases after Thm. 1."""
    n = Lvi.shape[0]
    row = Lvi.sum(1)          # e_s^T L_v^{-1} 1 (zero at v)
    tot = Lvi.sum()           # 1^T L_v^{-1} 1
    if s == v and t == v:
        return tot / n**2
    if t == v:
        return -row[s] / n + tot / n**2
    if s == v:
        return -row[t] / n + tot / n**2
    if s == t:
        return Lvi[s, s] - 2.0 * row[s] / n + tot / n**2
    return Lvi[s, t] - row[s] / n - row[t] / n + tot / n**2


def closeness(Ld):
    n = Ld.shape[0]
    return (n - 1) / (np.trace(Ld) + n * np.diag(Ld))


def kemeny_spectral(g):
    """sum_{i>=2} 1/sigma_i over the normalised Laplacian I - D^{-1/2} A D^{-1/2}."""
    A = adjacency(g)
    d = A.sum(1)
    Dm = 1.0 / np.sqrt(d)
    NL = np.eye(g.n) - Dm[:, None] * A * Dm[None, :]
    sig = np.linalg.eigvalsh(NL)
    return float(np.sum(1.0 / sig[1:]))


def kemeny_hitting(g):
    """Definition by hitting times: sum_u pi(u) h(s,u), the same for every s.
    h(s,u) from the linear system of the walk absorbed at u.  Returns the
    vector over s (all equal for a correct implementation)."""
    A = adjacency(g)
    d = A.sum(1)
    P = A / d[:, None]
    pi = d / d.sum()
    n = g.n
    H = np.zeros((n, n))
    for u in range(n):
        keep = [i for i in range(n) if i != u]
        M = np.eye(n - 1) - P[np.ix_(keep, keep)]
        H[keep, u] = np.linalg.solve(M, np.ones(n - 1))
    return H @ pi


def kemeny_lemma(L, v):
    """Sec. 5 lemma: kappa = Tr((I-P_v)^{-1}) - (1/2m) d_v^T L_v^{-1} d_v."""
    d = np.diag(L).copy()
    N = walk_green(L, v)
    Lvi = lv_inv(L, v)
    dv = d.copy()
    dv[v] = 0.0
    return float(np.trace(N) - dv @ Lvi @ dv / d.sum())


def kirchhoff_pairs(Ld):
    """Kirchhoff index by its definition: sum over unordered pairs of r(s,t)."""
    n = Ld.shape[0]
    return float(sum(resistance(Ld, s, t) for s in range(n) for t in range(s + 1, n)))


def resistance(Ld, s, t):
    return Ld[s, s] + Ld[t, t] - 2.0 * Ld[s, t]


def expected_counts(g, v):
    """Exact expectations of the sampled integer counts (per sample / walk):
      draws[u]   of a Wilson sample:   N_uu          (Lemma 4 and Sec. 3.4)
      total draws of a Wilson sample:  Tr N          (Sec. 3.3, Sec. 5)
      visits[u] of a uniform-start v-absorbed walk: (1/n) sum_s N_su  (Lemma 5)
      length of a stationary-start walk: sum_s pi(s) h(s, v)         (Sec. 5)
    with N = (I - P_v)^{-1}."""
    L = laplacian(g)
    N = walk_green(L, v)
    d = np.diag(L)
    h = N.sum(1)                      # h(s, v); zero at v
    return dict(draws=np.diag(N).copy(), total=float(np.trace(N)),
                visits_uniform=N.sum(0) / g.n,
                len_uniform=float(h.mean()),
                len_stationary=float((d / d.sum()) @ h),
                N=N)
