"""The oracle for Algorithm 1 of Escande & Weiss (arXiv:2005.09870, Section
3.2, Algorithm 1; Section 5): the wavelet representation of a
product-convolution operator H = sum_k U_k V_k, decomposed term by term.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  Plain dense FP64
numpy for small images (N = n1 n2 up to a few thousand); it shares nothing
with the GPU library.

With U_k the periodic convolution by u_k and V_k = diag(v_k),

    Theta = Psi^* H Psi = sum_k A_k B_k,   A_k = Psi^* U_k Psi,   B_k = Psi^* V_k Psi,

because Psi Psi^* = Id.  Algorithm 1 sets eps_k = eta / (m ||v_k||_inf),
replaces each A_k by a thresholded A~_k with ||A_k - A~_k||_2 <= eps_k and
returns Theta~ = sum_k A~_k B_k; since ||B_k||_2 = ||v_k||_inf (Psi is
orthogonal), ||Theta - Theta~||_2 <= eta (Section 5, the accuracy lemma).

Readings:
* the threshold of A_k is not specified beyond its accuracy; here A~_k keeps
  the entries with |a| > t_k, t_k the largest entry magnitude of A_k whose
  dropped part E satisfies the Schur test sqrt(||E||_1 ||E||_inf) <= eps_k
  (max column sum times max row sum of |E|), a certified bound on ||E||_2;
* matrices are indexed by Mallat-layout coefficients flattened row-major
  (i2 n1 + i1), the same layout as the transforms of the FISTA-Spa oracle;
* the dense construction column by column (each column one synthesis, one
  operator application and one analysis) stands in for the fast
  constructions of Section 5 (circulant sub-bands of A_k, sparse cascade for
  B_k, sparse products): it computes the same matrices.

parity unpinned: the nnz counts of the paper's Tables 2-3 (its image size,
its operators) are not reproduced.

Pins (tests/test_oracle_decomposition.py): the certificate ||Theta -
Theta~||_2 <= eta and ||A_k - A~_k||_2 <= eps_k by exact spectral norms; eta
= 0 with the full-rank expansion of Operator 1 gives the Theta of the
FISTA-W oracle (built from the C blur); the circulant sub-band structure of
A_k (Section 5.1); B_k symmetric with ||B_k||_2 = ||v_k||_inf and B = c Id
for a constant multiplier; supp B_k inside the support-intersection set I;
the Schur bound dominates the spectral norm.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from oracle import product_convolution as PC


def wavelet_matrix(apply, n2: int, n1: int, levels: int, h) -> np.ndarray:
    """Psi^* G Psi as a dense (N, N) matrix: column mu = Psi^* G Psi e_mu."""
    N = n1 * n2
    M = np.zeros((N, N))
    for mu in range(N):
        e = np.zeros(N)
        e[mu] = 1.0
        M[:, mu] = O.fwt(apply(O.ifwt(e.reshape(n2, n1), levels, h)), levels, h).ravel()
    return M


def conv_matrix(u_k: np.ndarray, n2: int, n1: int, levels: int, h) -> np.ndarray:
    """A_k = Psi^* U_k Psi for the periodic convolution by u_k (2R+1, 2R+1)."""
    ones = np.ones((1, n2, n1))
    return wavelet_matrix(lambda x: PC.apply_pc(u_k[None], ones, x), n2, n1, levels, h)


def mult_matrix(v_k: np.ndarray, levels: int, h) -> np.ndarray:
    """B_k = Psi^* diag(v_k) Psi for a per-pixel multiplier v_k (n2, n1)."""
    n2, n1 = v_k.shape
    return wavelet_matrix(lambda x: v_k * x, n2, n1, levels, h)


def schur_bound(E: np.ndarray) -> float:
    """sqrt(max column sum * max row sum) of |E|, an upper bound of ||E||_2."""
    a = np.abs(E)
    return float(np.sqrt(a.sum(axis=0).max() * a.sum(axis=1).max())) if a.size else 0.0


def threshold(A: np.ndarray, eps: float):
    """(A~, t): A~ keeps the entries of A with |a| > t, t the largest entry
    magnitude (or 0) whose dropped part has a Schur bound <= eps."""
    mags = np.unique(np.abs(A[A != 0]))
    best = 0.0
    lo, hi = 0, len(mags) - 1
    while lo <= hi:                       # the bound grows with t: bisect over the sorted magnitudes
        mid = (lo + hi) // 2
        t = float(mags[mid])
        if schur_bound(np.where(np.abs(A) <= t, A, 0.0)) <= eps:
            best = t
            lo = mid + 1
        else:
            hi = mid - 1
    return np.where(np.abs(A) > best, A, 0.0), best


def decompose(u: np.ndarray, v: np.ndarray, levels: int, h, eta: float):
    """Algorithm 1: Theta~ = sum_k A~_k B_k with eps_k = eta / (m ||v_k||_inf).
    u (m, 2R+1, 2R+1), v (m, n2, n1).  Returns dict(theta, eps, t, nnz_a)."""
    m, n2, n1 = v.shape
    theta = np.zeros((n1 * n2, n1 * n2))
    eps, ts, nnz_a = [], [], []
    for k in range(m):
        vinf = float(np.abs(v[k]).max())
        e_k = eta / (m * vinf) if vinf > 0 else np.inf
        A = conv_matrix(u[k], n2, n1, levels, h)
        At, t = threshold(A, e_k) if np.isfinite(e_k) else (np.zeros_like(A), np.inf)
        B = mult_matrix(v[k], levels, h)
        theta += At @ B
        eps.append(e_k)
        ts.append(t)
        nnz_a.append(int(np.count_nonzero(At)))
    return {"theta": theta, "eps": np.array(eps), "t": np.array(ts), "nnz_a": np.array(nnz_a)}


def band_of(i2: int, i1: int, n2: int, n1: int, levels: int):
    """(level, orientation) of a Mallat-layout position: level 1 finest ...
    levels, orientation 1..3 for details, (levels, 0) for the approximation."""
    for lev in range(1, levels + 1):
        h2, h1 = n2 >> lev, n1 >> lev
        if i2 >= h2 or i1 >= h1:
            return lev, (1 if i2 < h2 else (2 if i1 < h1 else 3))
    return levels, 0


def band_origin(lev: int, ori: int, n2: int, n1: int):
    """Top-left Mallat position of band (lev, ori) and its grid size."""
    h2, h1 = n2 >> lev, n1 >> lev
    o2 = h2 if ori in (2, 3) else 0
    o1 = h1 if ori in (1, 3) else 0
    return o2, o1, h2, h1
