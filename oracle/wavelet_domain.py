"""The oracle for FISTA in the wavelet domain (FISTA-W and FISTA-WP).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  Plain FP64 numpy /
scipy, written from the paper (Escande & Weiss, arXiv:2005.09870); it shares
nothing with the GPU library.

Section 4.3 replaces eq. 4.1 by its approximation in the wavelet domain,

    argmin_z  1/2 || Theta_L z - z0 ||^2 + ||z||_{1,w},   z0 = Psi^* f0,

with Theta_L an L-sparse approximation of Theta = Psi^* H Psi.  Appendix A.1
solves it by FISTA with a diagonal preconditioner Sigma:

    z(i)   = Prox^Sigma_{tau ||.||_{1,w}}( y(i) - tau Sigma Theta_L^T (Theta_L y(i) - z0) )
    y(i+1) = z(i) + (i-1)/(i+2) (z(i) - z(i-1)),

Sigma = Id ("FISTA-W") or the Jacobi preconditioner built from
diag(Theta_L^T Theta_L) ("FISTA-WP").  Readings (the paper is terse here):

* Prox^Sigma is the proximal map in the metric of Sigma^{-1}; for the weighted
  l1 norm it is soft-thresholding of coefficient l at tau * sigma_l * w_l.
* The Jacobi preconditioner is the INVERSE of the diagonal,
  sigma_l = 1 / sum_m Theta_L[m, l]^2 (a Jacobi step divides by the diagonal);
  a column of Theta_L that is entirely zero gets sigma_l = 1.
* tau <= 1 / ||Sigma^{1/2} Theta_L^T Theta_L Sigma^{1/2}||_2 (the step bound of
  the preconditioned problem), found by power iteration.
* Theta_L keeps the L entries of Theta of largest magnitude (every entry at
  least as large as the L-th largest), the rest set to zero.
* z(0) = y(1) = z0 unless the caller passes an initial state.

Parity pins (tests/test_oracle_wavelet.py): with Theta_L = Theta the
iteration is FISTA-Spa exactly; H = Id gives Theta = Id; a diagonal Theta_L is
solved in one preconditioned step; FISTA-WP equals FISTA-W on the rescaled
matrix Theta_L Sigma^{1/2}; the limit point equals an independent coordinate
descent minimiser; the power iteration matches a dense eigensolver.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle import oracle as O


def theta_dense(pb: O.Problem) -> np.ndarray:
    """Theta = Psi^* H Psi (N x N, N = n1 n2, single channel), column mu being
    Psi^* H Psi applied to the unit coefficient vector e_mu (Mallat order,
    row-major in the n2 x n1 plane)."""
    n1, n2 = pb.n1, pb.n2
    N = n1 * n2
    E = np.eye(N).reshape(N, n2, n1)
    X = O.ifwt(E, pb.levels, pb.h)
    Y = np.stack([O.apply_H(pb, X[k]) for k in range(N)])
    T = O.fwt(Y, pb.levels, pb.h).reshape(N, N)
    return np.ascontiguousarray(T.T)


def sparsify(theta: np.ndarray, L: int) -> sp.csr_matrix:
    """Theta_L: the entries of largest magnitude, at least L of them (ties at
    the L-th magnitude are all kept), as CSR with sorted column indices."""
    a = np.abs(theta)
    L = int(min(max(L, 1), a.size))
    thr = np.partition(a.ravel(), a.size - L)[a.size - L]
    keep = (a >= thr) & (a > 0)
    m = sp.csr_matrix(np.where(keep, theta, 0.0))
    m.sort_indices()
    return m


def csr_arrays(m: sp.csr_matrix):
    """(row_ptr int64, col int32, val float64) of a CSR matrix."""
    m = sp.csr_matrix(m)
    m.sort_indices()
    return (m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data.astype(np.float64))


def transpose(m: sp.csr_matrix) -> sp.csr_matrix:
    t = sp.csr_matrix(m.T)
    t.sort_indices()
    return t


def jacobi_sigma(m: sp.csr_matrix) -> np.ndarray:
    """sigma_l = 1 / (Theta_L^T Theta_L)[l, l] = 1 / sum_m Theta_L[m, l]^2, or 1
    for an empty column."""
    d = np.asarray(m.multiply(m).sum(axis=0)).ravel()
    out = np.ones_like(d)
    nz = d > 0
    out[nz] = 1.0 / d[nz]
    return out


def lipschitz(m: sp.csr_matrix, sigma=None, iters: int = 300, seed: int = 0) -> float:
    """||Sigma^{1/2} Theta_L^T Theta_L Sigma^{1/2}||_2 by power iteration."""
    n = m.shape[1]
    s = np.ones(n) if sigma is None else np.sqrt(sigma)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    x /= np.linalg.norm(x)
    lam = 0.0
    mt = m.T.tocsr()
    for _ in range(iters):
        y = s * (mt @ (m @ (s * x)))
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam


def step_size(m: sp.csr_matrix, sigma=None) -> float:
    return 1.0 / (lipschitz(m, sigma) * (1.0 + 1e-6))


def soft(v, t):
    """Soft-thresholding: sign(v) max(|v| - t, 0), zero on |v| <= t."""
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def fista_w(m: sp.csr_matrix, z0, w, tau, iters, sigma=None, init=None, log=False):
    """FISTA on the wavelet-domain problem.  m: Theta_L (N x N CSR); z0, w:
    length-N vectors (Mallat order); sigma: None (FISTA-W) or the diagonal of
    Sigma (FISTA-WP).  init: None (z(0) = z0) or (z(k), z(k-1), k) to resume at
    global iteration k.  Returns dict(z = z(K), z_prev = z(K-1), log) where log
    row i holds 1/2||Theta_L y(i) - z0||^2, sum w |y(i)|, ||z(i) - y(i)||^2."""
    z0 = np.asarray(z0, dtype=np.float64).ravel()
    w = np.asarray(w, dtype=np.float64).ravel()
    s = np.ones_like(z0) if sigma is None else np.asarray(sigma, dtype=np.float64).ravel()
    mt = m.T.tocsr()
    if init is None:
        z, zp, k0 = z0.copy(), z0.copy(), 0
    else:
        z, zp, k0 = np.array(init[0], dtype=np.float64).ravel(), np.array(init[1], dtype=np.float64).ravel(), init[2]
    lg = np.zeros((iters, 3))
    for it in range(iters):
        i = k0 + it + 1
        # y(i) = z(i-1) + (i-2)/(i+1) (z(i-1) - z(i-2)), and y(1) = z(0)
        beta = (i - 2) / (i + 1) if i >= 2 else 0.0
        y = z + beta * (z - zp)
        r = m @ y - z0
        g = mt @ r
        zn = soft(y - tau * s * g, tau * s * w)
        lg[it] = (0.5 * float(r @ r), float(np.sum(w * np.abs(y))), float(np.sum((zn - y) ** 2)))
        zp, z = z, zn
    return {"z": z, "z_prev": zp, "log": lg if log else None}


def energy_w(m: sp.csr_matrix, z0, w, z) -> float:
    r = m @ z - np.asarray(z0).ravel()
    return 0.5 * float(r @ r) + float(np.sum(np.asarray(w).ravel() * np.abs(z)))


def lasso_cd(m: sp.csr_matrix, z0, w, sweeps: int = 50000, tol: float = 1e-15):
    """Independent minimiser of 1/2||Theta_L z - z0||^2 + sum w |z| by cyclic
    coordinate descent on the dense matrix, then an exact solve of the
    optimality system on the detected support and signs."""
    A = m.toarray()
    b = np.asarray(z0, dtype=np.float64).ravel()
    w = np.asarray(w, dtype=np.float64).ravel()
    N = A.shape[1]
    z = np.zeros(N)
    r = b.copy()
    col2 = np.sum(A * A, 0)
    for _ in range(sweeps):
        zmax = 0.0
        for j in range(N):
            if col2[j] == 0.0:
                continue
            aj = A[:, j]
            u = z[j] + aj @ r / col2[j]
            zn = np.sign(u) * max(abs(u) - w[j] / col2[j], 0.0)
            if zn != z[j]:
                r -= aj * (zn - z[j])
                zmax = max(zmax, abs(zn - z[j]))
                z[j] = zn
        if zmax < tol:
            break
    S = np.nonzero(z)[0]
    AS = A[:, S]
    zz = np.zeros(N)
    zz[S] = np.linalg.solve(AS.T @ AS, AS.T @ b - w[S] * np.sign(z[S]))
    return zz
