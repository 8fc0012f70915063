"""The oracle for FISTA with a product-convolution operator (FISTA-PC).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  Plain FP64 numpy,
written from the paper (Escande & Weiss, arXiv:2005.09870); it shares
nothing with the GPU library.

A product-convolution expansion (Section 1, the expansion H f = sum_k
u_k * (v_k . f); Section 3.1 on how to obtain it) approximates an integral
operator G f(x) = sum_y K(x, y) f(y) through its space-varying impulse
responses S(., y) = K(. + y, y): if S(d, y) ~ sum_k u_k(d) v_k(y), then

    H f(x) = sum_k sum_y u_k(x - y) v_k(y) f(y) = sum_k (u_k * (v_k . f))(x),

with * the periodic convolution (u * g)(x) = sum_d u(d) g(x - d).  The
optimal rank-m pair in Frobenius norm comes from the truncated SVD of the
matrix S (Section 3.1; the paper uses a randomized SVD, the oracle an exact
one).  For Operator 1 of Section 4.1 the impulse response of source y is
the outer product of row y2's profile with itself, so S has only n2 distinct
columns and v_k(y) depends on y2 only.

Readings:
* S rows are indexed by the offset d = (d2, d1) in [-R, R]^2 (row-major,
  d2 slowest), columns by the source pixel; the SVD of the n2 distinct
  columns gives the same u_k, and v_k(y) = <S(., y), u_k>.
* H^T r = sum_k v_k . (u_k (x) r) with the correlation (u (x) r)(y) =
  sum_d u(d) r(y + d).
* FISTA-PC is the FISTA-Spa recursion of Appendix A.1 with H replaced by
  its expansion (Table 1), everything else unchanged.

Pins (tests/test_oracle_pc.py): the full-rank expansion is Operator 1
exactly; adjointness; orthonormal u_k; the Eckart-Young error of the
truncation; FISTA-PC with the full-rank expansion reproduces the pinned
FISTA-Spa oracle iterate by iterate; a unit kernel with unit multiplier is
the identity.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def svir_rows(kt: np.ndarray, R: int) -> np.ndarray:
    """Distinct columns of Operator 1's S: column i2 is the (2R+1)^2 response
    of source row i2 (row-major in (d2, d1)): kt[i2, d2+R] * kt[i2, d1+R]."""
    kt = np.asarray(kt, dtype=np.float64)
    return np.einsum("ia,ib->abi", kt, kt).reshape((2 * R + 1) ** 2, kt.shape[0])


def pc_expansion(kt: np.ndarray, R: int, m: int | None = None, rtol: float = 1e-14):
    """(u, v, sing): u (m, 2R+1, 2R+1) orthonormal kernels, v (m, n2) row
    multipliers, sing the singular values of S's distinct columns.  m None:
    every singular value above rtol * the largest (the exact expansion)."""
    S = svir_rows(kt, R)
    U, sv, _ = np.linalg.svd(S, full_matrices=False)
    if m is None:
        m = int(np.sum(sv > rtol * sv[0]))
    u = U[:, :m].T.copy()
    v = u @ S                      # v_k(i2) = <S(., i2), u_k>
    return u.reshape(m, 2 * R + 1, 2 * R + 1), v, sv


def rows_to_pixels(v: np.ndarray, n1: int) -> np.ndarray:
    """Per-row multipliers (m, n2) as per-pixel planes (m, n2, n1)."""
    return np.repeat(np.asarray(v, dtype=np.float64)[:, :, None], n1, axis=2)


def apply_pc(u: np.ndarray, v: np.ndarray, x: np.ndarray, transpose: bool = False) -> np.ndarray:
    """H x = sum_k u_k * (v_k . x), or H^T x = sum_k v_k . (u_k (x) x), on an
    (n2, n1) image with periodic boundaries; v per pixel (m, n2, n1)."""
    x = np.asarray(x, dtype=np.float64)
    m, W, _ = u.shape
    R = W // 2
    out = np.zeros_like(x)
    for k in range(m):
        g = x if transpose else v[k] * x
        acc = np.zeros_like(x)
        for a in range(W):
            for b in range(W):
                d2, d1 = a - R, b - R
                # convolution: g(x - d) = roll by +d; correlation: g(y + d) = roll by -d
                sh = (-d2, -d1) if transpose else (d2, d1)
                acc += u[k, a, b] * np.roll(g, sh, axis=(0, 1))
        out += v[k] * acc if transpose else acc
    return out


def fista_pc(u, v, h, levels, f0, w, tau, iters, log=False):
    """FISTA (Appendix A.1) on 1/2||H z - f0||^2 + ||z||_{1,w} in coefficient
    form with H the product-convolution expansion; z(0) = y(1) = Psi^* f0.
    Returns dict(z = z(K), f = Psi z(K), log) with log row i holding
    1/2||H Psi y(i) - f0||^2, sum w |y(i)|, ||z(i) - y(i)||^2."""
    f0 = np.asarray(f0, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    z = O.fwt(f0, levels, h)
    zp = z.copy()
    lg = np.zeros((iters, 3))
    for it in range(iters):
        i = it + 1
        beta = (i - 2) / (i + 1) if i >= 2 else 0.0
        y = z + beta * (z - zp)
        r = apply_pc(u, v, O.ifwt(y, levels, h)) - f0
        g = O.fwt(apply_pc(u, v, r, transpose=True), levels, h)
        vv = y - tau * g
        zn = np.sign(vv) * np.maximum(np.abs(vv) - tau * w, 0.0)
        lg[it] = (0.5 * float(np.sum(r * r)), float(np.sum(w * np.abs(y))), float(np.sum((zn - y) ** 2)))
        zp, z = z, zn
    return {"z": z, "f": O.ifwt(z, levels, h), "log": lg if log else None}


def lipschitz_pc(u, v, shape, iters: int = 300, seed: int = 0) -> float:
    """||H^T H||_2 by power iteration."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = apply_pc(u, v, apply_pc(u, v, x), transpose=True)
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam
