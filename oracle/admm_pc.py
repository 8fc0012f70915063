"""The oracle for ADMM with a product-convolution operator (ADMM-PC, Appendix
A.2 of Escande & Weiss, arXiv:2005.09870; Table 1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  Plain FP64 numpy;
shares nothing with the GPU library.

H = U V with U = (U_1 ... U_m) the convolutions by u_k and V = (V_1; ...; V_m)
the multipliers v_k.  With g = V f and z = Psi^* f the augmented Lagrangian
of eq. 4.1 is

  L = 1/2||U g - f0||^2 + ||z||_{1,w} + <xi, g - V f> + <zeta, z - Psi^* f>
      + beta1/2 ||g - V f||^2_D + beta2/2 ||z - Psi^* f||^2,  D = diag(gamma_k Id),

and one ADMM iteration is, in this order,

  g <- (U^T U + beta1 D)^-1 (U^T f0 - xi + beta1 D V f)
  z <- Prox_{||.||_{1,w}/beta2}(Psi^* f - zeta/beta2)
  f <- (beta1 sum_k gamma_k v_k^2 + beta2)^-1 (V^T (xi + beta1 D g) + Psi(beta2 z + zeta))
  xi <- xi + beta1 D (g - V f);   zeta <- zeta + beta2 (z - Psi^* f).

The g system is solved with the Woodbury identity: with A = beta1 D,
(U^T U + A)^-1 = A^-1 - A^-1 U^T (Id + U A^-1 U^T)^-1 U A^-1, where
Id + sum_k U_k U_k^T / (beta1 gamma_k) is diagonal in the Fourier basis.

Readings (the appendix is terse, and garbled in places):
* the printed Woodbury formula uses D_gamma^-1 alone and the middle matrix
  Id + sum_k gamma_k U_k U_k^*; the exact inverse of U^T U + beta1 D has
  (beta1 gamma_k)^-1 in both places, which is what is computed (the two agree
  for beta1 = 1 only in the first place);
* the printed f update writes x^(i) for f^(i);
* gamma_k = ||U_k||_2 (the largest |u_k^|) normalised to sum 1, as the
  appendix suggests; beta1 = beta2 = beta (a parameter);
* start: f = f0, g = V f0, z = Psi^* f0, xi = 0, zeta = 0;
* statistics per iteration: ||g - V f||^2_D, ||z - Psi^* f||^2 (the primal
  residuals) and ||z||_{1,w}.

Pins (tests/test_oracle_admm.py): the Woodbury/Fourier g-update equals a dense
solve of (U^T U + beta1 D) g = rhs; the f-update zeroes the f-gradient of L;
the Fourier multipliers of U_k match direct periodic convolution; the ADMM
limit equals the FISTA-PC limit (the same convex problem, different
algorithm) in energy.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def kernel_spectra(u: np.ndarray, n2: int, n1: int) -> np.ndarray:
    """u_k^ (m, n2, n1): the FFT of u_k placed at offsets (d2 mod n2, d1 mod n1)."""
    m, W, _ = u.shape
    R = W // 2
    pad = np.zeros((m, n2, n1))
    for a in range(W):
        for b in range(W):
            pad[:, (a - R) % n2, (b - R) % n1] += u[:, a, b]
    return np.fft.fft2(pad)


def gammas(uh: np.ndarray) -> np.ndarray:
    """gamma_k = ||U_k||_2 / sum_j ||U_j||_2 with ||U_k||_2 = max |u_k^|."""
    nr = np.abs(uh).reshape(uh.shape[0], -1).max(axis=1)
    return nr / nr.sum()


def conv(uh_k, g, transpose=False):
    """U_k g (or U_k^T g) for real g through the spectrum of u_k."""
    s = np.conj(uh_k) if transpose else uh_k
    return np.real(np.fft.ifft2(s * np.fft.fft2(g)))


def g_update(uh, gam, beta1, rhs):
    """(U^T U + beta1 D)^-1 rhs, rhs (m, n2, n1), by Woodbury in the Fourier basis."""
    a = rhs / (beta1 * gam)[:, None, None]
    th = np.sum(uh * np.fft.fft2(a), axis=0)
    mh = 1.0 + np.sum(np.abs(uh) ** 2 / (beta1 * gam)[:, None, None], axis=0)
    qh = th / mh
    corr = np.real(np.fft.ifft2(np.conj(uh) * qh[None]))
    return a - corr / (beta1 * gam)[:, None, None]


def admm_pc(u, v, h, levels, f0, w, beta, iters, log=False):
    """ADMM-PC on one (n2, n1) image; v per pixel (m, n2, n1).  Returns
    dict(f, z, log)."""
    f0 = np.asarray(f0, dtype=np.float64)
    n2, n1 = f0.shape
    uh = kernel_spectra(u, n2, n1)
    gam = gammas(uh)
    b1 = b2 = float(beta)
    Utf0 = np.stack([conv(uh[k], f0, transpose=True) for k in range(len(u))])
    f = f0.copy()
    g = v * f[None]
    z = O.fwt(f, levels, h)
    xi = np.zeros_like(g)
    zeta = np.zeros_like(z)
    den = b1 * np.sum(gam[:, None, None] * v * v, axis=0) + b2
    lg = np.zeros((iters, 3))
    for it in range(iters):
        g = g_update(uh, gam, b1, Utf0 - xi + b1 * gam[:, None, None] * v * f[None])
        vv = O.fwt(f, levels, h) - zeta / b2
        z = np.sign(vv) * np.maximum(np.abs(vv) - w / b2, 0.0)
        f = (np.sum(v * (xi + b1 * gam[:, None, None] * g), axis=0) + O.ifwt(b2 * z + zeta, levels, h)) / den
        rg = g - v * f[None]
        rz = z - O.fwt(f, levels, h)
        xi = xi + b1 * gam[:, None, None] * rg
        zeta = zeta + b2 * rz
        lg[it] = (float(np.sum(gam[:, None, None] * rg * rg)), float(np.sum(rz * rz)), float(np.sum(w * np.abs(z))))
    return {"f": f, "z": z, "log": lg if log else None}
