"""Pins of the ADMM-PC oracle (Appendix A.2, Table 1) against what the
mathematics fixes: the Fourier spectra of the kernels reproduce direct
periodic convolution; the Woodbury / Fourier g-update is the exact solution
of its linear system (checked by a dense solve); the f-update zeroes the
f-gradient of the augmented Lagrangian; and the ADMM limit is the minimiser
FISTA-PC reaches (same convex problem, different algorithm)."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import product_convolution as PC
from oracle import admm_pc as A
import syninputs as SI

H6 = O.symmlet(6)


def _pc(n1, n2, m):
    kt, R = O.op1_profiles(n2)
    u, v, _ = PC.pc_expansion(kt, R, m=m)
    return u, PC.rows_to_pixels(v, n1)


def test_spectra_are_periodic_convolution():
    u, v = _pc(24, 16, 3)
    uh = A.kernel_spectra(u, 16, 24)
    rng = np.random.default_rng(0)
    g = rng.standard_normal((16, 24))
    for k in range(3):
        one = np.ones((1, 16, 24))
        for tr in (False, True):
            ref = PC.apply_pc(u[k:k + 1], one, g, transpose=tr)
            assert np.abs(A.conv(uh[k], g, transpose=tr) - ref).max() < 1e-12


def test_g_update_solves_its_system():
    n2, n1, m = 8, 8, 2
    u, v = _pc(n1, n2, m)
    uh = A.kernel_spectra(u, n2, n1)
    gam = A.gammas(uh)
    assert abs(gam.sum() - 1.0) < 1e-15
    N = n1 * n2
    # dense U_k, column by column
    Us = []
    for k in range(m):
        cols = [A.conv(uh[k], np.eye(N)[j].reshape(n2, n1)).ravel() for j in range(N)]
        Us.append(np.stack(cols, axis=1))
    U = np.concatenate(Us, axis=1)                      # N x mN
    beta1 = 0.7
    D = np.kron(np.diag(gam), np.eye(N))
    rng = np.random.default_rng(1)
    rhs = rng.standard_normal((m, n2, n1))
    ref = np.linalg.solve(U.T @ U + beta1 * D, rhs.reshape(-1))
    got = A.g_update(uh, gam, beta1, rhs).reshape(-1)
    assert np.abs(got - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_f_update_zeroes_the_gradient():
    n, m, L = 16, 3, 4
    u, v = _pc(n, n, m)
    uh = A.kernel_spectra(u, n, n)
    gam = A.gammas(uh)
    rng = np.random.default_rng(2)
    g, xi = rng.standard_normal((2, m, n, n))
    z, zeta = rng.standard_normal((2, n, n))
    b1 = b2 = 1.3
    den = b1 * np.sum(gam[:, None, None] * v * v, axis=0) + b2
    f = (np.sum(v * (xi + b1 * gam[:, None, None] * g), axis=0) + O.ifwt(b2 * z + zeta, L, H6)) / den
    # dL/df = -V^T xi - Psi zeta - beta1 V^T D (g - V f) - beta2 Psi (z - Psi^* f)
    grad = (-np.sum(v * xi, axis=0) - O.ifwt(zeta, L, H6)
            - b1 * np.sum(v * gam[:, None, None] * (g - v * f[None]), axis=0)
            - b2 * O.ifwt(z - O.fwt(f, L, H6), L, H6))
    assert np.abs(grad).max() < 1e-12


def test_admm_limit_is_the_minimiser():
    """The ADMM limit against an independent minimiser: coordinate descent
    (with an exact active-set solve) on the dense matrix H Psi."""
    import scipy.sparse as sp
    from oracle import wavelet_domain as W
    n, m, L = 16, 3, 4
    u, v = _pc(n, n, m)
    c = SI.make_case(n, n, 1, 3, 2, "const", 0.05, 0.1, levels=L, seed=5)
    f0 = PC.apply_pc(u, v, c.clean[0]) + c.noise[0]
    w = O.expand_level_weights(c.level_w, n, n, L)[0]
    N = n * n
    HPsi = np.stack([PC.apply_pc(u, v, O.ifwt(np.eye(N)[j].reshape(n, n), L, H6)).ravel() for j in range(N)], axis=1)
    zs = W.lasso_cd(sp.csr_matrix(HPsi), f0.ravel(), w.ravel())
    estar = W.energy_w(sp.csr_matrix(HPsi), f0.ravel(), w.ravel(), zs)
    ad = A.admm_pc(u, v, H6, L, f0, w, 1.0, 3000, log=True)
    za = O.fwt(ad["f"], L, H6).ravel()
    ea = W.energy_w(sp.csr_matrix(HPsi), f0.ravel(), w.ravel(), za)
    assert abs(ea - estar) < 1e-8 * estar
    assert np.abs(za - zs).max() < 1e-5
    assert ad["log"][-1, 0] < 1e-14 and ad["log"][-1, 1] < 1e-14   # primal residuals vanish
