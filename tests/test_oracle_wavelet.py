"""Pins of the wavelet-domain FISTA oracle (FISTA-W / FISTA-WP, Section 4.3 and
Appendix A.1) against what the mathematics fixes:

* Theta = Psi^* H Psi is the identity for H = Id (Psi orthonormal, Section 2.2);
* with the untruncated Theta the wavelet-domain iteration IS FISTA-Spa
  (Theta^T (Theta y - Psi^* f0) = Psi^* H^T (H Psi y - f0) since Psi Psi^* = Id),
  so it must reproduce the pinned spatial-operator oracle iterate by iterate;
* a diagonal Theta_L decouples the problem; FISTA-WP with tau = 1 lands on the
  closed-form minimiser in one step;
* FISTA-WP is FISTA-W on the rescaled matrix Theta_L Sigma^{1/2};
* the limit equals an independent coordinate-descent minimiser;
* the step-size power iteration agrees with a dense symmetric eigensolver.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from oracle import wavelet_domain as W
import syninputs as SI

H6 = O.symmlet(6)


def _pb(n1=16, n2=16, levels=None, op="op1"):
    return O.Problem(n1, n2, 1, levels, h=H6, op=op)


@pytest.fixture(scope="module")
def theta16():
    pb = _pb()
    return pb, W.theta_dense(pb)


def _case(pb, seed=0, lam=0.05):
    c = SI.make_case(pb.n1, pb.n2, 1, 3, 2, "const", 0.05, lam, levels=pb.levels, seed=seed)
    f0 = O.apply_H(pb, c.clean[0]) + c.noise[0]
    w = O.expand_level_weights(c.level_w, pb.n1, pb.n2, pb.levels)[0]
    return f0, w


def test_theta_identity_operator():
    """H = Id: Theta = Psi^* Psi = Id (orthonormal basis, Section 2.2)."""
    pb = _pb(16, 8, 3, op="identity")
    T = W.theta_dense(pb)
    assert np.abs(T - np.eye(T.shape[0])).max() < 1e-12


def test_theta_columns_are_the_operator(theta16):
    """Column assembly: Theta x equals Psi^* H Psi x applied to whole vectors."""
    pb, T = theta16
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.standard_normal((pb.n2, pb.n1))
        direct = O.fwt(O.apply_H(pb, O.ifwt(x, pb.levels, pb.h)), pb.levels, pb.h).ravel()
        assert np.abs(T @ x.ravel() - direct).max() < 1e-12
    # H is not symmetric (the response depends on the source row), nor is Theta
    assert np.abs(T - T.T).max() > 1e-3


def test_full_theta_reproduces_fista_spa(theta16):
    """Untruncated Theta: FISTA-W = FISTA-Spa (App. A.1), iterate by iterate,
    energy terms included (||Theta y - z0|| = ||H Psi y - f0||)."""
    pb, T = theta16
    f0, w = _case(pb)
    pb.w = np.ascontiguousarray(w[None])
    tau = O.step_size(pb)
    ref = O.fista(pb, f0[None], tau, 40, log=True)
    m = sp.csr_matrix(T)
    z0 = O.fwt(f0, pb.levels, pb.h).ravel()
    out = W.fista_w(m, z0, w.ravel(), tau, 40, log=True)
    assert np.abs(out["z"] - ref["z"].ravel()).max() < 1e-11
    np.testing.assert_allclose(out["log"], ref["log"], rtol=1e-10, atol=1e-13)


def test_sparsify_keeps_the_largest(theta16):
    _, T = theta16
    N = T.shape[0]
    m = W.sparsify(T, 8 * N)
    assert m.nnz >= 8 * N
    kept = np.abs(m.data).min()
    dropped = np.abs(T - m.toarray())
    assert dropped.max() <= kept
    assert np.all(np.diff(m.indptr) >= 0) and m.has_sorted_indices


def test_jacobi_sigma_inverts_the_diagonal(theta16):
    _, T = theta16
    m = W.sparsify(T, 8 * T.shape[0])
    s = W.jacobi_sigma(m)
    d = np.diag(m.T @ m.toarray())
    nz = d > 0   # the blur all but removes the finest x1 detail under its widest rows
    np.testing.assert_allclose(s[nz] * d[nz], 1.0, rtol=1e-13)
    assert np.all(s[~nz] == 1.0)
    # an empty column gets sigma = 1
    m2 = sp.csr_matrix(np.diag([2.0, 0.0, 3.0]))
    np.testing.assert_allclose(W.jacobi_sigma(m2), [0.25, 1.0, 1.0 / 9.0])


def test_power_iteration_matches_eigensolver(theta16):
    _, T = theta16
    m = W.sparsify(T, 8 * T.shape[0])
    s = W.jacobi_sigma(m)
    A = m.toarray()
    for sig in (None, s):
        S = np.ones(A.shape[1]) if sig is None else np.sqrt(sig)
        M = (A * S[None, :]).T @ (A * S[None, :])
        lam = np.linalg.eigvalsh(M).max()
        assert abs(W.lipschitz(m, sig, iters=2000) - lam) < 1e-8 * lam


def test_diagonal_theta_one_step():
    """Diagonal Theta_L = diag(d): FISTA-WP with tau = 1 (Sigma^{1/2} Theta^T
    Theta Sigma^{1/2} = Id) gives z(1) = S(z0/d, w/d^2), the exact minimiser
    of sum 1/2 (d z - z0)^2 + w |z|, and stays there."""
    rng = np.random.default_rng(3)
    n = 200
    d = rng.uniform(0.2, 2.0, n) * rng.choice([-1.0, 1.0], n)
    z0 = rng.standard_normal(n)
    w = rng.uniform(0.0, 0.5, n)
    m = sp.csr_matrix(np.diag(d))
    s = W.jacobi_sigma(m)
    exact = np.sign(z0 / d) * np.maximum(np.abs(z0 / d) - w / d ** 2, 0.0)
    assert abs(W.lipschitz(m, s, iters=5) - 1.0) < 1e-14
    for K in (1, 5):
        out = W.fista_w(m, z0, w, 1.0, K, sigma=s)
        assert np.abs(out["z"] - exact).max() < 1e-14


def test_preconditioned_is_rescaled_plain(theta16):
    """FISTA-WP on (Theta_L, w) = Sigma^{1/2} x FISTA-W on (Theta_L Sigma^{1/2},
    w Sigma^{1/2}) started from Sigma^{-1/2} z0."""
    pb, T = theta16
    f0, w = _case(pb, seed=2)
    m = W.sparsify(T, 8 * T.shape[0])
    s = W.jacobi_sigma(m)
    tau = W.step_size(m, s)
    z0 = O.fwt(f0, pb.levels, pb.h).ravel()
    wp = W.fista_w(m, z0, w.ravel(), tau, 60, sigma=s, log=True)
    r = np.sqrt(s)
    ms = sp.csr_matrix(m.toarray() * r[None, :])
    u0 = z0 / r
    pl = W.fista_w(ms, z0, w.ravel() * r, tau, 60, init=(u0, u0, 0), log=True)
    assert np.abs(wp["z"] - r * pl["z"]).max() < 1e-11 * np.abs(wp["z"]).max()
    np.testing.assert_allclose(wp["log"][:, :2], pl["log"][:, :2], rtol=1e-10)


@pytest.mark.parametrize("precond", [False, True])
def test_limit_is_the_minimiser(theta16, precond):
    """Run to convergence; compare with coordinate descent (independent code)."""
    pb, T = theta16
    f0, w = _case(pb, seed=4, lam=0.1)
    m = W.sparsify(T, 8 * T.shape[0])
    s = W.jacobi_sigma(m) if precond else None
    tau = W.step_size(m, s)
    z0 = O.fwt(f0, pb.levels, pb.h).ravel()
    zf = W.fista_w(m, z0, w.ravel(), tau, 6000, sigma=s)["z"]
    zc = W.lasso_cd(m, z0, w.ravel())
    ef, ec = W.energy_w(m, z0, w, zf), W.energy_w(m, z0, w, zc)
    assert abs(ef - ec) < 1e-10 * abs(ec)
    assert np.abs(zf - zc).max() < 1e-6

