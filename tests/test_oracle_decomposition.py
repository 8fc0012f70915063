"""Pins of the Algorithm 1 oracle (Section 3.2, Algorithm 1; Section 5)
against what the mathematics fixes:

* the accuracy certificate ||Theta - Theta~||_2 <= eta, and ||A_k - A~_k||_2
  <= eps_k for each term, by exact spectral norms;
* eta = 0 with the full-rank expansion of Operator 1 reproduces the Theta of
  the wavelet-domain oracle, which is built from the C blur (another route);
* the sub-bands of A_k are circulant (Section 5.1): a source shifted by l'
  shifts a finer-or-equal target band by 2^(level' - level) l';
* B_k is symmetric, ||B_k||_2 = ||v_k||_inf, a constant multiplier gives c Id,
  and supp B_k lies in the support-intersection set I (Section 5.2) whose
  size obeys the per-row count bound;
* the Schur bound dominates the spectral norm and is tight for a diagonal.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import decomposition as D
from oracle import product_convolution as PC
from oracle import wavelet_domain as W

H6 = O.symmlet(6)


def _smooth_case(n2, n1, m, R, seed):
    """Random compact kernels and smooth positive multipliers (a non-separable
    product-convolution operator)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((m, 2 * R + 1, 2 * R + 1)) / (2 * R + 1)
    y2, y1 = np.meshgrid(np.arange(n2) / n2, np.arange(n1) / n1, indexing="ij")
    v = np.stack([1.0 + 0.5 * np.cos(2 * np.pi * (a * y1 + b * y2) + c)
                  for a, b, c in rng.uniform(0, 2, (m, 3))])
    return u, v


@pytest.fixture(scope="module")
def small():
    n2, n1, L = 16, 16, 2
    u, v = _smooth_case(n2, n1, 3, 2, 1)
    theta = D.wavelet_matrix(lambda x: PC.apply_pc(u, v, x), n2, n1, L, H6)
    return n2, n1, L, u, v, theta


@pytest.mark.parametrize("eta", [1e-3, 1e-2, 5e-2, 0.2])
def test_accuracy_certificate(small, eta):
    n2, n1, L, u, v, theta = small
    out = D.decompose(u, v, L, H6, eta)
    assert np.linalg.norm(theta - out["theta"], 2) <= eta * (1 + 1e-12)
    for k in range(len(u)):
        A = D.conv_matrix(u[k], n2, n1, L, H6)
        At, t = D.threshold(A, out["eps"][k])
        assert np.linalg.norm(A - At, 2) <= out["eps"][k] * (1 + 1e-12)
        assert t == out["t"][k]


def test_nnz_falls_with_eta(small):
    n2, n1, L, u, v, theta = small
    counts = [D.decompose(u, v, L, H6, eta)["nnz_a"].sum() for eta in (0.0, 1e-3, 1e-2, 1e-1)]
    assert all(b <= a for a, b in zip(counts, counts[1:])) and counts[-1] < counts[0]


def test_eta_zero_full_rank_operator1_is_theta():
    """The exact expansion of Operator 1 with eta = 0 gives Psi^* H Psi as
    built column by column from the C oracle's blur."""
    n = 16
    kt, R = O.op1_profiles(n)
    u, vr, _ = PC.pc_expansion(kt, R)
    v = PC.rows_to_pixels(vr, n)
    pb = O.Problem(n, n, 1, 2, h=H6)
    ref = W.theta_dense(pb)
    out = D.decompose(u, v, 2, H6, 0.0)
    assert np.abs(out["theta"] - ref).max() < 1e-11


def test_conv_subbands_are_circulant():
    n2, n1, L = 32, 32, 3
    rng = np.random.default_rng(2)
    u = rng.standard_normal((5, 5))
    A = D.conv_matrix(u, n2, n1, L, H6)
    bands = [(lev, o) for lev in range(1, L + 1) for o in (1, 2, 3)] + [(L, 0)]
    idx = lambda i2, i1: i2 * n1 + i1
    checked = 0
    for (ls, os_) in bands:
        s2, s1, g2, g1 = D.band_origin(ls, os_, n2, n1)
        col0 = A[:, idx(s2, s1)].reshape(n2, n1)
        for a2, a1 in ((1, 0), (0, 1), (g2 - 1, 3 % g1)):
            col = A[:, idx(s2 + a2, s1 + a1)].reshape(n2, n1)
            for (lt, ot) in bands:
                if lt > ls:
                    continue                       # coarser target: rows are the shifts
                t2, t1, h2, h1 = D.band_origin(lt, ot, n2, n1)
                f = 1 << (ls - lt)
                blk0 = col0[t2:t2 + h2, t1:t1 + h1]
                blk = col[t2:t2 + h2, t1:t1 + h1]
                assert np.abs(blk - np.roll(blk0, (f * a2, f * a1), axis=(0, 1))).max() < 1e-13
                checked += 1
    assert checked > 100


def test_mult_matrix_properties():
    n2, n1, L = 16, 16, 2
    _, v = _smooth_case(n2, n1, 1, 1, 3)
    B = D.mult_matrix(v[0], L, H6)
    assert np.abs(B - B.T).max() < 1e-13
    assert abs(np.linalg.norm(B, 2) - np.abs(v[0]).max()) < 1e-12
    assert np.abs(D.mult_matrix(np.full((n2, n1), 2.5), L, H6) - 2.5 * np.eye(n2 * n1)).max() < 1e-13


def test_mult_support_in_intersection_set():
    """B_k[lambda, mu] = 0 whenever supp psi_lambda and supp psi_mu are
    disjoint; the number of mu meeting a given lambda obeys the count bound
    (2 delta)^d ((2^d - 1) j + 2^(d (J - j))), delta = 6 for Symmlet-6."""
    n2 = n1 = 32
    L = 2
    N = n1 * n2
    psi = np.stack([O.ifwt(np.eye(N)[mu].reshape(n2, n1), L, H6).ravel() for mu in range(N)])
    S = (psi != 0.0).astype(np.int64)
    inter = (S @ S.T) > 0
    _, v = _smooth_case(n2, n1, 1, 1, 4)
    B = D.mult_matrix(v[0], L, H6)
    assert np.all(B[~inter] == 0.0)
    J, delta, d = 5, 6, 2
    for lam in range(0, N, 37):
        lev, _ = D.band_of(lam // n1, lam % n1, n2, n1, L)
        j = J - lev                                   # scale index: 0 coarsest ... J - 1 finest
        assert inter[lam].sum() <= (2 * delta) ** d * ((2 ** d - 1) * j + 2 ** (d * (J - j)))


def test_schur_bound():
    rng = np.random.default_rng(5)
    for _ in range(20):
        E = rng.standard_normal((30, 40)) * (rng.random((30, 40)) < 0.2)
        assert D.schur_bound(E) >= np.linalg.norm(E, 2) * (1 - 1e-12)
    dg = np.diag(rng.standard_normal(12))
    assert abs(D.schur_bound(dg) - np.linalg.norm(dg, 2)) < 1e-14
