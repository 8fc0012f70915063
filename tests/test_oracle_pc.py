"""Pins of the product-convolution oracle (FISTA-PC; Section 1's expansion,
Section 3.1's SVD construction, Table 1) against what the mathematics fixes:

* keeping every nonzero singular value reproduces Operator 1 exactly (the
  expansion is then an exact factorisation of the impulse responses);
* <H x, r> = <x, H^T r>;
* the u_k are orthonormal and the truncation error of S is the tail of its
  singular values (Eckart-Young);
* a unit kernel with a unit multiplier is the identity, a shifted unit
  kernel a periodic shift;
* FISTA-PC with the exact expansion reproduces the pinned FISTA-Spa oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import product_convolution as PC
import syninputs as SI

H6 = O.symmlet(6)


@pytest.fixture(scope="module")
def op32():
    kt, R = O.op1_profiles(32)
    return kt, R


def test_exact_expansion_is_operator1(op32):
    kt, R = op32
    u, v, sv = PC.pc_expansion(kt, R)
    vp = PC.rows_to_pixels(v, 24)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((32, 24))
    for tr in (False, True):
        ref = O.blur(x, kt, R, transpose=tr)
        assert np.abs(PC.apply_pc(u, vp, x, transpose=tr) - ref).max() < 1e-12


def test_adjoint_and_orthonormal(op32):
    kt, R = op32
    u, v, sv = PC.pc_expansion(kt, R, m=5)
    vp = PC.rows_to_pixels(v, 32)
    rng = np.random.default_rng(1)
    x, r = rng.standard_normal((2, 32, 32))
    a = float(np.sum(PC.apply_pc(u, vp, x) * r))
    b = float(np.sum(x * PC.apply_pc(u, vp, r, transpose=True)))
    assert abs(a - b) < 1e-12 * max(abs(a), 1.0)
    G = u.reshape(5, -1) @ u.reshape(5, -1).T
    assert np.abs(G - np.eye(5)).max() < 1e-13
    # singular values decreasing, positive
    assert np.all(np.diff(sv) <= 0) and sv[4] > 0


def test_truncation_error_is_the_singular_tail(op32):
    kt, R = op32
    S = PC.svir_rows(kt, R)
    for m in (1, 3, 5, 8):
        u, v, sv = PC.pc_expansion(kt, R, m=m)
        Sm = u.reshape(m, -1).T @ v
        err2 = float(np.sum((S - Sm) ** 2))
        assert abs(err2 - float(np.sum(sv[m:] ** 2))) < 1e-12 * max(float(np.sum(sv ** 2)), 1.0)


def test_unit_kernel_is_identity_and_shift():
    n2, n1 = 8, 12
    x = np.arange(n2 * n1, dtype=float).reshape(n2, n1)
    u = np.zeros((1, 3, 3))
    u[0, 1, 1] = 1.0
    v = np.ones((1, n2, n1))
    assert np.array_equal(PC.apply_pc(u, v, x), x)
    u2 = np.zeros((1, 3, 3))
    u2[0, 2, 1] = 1.0          # d = (d2, d1) = (1, 0): (u * x)(p) = x(p - (1, 0))
    out = PC.apply_pc(u2, v, x)
    assert np.array_equal(out, np.roll(x, 1, axis=0))
    assert np.array_equal(PC.apply_pc(u2, v, x, transpose=True), np.roll(x, -1, axis=0))


def test_fista_pc_exact_expansion_reproduces_fista_spa():
    n = 16
    kt, R = O.op1_profiles(n)
    c = SI.make_case(n, n, 1, 3, 2, "const", 0.05, 0.1, seed=21)
    pb = O.Problem(n, n, 1, c.levels, h=H6, w=O.expand_level_weights(c.level_w, n, n, c.levels))
    f0 = O.apply_H(pb, c.clean[0]) + c.noise[0]
    tau = O.step_size(pb)
    ref = O.fista(pb, f0[None], tau, 25, log=True)
    u, v, _ = PC.pc_expansion(kt, R)
    out = PC.fista_pc(u, PC.rows_to_pixels(v, n), H6, c.levels, f0, pb.w[0], tau, 25, log=True)
    assert np.abs(out["z"] - ref["z"][0]).max() < 1e-11
    np.testing.assert_allclose(out["log"], ref["log"], rtol=1e-10, atol=1e-13)


def test_operator_error_decreases_with_m(op32):
    kt, R = op32
    rng = np.random.default_rng(3)
    x = rng.standard_normal((32, 32))
    ref = O.blur(x, kt, R)
    errs = []
    for m in (1, 2, 5, 10):
        u, v, _ = PC.pc_expansion(kt, R, m=m)
        errs.append(float(np.linalg.norm(PC.apply_pc(u, PC.rows_to_pixels(v, 32), x) - ref)))
    assert all(b < a for a, b in zip(errs, errs[1:]))
