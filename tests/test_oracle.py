"""Pins of the oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them compares the oracle
with itself: they use hand-computed worked examples (tests/golden), closed
forms, textbook special cases (FFT convolution, soft-thresholding), algebraic
invariants (orthonormality, adjointness, vanishing moments) and an independent
minimiser (coordinate descent + exact active-set solve) on tiny images.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

H6 = O.symmlet(6)
HAAR = O.symmlet(1)


def _g(h):
    """High-pass filter of Section 2.1 as (k, g[k]) for k in [2-L, 1]."""
    L = len(h)
    ks = np.arange(2 - L, 2)
    return ks, np.array([(-1.0) ** (1 - k) * h[1 - k] for k in ks])


# ---------------------------------------------------------------- filters --
def test_symmlet_filter_identities():
    """P3 (Section 2.1): sum h = sqrt 2, orthonormal even shifts, exactly 6
    vanishing moments of g, support length 2M = 12."""
    h = H6
    assert len(h) == 12
    assert abs(h.sum() - math.sqrt(2.0)) < 1e-14
    for k in range(0, 6):
        s = float(np.dot(h[: len(h) - 2 * k], h[2 * k:]))
        assert abs(s - (1.0 if k == 0 else 0.0)) < 1e-13, (k, s)
    ks, g = _g(h)
    for p in range(6):
        scale = float(np.sum(np.abs(ks.astype(float)) ** p * np.abs(g)))
        assert abs(float(np.sum(ks.astype(float) ** p * g))) <= 1e-12 * max(scale, 1.0), p
    # the 7th moment does not vanish: M = 6 exactly
    assert abs(float(np.sum(ks.astype(float) ** 6 * g))) > 1.0


def test_symmlet_is_least_asymmetric_of_its_family():
    """The Symmlet is the Daubechies-6 factorisation with the most nearly linear
    phase; the extremal-phase (minimum phase) Daubechies filter of the same
    family must be strictly less linear.  Both have identical |m0|."""
    M = 6
    P = np.array([math.comb(M - 1 + k, k) for k in range(M)], float)
    yr = np.roots(P[::-1])
    zr = []
    for y in yr:
        b = 2 - 4 * y
        z1 = (b + np.sqrt(b * b - 4 + 0j)) / 2
        zr.append(z1 if abs(z1) < 1 else (b - np.sqrt(b * b - 4 + 0j)) / 2)
    q = np.real(np.poly(zr))[::-1]
    q /= q.sum()
    lo = np.array([1.0])
    for _ in range(M):
        lo = np.convolve(lo, [0.5, 0.5])
    hmin = math.sqrt(2) * np.convolve(lo, q)
    w = np.linspace(0, math.pi, 2049)
    def dev(h):
        ph = np.unwrap(np.angle(np.polyval(h[::-1], np.exp(-1j * w))))
        A = np.stack([np.ones_like(w), w], 1)
        c, *_ = np.linalg.lstsq(A, ph, rcond=None)
        return float(np.sum((ph - A @ c) ** 2))
    mag = lambda h: np.abs(np.polyval(h[::-1], np.exp(-1j * w)))
    np.testing.assert_allclose(mag(hmin), mag(H6), atol=1e-12)
    assert dev(H6) < 0.1 * dev(hmin)


# ------------------------------------------------------ wavelet transform --
def test_haar_hand_cases(golden_dir):
    """P6: hand-computed Haar transforms (tests/golden/haar_hand.json)."""
    data = json.load(open(os.path.join(golden_dir, "haar_hand.json")))
    for case in data["cases"]:
        img = np.array(case["image"], float)
        c = O.fwt(img, case["levels"], HAAR)
        np.testing.assert_allclose(c, np.array(case["coeffs"], float), atol=1e-13)
        np.testing.assert_allclose(O.ifwt(c, case["levels"], HAAR), img, atol=1e-13)


@pytest.mark.parametrize("shape,levels", [((8, 8), 3), ((64, 64), 6), ((96, 160), 5), ((32, 64), 4)])
def test_fwt_orthonormal(shape, levels):
    """P2 (Section 2.2): Psi Psi^* = Id and Parseval for the periodic basis."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape)
    c = O.fwt(x, levels, H6)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    np.testing.assert_allclose(O.ifwt(c, levels, H6), x, atol=1e-12)
    # adjointness <Psi^* f, c> = <f, Psi c>
    d = rng.standard_normal(shape)
    lhs = float(np.sum(O.fwt(x, levels, H6) * d))
    rhs = float(np.sum(x * O.ifwt(d, levels, H6)))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(d)


def test_dirac_coefficients_follow_filter_alignment():
    """Section 2.1: the level-1 coefficients of a Dirac at p are products of
    h[p - 2l] and g[p - 2l] (supp h = [0, L-1], supp g = [2-L, 1]), with the
    band that is high-pass along x1 stored top-right."""
    n1, n2 = 32, 16
    p1, p2 = 13, 6
    img = np.zeros((n2, n1))
    img[p2, p1] = 1.0
    c = O.fwt(img, 1, H6)
    L = len(H6)
    def hh(k):
        return H6[k] if 0 <= k < L else 0.0
    def gg(k):
        return (-1.0) ** (1 - k) * H6[1 - k] if 2 - L <= k <= 1 else 0.0
    def per(f, p, l, n):
        # periodic: all k = p - 2l + m n
        return sum(f(p - 2 * l + m * n) for m in (-2, -1, 0, 1, 2))
    ref = np.zeros((n2, n1))
    for l2 in range(n2 // 2):
        for l1 in range(n1 // 2):
            ref[l2, l1] = per(hh, p1, l1, n1) * per(hh, p2, l2, n2)
            ref[l2, n1 // 2 + l1] = per(gg, p1, l1, n1) * per(hh, p2, l2, n2)
            ref[n2 // 2 + l2, l1] = per(hh, p1, l1, n1) * per(gg, p2, l2, n2)
            ref[n2 // 2 + l2, n1 // 2 + l1] = per(gg, p1, l1, n1) * per(gg, p2, l2, n2)
    np.testing.assert_allclose(c, ref, atol=1e-15)


def test_vanishing_moments_locate_wrap_region():
    """Section 2.1 (M vanishing moments, supp g = [-(2M-2), 1]): for a signal
    that is a polynomial of degree 5 in x1 on [0, n1), the x1-detail
    coefficients vanish exactly where the filter window [2l-10, 2l+1] does not
    wrap, i.e. l = 5 .. n1/2-1, and not for l < 5.  A filter shifted to the
    support [0, 11] would instead leave the last coefficients non-zero."""
    n1, n2 = 64, 4
    x1 = np.arange(n1, dtype=float) / n1
    img = np.tile(1 + x1 - 2 * x1**2 + 3 * x1**3 - x1**4 + 0.5 * x1**5, (n2, 1))
    c = O.fwt(img, 1, H6)
    det = c[: n2 // 2, n1 // 2:]  # high along x1, low along x2
    assert np.abs(det[:, 5:]).max() < 1e-12
    assert np.abs(det[:, :5]).max() > 1e-3


def test_constant_image_has_no_details():
    """P4: a constant image has zero periodic detail coefficients; its
    approximation band carries c * 2^levels per coefficient (orthonormal
    low-pass with sum h = sqrt 2 along two axes)."""
    for shape, L in [((64, 64), 6), ((96, 160), 5)]:
        c = O.fwt(np.full(shape, 0.7), L, H6)
        k = O.band_of(shape[1], shape[0], L)
        assert np.abs(c[k > 0]).max() < 1e-13
        np.testing.assert_allclose(c[k == 0], 0.7 * 2.0**L, rtol=1e-13)


# ---------------------------------------------------------------- blur -----
def test_operator1_support_matches_paper(golden_dir):
    """P9: largest impulse-response support 19 x 19 at sigma = 3 (Section 4.1)."""
    g = json.load(open(os.path.join(golden_dir, "operator1.json")))
    for n2 in (16, 64, 512, 1024):
        kt, R = O.op1_profiles(n2, g["sigma_max"], g["mass"])
        assert (2 * R + 1, 2 * R + 1) == tuple(g["largest_support"])
        last = kt[-1]
        assert np.count_nonzero(last) == 2 * R + 1
        np.testing.assert_allclose(kt.sum(1), 1.0, rtol=1e-14)
    # first row: sigma = 0 -> Dirac
    kt, R = O.op1_profiles(64)
    assert kt[0, R] == 1.0 and np.count_nonzero(kt[0]) == 1


@pytest.mark.parametrize("shape", [(8, 8), (64, 64), (96, 160)])
def test_blur_adjoint(shape):
    """P1: <H x, r> = <x, H^T r> to 1e-12 relative (H and H^T are coded as
    two separate gathers)."""
    n2, n1 = shape
    kt, R = O.op1_profiles(n2)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(shape)
    r = rng.standard_normal(shape)
    lhs = float(np.sum(O.blur(x, kt, R) * r))
    rhs = float(np.sum(x * O.blur(r, kt, R, transpose=True)))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(r)


def test_blur_columns_are_impulse_responses():
    """Section 1 (S(., y) = K(. + y, y)) and Section 4.1: H applied to a Dirac
    at source y is the isotropic response of the SOURCE row, the outer
    product of one profile with itself, centred on y, with unit sum; the
    columns of H therefore sum to one (H^T 1 = 1)."""
    n1, n2 = 48, 40
    kt, R = O.op1_profiles(n2)
    for (y1, y2) in [(5, 3), (20, 39), (47, 20)]:
        d = np.zeros((n2, n1))
        d[y2, y1] = 1.0
        resp = O.blur(d, kt, R)
        resp = np.roll(np.roll(resp, R - y1, 1), R - y2, 0)[: 2 * R + 1, : 2 * R + 1]
        prof = kt[y2]
        np.testing.assert_allclose(resp, np.outer(prof, prof), atol=1e-15)
        # isotropic Gaussian of std sigma(y2): variance of the profile
        s = O.op1_sigma(n2)[y2]
        dd = np.arange(-R, R + 1)
        var = float(np.sum(prof * dd * dd))
        if s > 1.0:
            assert abs(var - s * s) < 0.05 * s * s
    ones = np.ones((n2, n1))
    np.testing.assert_allclose(O.blur(ones, kt, R, transpose=True), 1.0, rtol=1e-14)


def test_blur_constant_profile_is_circular_convolution():
    """With one profile for every row the operator is a circular convolution
    with the outer-product kernel: compare with an FFT convolution."""
    n1, n2, R = 40, 24, 4
    rng = np.random.default_rng(3)
    prof = rng.random(2 * R + 1)
    kt = np.tile(prof, (n2, 1))
    x = rng.standard_normal((n2, n1))
    ker = np.zeros((n2, n1))
    for d2 in range(-R, R + 1):
        for d1 in range(-R, R + 1):
            ker[d2 % n2, d1 % n1] += prof[d1 + R] * prof[d2 + R]
    ref = np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(ker)))
    np.testing.assert_allclose(O.blur(x, kt, R), ref, atol=1e-12)
    refT = np.real(np.fft.ifft2(np.fft.fft2(x) * np.conj(np.fft.fft2(ker))))
    np.testing.assert_allclose(O.blur(x, kt, R, transpose=True), refT, atol=1e-12)


# --------------------------------------------------------------- FISTA -----
def test_soft_threshold_hand(golden_dir):
    """Appendix A.1 prox with H = Id, tau = 1: z(1) = S_w(Psi^* f0) (hand values)."""
    g = json.load(open(os.path.join(golden_dir, "soft_threshold_hand.json")))
    c = np.array(g["coeffs"])
    f0 = O.ifwt(c, 1, HAAR)
    pb = O.Problem(2, 2, levels=1, h=HAAR, op="identity", w=np.array(g["weights"])[None])
    out = O.fista(pb, f0[None], tau=1.0, iters=1)
    np.testing.assert_allclose(out["z"][0], np.array(g["z1"]), atol=1e-15)


def test_momentum_worked_example(golden_dir):
    """Appendix A.1 recursion, momentum (i-1)/(i+2): hand iterates of the
    worked example in tests/golden/momentum_hand.json."""
    g = json.load(open(os.path.join(golden_dir, "momentum_hand.json")))
    rng = np.random.default_rng(4)
    f0 = rng.standard_normal((1, 8, 8))
    pb = O.Problem(8, 8, levels=3, op="identity")
    c = O.fwt(f0, 3, pb.h)
    for i, ratio in enumerate(g["z_over_c"], start=1):
        out = O.fista(pb, f0, tau=g["tau"], iters=i, init=np.zeros((1, 8, 8)))
        np.testing.assert_allclose(out["z"], ratio * c, rtol=1e-13, atol=1e-14)


def test_identity_operator_closed_form():
    """P5: with H = Id eq. 4.1 is solved by wavelet soft-thresholding,
    f* = Psi S_w(Psi^* f0).  FISTA with tau = 1 reaches it at iteration 1 and
    stays there; with tau = 1/2 it converges to it; the duality gap of the
    H = Id problem vanishes at f*."""
    rng = np.random.default_rng(5)
    n = 32
    L = 5
    f0 = rng.standard_normal((1, n, n))
    w = O.expand_level_weights(O.paper_level_weights(L, 0.3), n, n, L)
    pb = O.Problem(n, n, levels=L, op="identity", w=w)
    c = O.fwt(f0, L, pb.h)
    zstar = np.sign(c) * np.maximum(np.abs(c) - w, 0.0)
    fstar = O.ifwt(zstar, L, pb.h)
    for K in (1, 2, 7):
        out = O.fista(pb, f0, tau=1.0, iters=K)
        np.testing.assert_allclose(out["z"], zstar, atol=1e-13)
        np.testing.assert_allclose(out["f"], fstar, atol=1e-13)
    out = O.fista(pb, f0, tau=0.5, iters=200)
    np.testing.assert_allclose(out["z"], zstar, atol=1e-10)
    # duality gap: primal E(f*) vs dual D(q) = <q, f0> - |q|^2/2 with
    # q = f0 - f* feasible (|Psi^* q| <= w), gap 0 at the optimum
    E, _ = O.energy(pb, f0, zstar)
    q = f0 - fstar
    assert np.all(np.abs(O.fwt(q, L, pb.h)) <= w + 1e-12)
    D = float(np.sum(q * f0) - 0.5 * np.sum(q * q))
    assert abs(E - D) < 1e-12 * abs(E)


def test_identity_operator_constant_image():
    """P4: H = Id, constant observation, zero weight on the approximation band:
    the minimiser reproduces the constant image exactly."""
    pb = O.Problem(16, 16, levels=4, op="identity",
                   w=O.expand_level_weights([0, 0.5, 0.5, 0.5, 0.5], 16, 16, 4))
    f0 = np.full((1, 16, 16), 0.3)
    out = O.fista(pb, f0, tau=1.0, iters=3)
    np.testing.assert_allclose(out["f"], f0, atol=1e-14)


def _tiny_problem(sigma_max=1.0):
    n, L = 8, 3
    rng = np.random.default_rng(6)
    clean = np.zeros((n, n))
    clean[2:6, 1:5] = 1.0
    clean[5:8, 4:8] += 0.5
    kt, R = O.op1_profiles(n, sigma_max)
    f0 = O.blur(clean, kt, R) + 0.05 * rng.standard_normal((n, n))
    w = O.expand_level_weights([0.0, 0.02, 0.04, 0.06], n, n, L)
    pb = O.Problem(n, n, levels=L, op=(kt, R), w=w)
    return pb, f0[None]


@pytest.mark.parametrize("sigma_max", [1.0, 3.0])
def test_fista_limit_matches_independent_minimiser(sigma_max):
    """P7: on an 8x8 image with Operator 1, FISTA run long reaches the same
    energy as an independent coordinate-descent + exact active-set minimiser,
    satisfies the optimality (KKT) conditions, and matches the minimiser
    where it is unique (well-conditioned operator)."""
    pb, f0 = _tiny_problem(sigma_max)
    tau = O.step_size(pb)
    out = O.fista(pb, f0, tau, 20000)
    zf = out["z"]
    zx, A = O.lasso_exact(pb, f0[0])
    Ef, _ = O.energy(pb, f0, zf)
    Ex, _ = O.energy(pb, f0, zx[None])
    assert abs(Ef - Ex) <= 1e-11 * abs(Ex)
    assert O.kkt_residual(pb, f0, zx[None]) < 1e-10
    assert O.kkt_residual(pb, f0, zf) < 1e-8
    if np.linalg.cond(A) < 1e6:
        np.testing.assert_allclose(zf[0], zx, atol=1e-8)


def test_fista_rate_bound():
    """P8: Beck & Teboulle's bound for FISTA with step tau = 1/L,
    E(z_i) - E* <= 2 ||z_0 - z*||^2 / (tau (i+1)^2), at every iterate."""
    pb, f0 = _tiny_problem(3.0)
    tau = O.step_size(pb)
    zstar = O.fista(pb, f0, tau, 20000)["z"]
    Estar, _ = O.energy(pb, f0, zstar)
    z0 = O.fwt(f0, pb.levels, pb.h)
    R2 = float(np.sum((z0 - zstar) ** 2))
    for i in (1, 2, 3, 5, 10, 20, 50, 100):
        z = O.fista(pb, f0, tau, i)["z"]
        E, _ = O.energy(pb, f0, z)
        assert E - Estar <= 2 * R2 / (tau * (i + 1) ** 2) + 1e-14


def test_energy_log_terms():
    """The per-iteration log holds the two terms of eq. 4.1 at y(i) and
    ||z(i) - y(i)||^2; at i = 1, y(1) = Psi^* f0."""
    pb, f0 = _tiny_problem(3.0)
    tau = O.step_size(pb)
    out = O.fista(pb, f0, tau, 5, log=True)
    y1 = O.fwt(f0, pb.levels, pb.h)
    E, terms = O.energy(pb, f0, y1)
    np.testing.assert_allclose(out["log"][0, :2], terms, rtol=1e-13)
    z1 = O.fista(pb, f0, tau, 1)["z"]
    np.testing.assert_allclose(out["log"][0, 2], np.sum((z1 - y1) ** 2), rtol=1e-13)


# -------------------------------------------------------------- reverse -----
def test_reverse_mode_matches_finite_differences():
    """P10: the oracle's reverse pass equals FP64 central differences of the
    forward recursion (loss 1/2 ||f_K - clean||^2) in random directions of f0
    and of the weight map."""
    n, L, K = 16, 4, 10
    rng = np.random.default_rng(7)
    kt, R = O.op1_profiles(n)
    clean = rng.random((1, n, n))
    f0 = O.blur(clean[0], kt, R)[None] + 0.1 * rng.standard_normal((1, n, n))
    w = np.log1p(np.exp(rng.normal(-2.0, 0.1, (1, n, n))))
    pb = O.Problem(n, n, levels=L, op=(kt, R), w=w)
    tau = O.step_size(pb)

    def loss(f0_, w_):
        pb.w = np.ascontiguousarray(w_)
        f = O.fista(pb, f0_, tau, K)["f"]
        return 0.5 * float(np.sum((f - clean) ** 2))

    pb.w = w.copy()
    out = O.fista(pb, f0, tau, K, tape=True)
    # margin from the kinks
    margin = np.min(np.abs(np.abs(out["tape"]) - tau * w[None]))
    assert margin > 1e-7
    f0b, wb = O.fista_reverse(pb, tau, K, out["tape"], out["f"] - clean)
    eps = 1e-6
    for t in range(10):
        d = rng.standard_normal((1, n, n))
        fd = (loss(f0 + eps * d, w) - loss(f0 - eps * d, w)) / (2 * eps)
        an = float(np.sum(f0b * d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("f0", t, fd, an)
        d = rng.standard_normal((1, n, n)) * w
        fd = (loss(f0, w + eps * d) - loss(f0, w - eps * d)) / (2 * eps)
        an = float(np.sum(wb * d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("w", t, fd, an)


# ------------------------------------------------ colour extension, bands ----
def _joint_problem(g):
    w = np.broadcast_to(np.array(g["weights"]), (3, 2, 2))
    return O.Problem(2, 2, 3, levels=1, h=HAAR, op="identity", w=w, joint=True)


def test_joint_prox_hand(golden_dir):
    """Group soft-thresholding of the channel vector (the colour extension of
    the Appendix A.1 prox): hand values of tests/golden/joint_prox_hand.json,
    including the tie ||v|| = tau w and v = 0, reached as the first FISTA
    iterate with H = Id and tau = 1."""
    g = json.load(open(os.path.join(golden_dir, "joint_prox_hand.json")))
    c = np.array(g["coeffs"])
    f0 = O.ifwt(c, 1, HAAR)
    out = O.fista(_joint_problem(g), f0, tau=1.0, iters=1)
    np.testing.assert_allclose(out["z"], np.array(g["z1"]), atol=1e-14)
    # tau scales the threshold: tau = 1/2 halves it at (0,0): 1 - 1.25/5 = 3/4
    half = O.fista(_joint_problem(g), f0, tau=0.5, iters=1)
    np.testing.assert_allclose(half["z"][:, 0, 0], [2.25, 3.0, 0.0], atol=1e-14)


def test_joint_penalty_hand(golden_dir):
    """Penalty of eq. 4.1 in the colour extension, sum w ||z||_2 over the
    channel vectors (hand values), via the energy and via the FISTA log, whose
    second term is the penalty at y(1) = Psi^* f0."""
    g = json.load(open(os.path.join(golden_dir, "joint_prox_hand.json")))
    pb = _joint_problem(g)
    c = np.array(g["coeffs"])
    f0 = O.ifwt(c, 1, HAAR)
    _, terms = O.energy(pb, f0, np.array(g["z1"]))
    assert abs(terms[1] - g["penalty_at_z1"]) < 1e-13
    _, terms = O.energy(pb, f0, c)
    assert abs(terms[1] - g["penalty_at_coeffs"]) < 1e-13
    assert abs(terms[0]) < 1e-25  # H = Id and f = f0: no data misfit
    lg = O.fista(pb, f0, tau=1.0, iters=1, log=True)["log"]
    assert abs(lg[0, 1] - g["penalty_at_coeffs"]) < 1e-12


def test_band_map_hand(golden_dir):
    """Band index of every Mallat position and the Fig. 5 weights
    w = 2e-2 |lambda| (hand-drawn maps, tests/golden/band_map_hand.json)."""
    g = json.load(open(os.path.join(golden_dir, "band_map_hand.json")))
    for case in g["cases"]:
        n1, n2, L = case["n1"], case["n2"], case["levels"]
        np.testing.assert_array_equal(O.band_of(n1, n2, L), np.array(case["band"]))
        np.testing.assert_allclose(O.paper_level_weights(L), case["paper_weights"], atol=1e-17)
        w = O.expand_level_weights(O.paper_level_weights(L), n1, n2, L, C=2)
        np.testing.assert_allclose(w, np.broadcast_to(np.array(case["paper_weights"])[np.array(case["band"])],
                                                      (2, n2, n1)), atol=1e-17)


def _circular_extent(mask):
    """Length of the shortest circular interval that holds every True entry."""
    idx = np.nonzero(mask)[0]
    n = len(mask)
    gaps = np.diff(np.concatenate([idx, idx[:1] + n]))
    return n - int(gaps.max()) + 1


def test_band_index_is_the_scale():
    """Section 2.1: supp psi_{j,0} and supp phi_{j,0} span (2^(J-j) - 1)(2 delta - 1) + 1
    samples.  The synthesis of a unit coefficient of band k (Symmlet-6,
    delta = 6, 64 x 64, J = 6) spans exactly that many rows and columns with
    j = k - 1, which fixes the band order of the weights (finest band = largest
    j = largest weight)."""
    n, J = 64, 6
    band = O.band_of(n, n, J)
    for lev in (1, 2):  # levels whose support does not wrap around the torus
        h2 = n >> lev
        for (r, c) in ((0, h2), (h2, 0), (h2, h2)):  # one coefficient of each orientation
            k = int(band[r + 1, c + 1])
            j = k - 1
            e = np.zeros((n, n))
            e[r + 1, c + 1] = 1.0
            x = O.ifwt(e, J, H6)
            nz = np.abs(x) > 1e-14
            span = (2 ** (J - j) - 1) * (2 * 6 - 1) + 1
            assert _circular_extent(nz.any(0)) == span, (lev, r, c, k)
            assert _circular_extent(nz.any(1)) == span, (lev, r, c, k)


@pytest.mark.parametrize("n", [8, 16])
def test_step_size_is_the_spectral_bound(n):
    """Appendix A.1 asks tau <= ||H||^-2: the oracle's power iteration gives
    ||H^T H|| to 1e-12 of the largest eigenvalue of the dense H^T H
    (numpy.linalg.eigvalsh on Operator 1 built column by column), and its
    step satisfies the bound."""
    pb = O.Problem(n, n, 1)
    N = n * n
    H = np.zeros((N, N))
    for j in range(N):
        e = np.zeros((n, n))
        e.flat[j] = 1.0
        H[:, j] = O.apply_H(pb, e).ravel()
    lam = np.linalg.eigvalsh(H.T @ H)[-1]
    assert abs(O.lipschitz(pb) - lam) <= 1e-12 * lam
    tau = O.step_size(pb)
    assert tau * lam <= 1.0 and tau * lam > 1.0 - 1e-5
    assert O.step_size(O.Problem(n, n, 1, op="identity")) * 1.0 <= 1.0
