"""GPU parity of FISTA in the wavelet domain (FISTA-W / FISTA-WP, Section 4.3
and Appendix A.1): the HIP path through the C ABI against the oracle.

Theta_L is the oracle's: the exact Theta = Psi^* H Psi of a small image
(Operator 1) with all but its L largest entries set to zero.  Tolerances as
for the spatial-operator solver: FP64 GPU vs FP64 oracle 1e-10 on iterates,
FP32 GPU vs FP64 oracle 1e-5 max-abs on iterates of [0, 1]-scale images;
the CSR transpose is integer / permutation work and must be bit-exact.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from oracle import wavelet_domain as W  # noqa: E402
import syninputs as SI  # noqa: E402
import paper_2005_09870_amd as P  # noqa: E402
from paper_2005_09870_amd import _lib as C  # noqa: E402

DEV = "cuda"
H6 = O.symmlet(6)
_CACHE = {}


def _theta(n1, n2, levels=None, mult=16):
    key = (n1, n2, levels, mult)
    if key not in _CACHE:
        pb = O.Problem(n1, n2, 1, levels, h=H6)
        T = W.theta_dense(pb)
        _CACHE[key] = (pb, W.sparsify(T, mult * n1 * n2))
    return _CACHE[key]


def _case(pb, seed, lam=0.1):
    c = SI.make_case(pb.n1, pb.n2, 1, 4, 3, "const", 0.1, lam, levels=pb.levels, seed=seed)
    f0 = O.apply_H(pb, c.clean[0]) + c.noise[0]
    z0 = O.fwt(f0, pb.levels, pb.h)
    return z0, c.level_w


def _gpu(m, dtype):
    return P.Csr.from_arrays(m.indptr, m.indices, m.data, dtype=dtype, device=DEV)


def _t(a, dtype):
    return torch.as_tensor(np.array(a, dtype=np.float64), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_transpose_is_exact(dtype):
    pb, m = _theta(32, 32)
    a = _gpu(m, dtype)
    t = P.pd_csr_transpose(a)
    ref = W.transpose(m)
    assert np.array_equal(t.row_ptr.cpu().numpy(), ref.indptr.astype(np.int64))
    assert np.array_equal(t.col.cpu().numpy(), ref.indices.astype(np.int32))
    want = torch.as_tensor(ref.data, dtype=dtype).numpy()
    assert np.array_equal(t.val.cpu().numpy(), want)


def test_transpose_rejects_malformed():
    rp = np.array([0, 2, 3, 3], np.int64)
    bad_order = P.Csr.from_arrays(rp, np.array([1, 0, 2], np.int32), np.ones(3), device=DEV)
    out_of_range = P.Csr.from_arrays(rp, np.array([0, 1, 3], np.int32), np.ones(3), device=DEV)
    bad_rp = P.Csr.from_arrays(np.array([0, 2, 1, 3], np.int64), np.array([0, 1, 2], np.int32), np.ones(3),
                               device=DEV)
    for a in (bad_order, out_of_range, bad_rp):
        with pytest.raises(C.PDError) as e:
            P.pd_csr_transpose(a)
        assert e.value.code == C.PD_ERR_ARG


@pytest.mark.parametrize("mult", [4, 16, 48])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 2e-6)])
def test_spmv_and_jacobi_match_oracle(mult, dtype, tol):
    """Row lengths of 4N .. 48N matrices select every row-group width."""
    pb, m = _theta(32, 32, mult=mult)
    rng = np.random.default_rng(mult)
    x = rng.standard_normal(m.shape[0])
    a = _gpu(m, dtype)
    y = _np(P.pd_spmv(a, _t(x, dtype)))
    ref = m @ x
    assert np.abs(y - ref).max() < tol * max(1.0, np.abs(ref).max()) * 10
    s = _np(P.pd_wjacobi(P.pd_csr_transpose(a)))
    np.testing.assert_allclose(s, W.jacobi_sigma(m), rtol=tol * 10)


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_wsolve_matches_oracle(precond, dtype, tol):
    """32 x 32, Operator 1, Theta_L with 16N entries, 200 iterations."""
    pb, m = _theta(32, 32)
    z0, lw = _case(pb, seed=7)
    w = O.expand_level_weights(lw, pb.n1, pb.n2, pb.levels)[0]
    sig = W.jacobi_sigma(m) if precond else None
    tau = W.step_size(m, sig)
    ref = W.fista_w(m, z0, w, tau, 200, sigma=sig, log=True)
    a = _gpu(m, dtype)
    out = P.pd_wsolve(_t(z0, dtype), a, P.pd_csr_transpose(a), pb.levels, tau, 200, precond=precond,
                      level_w=lw, stats=True, check_finite=True)
    assert np.abs(_np(out["z_cur"]).ravel() - ref["z"]).max() < tol
    assert np.abs(_np(out["z_prev"]).ravel() - ref["z_prev"]).max() < tol
    st = _np(out["stats"])
    rt = 1e-9 if dtype == torch.float64 else 1e-4
    np.testing.assert_allclose(st[:, :2], ref["log"][:, :2], rtol=rt)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_wsolve_ragged_coeff_weights(dtype, tol):
    """Non-square 32 x 16 plane with 4 levels (row count not a multiple of a
    workgroup's rows), per-coefficient weights, odd iteration count."""
    pb, m = _theta(32, 16, levels=4, mult=8)
    z0, _ = _case(pb, seed=8)
    rng = np.random.default_rng(9)
    w = rng.uniform(0.0, 0.2, z0.shape)
    sig = W.jacobi_sigma(m)
    tau = W.step_size(m, sig)
    ref = W.fista_w(m, z0, w, tau, 77, sigma=sig)
    a = _gpu(m, dtype)
    out = P.pd_wsolve(_t(z0, dtype), a, P.pd_csr_transpose(a), pb.levels, tau, 77, precond=True,
                      coeff_w=_t(w, dtype))
    assert np.abs(_np(out["z_cur"]).ravel() - ref["z"]).max() < tol


def test_wsolve_resume_is_bitwise():
    pb, m = _theta(32, 32)
    z0, lw = _case(pb, seed=10)
    a = _gpu(m, torch.float32)
    at = P.pd_csr_transpose(a)
    tau = W.step_size(m)
    z0t = _t(z0, torch.float32)
    one = P.pd_wsolve(z0t, a, at, pb.levels, tau, 100, level_w=lw)
    first = P.pd_wsolve(z0t, a, at, pb.levels, tau, 37, level_w=lw)
    two = P.pd_wsolve(z0t, a, at, pb.levels, tau, 63, level_w=lw, z_cur=first["z_cur"],
                      z_prev=first["z_prev"], init=False, iter_offset=37)
    assert torch.equal(one["z_cur"], two["z_cur"]) and torch.equal(one["z_prev"], two["z_prev"])


def test_full_theta_equals_spatial_solver():
    """Untruncated Theta: FISTA-W on the GPU equals FISTA-Spa on the GPU (and
    the oracle) in FP64, the identity Theta^T (Theta y - Psi^* f0) =
    Psi^* H^T (H Psi y - f0)."""
    pb = O.Problem(16, 16, 1, None, h=H6)
    m = sp.csr_matrix(W.theta_dense(pb))
    c = SI.make_case(16, 16, 1, 3, 2, "const", 0.05, 0.05, seed=11)
    f0 = O.apply_H(pb, c.clean[0]) + c.noise[0]
    tau = O.step_size(pb)
    z0 = O.fwt(f0, pb.levels, pb.h)
    a = _gpu(m, torch.float64)
    out = P.pd_wsolve(_t(z0, torch.float64), a, P.pd_csr_transpose(a), pb.levels, tau, 60, level_w=c.level_w)
    op = P.Operator.from_taps(pb.kt, pb.R, dtype=torch.float64)
    spa = P.pd_solve(_t(f0[None], torch.float64), op, H6, pb.levels, tau, 60, level_w=c.level_w)
    assert np.abs(_np(out["z_cur"]) - _np(spa["z_cur"])[0]).max() < 1e-10


def test_wsolve_zero_iterations_and_nonfinite():
    pb, m = _theta(32, 32)
    z0, lw = _case(pb, seed=12)
    a = _gpu(m, torch.float32)
    at = P.pd_csr_transpose(a)
    z0t = _t(z0, torch.float32)
    out = P.pd_wsolve(z0t, a, at, pb.levels, 0.5, 0, level_w=lw)
    assert torch.equal(out["z_cur"], z0t) and torch.equal(out["z_prev"], z0t)
    bad = z0t.clone()
    bad[3, 5] = float("nan")
    with pytest.raises(C.PDError) as e:
        P.pd_wsolve(bad, a, at, pb.levels, 0.5, 3, level_w=lw, check_finite=True)
    assert e.value.code == C.PD_ERR_NONFINITE


def test_wstep_size_matches_oracle():
    pb, m = _theta(32, 32)
    a = _gpu(m, torch.float64)
    at = P.pd_csr_transpose(a)
    for sig in (None, W.jacobi_sigma(m)):
        ref = W.lipschitz(m, sig, iters=500)   # both converged to ~1e-13 by then
        got = P.wlipschitz(a, at, None if sig is None else _t(sig, torch.float64), iters=500)
        assert abs(got - ref) < 1e-9 * ref


# ------------------------------------------------------ Theta_L by probing ---
def test_theta_builder_on_gpu_matches_dense():
    """The probed Theta_L (libpd transforms and blur, FP64) equals the oracle's
    dense Theta thresholded at eta, entry for entry."""
    from paper_2005_09870_amd import theta as TH
    n, L, eta = 64, 6, 3e-3
    pb = O.Problem(n, n, 1, L, h=H6)
    T = W.theta_dense(pb)
    op = P.Operator.from_taps(pb.kt, pb.R, dtype=torch.float64)
    m = TH.theta_rowblur(op, H6, n, n, L, eta, dtype=torch.float64)
    A = sp.csr_matrix((m.val.cpu().numpy(), m.col.cpu().numpy(), m.row_ptr.cpu().numpy()), shape=T.shape)
    keep = np.abs(T) >= eta
    # entries within rounding of the threshold may fall either way
    near = np.abs(np.abs(T) - eta) < 1e-12
    got = A.toarray() != 0
    assert not np.any((got != keep) & ~near)
    assert np.abs(np.where(got & keep, A.toarray() - T, 0.0)).max() < 1e-12


def test_wavelet_solver_at_1024_full_size():
    """The 1024 x 1024 workload (Operator 1, 10 levels, Theta_L = entries of
    magnitude >= 3e-3): sampled columns of the probed Theta_L against the
    oracle's Psi^* H Psi e, then 4 FISTA-WP iterations in FP32 against the
    oracle on the same matrix (every coefficient)."""
    from paper_2005_09870_amd import theta as TH
    n, L, eta = 1024, 10, 3e-3
    kt, R = O.op1_profiles(n)
    op = P.Operator.from_taps(kt, R, dtype=torch.float64)
    m64 = TH.theta_rowblur(op, H6, n, n, L, eta, dtype=torch.float64)
    mt64 = P.pd_csr_transpose(m64)
    rp, col, val = mt64.row_ptr.cpu().numpy(), mt64.col.cpu().numpy(), mt64.val.cpu().numpy()
    pb = O.Problem(n, n, 1, L, h=H6)
    for mu in (5 * n + 700, 300 * n + 40, 3 * n + 2, 0):   # level-1, level-2, coarse detail, approximation
        e = np.zeros((n, n))
        e.flat[mu] = 1.0
        colref = O.fwt(O.apply_H(pb, O.ifwt(e, L, H6)), L, H6).ravel()
        keep = np.nonzero(np.abs(colref) >= eta)[0]
        lo, hi = rp[mu], rp[mu + 1]
        near = np.abs(np.abs(colref) - eta) < 1e-12
        assert set(col[lo:hi]) ^ set(keep) <= set(np.nonzero(near)[0])
        np.testing.assert_allclose(val[lo:hi], colref[col[lo:hi]], rtol=0, atol=1e-12)
    # FISTA-WP, FP32 on the GPU vs the oracle (FP64) on the FP32-rounded matrix
    a = P.Csr(m64.row_ptr, m64.col, m64.val.float())
    at = P.pd_csr_transpose(a)
    c = SI.make_case(n, n, 1, 160, 100, "ramp", 0.05, 0.08, seed=13)
    f0 = O.apply_H(pb, c.clean[0]) + c.noise[0]
    z0 = O.fwt(f0, L, H6)
    A = sp.csr_matrix((a.val.double().cpu().numpy(), a.col.cpu().numpy(), a.row_ptr.cpu().numpy()),
                      shape=(n * n, n * n))
    sig = W.jacobi_sigma(A)
    tau = 0.9 / W.lipschitz(A, sig, iters=30)
    w = O.expand_level_weights(c.level_w, n, n, L)[0]
    ref = W.fista_w(A, z0, w, tau, 4, sigma=sig)
    out = P.pd_wsolve(_t(z0, torch.float32), a, at, L, tau, 4, precond=True, level_w=c.level_w)
    # compared on f = Psi z (pixel scale): the approximation coefficient is ~400 here
    fg = O.ifwt(_np(out["z_cur"]).reshape(n, n), L, H6)
    fr = O.ifwt(ref["z"].reshape(n, n), L, H6)
    assert np.abs(fg - fr).max() < 1e-5
