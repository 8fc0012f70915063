"""CPU checks of the C ABI: the library loads, exports every declared symbol,
its host-side set-up matches the oracle, and argument errors are reported
before any GPU work is enqueued (no device calls happen in these tests)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_09870_amd import _lib as C
from paper_2005_09870_amd import solver as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "pd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = C.load()
    syms = declared_symbols()
    assert len(syms) >= 11
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(C.EXPORTS) == syms


def test_symmlet_matches_oracle():
    for M in range(1, 9):
        np.testing.assert_allclose(S.pd_symmlet(M), O.symmlet(M), atol=5e-15)


def test_op1_taps_match_oracle():
    for n2 in (2, 8, 64, 96, 512, 2048):
        t, R = S.pd_op1_taps(n2)
        kt, RR = O.op1_profiles(n2)
        assert R == RR
        np.testing.assert_allclose(t, kt, atol=1e-15)


def _svir(taps):
    """S of a row-profile operator, dense: S[(a, b), y] = taps[y, a] taps[y, b]."""
    n2, W = taps.shape
    return np.einsum("ya,yb->aby", taps, taps).reshape(W * W, n2)


def test_pc_expansion_matches_exact_svd():
    """pd_pc_expansion (randomized SVD, Section 3.3.3) against the oracle's exact
    SVD of the same S: the singular values and the rank-m truncation
    sum_k u_k v_k^T (unique while sigma_m > sigma_m+1), Operator 1 at several
    heights and ranks, and the oracle's own u, v up to the sign of each term."""
    from oracle import product_convolution as PC
    for n2, m in ((64, 5), (256, 5), (512, 12), (128, 25), (1024, 5)):
        taps, R = S.pd_op1_taps(n2)
        u, v, sv = S.pd_pc_expansion(taps, R, m)
        ue, ve, sve = PC.pc_expansion(taps, R, m)
        k = min(m, ue.shape[0])
        assert u.shape == (k, 2 * R + 1, 2 * R + 1) and v.shape == (k, n2)
        np.testing.assert_allclose(sv, sve[:k], rtol=1e-10, atol=1e-12 * sve[0])
        W2 = (2 * R + 1) ** 2
        approx = u.reshape(k, W2).T @ v
        exact = ue.reshape(-1, W2)[:k].T @ ve[:k]
        np.testing.assert_allclose(approx, exact, atol=1e-10 * sve[0])
        for t in range(k):
            if t + 1 < k and sve[t] - sve[t + 1] < 1e-6 * sve[0]:
                continue  # a near-degenerate pair: only the truncation is unique
            s = np.sign(np.dot(u[t].ravel(), ue[t].ravel()))
            np.testing.assert_allclose(u[t] * s, ue[t], atol=1e-8)
            np.testing.assert_allclose(v[t] * s, ve[t], atol=1e-8 * sve[0])


def test_pc_expansion_pins():
    """Pins of pd_pc_expansion that do not use the oracle: at full rank the terms
    rebuild S exactly and sum sigma^2 = ||S||_F^2; the kernels are orthonormal
    with their largest entry positive; v_k = S^T u_k and ||v_k|| = sigma_k; a
    single profile (rank-one S) gives one term whatever the request; the
    result does not depend on the seed beyond rounding."""
    taps, R = S.pd_op1_taps(48)
    Sm = _svir(taps)
    full = min(Sm.shape)
    u, v, sv = S.pd_pc_expansion(taps, R, full, oversample=0, power_iters=1)
    k = u.shape[0]
    U = u.reshape(k, -1)
    np.testing.assert_allclose(U.T @ v, Sm, atol=1e-12 * sv[0])
    np.testing.assert_allclose(np.sum(sv ** 2), np.sum(Sm ** 2), rtol=1e-12)
    np.testing.assert_allclose(U @ U.T, np.eye(k), atol=1e-12)
    assert np.all(np.diff(sv) <= 0)
    for t in range(k):
        assert U[t, np.argmax(np.abs(U[t]))] > 0
    np.testing.assert_allclose(v, U @ Sm, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), sv, rtol=1e-10, atol=1e-13 * sv[0])
    one = np.tile(np.array([[0.25, 0.5, 0.25]]), (10, 1))
    u1, v1, s1 = S.pd_pc_expansion(one, 1, 5)
    assert u1.shape[0] == 1
    np.testing.assert_allclose(u1[0], np.outer(one[0], one[0]) / np.linalg.norm(np.outer(one[0], one[0])),
                               atol=1e-15)
    a = S.pd_pc_expansion(taps, R, 5, seed=1)
    b = S.pd_pc_expansion(taps, R, 5, seed=12345)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, atol=1e-10)


def test_pc_expansion_argument_errors():
    L = C.load()
    taps, R = S.pd_op1_taps(16)
    u = np.zeros((5, (2 * R + 1) ** 2))
    v = np.zeros((5, 16))
    m = ctypes.c_int32()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    ok = (dp(taps), 16, R, 5, 10, 2, 0, dp(u), dp(v), None, ctypes.byref(m))
    assert L.pd_pc_expansion(*ok) == C.PD_OK and m.value == 5
    for i, bad in ((0, None), (1, 0), (2, -1), (2, 65), (3, 0), (4, -1), (5, 17), (7, None), (8, None),
                   (10, None)):
        args = list(ok)
        args[i] = bad
        assert L.pd_pc_expansion(*args) == C.PD_ERR_ARG, i
    zero = np.zeros_like(taps)
    assert L.pd_pc_expansion(dp(zero), 16, R, 5, 10, 2, 0, dp(u), dp(v), None, ctypes.byref(m)) == C.PD_ERR_ARG


def _fake(n):
    return ctypes.c_void_p(0x1000 * n)


def _call_solve(shape, dtype=C.PD_F32, op=None, wav=None, w=None, prm=None, f0=1, zc=2, zp=3,
                ws=4, ws_bytes=None):
    L = C.load()
    h = S.pd_symmlet(6)
    wav = wav or C.pd_wavelet(12, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    lw = np.zeros(shape.levels + 1 if shape.levels > 0 else 1)
    w = w or C.pd_weights(lw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0)
    op = op or C.pd_operator(C.PD_OP_IDENTITY, 0, None)
    prm = prm or C.pd_params(0.5, 10, 0, 0)
    if ws_bytes is None:
        ws_bytes = 1 << 40
    return L.pd_solve(ctypes.byref(shape), dtype, ctypes.byref(op), ctypes.byref(wav), ctypes.byref(w),
                      ctypes.byref(prm), _fake(f0) if f0 else None, _fake(zc) if zc else None,
                      _fake(zp) if zp else None, 1, None, None, _fake(ws) if ws else None,
                      ws_bytes, None)


def test_argument_errors_are_reported_without_gpu_work():
    ok = C.pd_shape(64, 64, 1, 6)
    assert _call_solve(C.pd_shape(100, 64, 1, 3)) == C.PD_ERR_SHAPE      # 100 % 8 != 0
    assert _call_solve(C.pd_shape(64, 64, 1, 7)) == C.PD_ERR_SHAPE       # too deep
    assert _call_solve(C.pd_shape(64, 64, 0, 3)) == C.PD_ERR_SHAPE       # no channel
    assert _call_solve(C.pd_shape(64, 64, 5, 3)) == C.PD_ERR_SHAPE       # too many channels
    assert _call_solve(ok, dtype=7) == C.PD_ERR_ARG
    assert _call_solve(ok, f0=0) == C.PD_ERR_ARG
    assert _call_solve(ok, zc=2, zp=2) == C.PD_ERR_ARG                   # aliased state
    assert _call_solve(ok, prm=C.pd_params(0.0, 10, 0, 0)) == C.PD_ERR_TAU
    assert _call_solve(ok, prm=C.pd_params(float("nan"), 10, 0, 0)) == C.PD_ERR_TAU
    assert _call_solve(ok, prm=C.pd_params(0.5, -1, 0, 0)) == C.PD_ERR_ARG
    assert _call_solve(ok, op=C.pd_operator(9, 0, None)) == C.PD_ERR_ARG
    assert _call_solve(ok, op=C.pd_operator(C.PD_OP_ROWBLUR, 9, None)) == C.PD_ERR_ARG
    assert _call_solve(ok, op=C.pd_operator(C.PD_OP_ROWBLUR, 12, _fake(9))) == C.PD_ERR_UNSUPPORTED
    # product-convolution expansion: kernels, multipliers and 1..64 terms required
    assert _call_solve(ok, op=C.pd_operator(C.PD_OP_PC, 3, _fake(9), 0, _fake(10))) == C.PD_ERR_ARG
    assert _call_solve(ok, op=C.pd_operator(C.PD_OP_PC, 3, _fake(9), 5, None)) == C.PD_ERR_ARG
    assert _call_solve(ok, op=C.pd_operator(C.PD_OP_PC, 3, _fake(9), 65, _fake(10))) == C.PD_ERR_UNSUPPORTED
    assert _call_solve(ok, op=C.pd_operator(C.PD_OP_PC, 10, _fake(9), 5, _fake(10))) == C.PD_ERR_UNSUPPORTED
    h3 = np.zeros(3)
    assert _call_solve(ok, wav=C.pd_wavelet(3, h3.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))) \
        == C.PD_ERR_UNSUPPORTED
    both = C.pd_weights(None, None, 0)
    assert _call_solve(ok, w=both) == C.PD_ERR_ARG
    need = C.load().pd_workspace_size(ctypes.byref(ok), C.PD_F32)
    assert need > 0
    assert _call_solve(ok, ws_bytes=need - 1) == C.PD_ERR_WORKSPACE


def test_workspace_size_rejects_bad_shapes():
    L = C.load()
    assert L.pd_workspace_size(ctypes.byref(C.pd_shape(100, 64, 1, 3)), C.PD_F32) == 0
    a = L.pd_workspace_size(ctypes.byref(C.pd_shape(512, 512, 1, 9)), C.PD_F32)
    b = L.pd_workspace_size(ctypes.byref(C.pd_shape(512, 512, 1, 9)), C.PD_F64)
    assert 2 * 512 * 512 * 4 < a < b


def test_strerror_covers_codes():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert C.strerror(code) != "unknown status"


def _call_wsolve(shape, dtype=C.PD_F32, th=None, tht=None, w=None, prm=None, z0=1, zc=2, zp=3, ws=4,
                 ws_bytes=None, lw_len=None):
    L = C.load()
    n = shape.n1 * shape.n2
    csr = C.pd_csr(n, 10, _fake(5), _fake(6), _fake(7))
    th = csr if th is None else th
    tht = csr if tht is None else tht
    lw = np.zeros(shape.levels + 1 if shape.levels > 0 else 1)
    w = w or C.pd_weights(lw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0)
    prm = prm or C.pd_params(0.5, 10, 0, 0)
    if ws_bytes is None:
        ws_bytes = 1 << 40
    return L.pd_wsolve(ctypes.byref(shape), dtype, ctypes.byref(th) if th else None,
                       ctypes.byref(tht) if tht else None, ctypes.byref(w), ctypes.byref(prm), 1,
                       _fake(z0) if z0 else None, _fake(zc) if zc else None, _fake(zp) if zp else None, 1, None,
                       _fake(ws) if ws else None, ws_bytes, None)


def test_wavelet_domain_argument_errors_without_gpu_work():
    """pd_wsolve / pd_csr_transpose / pd_spmv reject bad arguments before any
    device work (the pointers here are never dereferenced)."""
    L = C.load()
    ok = C.pd_shape(64, 64, 1, 6)
    assert _call_wsolve(C.pd_shape(64, 64, 2, 6)) == C.PD_ERR_SHAPE      # one channel only
    assert _call_wsolve(C.pd_shape(100, 64, 1, 3)) == C.PD_ERR_SHAPE
    assert _call_wsolve(ok, dtype=5) == C.PD_ERR_ARG
    assert _call_wsolve(ok, th=C.pd_csr(64 * 64 + 1, 10, _fake(5), _fake(6), _fake(7))) == C.PD_ERR_SHAPE
    assert _call_wsolve(ok, th=C.pd_csr(4096, 10, None, _fake(6), _fake(7))) == C.PD_ERR_ARG
    assert _call_wsolve(ok, th=C.pd_csr(4096, -1, _fake(5), _fake(6), _fake(7))) == C.PD_ERR_ARG
    assert _call_wsolve(ok, prm=C.pd_params(-1.0, 10, 0, 0)) == C.PD_ERR_TAU
    assert _call_wsolve(ok, prm=C.pd_params(0.5, -2, 0, 0)) == C.PD_ERR_ARG
    assert _call_wsolve(ok, zc=3, zp=3) == C.PD_ERR_ARG
    assert _call_wsolve(ok, z0=2) == C.PD_ERR_ARG
    assert _call_wsolve(ok, w=C.pd_weights(None, None, 0)) == C.PD_ERR_ARG
    need = L.pd_wsolve_workspace_size(ctypes.byref(ok), C.PD_F32)
    assert need >= 3 * 4096 * 4
    assert L.pd_wsolve_workspace_size(ctypes.byref(C.pd_shape(64, 64, 3, 6)), C.PD_F32) == 0
    assert _call_wsolve(ok, ws_bytes=need - 1) == C.PD_ERR_WORKSPACE
    bad = C.pd_csr(0, 0, _fake(5), None, None)
    assert L.pd_csr_transpose(ctypes.byref(bad), C.PD_F32, _fake(1), _fake(2), _fake(3), _fake(4), 1 << 30,
                              None) == C.PD_ERR_ARG
    a = C.pd_csr(100, 10, _fake(5), _fake(6), _fake(7))
    assert L.pd_csr_transpose(ctypes.byref(a), C.PD_F32, _fake(1), _fake(2), _fake(3), _fake(4), 8,
                              None) == C.PD_ERR_WORKSPACE
    assert L.pd_spmv(ctypes.byref(a), C.PD_F32, None, _fake(2), None) == C.PD_ERR_ARG
    assert L.pd_wjacobi(ctypes.byref(a), C.PD_F32, None, None) == C.PD_ERR_ARG


def _call_admm(shape, dtype=C.PD_F32, op=None, w=None, beta=1.0, iters=5, f0=1, fo=2, zo=3, ws=4,
               ws_bytes=None):
    L = C.load()
    h = S.pd_symmlet(6)
    wav = C.pd_wavelet(12, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    lw = np.zeros(shape.levels + 1 if shape.levels > 0 else 1)
    w = w or C.pd_weights(lw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0)
    op = op or C.pd_operator(C.PD_OP_PC, 2, _fake(8), 3, _fake(9))
    if ws_bytes is None:
        ws_bytes = 1 << 40
    return L.pd_admm_solve(ctypes.byref(shape), dtype, ctypes.byref(op), ctypes.byref(wav), ctypes.byref(w),
                           beta, iters, _fake(f0) if f0 else None, _fake(fo) if fo else None,
                           _fake(zo) if zo else None, None, _fake(ws) if ws else None, ws_bytes, None)


def test_admm_argument_errors_without_gpu_work():
    """pd_admm_solve / pd_fft2 reject bad arguments before any device work."""
    L = C.load()
    ok = C.pd_shape(64, 32, 2, 4)
    assert _call_admm(C.pd_shape(96, 64, 1, 3)) == C.PD_ERR_UNSUPPORTED       # 96 is not a power of two
    assert _call_admm(C.pd_shape(4096, 64, 1, 3), dtype=C.PD_F64) == C.PD_ERR_UNSUPPORTED  # FP64 LDS limit
    assert _call_admm(C.pd_shape(64, 64, 0, 3)) == C.PD_ERR_SHAPE
    assert _call_admm(ok, dtype=7) == C.PD_ERR_ARG
    assert _call_admm(ok, op=C.pd_operator(C.PD_OP_ROWBLUR, 2, _fake(8), 0, None)) == C.PD_ERR_UNSUPPORTED
    assert _call_admm(ok, op=C.pd_operator(C.PD_OP_PC, 2, _fake(8), 0, _fake(9))) == C.PD_ERR_ARG
    assert _call_admm(ok, op=C.pd_operator(C.PD_OP_PC, 2, _fake(8), 65, _fake(9))) == C.PD_ERR_UNSUPPORTED
    assert _call_admm(ok, beta=0.0) == C.PD_ERR_TAU
    assert _call_admm(ok, beta=float("nan")) == C.PD_ERR_TAU
    assert _call_admm(ok, iters=-1) == C.PD_ERR_ARG
    assert _call_admm(ok, fo=1) == C.PD_ERR_ARG              # f_out aliases f0
    assert _call_admm(ok, zo=2) == C.PD_ERR_ARG              # z_out aliases f_out
    assert _call_admm(ok, f0=0) == C.PD_ERR_ARG
    assert _call_admm(ok, w=C.pd_weights(None, None, 0)) == C.PD_ERR_ARG
    lw = np.zeros(5)
    joint = C.pd_weights(lw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 1)
    assert _call_admm(ok, w=joint) == C.PD_ERR_UNSUPPORTED
    need = L.pd_admm_workspace_size(ctypes.byref(ok), C.PD_F32, 3)
    assert need > (3 * 3 + 2 * 3 * 2) * 64 * 32 * 4
    assert L.pd_admm_workspace_size(ctypes.byref(ok), C.PD_F32, 4) > need
    assert L.pd_admm_workspace_size(ctypes.byref(ok), C.PD_F32, 0) == 0
    assert _call_admm(ok, ws_bytes=need - 1) == C.PD_ERR_WORKSPACE
    # FFT utility
    assert L.pd_fft2_workspace_size(64, 32, C.PD_F32) > 0
    assert L.pd_fft2_workspace_size(48, 32, C.PD_F32) == 0
    assert L.pd_fft2_workspace_size(4096, 8, C.PD_F64) == 0
    assert L.pd_fft2(48, 32, 1, C.PD_F32, 0, _fake(1), _fake(2), 1 << 20, None) == C.PD_ERR_UNSUPPORTED
    assert L.pd_fft2(64, 32, -1, C.PD_F32, 0, _fake(1), _fake(2), 1 << 20, None) == C.PD_ERR_ARG
    assert L.pd_fft2(64, 32, 1, C.PD_F32, 0, None, _fake(2), 1 << 20, None) == C.PD_ERR_ARG
    assert L.pd_fft2(64, 32, 1, C.PD_F32, 0, _fake(1), _fake(2), 8, None) == C.PD_ERR_WORKSPACE
    assert L.pd_fft2(64, 32, 0, C.PD_F32, 0, None, None, 0, None) == C.PD_OK


def test_decompose_argument_errors_without_gpu_work():
    L = C.load()
    h = S.pd_symmlet(6)
    wav = C.pd_wavelet(12, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    op = C.pd_operator(C.PD_OP_PC, 1, _fake(8), 2, _fake(9))
    nnz = ctypes.c_int64(0)

    def call(shape, op=op, eta=0.1, cap=0, rows=None, vals=None, ws=4, ws_bytes=1 << 40, cp=5):
        return L.pd_decompose(ctypes.byref(shape), ctypes.byref(op), ctypes.byref(wav), eta, cap, ctypes.byref(nnz),
                              _fake(cp) if cp else None, rows, vals, _fake(ws) if ws else None, ws_bytes, None)

    ok = C.pd_shape(32, 16, 1, 2)
    assert call(C.pd_shape(32, 16, 2, 2)) == C.PD_ERR_SHAPE
    assert call(C.pd_shape(32, 16, 1, 0)) == C.PD_ERR_SHAPE
    assert call(ok, op=C.pd_operator(C.PD_OP_ROWBLUR, 1, _fake(8), 0, None)) == C.PD_ERR_UNSUPPORTED
    assert call(ok, eta=-1.0) == C.PD_ERR_TAU
    assert call(ok, eta=float("inf")) == C.PD_ERR_TAU
    assert call(ok, cap=-1) == C.PD_ERR_ARG
    assert call(ok, cap=10) == C.PD_ERR_ARG          # capacity without rows / vals
    assert call(ok, cp=0) == C.PD_ERR_ARG
    need = L.pd_decompose_workspace_size(ctypes.byref(ok), 2)
    assert need > 4 * 256 * 512 * 8
    assert L.pd_decompose_workspace_size(ctypes.byref(ok), 3) > need
    assert L.pd_decompose_workspace_size(ctypes.byref(ok), 0) == 0
    assert call(ok, ws_bytes=need - 1) == C.PD_ERR_WORKSPACE


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N > 1 exits with a message (the solver runs on one GPU),
    before importing torch or touching a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_batched_argument_errors_without_gpu_work():
    """pd_solve_batched checks every descriptor on the host first: one prox kind
    per batch (and one channel count when joint), weights as for pd_solve,
    images packed back to back, a large enough workspace."""
    L = C.load()
    h = S.pd_symmlet(6)
    wav = C.pd_wavelet(12, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    lw = np.full(4, 0.1)
    lwp = lw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def descs(specs):
        d = (C.pd_image_desc * len(specs))()
        off = 0
        for b, (n, ch, joint, coeff) in enumerate(specs):
            d[b].shape = C.pd_shape(n, n, ch, 3)
            d[b].offset = off
            d[b].tau = 0.5
            d[b].op = C.pd_operator(C.PD_OP_ROWBLUR, 9, _fake(7))
            d[b].w = C.pd_weights(None if coeff else lwp, _fake(8) if coeff else None, joint)
            off += n * n * ch
        return d

    def call(d, ws_bytes=1 << 40):
        return L.pd_solve_batched(len(d), d, C.PD_F32, ctypes.byref(wav), 10, _fake(1), _fake(2), None,
                                  _fake(3), ws_bytes, None)

    assert call(descs([(32, 3, 1, 0), (64, 1, 0, 0)])) == C.PD_ERR_UNSUPPORTED   # joint and scalar mixed
    assert call(descs([(32, 3, 1, 0), (64, 2, 1, 0)])) == C.PD_ERR_UNSUPPORTED   # joint, channel counts differ
    assert call(descs([(32, 2, 1, 1)])) == C.PD_ERR_UNSUPPORTED                  # joint needs band weights
    both = descs([(32, 1, 0, 0)])
    both[0].w = C.pd_weights(lwp, _fake(8), 0)
    assert call(both) == C.PD_ERR_ARG                                             # exactly one weight kind
    d = descs([(32, 1, 0, 0), (64, 1, 0, 1)])
    d[1].offset += 1
    assert call(d) == C.PD_ERR_ARG                                                # not packed back to back
    d = descs([(32, 1, 0, 0), (64, 1, 0, 1)])
    need = L.pd_batched_workspace_size(2, d, C.PD_F32)
    assert need > 0 and call(d, need - 1) == C.PD_ERR_WORKSPACE


def test_noalloc_size_limit_without_gpu_work():
    """pd_solve_noalloc rejects a problem whose workspace exceeds its fixed
    scratch (PD_NOALLOC_SCRATCH_BYTES, 16 MiB) before touching the device."""
    L = C.load()
    h = S.pd_symmlet(6)
    wav = C.pd_wavelet(12, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    big = C.pd_shape(2048, 2048, 1, 11)
    small = C.pd_shape(1024, 1024, 1, 10)
    assert L.pd_workspace_size(ctypes.byref(big), C.PD_F32) > (16 << 20)
    assert L.pd_workspace_size(ctypes.byref(small), C.PD_F32) <= (16 << 20)
    lw = np.zeros(12)
    w = C.pd_weights(lw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0)
    op = C.pd_operator(C.PD_OP_IDENTITY, 0, None)
    prm = C.pd_params(0.5, 10, 0, 0)
    rc = L.pd_solve_noalloc(ctypes.byref(big), C.PD_F32, ctypes.byref(op), ctypes.byref(wav), ctypes.byref(w),
                            ctypes.byref(prm), _fake(1), _fake(2), _fake(3), 1, None, None, None)
    assert rc == C.PD_ERR_WORKSPACE
    bad = C.pd_shape(100, 64, 1, 3)
    rc = L.pd_solve_noalloc(ctypes.byref(bad), C.PD_F32, ctypes.byref(op), ctypes.byref(wav), ctypes.byref(w),
                            ctypes.byref(prm), _fake(1), _fake(2), _fake(3), 1, None, None, None)
    assert rc == C.PD_ERR_SHAPE
