"""Python binding of libpd: argument marshalling over torch device tensors.

Every step of the solver runs in libpd's HIP kernels; torch only provides
device memory and the current HIP stream.  Names follow the C ABI
(include/pd.h).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as C

_DT = {torch.float32: C.PD_F32, torch.float64: C.PD_F64}


def _dtype_code(dtype: torch.dtype) -> int:
    if dtype not in _DT:
        raise TypeError(f"unsupported dtype {dtype}; use float32 or float64")
    return _DT[dtype]


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_dev(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("libpd needs contiguous device tensors")


# ------------------------------------------------------------------- set-up --
def pd_symmlet(moments: int = 6) -> np.ndarray:
    """Low-pass filter of the Symmlet with `moments` vanishing moments (host)."""
    h = np.zeros(2 * moments)
    C.check(C.load().pd_symmlet(moments, _dptr(h)), "pd_symmlet")
    return h


def pd_op1_taps(n2: int, sigma_max: float = 3.0, mass: float = 0.99):
    """Operator-1 profile table (n2, 2R+1) of source rows and its half-width R."""
    r = ctypes.c_int32()
    L = C.load()
    C.check(L.pd_op1_taps(n2, sigma_max, mass, ctypes.byref(r), None), "pd_op1_taps")
    taps = np.zeros((n2, 2 * r.value + 1))
    C.check(L.pd_op1_taps(n2, sigma_max, mass, ctypes.byref(r), _dptr(taps)), "pd_op1_taps")
    return taps, r.value


def pd_pc_expansion(taps, radius: int, terms: int, oversample: int = 10, power_iters: int = 2, seed: int = 0):
    """Rank-`terms` product-convolution expansion of a row-profile operator by
    libpd's randomized SVD of its impulse responses (Section 3.3.3).  Returns
    (u (m, 2R+1, 2R+1), v (m, n2), singular values (m,)), m <= terms."""
    taps = np.ascontiguousarray(taps, dtype=np.float64)
    n2, W = taps.shape
    if W != 2 * radius + 1:
        raise ValueError("taps must be (n2, 2R+1)")
    u = np.zeros((terms, W * W))
    v = np.zeros((terms, n2))
    sv = np.zeros(terms)
    m = ctypes.c_int32()
    C.check(C.load().pd_pc_expansion(_dptr(taps), n2, radius, terms, oversample, power_iters, seed, _dptr(u),
                                     _dptr(v), _dptr(sv), ctypes.byref(m)), "pd_pc_expansion")
    k = m.value
    return u[:k].reshape(k, W, W).copy(), v[:k].copy(), sv[:k].copy()


@dataclass
class Operator:
    """Blur operator on the device: PD_OP_IDENTITY, a row-profile table
    (PD_OP_ROWBLUR) or a product-convolution expansion (PD_OP_PC: kernels
    `taps` (m, 2R+1, 2R+1) and multipliers `mult` (m, n2, n1))."""
    kind: int
    radius: int = 0
    taps: torch.Tensor | None = None
    mult: torch.Tensor | None = None

    @staticmethod
    def pc(u, v, dtype=torch.float32, device="cuda") -> "Operator":
        """H f = sum_k u_k * (v_k . f): u (m, 2R+1, 2R+1) kernels, v (m, n2, n1)
        per-pixel multipliers."""
        ut = torch.as_tensor(np.asarray(u), dtype=dtype, device=device).contiguous()
        vt = torch.as_tensor(np.asarray(v), dtype=dtype, device=device).contiguous()
        if ut.dim() != 3 or ut.shape[1] != ut.shape[2] or ut.shape[1] % 2 == 0 or vt.dim() != 3 \
                or vt.shape[0] != ut.shape[0]:
            raise ValueError("u must be (m, 2R+1, 2R+1) and v (m, n2, n1)")
        return Operator(C.PD_OP_PC, int(ut.shape[1] // 2), ut, vt)

    @staticmethod
    def identity() -> "Operator":
        return Operator(C.PD_OP_IDENTITY)

    @staticmethod
    def op1(n2: int, dtype=torch.float32, device="cuda", sigma_max=3.0, mass=0.99) -> "Operator":
        taps, R = pd_op1_taps(n2, sigma_max, mass)
        return Operator(C.PD_OP_ROWBLUR, R, torch.as_tensor(taps, dtype=dtype, device=device).contiguous())

    @staticmethod
    def from_taps(taps, radius: int, dtype=torch.float32, device="cuda") -> "Operator":
        t = torch.as_tensor(np.asarray(taps), dtype=dtype, device=device).contiguous()
        return Operator(C.PD_OP_ROWBLUR, int(radius), t)

    def c(self) -> C.pd_operator:
        return C.pd_operator(self.kind, self.radius, None if self.taps is None else self.taps.data_ptr(),
                             0 if self.mult is None else int(self.mult.shape[0]),
                             None if self.mult is None else self.mult.data_ptr())


def _shape(x: torch.Tensor, levels: int) -> C.pd_shape:
    if x.dim() != 3:
        raise ValueError("expected a (C, n2, n1) tensor")
    c, n2, n1 = x.shape
    return C.pd_shape(n1, n2, c, levels)


def _wavelet(h) -> tuple[C.pd_wavelet, np.ndarray]:
    h = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
    return C.pd_wavelet(len(h), _dptr(h)), h


def pd_workspace_size(shape: C.pd_shape, dtype: torch.dtype) -> int:
    return int(C.load().pd_workspace_size(ctypes.byref(shape), _dtype_code(dtype)))


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------- solve ---
def pd_solve(f0: torch.Tensor, op: Operator, h, levels: int, tau: float, iters: int,
             level_w=None, coeff_w: torch.Tensor | None = None, joint: bool = False,
             z_cur: torch.Tensor | None = None, z_prev: torch.Tensor | None = None,
             init: bool = True, iter_offset: int = 0, want_f: bool = True,
             stats: bool = False, check_finite: bool = False,
             ws: torch.Tensor | None = None):
    """Run `iters` FISTA iterations on eq. 4.1.  Returns a dict with f (Psi z),
    z_cur, z_prev and stats ((iters, 3) FP64: data term and regulariser at
    y(i), ||z(i) - y(i)||^2)."""
    _check_dev(f0, coeff_w, z_cur, z_prev)
    dt = _dtype_code(f0.dtype)
    shape = _shape(f0, levels)
    wav, hh = _wavelet(h)
    lw = None
    if level_w is not None:
        lw = np.ascontiguousarray(np.asarray(level_w, dtype=np.float64))
        if lw.shape != (levels + 1,):
            raise ValueError("level_w needs levels+1 entries")
    w = C.pd_weights(_dptr(lw) if lw is not None else None,
                     None if coeff_w is None else coeff_w.data_ptr(), 1 if joint else 0)
    prm = C.pd_params(float(tau), int(iters), int(iter_offset), 1 if check_finite else 0)
    if z_cur is None:
        z_cur = torch.empty_like(f0)
    if z_prev is None:
        z_prev = torch.empty_like(f0)
    f = torch.empty_like(f0) if want_f else None
    st = torch.zeros((max(iters, 1), 3), dtype=torch.float64, device=f0.device) if stats else None
    need = pd_workspace_size(shape, f0.dtype)
    if ws is None or ws.numel() < need:
        ws = workspace(need, f0.device)
    opc = op.c()
    rc = C.load().pd_solve(ctypes.byref(shape), dt, ctypes.byref(opc), ctypes.byref(wav),
                           ctypes.byref(w), ctypes.byref(prm), _ptr(f0), _ptr(z_cur), _ptr(z_prev),
                           1 if init else 0, _ptr(f), _ptr(st), _ptr(ws), ws.numel(),
                           _stream(f0.device))
    C.check(rc, "pd_solve")
    return {"f": f, "z_cur": z_cur, "z_prev": z_prev,
            "stats": None if st is None else st[:iters]}


def pd_fwt(x: torch.Tensor, h, levels: int, inverse: bool = False,
           ws: torch.Tensor | None = None) -> torch.Tensor:
    """Psi^* x (forward) or Psi x (inverse) for a (C, n2, n1) tensor."""
    _check_dev(x)
    shape = _shape(x, levels)
    wav, hh = _wavelet(h)
    out = torch.empty_like(x)
    need = pd_workspace_size(shape, x.dtype)
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    rc = C.load().pd_fwt(ctypes.byref(shape), _dtype_code(x.dtype), ctypes.byref(wav),
                         1 if inverse else 0, _ptr(x), _ptr(out), _ptr(ws), ws.numel(),
                         _stream(x.device))
    C.check(rc, "pd_fwt")
    return out


def pd_apply_op(x: torch.Tensor, op: Operator, transpose: bool = False) -> torch.Tensor:
    """H x or H^T x for a (C, n2, n1) tensor."""
    _check_dev(x)
    shape = _shape(x, 1 if x.shape[1] % 2 == 0 and x.shape[2] % 2 == 0 else 0)
    shape.levels = 1
    out = torch.empty_like(x)
    opc = op.c()
    rc = C.load().pd_apply_op(ctypes.byref(shape), _dtype_code(x.dtype), ctypes.byref(opc),
                              1 if transpose else 0, _ptr(x), _ptr(out), _stream(x.device))
    C.check(rc, "pd_apply_op")
    return out


def lipschitz(op: Operator, n1: int, n2: int, iters: int = 200, seed: int = 0,
              dtype=torch.float64, device="cuda") -> float:
    """||H^T H||_2 by power iteration on the GPU (host-side normalisation)."""
    if op.kind == C.PD_OP_IDENTITY:
        return 1.0
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn((1, n2, n1), generator=g, dtype=torch.float64).to(device=device, dtype=dtype)
    x /= torch.linalg.vector_norm(x)
    lam = 0.0
    opd = op if op.taps is None or op.taps.dtype == dtype else \
        Operator(op.kind, op.radius, op.taps.to(dtype), None if op.mult is None else op.mult.to(dtype))
    for _ in range(iters):
        y = pd_apply_op(pd_apply_op(x, opd), opd, transpose=True)
        lam = float(torch.linalg.vector_norm(y))
        x = y / lam
    return lam


def step_size(op: Operator, n1: int, n2: int, device="cuda") -> float:
    return 1.0 / (lipschitz(op, n1, n2, device=device) * (1.0 + 1e-6))


BLUR_VARIANTS = (32, 48, 1020, 1039, 1058)


def pd_tune(f0: torch.Tensor, op: Operator, levels: int, pin: int = 0) -> int:
    """Autotune the blur for f0's size and this operator (cached in the
    library for later solves of the same size); returns the chosen variant
    code (0: nothing to tune): 32 / 48 = one fused kernel with that many
    output rows per workgroup, 1020 / 1039 / 1058 = two marching kernels with
    20 / 39 / 58 rows per wave.  pin = one of BLUR_VARIANTS records that
    variant untimed.  Results never depend on the variant."""
    _check_dev(f0)
    shape = _shape(f0, levels)
    ws = workspace(pd_workspace_size(shape, f0.dtype), f0.device)
    ch = ctypes.c_int32(int(pin))
    opc = op.c()
    rc = C.load().pd_tune(ctypes.byref(shape), _dtype_code(f0.dtype), ctypes.byref(opc), _ptr(ws), ws.numel(),
                          ctypes.byref(ch), _stream(f0.device))
    C.check(rc, "pd_tune")
    return int(ch.value)


def pd_solve_noalloc(f0: torch.Tensor, op: Operator, h, levels: int, tau: float, iters: int,
                     level_w=None, coeff_w: torch.Tensor | None = None, joint: bool = False,
                     z_cur: torch.Tensor | None = None, z_prev: torch.Tensor | None = None,
                     init: bool = True, iter_offset: int = 0, f_out: torch.Tensor | None = None,
                     stats: torch.Tensor | None = None, check_finite: bool = False):
    """pd_solve on the library's fixed scratch (no workspace argument, no
    device allocation inside the call).  Every output buffer the caller does
    not pass is allocated here, by torch, before the call."""
    _check_dev(f0, coeff_w, z_cur, z_prev, f_out, stats)
    shape = _shape(f0, levels)
    wav, hh = _wavelet(h)
    lw = None
    if level_w is not None:
        lw = np.ascontiguousarray(np.asarray(level_w, dtype=np.float64))
        if lw.shape != (levels + 1,):
            raise ValueError("level_w needs levels+1 entries")
    w = C.pd_weights(_dptr(lw) if lw is not None else None,
                     None if coeff_w is None else coeff_w.data_ptr(), 1 if joint else 0)
    prm = C.pd_params(float(tau), int(iters), int(iter_offset), 1 if check_finite else 0)
    z_cur = torch.empty_like(f0) if z_cur is None else z_cur
    z_prev = torch.empty_like(f0) if z_prev is None else z_prev
    opc = op.c()
    rc = C.load().pd_solve_noalloc(ctypes.byref(shape), _dtype_code(f0.dtype), ctypes.byref(opc),
                                   ctypes.byref(wav), ctypes.byref(w), ctypes.byref(prm), _ptr(f0), _ptr(z_cur),
                                   _ptr(z_prev), 1 if init else 0, _ptr(f_out), _ptr(stats), _stream(f0.device))
    C.check(rc, "pd_solve_noalloc")
    return {"f": f_out, "z_cur": z_cur, "z_prev": z_prev, "stats": stats}


# ----------------------------------------------------------------- batched ---
def pd_solve_batched(f0s: list[torch.Tensor], ops: list[Operator], level_ws, taus, h,
                     levels: list[int], iters: int, stats: bool = False, coeff_ws=None, joint: bool = False):
    """Solve a batch of uneven-size problems in lock-step launches; returns the
    list of f = Psi z and the (batch, iters, 3) FP64 statistics (or None).
    Weights per image: level_ws[b] (host band weights) or, when coeff_ws is
    given and coeff_ws[b] is not None, that image's device weight map; joint
    applies the group prox to every image (all with one channel count)."""
    dev = f0s[0].device
    dtype = f0s[0].dtype
    _check_dev(*f0s, *([] if coeff_ws is None else [c for c in coeff_ws if c is not None]))
    sizes = [t.numel() for t in f0s]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    f0p = torch.cat([t.reshape(-1) for t in f0s]).contiguous()
    fo = torch.empty_like(f0p)
    descs = (C.pd_image_desc * len(f0s))()
    keep = []
    for b, t in enumerate(f0s):
        cw = None if coeff_ws is None else coeff_ws[b]
        lw = None
        if cw is None:
            lw = np.ascontiguousarray(np.asarray(level_ws[b], dtype=np.float64))
            if lw.shape != (levels[b] + 1,):
                raise ValueError("level_w needs levels+1 entries")
            keep.append(lw)
        elif cw.shape != t.shape or cw.dtype != dtype or not cw.is_contiguous():
            raise ValueError("coeff_w must match its image's shape and dtype, contiguous")
        descs[b].shape = _shape(t, levels[b])
        descs[b].offset = int(offs[b])
        descs[b].tau = float(taus[b])
        descs[b].op = ops[b].c()
        descs[b].w = C.pd_weights(_dptr(lw) if lw is not None else None, None if cw is None else cw.data_ptr(),
                                  1 if joint else 0)
    wav, hh = _wavelet(h)
    L = C.load()
    dt = _dtype_code(dtype)
    need = L.pd_batched_workspace_size(len(f0s), descs, dt)
    if need == 0:
        raise C.PDError(C.PD_ERR_SHAPE, "pd_batched_workspace_size")
    ws = workspace(need, dev)
    st = torch.zeros((len(f0s), max(iters, 1), 3), dtype=torch.float64, device=dev) if stats else None
    rc = L.pd_solve_batched(len(f0s), descs, dt, ctypes.byref(wav), int(iters), _ptr(f0p), _ptr(fo),
                            _ptr(st), _ptr(ws), ws.numel(), _stream(dev))
    C.check(rc, "pd_solve_batched")
    outs = [fo[o:o + n].view_as(t) for o, n, t in zip(offs, sizes, f0s)]
    return outs, st


# ------------------------------------------------------------- diagnostics ---
def pd_fuse_enable(enable: bool = True) -> None:
    """Fusion of the coarsest fine synthesis levels (three, or two) and of the two coarsest
    fine analysis levels of an iteration into one launch each (bitwise-identical results)."""
    C.check(C.load().pd_fuse_enable(1 if enable else 0), "pd_fuse_enable")


def pd_graphs_enable(enable: bool = True) -> None:
    """Graph replay of pd_solve's middle iterations (bitwise-identical results)."""
    C.check(C.load().pd_graphs_enable(1 if enable else 0), "pd_graphs_enable")


def pd_timing_enable(enable: bool = True) -> None:
    C.check(C.load().pd_timing_enable(1 if enable else 0), "pd_timing_enable")


def pd_timing_read() -> list[dict]:
    """Per (kernel class, level): launches and total milliseconds, measured by
    HIP events the library recorded on the launch stream."""
    L = C.load()
    rows = ctypes.c_int32()
    C.check(L.pd_timing_read(0, None, None, None, None, ctypes.byref(rows)), "pd_timing_read")
    n = rows.value
    kc = (ctypes.c_int32 * max(n, 1))()
    lv = (ctypes.c_int32 * max(n, 1))()
    la = (ctypes.c_int64 * max(n, 1))()
    ms = (ctypes.c_double * max(n, 1))()
    C.check(L.pd_timing_read(n, kc, lv, la, ms, ctypes.byref(rows)), "pd_timing_read")
    return [{"kernel": C.KCLASS_NAMES.get(kc[i], str(kc[i])), "kclass": kc[i], "level": lv[i],
             "launches": la[i], "total_ms": ms[i], "avg_us": 1e3 * ms[i] / max(la[i], 1)}
            for i in range(n)]


# ---------------------------------------------------------------- backward ---
def _bwd_args(f0, op, h, levels, tau, iters, level_w, coeff_w, checkpoint_every):
    dt = _dtype_code(f0.dtype)
    shape = _shape(f0, levels)
    wav, hh = _wavelet(h)
    lw = None if level_w is None else np.ascontiguousarray(np.asarray(level_w, dtype=np.float64))
    w = C.pd_weights(_dptr(lw) if lw is not None else None,
                     None if coeff_w is None else coeff_w.data_ptr(), 0)
    prm = C.pd_params(float(tau), int(iters), 0, 0)
    need = C.load().pd_backward_workspace_size(ctypes.byref(shape), dt, int(iters), int(checkpoint_every))
    if need == 0:
        raise C.PDError(C.PD_ERR_ARG, "pd_backward_workspace_size")
    return dt, shape, wav, (hh, lw), w, prm, need


def pd_backward(f0: torch.Tensor, op: Operator, h, levels: int, tau: float, iters: int,
                grad_f: torch.Tensor, level_w=None, coeff_w: torch.Tensor | None = None,
                checkpoint_every: int = 20, want_f0: bool = True, want_w: bool = True,
                ws: torch.Tensor | None = None):
    """Reverse mode of pd_solve (init = Psi^* f0): returns (dL/df0, dL/dw) for
    dL/df = grad_f.  dL/dw is per coefficient (Mallat layout).  With ws from
    pd_solve_checkpointed (same arguments), the stored checkpoints are used
    (pd_backward_checkpointed) instead of a forward pass."""
    _check_dev(f0, grad_f, coeff_w, ws)
    dt, shape, wav, keep, w, prm, need = _bwd_args(f0, op, h, levels, tau, iters, level_w, coeff_w,
                                                   checkpoint_every)
    gf0 = torch.empty_like(f0) if want_f0 else None
    gw = torch.empty_like(f0) if want_w else None
    have = ws is not None
    if ws is None:
        ws = workspace(need, f0.device)
    elif ws.numel() < need:
        raise ValueError("workspace smaller than pd_backward_workspace_size")
    opc = op.c()
    fn = C.load().pd_backward_checkpointed if have else C.load().pd_backward
    rc = fn(ctypes.byref(shape), dt, ctypes.byref(opc), ctypes.byref(wav), ctypes.byref(w),
            ctypes.byref(prm), _ptr(f0), _ptr(grad_f.contiguous()), _ptr(gf0), _ptr(gw),
            int(checkpoint_every), _ptr(ws), ws.numel(), _stream(f0.device))
    C.check(rc, "pd_backward_checkpointed" if have else "pd_backward")
    return gf0, gw


def pd_solve_checkpointed(f0: torch.Tensor, op: Operator, h, levels: int, tau: float, iters: int,
                          level_w=None, coeff_w: torch.Tensor | None = None, checkpoint_every: int = 20):
    """Forward solve from Psi^* f0 keeping the reverse mode's checkpoints:
    returns (f = Psi z(K), ws), ws to be passed to pd_backward."""
    _check_dev(f0, coeff_w)
    dt, shape, wav, keep, w, prm, need = _bwd_args(f0, op, h, levels, tau, iters, level_w, coeff_w,
                                                   checkpoint_every)
    ws = workspace(need, f0.device)
    f = torch.empty_like(f0)
    opc = op.c()
    rc = C.load().pd_solve_checkpointed(ctypes.byref(shape), dt, ctypes.byref(opc), ctypes.byref(wav),
                                        ctypes.byref(w), ctypes.byref(prm), _ptr(f0), _ptr(f),
                                        int(checkpoint_every), _ptr(ws), ws.numel(), _stream(f0.device))
    C.check(rc, "pd_solve_checkpointed")
    return f, ws


class FistaSolve(torch.autograd.Function):
    """f = Psi z(K) of pd_solve as a differentiable function of the observation
    f0 and the per-coefficient weights w.  The forward pass keeps the reverse
    mode's checkpoints (pd_solve_checkpointed); the backward pass runs
    pd_backward_checkpointed on them."""

    @staticmethod
    def forward(ctx, f0, w, op, h, levels, tau, iters, checkpoint_every):
        f0 = f0.contiguous()
        w = w.contiguous()
        out, ws = pd_solve_checkpointed(f0, op, h, levels, tau, iters, coeff_w=w,
                                        checkpoint_every=checkpoint_every)
        ctx.save_for_backward(f0, w)
        ctx.ws = ws
        ctx.cfg = (op, h, levels, tau, iters, checkpoint_every)
        return out

    @staticmethod
    def backward(ctx, grad_f):
        f0, w = ctx.saved_tensors
        op, h, levels, tau, iters, ce = ctx.cfg
        gf0, gw = pd_backward(f0, op, h, levels, tau, iters, grad_f.contiguous(), coeff_w=w,
                              checkpoint_every=ce, want_f0=ctx.needs_input_grad[0],
                              want_w=ctx.needs_input_grad[1], ws=ctx.ws)
        return gf0, gw, None, None, None, None, None, None


def solve_autograd(f0: torch.Tensor, theta: torch.Tensor, op: Operator, h, levels: int, tau: float,
                   iters: int, checkpoint_every: int = 20) -> torch.Tensor:
    """Differentiable solve with weights w = softplus(theta) (per coefficient)."""
    w = torch.nn.functional.softplus(theta)
    return FistaSolve.apply(f0, w, op, h, levels, tau, iters, checkpoint_every)


# --------------------------------------------- FISTA in the wavelet domain ---
@dataclass
class Csr:
    """A square CSR matrix on the device (row_ptr int64 [n+1], col int32 [nnz],
    val float32/float64 [nnz]); rows and columns are Mallat positions."""
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.row_ptr.numel() - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @staticmethod
    def from_arrays(row_ptr, col, val, dtype=torch.float32, device="cuda") -> "Csr":
        return Csr(torch.as_tensor(np.asarray(row_ptr, dtype=np.int64), device=device),
                   torch.as_tensor(np.asarray(col, dtype=np.int32), device=device),
                   torch.as_tensor(np.asarray(val, dtype=np.float64), dtype=dtype, device=device))

    def c(self) -> C.pd_csr:
        _check_dev(self.row_ptr, self.col, self.val)
        if self.row_ptr.dtype != torch.int64 or self.col.dtype != torch.int32:
            raise TypeError("row_ptr must be int64 and col int32")
        return C.pd_csr(self.n, self.nnz, self.row_ptr.data_ptr(),
                        self.col.data_ptr() if self.nnz else None,
                        self.val.data_ptr() if self.nnz else None)


def pd_csr_transpose(a: Csr) -> Csr:
    """The transpose of a (each row's columns sorted)."""
    dev = a.row_ptr.device
    t = Csr(torch.empty(a.n + 1, dtype=torch.int64, device=dev),
            torch.empty(max(a.nnz, 1), dtype=torch.int32, device=dev)[:a.nnz],
            torch.empty(max(a.nnz, 1), dtype=a.val.dtype, device=dev)[:a.nnz])
    need = int(C.load().pd_csr_transpose_workspace_size(a.n))
    ws = workspace(need, dev)
    ac = a.c()
    rc = C.load().pd_csr_transpose(ctypes.byref(ac), _dtype_code(a.val.dtype), _ptr(t.row_ptr),
                                   _ptr(t.col), _ptr(t.val), _ptr(ws), ws.numel(), _stream(dev))
    C.check(rc, "pd_csr_transpose")
    return t


def pd_spmv(a: Csr, x: torch.Tensor) -> torch.Tensor:
    """a @ x for a device vector x of length n."""
    _check_dev(x)
    y = torch.empty_like(x)
    ac = a.c()
    rc = C.load().pd_spmv(ctypes.byref(ac), _dtype_code(x.dtype), _ptr(x), _ptr(y), _stream(x.device))
    C.check(rc, "pd_spmv")
    return y


def pd_wjacobi(theta_t: Csr) -> torch.Tensor:
    """Jacobi preconditioner of FISTA-WP from Theta_L^T."""
    s = torch.empty(theta_t.n, dtype=theta_t.val.dtype, device=theta_t.val.device)
    tc = theta_t.c()
    rc = C.load().pd_wjacobi(ctypes.byref(tc), _dtype_code(s.dtype), _ptr(s), _stream(s.device))
    C.check(rc, "pd_wjacobi")
    return s


def wlipschitz(theta: Csr, theta_t: Csr, sigma: torch.Tensor | None = None, iters: int = 200,
               seed: int = 0) -> float:
    """||Sigma^{1/2} Theta_L^T Theta_L Sigma^{1/2}||_2 by power iteration with
    the library's sparse products (host-side normalisation)."""
    dev = theta.val.device
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(theta.n, generator=g, dtype=torch.float64).to(device=dev, dtype=theta.val.dtype)
    r = None if sigma is None else torch.sqrt(sigma)
    x /= torch.linalg.vector_norm(x)
    lam = 0.0
    for _ in range(iters):
        v = x if r is None else r * x
        y = pd_spmv(theta_t, pd_spmv(theta, v))
        if r is not None:
            y = r * y
        lam = float(torch.linalg.vector_norm(y))
        x = y / lam
    return lam


def wstep_size(theta: Csr, theta_t: Csr, sigma: torch.Tensor | None = None) -> float:
    return 1.0 / (wlipschitz(theta, theta_t, sigma) * (1.0 + 1e-6))


def pd_wsolve_workspace_size(n1: int, n2: int, levels: int, dtype: torch.dtype) -> int:
    shape = C.pd_shape(n1, n2, 1, levels)
    return int(C.load().pd_wsolve_workspace_size(ctypes.byref(shape), _dtype_code(dtype)))


def pd_wsolve(z0: torch.Tensor, theta: Csr, theta_t: Csr, levels: int, tau: float, iters: int,
              precond: bool = False, level_w=None, coeff_w: torch.Tensor | None = None,
              z_cur: torch.Tensor | None = None, z_prev: torch.Tensor | None = None,
              init: bool = True, iter_offset: int = 0, stats: bool = False,
              check_finite: bool = False, ws: torch.Tensor | None = None):
    """FISTA-W (precond False) or FISTA-WP on 1/2||Theta_L z - z0||^2 + ||z||_{1,w}.
    z0: (n2, n1) or (1, n2, n1) Mallat coefficients Psi^* f0.  Returns a dict
    with z_cur = z(K), z_prev = z(K-1) (shaped like z0) and stats ((iters, 3)
    FP64: 1/2||Theta_L y(i) - z0||^2, ||y(i)||_{1,w}, ||z(i) - y(i)||^2)."""
    _check_dev(z0, coeff_w, z_cur, z_prev)
    n2, n1 = z0.shape[-2:]
    shape = C.pd_shape(int(n1), int(n2), 1, int(levels))
    lw = None
    if level_w is not None:
        lw = np.ascontiguousarray(np.asarray(level_w, dtype=np.float64))
        if lw.shape != (levels + 1,):
            raise ValueError("level_w needs levels+1 entries")
    w = C.pd_weights(_dptr(lw) if lw is not None else None,
                     None if coeff_w is None else coeff_w.data_ptr(), 0)
    prm = C.pd_params(float(tau), int(iters), int(iter_offset), 1 if check_finite else 0)
    if z_cur is None:
        z_cur = torch.empty_like(z0)
    if z_prev is None:
        z_prev = torch.empty_like(z0)
    st = torch.zeros((max(iters, 1), 3), dtype=torch.float64, device=z0.device) if stats else None
    need = pd_wsolve_workspace_size(n1, n2, levels, z0.dtype)
    if ws is None or ws.numel() < need:
        ws = workspace(need, z0.device)
    tc, ttc = theta.c(), theta_t.c()
    rc = C.load().pd_wsolve(ctypes.byref(shape), _dtype_code(z0.dtype), ctypes.byref(tc), ctypes.byref(ttc),
                            ctypes.byref(w), ctypes.byref(prm), 1 if precond else 0, _ptr(z0), _ptr(z_cur),
                            _ptr(z_prev), 1 if init else 0, _ptr(st), _ptr(ws), ws.numel(),
                            _stream(z0.device))
    C.check(rc, "pd_wsolve")
    return {"z_cur": z_cur, "z_prev": z_prev, "stats": None if st is None else st[:iters]}


def pd_admm_workspace_size(n1: int, n2: int, channels: int, levels: int, terms: int, dtype: torch.dtype) -> int:
    shape = C.pd_shape(n1, n2, channels, levels)
    return int(C.load().pd_admm_workspace_size(ctypes.byref(shape), _dtype_code(dtype), int(terms)))


def pd_admm_solve(f0: torch.Tensor, op: Operator, h, levels: int, beta: float, iters: int,
                  level_w=None, coeff_w: torch.Tensor | None = None, stats: bool = False,
                  ws: torch.Tensor | None = None):
    """ADMM-PC (Appendix A.2) on 1/2||H Psi z - f0||^2 + ||z||_{1,w} with H the
    product-convolution expansion `op` (Operator.pc).  f0: (n2, n1) or
    (C, n2, n1).  Returns dict(f, z, stats) with stats (iters, 3) FP64:
    ||g - V f||^2_D, ||z - Psi^* f||^2, ||z||_{1,w} per iteration."""
    _check_dev(f0, coeff_w)
    if op.kind != C.PD_OP_PC:
        raise ValueError("pd_admm_solve needs a product-convolution operator")
    shape = _shape(f0, levels)
    wav, _hk = _wavelet(h)
    lw = None
    if level_w is not None:
        lw = np.ascontiguousarray(np.asarray(level_w, dtype=np.float64))
        if lw.shape != (levels + 1,):
            raise ValueError("level_w needs levels+1 entries")
    w = C.pd_weights(_dptr(lw) if lw is not None else None,
                     None if coeff_w is None else coeff_w.data_ptr(), 0)
    f = torch.empty_like(f0)
    z = torch.empty_like(f0)
    st = torch.empty((max(iters, 1), 3), dtype=torch.float64, device=f0.device) if stats else None
    need = int(C.load().pd_admm_workspace_size(ctypes.byref(shape), _dtype_code(f0.dtype), int(op.mult.shape[0])))
    if need == 0:
        raise ValueError("pd_admm_solve: unsupported shape or terms")
    if ws is None or ws.numel() < need:
        ws = workspace(need, f0.device)
    oc = op.c()
    rc = C.load().pd_admm_solve(ctypes.byref(shape), _dtype_code(f0.dtype), ctypes.byref(oc), ctypes.byref(wav),
                                ctypes.byref(w), float(beta), int(iters), _ptr(f0), _ptr(f), _ptr(z), _ptr(st),
                                _ptr(ws), ws.numel(), _stream(f0.device))
    C.check(rc, "pd_admm_solve")
    return {"f": f, "z": z, "stats": None if st is None else st[:iters]}


def pd_fft2(x: torch.Tensor, inverse: bool = False) -> torch.Tensor:
    """2-D DFT over the last two axes of a complex64/complex128 tensor (a copy)."""
    _check_dev(x)
    if x.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("pd_fft2 needs complex64 or complex128")
    y = x.contiguous().clone()
    n2, n1 = y.shape[-2:]
    batch = y.numel() // (n1 * n2) if y.numel() else 0
    dt = C.PD_F32 if y.dtype == torch.complex64 else C.PD_F64
    need = int(C.load().pd_fft2_workspace_size(int(n1), int(n2), dt))
    if need == 0:
        raise ValueError("pd_fft2: sizes must be powers of two within the LDS limit")
    ws = workspace(need, y.device)
    rc = C.load().pd_fft2(int(n1), int(n2), int(batch), dt, 1 if inverse else 0, _ptr(y), _ptr(ws), ws.numel(),
                          _stream(y.device))
    C.check(rc, "pd_fft2")
    return y


# ------------------------------------------------------------- Algorithm 1 ---
def pd_decompose_workspace_size(n1: int, n2: int, levels: int, terms: int) -> int:
    shape = C.pd_shape(n1, n2, 1, levels)
    return int(C.load().pd_decompose_workspace_size(ctypes.byref(shape), int(terms)))


def pd_decompose(op: Operator, h, levels: int, n2: int, n1: int, eta: float, capacity: int | None = None,
                 ws: torch.Tensor | None = None) -> Csr:
    """Algorithm 1 (Section 3.2): Theta~ = sum_k A~_k B_k for the FP64
    product-convolution operator `op` (Operator.pc with dtype float64) on an
    n2 x n1 image, eps_k = eta / (m ||v_k||_inf).  Returns Theta~ by columns,
    i.e. the CSR of its transpose (pd_csr_transpose gives Theta~ by rows).
    capacity None: a first call sizes the output, a second fills it."""
    if op.kind != C.PD_OP_PC or op.taps.dtype != torch.float64 or op.mult.dtype != torch.float64:
        raise ValueError("pd_decompose needs a float64 product-convolution operator")
    _check_dev(op.taps, op.mult)
    dev = op.taps.device
    shape = C.pd_shape(int(n1), int(n2), 1, int(levels))
    wav, _hk = _wavelet(h)
    oc = op.c()
    m = int(op.mult.shape[0])
    need = pd_decompose_workspace_size(n1, n2, levels, m)
    if need == 0:
        raise ValueError("pd_decompose: unsupported shape or terms")
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    N = int(n1) * int(n2)
    col_ptr = torch.empty(N + 1, dtype=torch.int64, device=dev)
    nnz = ctypes.c_int64(0)
    L = C.load()
    st = _stream(dev)

    def call(cap, rows, vals):
        return L.pd_decompose(ctypes.byref(shape), ctypes.byref(oc), ctypes.byref(wav), float(eta), int(cap),
                              ctypes.byref(nnz), _ptr(col_ptr), _ptr(rows), _ptr(vals), _ptr(ws), ws.numel(), st)

    sized = capacity is None
    if sized:
        rc = call(0, None, None)
        if rc not in (C.PD_OK, C.PD_ERR_WORKSPACE):
            C.check(rc, "pd_decompose")
        # the FP64 atomic sums are not bitwise reproducible, so an entry that cancels can be
        # exactly zero in one call and not in the next: size with slack, refit if still short
        capacity = nnz.value + max(1024, nnz.value // 64)
    for attempt in range(3):
        rows = torch.empty(max(int(capacity), 1), dtype=torch.int32, device=dev)
        vals = torch.empty(max(int(capacity), 1), dtype=torch.float64, device=dev)
        rc = call(capacity, rows if capacity else None, vals if capacity else None)
        if rc == C.PD_ERR_WORKSPACE and sized and attempt < 2:
            capacity = nnz.value + max(1024, nnz.value // 64)
            continue
        C.check(rc, "pd_decompose")
        break
    k = nnz.value
    return Csr(col_ptr, rows[:k], vals[:k])
