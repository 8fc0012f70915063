"""ctypes declarations of libpd's C ABI (include/pd.h).  Loading fails loudly
when the library has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpd.so")

PD_OK = 0
PD_ERR_ARG = -1
PD_ERR_SHAPE = -2
PD_ERR_WORKSPACE = -3
PD_ERR_TAU = -4
PD_ERR_NONFINITE = -5
PD_ERR_HIP = -6
PD_ERR_UNSUPPORTED = -7

PD_F32 = 0
PD_F64 = 1
PD_OP_IDENTITY = 0
PD_OP_ROWBLUR = 1
PD_OP_PC = 2


class pd_shape(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("levels", ctypes.c_int32)]


class pd_operator(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("radius", ctypes.c_int32), ("taps", ctypes.c_void_p),
                ("terms", ctypes.c_int32), ("mult", ctypes.c_void_p)]


class pd_wavelet(ctypes.Structure):
    _fields_ = [("len", ctypes.c_int32), ("h", ctypes.POINTER(ctypes.c_double))]


class pd_weights(ctypes.Structure):
    _fields_ = [("level_w", ctypes.POINTER(ctypes.c_double)), ("coeff_w", ctypes.c_void_p),
                ("joint", ctypes.c_int32)]


class pd_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("iters", ctypes.c_int32),
                ("iter_offset", ctypes.c_int32), ("check_finite", ctypes.c_int32)]


class pd_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class pd_image_desc(ctypes.Structure):
    _fields_ = [("shape", pd_shape), ("offset", ctypes.c_int64), ("tau", ctypes.c_double),
                ("op", pd_operator), ("w", pd_weights)]


# every symbol include/pd.h declares
EXPORTS = [
    "pd_workspace_size", "pd_solve", "pd_solve_noalloc", "pd_batched_workspace_size", "pd_solve_batched",
    "pd_backward_workspace_size", "pd_backward", "pd_solve_checkpointed", "pd_backward_checkpointed", "pd_fwt", "pd_apply_op", "pd_tune", "pd_symmlet",
    "pd_op1_taps", "pd_pc_expansion", "pd_strerror", "pd_timing_enable", "pd_timing_read", "pd_graphs_enable", "pd_fuse_enable",
    "pd_csr_transpose_workspace_size", "pd_csr_transpose", "pd_spmv", "pd_wjacobi",
    "pd_wsolve_workspace_size", "pd_wsolve", "pd_admm_workspace_size", "pd_admm_solve",
    "pd_fft2_workspace_size", "pd_fft2", "pd_decompose_workspace_size", "pd_decompose",
]

PD_K_BLUR, PD_K_SYNTH, PD_K_ANALYSIS, PD_K_COARSE, PD_K_OTHER = 1, 2, 3, 4, 5
PD_K_WRES, PD_K_WPROX = 6, 7
PD_K_FFT, PD_K_ADMM, PD_K_DECOMP, PD_K_SYNTH2, PD_K_JPROX, PD_K_SYNTH3, PD_K_ANALYSIS2 = 8, 9, 10, 11, 12, 13, 14
KCLASS_NAMES = {1: "blur", 2: "synthesis", 3: "analysis", 4: "coarse", 5: "other",
                6: "wres", 7: "wprox", 8: "fft", 9: "admm", 10: "decomp", 11: "synthesis2",
                12: "jprox", 13: "synthesis3", 14: "analysis2"}

_lib = None


class PDError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpd.so not built at {LIB_PATH}; run `python -m paper_2005_09870_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, sz, i32, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    dp = P(ctypes.c_double)
    L.pd_workspace_size.argtypes = [P(pd_shape), i32]
    L.pd_workspace_size.restype = sz
    L.pd_solve.argtypes = [P(pd_shape), i32, P(pd_operator), P(pd_wavelet), P(pd_weights),
                           P(pd_params), vp, vp, vp, i32, vp, vp, vp, sz, vp]
    L.pd_solve.restype = ctypes.c_int
    L.pd_solve_noalloc.argtypes = [P(pd_shape), i32, P(pd_operator), P(pd_wavelet), P(pd_weights),
                                   P(pd_params), vp, vp, vp, i32, vp, vp, vp]
    L.pd_solve_noalloc.restype = ctypes.c_int
    L.pd_batched_workspace_size.argtypes = [i32, P(pd_image_desc), i32]
    L.pd_batched_workspace_size.restype = sz
    L.pd_solve_batched.argtypes = [i32, P(pd_image_desc), i32, P(pd_wavelet), i32, vp, vp, vp,
                                   vp, sz, vp]
    L.pd_solve_batched.restype = ctypes.c_int
    L.pd_backward_workspace_size.argtypes = [P(pd_shape), i32, i32, i32]
    L.pd_backward_workspace_size.restype = sz
    L.pd_backward.argtypes = [P(pd_shape), i32, P(pd_operator), P(pd_wavelet), P(pd_weights),
                              P(pd_params), vp, vp, vp, vp, i32, vp, sz, vp]
    L.pd_backward.restype = ctypes.c_int
    L.pd_solve_checkpointed.argtypes = [P(pd_shape), i32, P(pd_operator), P(pd_wavelet), P(pd_weights),
                                        P(pd_params), vp, vp, i32, vp, sz, vp]
    L.pd_solve_checkpointed.restype = ctypes.c_int
    L.pd_backward_checkpointed.argtypes = L.pd_backward.argtypes
    L.pd_backward_checkpointed.restype = ctypes.c_int
    L.pd_fwt.argtypes = [P(pd_shape), i32, P(pd_wavelet), i32, vp, vp, vp, sz, vp]
    L.pd_fwt.restype = ctypes.c_int
    L.pd_apply_op.argtypes = [P(pd_shape), i32, P(pd_operator), i32, vp, vp, vp]
    L.pd_apply_op.restype = ctypes.c_int
    L.pd_tune.argtypes = [P(pd_shape), i32, P(pd_operator), vp, sz, P(i32), vp]
    L.pd_tune.restype = ctypes.c_int
    L.pd_symmlet.argtypes = [i32, dp]
    L.pd_symmlet.restype = ctypes.c_int
    L.pd_op1_taps.argtypes = [i32, d, d, P(i32), dp]
    L.pd_op1_taps.restype = ctypes.c_int
    L.pd_pc_expansion.argtypes = [dp, i32, i32, i32, i32, i32, ctypes.c_uint64, dp, dp, dp, P(i32)]
    L.pd_pc_expansion.restype = ctypes.c_int
    L.pd_timing_enable.argtypes = [i32]
    L.pd_timing_enable.restype = ctypes.c_int
    L.pd_fuse_enable.argtypes = [i32]
    L.pd_fuse_enable.restype = ctypes.c_int
    L.pd_graphs_enable.argtypes = [i32]
    L.pd_graphs_enable.restype = ctypes.c_int
    L.pd_timing_read.argtypes = [i32, P(i32), P(i32), P(ctypes.c_int64), dp, P(i32)]
    L.pd_timing_read.restype = ctypes.c_int
    L.pd_csr_transpose_workspace_size.argtypes = [i32]
    L.pd_csr_transpose_workspace_size.restype = sz
    L.pd_csr_transpose.argtypes = [P(pd_csr), i32, vp, vp, vp, vp, sz, vp]
    L.pd_csr_transpose.restype = ctypes.c_int
    L.pd_spmv.argtypes = [P(pd_csr), i32, vp, vp, vp]
    L.pd_spmv.restype = ctypes.c_int
    L.pd_wjacobi.argtypes = [P(pd_csr), i32, vp, vp]
    L.pd_wjacobi.restype = ctypes.c_int
    L.pd_wsolve_workspace_size.argtypes = [P(pd_shape), i32]
    L.pd_wsolve_workspace_size.restype = sz
    L.pd_wsolve.argtypes = [P(pd_shape), i32, P(pd_csr), P(pd_csr), P(pd_weights), P(pd_params), i32,
                            vp, vp, vp, i32, vp, vp, sz, vp]
    L.pd_wsolve.restype = ctypes.c_int
    L.pd_admm_workspace_size.argtypes = [P(pd_shape), i32, i32]
    L.pd_admm_workspace_size.restype = sz
    L.pd_admm_solve.argtypes = [P(pd_shape), i32, P(pd_operator), P(pd_wavelet), P(pd_weights), d, i32,
                                vp, vp, vp, vp, vp, sz, vp]
    L.pd_admm_solve.restype = ctypes.c_int
    L.pd_fft2_workspace_size.argtypes = [i32, i32, i32]
    L.pd_fft2_workspace_size.restype = sz
    L.pd_fft2.argtypes = [i32, i32, i32, i32, i32, vp, vp, sz, vp]
    L.pd_fft2.restype = ctypes.c_int
    L.pd_decompose_workspace_size.argtypes = [P(pd_shape), i32]
    L.pd_decompose_workspace_size.restype = sz
    L.pd_decompose.argtypes = [P(pd_shape), P(pd_operator), P(pd_wavelet), d, ctypes.c_int64,
                               P(ctypes.c_int64), vp, vp, vp, vp, sz, vp]
    L.pd_decompose.restype = ctypes.c_int
    L.pd_strerror.argtypes = [i32]
    L.pd_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return load().pd_strerror(int(code)).decode()
    except ImportError:
        return f"status {code}"


def check(code: int, where: str) -> None:
    if code != PD_OK:
        raise PDError(code, where)
