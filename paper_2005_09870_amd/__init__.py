"""MI355X-native FISTA solver for the wavelet-l1 deblurring energy of
Escande & Weiss (arXiv:2005.09870, eq. 4.1, Appendix A.1).

The compute path is libpd.so (hand-written HIP for gfx950 behind the C ABI in
include/pd.h); this package only marshals torch device tensors into it.
"""
from ._lib import PDError, load  # noqa: F401
from .solver import (  # noqa: F401
    BLUR_VARIANTS,
    Csr,
    FistaSolve,
    Operator,
    pd_backward,
    pd_solve_checkpointed,
    solve_autograd,
    lipschitz,
    pd_admm_solve,
    pd_admm_workspace_size,
    pd_apply_op,
    pd_decompose,
    pd_decompose_workspace_size,
    pd_fft2,
    pd_fwt,
    pd_graphs_enable,
    pd_fuse_enable,
    pd_op1_taps,
    pd_pc_expansion,
    pd_solve,
    pd_solve_batched,
    pd_solve_noalloc,
    pd_symmlet,
    pd_tune,
    pd_workspace_size,
    pd_csr_transpose,
    pd_spmv,
    pd_wjacobi,
    pd_wsolve,
    pd_wsolve_workspace_size,
    step_size,
    wlipschitz,
    wstep_size,
)
