"""Product-convolution expansions for the FISTA-PC operator (PD_OP_PC).

Set-up, not the iteration.  Section 3.1: when an operator's impulse
responses S(., y) are known, the best rank-m expansion
H f = sum_k u_k * (v_k . f) in Frobenius norm comes from the truncated SVD of
the matrix S (rows: offsets d in [-R, R]^2, columns: sources y), with
v_k(y) = <S(., y), u_k>; the paper computes it with a randomized SVD, this
module with an exact one (torch.linalg.svd, FP64).

For a row blur (pd_operator PD_OP_ROWBLUR, Operator 1 of Section 4.1) the
response of source y is the outer product of row y2's profile with itself,
so S has one distinct column per row and v_k depends on y2 only.
"""
from __future__ import annotations

import numpy as np
import torch

from . import solver as S


def rowblur_expansion(taps, radius: int, m: int, n1: int):
    """(u, v) for S.Operator.pc: u (m, 2R+1, 2R+1) orthonormal kernels, v
    (m, n2, n1) multipliers, from a row-profile table taps (n2, 2R+1)."""
    p = torch.as_tensor(np.asarray(taps), dtype=torch.float64)
    n2, W = p.shape
    if W != 2 * radius + 1:
        raise ValueError("taps must be (n2, 2R+1)")
    cols = (p[:, :, None] * p[:, None, :]).reshape(n2, W * W).T  # (W*W, n2): column i2 = response of row i2
    U, sv, _ = torch.linalg.svd(cols, full_matrices=False)
    m = int(min(m, int((sv > 0).sum())))
    u = U[:, :m].T.contiguous()                  # (m, W*W)
    v = u @ cols                                 # (m, n2): <S(., i2), u_k>
    return (u.reshape(m, W, W).numpy(), v[:, :, None].expand(m, n2, n1).contiguous().numpy())


def rowblur_pc_operator(taps, radius: int, m: int, n1: int, dtype=torch.float32, device="cuda") -> S.Operator:
    u, v = rowblur_expansion(taps, radius, m, n1)
    return S.Operator.pc(u, v, dtype=dtype, device=device)
