"""Product-convolution expansions for the FISTA-PC operator (PD_OP_PC).

Set-up, not the iteration.  Section 3.3.3: when an operator's impulse
responses S(., y) are known, the best rank-m expansion
H f = sum_k u_k * (v_k . f) in Frobenius norm comes from the truncated SVD of
the matrix S (rows: offsets d in [-R, R]^2, columns: sources y), with
v_k(y) = <S(., y), u_k>; libpd computes it with a randomized SVD
(pd_pc_expansion), this module only lays the result out.

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
    u, v, _ = S.pd_pc_expansion(np.asarray(taps, dtype=np.float64), radius, m)
    return u, np.repeat(v[:, :, None], n1, axis=2)


def rowblur_pc_operator(taps, radius: int, m: int, n1: int, dtype=torch.float32, device="cuda") -> S.Operator:
    u, v = rowblur_expansion(taps, radius, m, n1)
    return S.Operator.pc(u, v, dtype=dtype, device=device)
