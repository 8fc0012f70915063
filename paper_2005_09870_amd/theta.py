"""Theta_L for the wavelet-domain solver: the entries of Theta = Psi^* H Psi
(Section 4.3) of magnitude at least eta, for a row blur H (pd_operator
PD_OP_ROWBLUR: the impulse response depends on the source row only, so H
commutes with periodic shifts along x1, as Operator 1 of Section 4.1 does).

Set-up, not the iteration.  Columns of Theta are probed with the library's own
transforms and blur (pd_fwt, pd_apply_op): Theta e = Psi^* H Psi e for probe
vectors e holding unit coefficients of one band at x1-position 0 and rows
spaced far enough apart that every coefficient of the result is reached by at
most one of them.  Shift covariance fills in the other x1-positions:

* for a row coefficient at level j <= j' (the column's level), moving the
  column by one position (2^j' pixels) moves the row by 2^(j'-j) positions,
  so a probe at x1-position 0 gives the whole column family;
* entries whose row is coarser than its column (j > j') are probed from the
  row side with H^T (Theta^T e = Psi^* H^T Psi e) and shifted the same way.

Every entry of Theta is produced exactly once.  The probes run in FP64 and the
result is sorted into CSR (columns increasing within a row).  torch is used
here only for index bookkeeping on the probes' outputs.
"""
from __future__ import annotations

import math

import torch

from . import solver as S


def _geometry(n1: int, n2: int, L: int, device):
    """Band level, orientation and in-band position of every Mallat position."""
    i2, i1 = torch.meshgrid(torch.arange(n2, device=device), torch.arange(n1, device=device), indexing="ij")
    i1 = i1.reshape(-1)
    i2 = i2.reshape(-1)
    t1 = sum((i1 < (n1 >> t)).long() for t in range(1, L + 1))
    t2 = sum((i2 < (n2 >> t)).long() for t in range(1, L + 1))
    t = torch.minimum(t1, t2)
    lev = torch.where(t == L, torch.full_like(t, L), t + 1)
    s1 = torch.div(torch.full_like(lev, n1), 2 ** lev, rounding_mode="floor")
    s2 = torch.div(torch.full_like(lev, n2), 2 ** lev, rounding_mode="floor")
    hi1 = ((t < L) & (i1 >= s1)).long()
    hi2 = ((t < L) & (i2 >= s2)).long()
    return {"i1": i1, "i2": i2, "lev": lev, "hi1": hi1, "l1": i1 - hi1 * s1, "l2": i2 - hi2 * s2,
            "P1": s1}


def _bands(L: int):
    """(level, orientation) of every band: approximation (L, 0), details
    (j, 1) high along x1, (j, 2) high along x2, (j, 3) both."""
    return [(L, 0)] + [(j, e) for j in range(1, L + 1) for e in (1, 2, 3)]


def _origin(n1: int, n2: int, j: int, e: int):
    return (n2 >> j if e in (2, 3) else 0), (n1 >> j if e in (1, 3) else 0)


def theta_rowblur(op: S.Operator, h, n1: int, n2: int, levels: int, eta: float,
                  dtype=torch.float32, device="cuda", batch: int = 4, apply=None) -> S.Csr:
    """Theta_L (CSR on `device`, values in `dtype`) for the row blur `op`
    (radius op.radius), wavelet filter h and an n1 x n2 plane with `levels`
    levels: every entry of Theta = Psi^* H Psi with |value| >= eta.  `apply`
    (x, transpose) -> Psi^* H Psi x (or Psi^* H^T Psi x) on a (batch, n2, n1)
    FP64 tensor; by default libpd's pd_fwt and pd_apply_op."""
    L = levels
    lf = len(h)
    R = int(op.radius)
    N = n1 * n2
    if apply is None:
        op64 = op if op.taps is None or op.taps.dtype == torch.float64 else \
            S.Operator(op.kind, op.radius, op.taps.to(torch.float64))
        ws = S.workspace(S.pd_workspace_size(S.C.pd_shape(n1, n2, batch, L), torch.float64), device)

        def apply(x, transpose):
            return S.pd_fwt(S.pd_apply_op(S.pd_fwt(x, h, L, inverse=True, ws=ws), op64, transpose=transpose),
                            h, L, ws=ws)
    g = _geometry(n1, n2, L, device)
    lev, l1, hi1, i2 = g["lev"], g["l1"], g["hi1"], g["i2"]
    width = lambda j: (lf - 1) * (2 ** j - 1) + 1          # pixels a level-j coefficient spans
    off = lambda j: (lf - 1) * (2 ** j - 1) / 2.0          # its centre from 2^j * position
    centre2 = (2.0 ** lev) * g["l2"].double() + (lf - 1) * (2.0 ** lev - 1) / 2.0
    rows, cols, vals = [], [], []
    for transpose in (False, True):
        for (jb, eb) in _bands(L):
            # column probes find rows at levels <= jb; row probes (H^T) columns at levels < jb
            target = (lev < jb) if transpose else (lev <= jb)
            if not bool(target.any()):
                continue
            P1, P2 = n1 >> jb, n2 >> jb
            o2, o1 = _origin(n1, n2, jb, eb)
            dmin = math.floor((2 * width(jb) + 2 * R) / 2 ** jb) + 1
            D = next((d for d in range(dmin, P2 + 1) if P2 % d == 0), P2)
            K = P2 // D
            found = []
            for r0 in range(0, D, batch):
                Cn = min(batch, D - r0)
                x = torch.zeros((batch, n2, n1), dtype=torch.float64, device=device)
                for c in range(Cn):
                    x[c, o2 + r0 + c + D * torch.arange(K, device=device), o1] = 1.0
                y = apply(x, transpose)
                for c in range(Cn):
                    yc = y[c].reshape(-1)
                    idx = torch.nonzero(target & (yc.abs() >= eta)).reshape(-1)
                    if idx.numel() == 0:
                        continue
                    # the probe whose row is nearest (periodically) to the coefficient's
                    d = (centre2[idx] - off(jb) - 2.0 ** jb * (r0 + c)) / (2.0 ** jb * D)
                    k = torch.remainder(torch.floor(d + 0.5).long(), K)
                    found.append((idx, r0 + c + D * k, yc[idx]))
            if not found:
                continue
            idx = torch.cat([f[0] for f in found])
            pl2 = torch.cat([f[1] for f in found])
            v = torch.cat([f[2] for f in found])
            # shift covariance along x1: probe at x1-position s, the other coefficient by 2^(jb-j) s
            s = torch.arange(P1, device=device)
            j = lev[idx]
            P1o = g["P1"][idx]
            lo = torch.remainder(l1[idx][:, None] + (2 ** (jb - j))[:, None] * s[None, :], P1o[:, None])
            other = (i2[idx][:, None] * n1 + lo + (hi1[idx] * P1o)[:, None]).reshape(-1)
            probe = ((o2 + pl2)[:, None] * n1 + o1 + s[None, :]).reshape(-1)
            vv = v[:, None].expand(-1, P1).reshape(-1)
            if transpose:
                rows.append(probe)
                cols.append(other)
            else:
                rows.append(other)
                cols.append(probe)
            vals.append(vv)
    r = torch.cat(rows)
    c = torch.cat(cols)
    v = torch.cat(vals)
    key, order = torch.sort(r * N + c)
    r, c, v = r[order], c[order], v[order]
    if key.numel() > 1 and bool((key[1:] == key[:-1]).any()):
        raise RuntimeError("theta_rowblur: an entry was produced twice")
    counts = torch.bincount(r, minlength=N)
    rp = torch.zeros(N + 1, dtype=torch.int64, device=device)
    rp[1:] = torch.cumsum(counts, 0)
    return S.Csr(rp, c.to(torch.int32), v.to(dtype))
