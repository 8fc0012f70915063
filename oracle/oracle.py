"""The oracle: plain FP64 CPU reference for the wavelet-l1 deblurring solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code,
table or constant generator with the GPU library: the Symmlet filter, the
Operator-1 impulse responses and the step size are all derived here, by
methods of its own, from the paper (Escande & Weiss, arXiv:2005.09870).

The heavy loops (wavelet transforms, the blur as an integral operator, the
FISTA recursion and its reverse mode) live in ``oracle.c``; this module builds
and loads that library and adds the pieces that are easiest to state in numpy:

* ``symmlet(M)``          -- Daubechies spectral factorisation (Section 2.1:
  a filter bank (h, g) with M vanishing moments, supp h = [0, 2M-1]), root set
  chosen for the most nearly linear phase ("Symmlet", Section 4.2 / 4.3).
* ``op1_profiles(n2)``    -- Operator 1 of Section 4.1: isotropic Gaussian
  impulse responses, standard deviation 3*y2 (y2 in [0,1] the vertical source
  coordinate), truncated to keep 99% of the mass.
* ``fista`` / ``energy`` / ``grad`` / ``fista_reverse`` -- thin wrappers over
  the C library (Appendix A.1, eq. 4.1).
* ``lasso_exact``         -- an independent minimiser of eq. 4.1 for tiny
  images (coordinate descent + exact active-set solve), used to pin FISTA.

parity unpinned: none of the paper's printed image-quality figures (SNR, pSNR,
iteration counts) can be reproduced, because its test image is not available.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from itertools import product

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        d = ctypes.c_double
        L.or_threads.argtypes = []
        L.or_threads.restype = i
        L.or_fwt2.argtypes = [dp, i, i, i, dp, i]
        L.or_ifwt2.argtypes = [dp, i, i, i, dp, i]
        L.or_blur.argtypes = [dp, dp, i, i, dp, i, i]
        L.or_grad.argtypes = [i, i, i, i, dp, i, dp, i, i, dp, dp, dp, dp]
        L.or_energy.argtypes = [i, i, i, i, dp, i, dp, i, i, dp, i, dp, dp, dp]
        L.or_energy.restype = d
        L.or_fista.argtypes = [i, i, i, i, dp, i, dp, i, i, dp, i, d, i, dp, dp, dp, dp, dp, dp]
        L.or_fista_reverse.argtypes = [i, i, i, i, dp, i, dp, i, i, dp, d, i, dp, dp, dp, dp]
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_threads())


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Symmlet filter: Daubechies spectral factorisation (Section 2.1).
# ---------------------------------------------------------------------------
def _binom(a, b):
    return math.comb(a, b)


def symmlet(M: int = 6) -> np.ndarray:
    """Low-pass filter h (length 2M) of the orthogonal wavelet with M vanishing
    moments and minimal support whose phase is closest to linear.

    |m0(w)|^2 = cos^{2M}(w/2) P(sin^2(w/2)),  P(y) = sum_{k<M} C(M-1+k, k) y^k.
    Each root y_k of P gives a reciprocal pair of roots of z + 1/z = 2 - 4 y_k;
    one root of every pair (conjugates together) is kept.  Among the choices,
    the one whose residual phase (after removing the best straight line, over
    [0, pi]) has the least squared deviation is selected.  Of the two mirror
    images (time-reversed filters, equal phase deviation) the one whose energy
    centroid sum n h[n]^2 lies in the upper half of [0, 2M-1] is returned.
    h is normalised so that sum h = sqrt(2).
    """
    if M == 1:
        return np.array([1.0, 1.0]) / math.sqrt(2.0)
    P = np.array([_binom(M - 1 + k, k) for k in range(M)], dtype=np.float64)
    yroots = np.roots(P[::-1])
    groups = []  # each group: list of z-roots inside the unit circle
    used = np.zeros(len(yroots), bool)
    for a, y in enumerate(yroots):
        if used[a]:
            continue
        used[a] = True
        b = 2.0 - 4.0 * y
        z1 = (b + np.sqrt(b * b - 4.0 + 0j)) / 2.0
        z2 = (b - np.sqrt(b * b - 4.0 + 0j)) / 2.0
        zin = z1 if abs(z1) < 1.0 else z2
        if abs(y.imag) > 1e-9 * max(1.0, abs(y)):
            # pair with the conjugate y root
            c = int(np.argmin([abs(yy - np.conj(y)) if not used[q] else np.inf
                               for q, yy in enumerate(yroots)]))
            used[c] = True
            groups.append([zin, np.conj(zin)])
        else:
            groups.append([complex(zin.real, 0.0)])
    w = np.linspace(0.0, math.pi, 4097)
    e = np.exp(-1j * w)
    best = None
    # group 0 is held "inside" to enumerate each mirror pair once
    for choice in product([0, 1], repeat=len(groups) - 1):
        flags = (0,) + choice
        roots = []
        for g, f in zip(groups, flags):
            roots.extend(g if f == 0 else [1.0 / z for z in g])
        q = np.poly(roots)  # highest power first
        val = np.polyval(q, e)
        ph = np.unwrap(np.angle(val))
        A = np.stack([np.ones_like(w), w], 1)
        coef, *_ = np.linalg.lstsq(A, ph, rcond=None)
        score = float(np.sum((ph - A @ coef) ** 2))
        if best is None or score < best[0]:
            best = (score, roots)
    roots = best[1]
    q = np.real(np.poly(roots))[::-1]  # increasing powers
    q = q / np.sum(q)  # L(1) = 1
    lo = np.array([1.0])
    for _ in range(M):
        lo = np.convolve(lo, [0.5, 0.5])
    h = math.sqrt(2.0) * np.convolve(lo, q)
    n = np.arange(len(h))
    if np.sum(n * h * h) < (len(h) - 1) / 2.0:
        h = h[::-1].copy()
    return h


# ---------------------------------------------------------------------------
# Operator 1 (Section 4.1).
# ---------------------------------------------------------------------------
def op1_sigma(n2: int, sigma_max: float = 3.0) -> np.ndarray:
    """Standard deviation (pixels) of the impulse response emitted by source row
    i2: sigma = sigma_max * y2 with y2 = i2 / (n2 - 1) in [0, 1]."""
    if n2 == 1:
        return np.zeros(1)
    return sigma_max * np.arange(n2, dtype=np.float64) / (n2 - 1)


def op1_radius(sigma: float, mass: float = 0.99) -> int:
    """Half-width keeping the fraction `mass` of a 2-D isotropic Gaussian in a
    square window: per-axis mass sqrt(mass), half-width sigma*sqrt(2)*erfinv(sqrt(mass))."""
    from scipy.special import erfinv
    if sigma <= 0.0:
        return 0
    return int(math.ceil(sigma * math.sqrt(2.0) * float(erfinv(math.sqrt(mass)))))


def op1_profiles(n2: int, sigma_max: float = 3.0, mass: float = 0.99):
    """Per-source-row 1-D profile table kt[i2, d + R] (d in [-R, R]) of Operator
    1 and its common half-width R.  The 2-D impulse response of source row i2
    is the outer product of row i2's profile with itself, normalised to unit
    sum (truncation per the 99% rule, then renormalisation)."""
    sig = op1_sigma(n2, sigma_max)
    radii = [op1_radius(s, mass) for s in sig]
    R = max(radii)
    kt = np.zeros((n2, 2 * R + 1))
    for i2, (s, r) in enumerate(zip(sig, radii)):
        if r == 0:
            kt[i2, R] = 1.0
            continue
        d = np.arange(-r, r + 1, dtype=np.float64)
        p = np.exp(-d * d / (2.0 * s * s))
        kt[i2, R - r:R + r + 1] = p / p.sum()
    return kt, R


# ---------------------------------------------------------------------------
# Weights (Section 4.3): one weight per wavelet coefficient, Mallat layout.
# ---------------------------------------------------------------------------
def band_of(n1: int, n2: int, levels: int):
    """Band index map k[i2, i1] of the Mallat layout: k = 0 for the coarsest
    approximation band, k = 1..levels for the detail bands from the coarsest
    (decomposition level `levels`) to the finest (level 1).  k equals the
    paper's scale |lambda| = j plus one for full-depth transforms."""
    k = np.zeros((n2, n1), dtype=np.int64)
    i2, i1 = np.meshgrid(np.arange(n2), np.arange(n1), indexing="ij")
    assigned = np.zeros((n2, n1), bool)
    for lev in range(1, levels + 1):
        det = ((i1 >= (n1 >> lev)) | (i2 >= (n2 >> lev))) & ~assigned
        k[det] = levels + 1 - lev
        assigned |= det
    return k


def expand_level_weights(level_w, n1, n2, levels, C=1):
    """Per-coefficient weight map (C, n2, n1) from a per-band table level_w[k]."""
    kmap = band_of(n1, n2, levels)
    w = np.asarray(level_w, dtype=np.float64)[kmap]
    return np.broadcast_to(w, (C, n2, n1)).copy()


def paper_level_weights(levels: int, scale: float = 2e-2) -> np.ndarray:
    """w[lambda] = scale * |lambda| (Fig. 5 caption): band k has |lambda| = k-1
    for detail bands; the approximation band (|lambda| = 0) gets 0."""
    w = np.zeros(levels + 1)
    w[1:] = scale * np.arange(levels)
    return w


# ---------------------------------------------------------------------------
# Wrappers over the C library.
# ---------------------------------------------------------------------------
class Problem:
    """Everything that defines one instance of eq. 4.1 for the oracle."""

    def __init__(self, n1, n2, C=1, levels=None, h=None, op="op1", sigma_max=3.0,
                 mass=0.99, w=None, joint=False):
        self.n1, self.n2, self.C = int(n1), int(n2), int(C)
        if levels is None:
            levels = min((n1 & -n1).bit_length() - 1, (n2 & -n2).bit_length() - 1)
        self.levels = int(levels)
        self.h = _c(symmlet(6) if h is None else h)
        self.op_identity = 1 if op == "identity" else 0
        if self.op_identity:
            self.kt, self.R = np.ones((n2, 1)), 0
        elif isinstance(op, tuple):
            self.kt, self.R = _c(op[0]), int(op[1])
        else:
            self.kt, self.R = op1_profiles(n2, sigma_max, mass)
        self.kt = _c(self.kt)
        if w is None:
            w = np.zeros((C, n2, n1))
        self.w = _c(np.broadcast_to(w, (C, n2, n1)))
        self.joint = 1 if joint else 0

    @property
    def shape(self):
        return (self.C, self.n2, self.n1)

    def _args(self):
        return (self.n1, self.n2, self.C, self.levels, _p(self.h), len(self.h),
                _p(self.kt), self.R, self.op_identity)


def fwt(a, levels, h):
    a = _c(a).copy()
    n2, n1 = a.shape[-2:]
    flat = a.reshape(-1, n2, n1)
    for c in range(flat.shape[0]):
        blk = np.ascontiguousarray(flat[c])
        lib().or_fwt2(_p(blk), n1, n2, levels, _p(_c(h)), len(h))
        flat[c] = blk
    return flat.reshape(a.shape)


def ifwt(a, levels, h):
    a = _c(a).copy()
    n2, n1 = a.shape[-2:]
    flat = a.reshape(-1, n2, n1)
    for c in range(flat.shape[0]):
        blk = np.ascontiguousarray(flat[c])
        lib().or_ifwt2(_p(blk), n1, n2, levels, _p(_c(h)), len(h))
        flat[c] = blk
    return flat.reshape(a.shape)


def blur(x, kt, R, transpose=False):
    x = _c(x)
    n2, n1 = x.shape[-2:]
    out = np.empty_like(x)
    fx = x.reshape(-1, n2, n1)
    fo = out.reshape(-1, n2, n1)
    for c in range(fx.shape[0]):
        src = np.ascontiguousarray(fx[c])
        dst = np.empty_like(src)
        lib().or_blur(_p(src), _p(dst), n1, n2, _p(_c(kt)), int(R), 1 if transpose else 0)
        fo[c] = dst
    return out


def grad(pb: Problem, f0, y):
    f0 = _c(f0).reshape(pb.shape)
    y = _c(y).reshape(pb.shape)
    g = np.empty(pb.shape)
    r = np.empty(pb.shape)
    lib().or_grad(*pb._args(), _p(f0), _p(y), _p(g), _p(r))
    return g, r


def energy(pb: Problem, f0, z):
    f0 = _c(f0).reshape(pb.shape)
    z = _c(z).reshape(pb.shape)
    terms = np.zeros(2)
    e = lib().or_energy(*pb._args(), _p(pb.w), pb.joint, _p(f0), _p(z), _p(terms))
    return e, terms


def fista(pb: Problem, f0, tau, iters, init=None, log=False, tape=False):
    """Run the FISTA recursion; returns dict(z, f, log, tape)."""
    f0 = _c(f0).reshape(pb.shape)
    z = np.empty(pb.shape)
    f = np.empty(pb.shape)
    lg = np.zeros((max(iters, 1), 3)) if log else None
    tp = np.zeros((max(iters, 1),) + pb.shape) if tape else None
    ini = None if init is None else _c(init).reshape(pb.shape)
    lib().or_fista(*pb._args(), _p(pb.w), pb.joint, float(tau), int(iters), _p(f0),
                   _p(ini), _p(z), _p(f), _p(lg), _p(tp))
    return {"z": z, "f": f, "log": None if lg is None else lg[:iters],
            "tape": None if tp is None else tp[:iters]}


def fista_reverse(pb: Problem, tau, iters, tape, fbar):
    """Reverse mode of `fista` with init = Psi^* f0 (scalar prox): returns
    (dLoss/df0, dLoss/dw) for dLoss/df = fbar."""
    assert not pb.joint
    tape = _c(tape)
    fbar = _c(fbar).reshape(pb.shape)
    f0b = np.empty(pb.shape)
    wb = np.empty(pb.shape)
    lib().or_fista_reverse(*pb._args(), _p(pb.w), float(tau), int(iters), _p(tape),
                           _p(fbar), _p(f0b), _p(wb))
    return f0b, wb


def apply_H(pb: Problem, x, transpose=False):
    if pb.op_identity:
        return _c(x).copy()
    return blur(x, pb.kt, pb.R, transpose)


def lipschitz(pb: Problem, iters: int = 300, seed: int = 0) -> float:
    """||H^T H||_2 by power iteration (Appendix A.1 asks tau <= ||H||^{-2})."""
    if pb.op_identity:
        return 1.0
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((pb.n2, pb.n1))
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = blur(blur(x, pb.kt, pb.R), pb.kt, pb.R, transpose=True)
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam


def step_size(pb: Problem) -> float:
    return 1.0 / (lipschitz(pb) * (1.0 + 1e-6))


def kkt_residual(pb: Problem, f0, z):
    """Optimality residual of eq. 4.1 in coefficient form (scalar weights):
    max over coefficients of |g + w sign z| (z != 0) or max(0, |g| - w) (z = 0),
    with g the gradient of the data term at z."""
    g, _ = grad(pb, f0, z)
    w = pb.w.reshape(pb.shape)
    nz = z != 0
    res = np.where(nz, np.abs(g + w * np.sign(z)), np.maximum(0.0, np.abs(g) - w))
    return float(res.max())


def dense_A(pb: Problem):
    """A = H Psi as a dense (N x N) matrix, column by column (single channel)."""
    N = pb.n1 * pb.n2
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros((pb.n2, pb.n1))
        e.flat[j] = 1.0
        A[:, j] = apply_H(pb, ifwt(e, pb.levels, pb.h)).ravel()
    return A


def lasso_exact(pb: Problem, f0, sweeps: int = 20000, tol: float = 1e-14):
    """Minimiser of 1/2 ||A z - f0||^2 + sum w |z| for a tiny single-channel
    problem, by cyclic coordinate descent followed by an exact solve of the
    optimality system on the detected support and signs.  Shares nothing with
    the FISTA recursion.  Returns (z, A)."""
    A = dense_A(pb)
    b = _c(f0).ravel()
    w = pb.w.reshape(-1)
    N = A.shape[1]
    z = np.zeros(N)
    r = b.copy()
    col2 = np.sum(A * A, 0)
    for _ in range(sweeps):
        zmax = 0.0
        for j in range(N):
            aj = A[:, j]
            u = z[j] + aj @ r / col2[j]
            t = w[j] / col2[j]
            zn = np.sign(u) * max(abs(u) - t, 0.0)
            if zn != z[j]:
                r -= aj * (zn - z[j])
                zmax = max(zmax, abs(zn - z[j]))
                z[j] = zn
        if zmax < tol:
            break
    S = np.nonzero(z)[0]
    s = np.sign(z[S])
    AS = A[:, S]
    zS = np.linalg.solve(AS.T @ AS, AS.T @ b - w[S] * s)
    zz = np.zeros(N)
    zz[S] = zS
    return zz.reshape(pb.n2, pb.n1), A
