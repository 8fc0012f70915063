"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Holds none of the method's arithmetic: it paints piecewise-constant scenes
(axis-aligned rectangles and disks on a constant or ramp background), draws
Gaussian noise, salt-and-pepper masks, batch shapes and weight parameters.
The observation f0 = H clean + noise (Section 4.3's model) is formed by each
side with its own operator.

All draws use numpy's PCG64 generator with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def scene(n1: int, n2: int, n_rect: int, n_disk: int, background: str = "const",
          rng: np.random.Generator | None = None, seed: int = 0) -> np.ndarray:
    """Piecewise-constant image (n2, n1) in float64.

    background "const": 0.2 everywhere; "ramp": 0.1 + 0.3 (x1/n1 + x2/n2)/2.
    Rectangles: corner uniform in the image, sides uniform in
    [n/16, n/4] (n the side along that axis), clipped at the border.
    Disks: centre uniform, radius uniform in [m/32, m/8], m = min(n1, n2).
    Each shape gets an intensity uniform in [0, 1]; later shapes overwrite
    earlier ones.  Rectangles are drawn first, then disks."""
    if rng is None:
        rng = np.random.default_rng(seed)
    if background == "ramp":
        i2, i1 = np.meshgrid(np.arange(n2), np.arange(n1), indexing="ij")
        img = 0.1 + 0.3 * (i1 / n1 + i2 / n2) / 2.0
    else:
        img = np.full((n2, n1), 0.2)
    for _ in range(n_rect):
        c1 = rng.integers(0, n1)
        c2 = rng.integers(0, n2)
        s1 = int(rng.uniform(n1 / 16, n1 / 4))
        s2 = int(rng.uniform(n2 / 16, n2 / 4))
        img[c2:c2 + s2, c1:c1 + s1] = rng.uniform(0.0, 1.0)
    m = min(n1, n2)
    for _ in range(n_disk):
        c1 = rng.uniform(0, n1)
        c2 = rng.uniform(0, n2)
        r = rng.uniform(m / 32, m / 8)
        # the test only on the disk's bounding box (one pixel of margin)
        a1, b1 = max(0, int(np.floor(c1 - r)) - 1), min(n1, int(np.ceil(c1 + r)) + 2)
        a2, b2 = max(0, int(np.floor(c2 - r)) - 1), min(n2, int(np.ceil(c2 + r)) + 2)
        j2, j1 = np.meshgrid(np.arange(a2, b2), np.arange(a1, b1), indexing="ij")
        box = img[a2:b2, a1:b1]
        box[(j1 - c1) ** 2 + (j2 - c2) ** 2 <= r * r] = rng.uniform(0.0, 1.0)
    return img


def gaussian_noise(shape, sigma: float, rng: np.random.Generator) -> np.ndarray:
    return sigma * rng.standard_normal(shape)


def salt_pepper(shape2d, frac: float, rng: np.random.Generator):
    """Pixel mask (n2, n1) with fraction `frac` set, and the value (0 or 1,
    probability 1/2 each) those pixels take in every channel."""
    mask = rng.random(shape2d) < frac
    val = (rng.random(shape2d) < 0.5).astype(np.float64)
    return mask, val


def level_profile(levels: int, lam: float) -> np.ndarray:
    """Per-band weights, linear in the scale index as in the paper's
    w = c |lambda| profile, scaled so the finest detail band gets `lam`:
    band k = 0 (coarsest approximation) -> 0, detail band k = 1..levels
    (coarse to fine) -> lam (k-1)/(levels-1)."""
    w = np.zeros(levels + 1)
    if levels >= 2:
        w[1:] = lam * np.arange(levels) / (levels - 1)
    elif levels == 1:
        w[1] = lam
    return w


def two_adic_levels(n1: int, n2: int) -> int:
    """Largest L with n1 and n2 both divisible by 2^L."""
    v = lambda n: (n & -n).bit_length() - 1
    return min(v(n1), v(n2))


@dataclass
class ImageCase:
    n1: int
    n2: int
    C: int
    levels: int
    clean: np.ndarray          # (C, n2, n1)
    noise: np.ndarray          # (C, n2, n1), added after the blur
    level_w: np.ndarray        # (levels+1,)
    sp_mask: np.ndarray | None = None   # salt-and-pepper pixels (n2, n1)
    sp_val: np.ndarray | None = None
    theta: np.ndarray | None = None     # per-coefficient weight parameters


def make_case(n1, n2, C=1, n_rect=6, n_disk=4, background="const", sigma=0.1,
              lam=0.1, levels=None, seed=0, sp_frac=0.0, theta=None) -> ImageCase:
    """One image case: independent scene per channel, noise, weights."""
    rng = np.random.default_rng(seed)
    clean = np.stack([scene(n1, n2, n_rect, n_disk, background, rng) for _ in range(C)])
    noise = gaussian_noise(clean.shape, sigma, rng)
    L = two_adic_levels(n1, n2) if levels is None else levels
    mask = val = None
    if sp_frac > 0:
        mask, val = salt_pepper((n2, n1), sp_frac, rng)
    th = None
    if theta is not None:
        mu, sd = theta
        th = rng.normal(mu, sd, clean.shape)
    return ImageCase(n1, n2, C, L, clean, noise, level_profile(L, lam), mask, val, th)


def scaled_counts(n1, n2, base_side=512, base_rect=40, base_disk=25):
    """Shape counts scaled by area relative to a base image."""
    a = (n1 * n2) / float(base_side * base_side)
    return max(1, int(round(base_rect * a))), max(1, int(round(base_disk * a)))


# The workloads (seeded stand-ins for the paper's deblurring experiment).
def case_small(seed=1):
    """64x64 grayscale, 6 rectangles + 4 disks on 0.2, noise 0.1, lambda 0.1."""
    return make_case(64, 64, 1, 6, 4, "const", 0.1, 0.1, seed=seed)


def case_512(seed=2):
    """512x512 grayscale, 40 rectangles + 25 disks, ramp background, noise
    0.05, lambda 0.08."""
    return make_case(512, 512, 1, 40, 25, "ramp", 0.05, 0.08, seed=seed)


def case_colour(seed=3, n=2048):
    """n x n x 3, independent shapes per channel, noise 0.1 plus 5%
    salt-and-pepper pixels, lambda 0.1."""
    r, d = scaled_counts(n, n)
    return make_case(n, n, 3, r, d, "ramp", 0.1, 0.1, seed=seed, sp_frac=0.05)


def batch_shapes(count=64, seed=4, lo=96, hi=1024, step=32):
    """Uneven sizes: sides i.i.d. uniform on {lo, lo+step, ..., hi}, and a
    per-image lambda uniform in [0.03, 0.2]."""
    rng = np.random.default_rng(seed)
    sides = np.arange(lo, hi + 1, step)
    n1 = rng.choice(sides, count)
    n2 = rng.choice(sides, count)
    lam = rng.uniform(0.03, 0.2, count)
    return [(int(a), int(b), float(c)) for a, b, c in zip(n1, n2, lam)]


def case_batch(count=64, seed=4, **kw):
    out = []
    for b, (n1, n2, lam) in enumerate(batch_shapes(count, seed, **kw)):
        r, d = scaled_counts(n1, n2)
        out.append(make_case(n1, n2, 1, r, d, "const", 0.1, lam, seed=seed * 1000 + b))
    return out


def case_grad(count=16, seed=5, n=256):
    """16 x 256^2 with clean targets, noise 0.1, per-coefficient weight
    parameters theta ~ N(-2, 0.1^2) (weights softplus(theta))."""
    out = []
    for b in range(count):
        r, d = scaled_counts(n, n)
        out.append(make_case(n, n, 1, r, d, "const", 0.1, 0.1, seed=seed * 1000 + b,
                             theta=(-2.0, 0.1)))
    return out
