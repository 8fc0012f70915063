"""Writes the sampled full-size fixtures the GPU parity tests compare with.

Calls only the oracle (plain FP64 CPU code) and the seeded input generators:

  fullsize_512.npz    the 512 x 512 workload (Operator 1, Symmlet-6, 9 levels,
                      40 rectangles + 25 disks on a ramp, noise 0.05, lambda
                      0.08) after 2000 FISTA iterations (Appendix A.1) with the
                      oracle's step 1/||H^T H||: f = Psi z(K) and z(K) on four
                      full rows and 4096 seeded pixels, and the per-iteration
                      energy log.
  fullsize_colour.npz the 2048 x 2048 x 3 workload (joint shrinkage, noise 0.1
                      plus 5% salt-and-pepper pixels, lambda 0.1, 11 levels)
                      after 100 iterations with tau = 0.89: f and z on one full
                      row and 2048 seeded pixels per channel, and the log.
  fullsize_batch.npz  the four smallest images of the 64-image batch of uneven
                      sizes (sides uniform on {96, ..., 1024}, per-image
                      lambda) after 1000 iterations with each image's oracle
                      step: f on two full rows and 1024 seeded pixels, and the
                      log.

    python tests/golden/make_fullsize.py [512] [colour] [batch]

The oracle needs a few minutes per fixture on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
import syninputs as SI  # noqa: E402

ROWS_512 = np.array([0, 1, 257, 511])
SAMPLE_SEED = 12345


def samples(n_pix, count, seed):
    return np.sort(np.random.default_rng(seed).choice(n_pix, count, replace=False))


def make_512(path, iters=2000):
    case = SI.case_512()
    n = 512
    pb = O.Problem(n, n, 1, case.levels, h=O.symmlet(6),
                   w=O.expand_level_weights(case.level_w, n, n, case.levels))
    f0 = O.apply_H(pb, case.clean) + case.noise
    tau = O.step_size(pb)
    t = time.time()
    ref = O.fista(pb, f0, tau, iters, log=True)
    print(f"512: {iters} iterations in {time.time() - t:.1f} s, tau = {tau:.9f}", flush=True)
    idx = samples(n * n, 4096, SAMPLE_SEED)
    f, z = ref["f"][0], ref["z"][0]
    np.savez_compressed(path, tau=tau, iters=iters, rows=ROWS_512, f_rows=f[ROWS_512], z_rows=z[ROWS_512],
                        idx=idx, f_idx=f.ravel()[idx], z_idx=z.ravel()[idx], log=ref["log"],
                        f_sum=f.sum(), f_sq=(f * f).sum(), z_abs=np.abs(z).sum())


def make_colour(path, iters=100):
    c = SI.case_colour()
    n = 2048
    pb = O.Problem(n, n, 3, c.levels, h=O.symmlet(6), w=O.expand_level_weights(c.level_w, n, n, c.levels, 3),
                   joint=True)
    f0 = np.stack([O.apply_H(pb, c.clean[k]) for k in range(3)]) + c.noise
    f0 = np.where(c.sp_mask[None], c.sp_val[None], f0)
    tau = 0.89
    t = time.time()
    ref = O.fista(pb, f0, tau, iters, log=True)
    print(f"colour: {iters} iterations in {time.time() - t:.1f} s", flush=True)
    rows = np.array([1500])
    idx = np.stack([samples(n * n, 2048, SAMPLE_SEED + k) for k in range(3)])
    f, z = ref["f"], ref["z"]
    np.savez_compressed(path, tau=tau, iters=iters, rows=rows, f_rows=f[:, rows], z_rows=z[:, rows], idx=idx,
                        f_idx=np.stack([f[k].ravel()[idx[k]] for k in range(3)]),
                        z_idx=np.stack([z[k].ravel()[idx[k]] for k in range(3)]), log=ref["log"],
                        f_sum=f.sum(), f_sq=(f * f).sum(), z_abs=np.abs(z).sum())


BATCH_SMALLEST = 4


def batch_smallest(count=64):
    """Indices of the BATCH_SMALLEST smallest images of the batch draw (by area, then index)."""
    shapes = SI.batch_shapes(count)
    return sorted(range(count), key=lambda b: (shapes[b][0] * shapes[b][1], b))[:BATCH_SMALLEST]


def make_batch(path, iters=1000):
    cases = SI.case_batch(64)
    out = {"iters": iters, "images": np.array(batch_smallest())}
    for j, b in enumerate(out["images"]):
        c = cases[b]
        pb = O.Problem(c.n1, c.n2, 1, c.levels, h=O.symmlet(6),
                       w=O.expand_level_weights(c.level_w, c.n1, c.n2, c.levels))
        f0 = O.apply_H(pb, c.clean) + c.noise
        tau = O.step_size(pb)
        t = time.time()
        ref = O.fista(pb, f0, tau, iters, log=True)
        print(f"batch image {b} ({c.n1} x {c.n2}): {iters} iterations in {time.time() - t:.1f} s", flush=True)
        f = ref["f"][0]
        rows = np.array([0, c.n2 // 2 + 1])
        idx = samples(c.n1 * c.n2, 1024, SAMPLE_SEED + b)
        out.update({f"tau_{j}": tau, f"rows_{j}": rows, f"f_rows_{j}": f[rows], f"idx_{j}": idx,
                    f"f_idx_{j}": f.ravel()[idx], f"log_{j}": ref["log"], f"f_sum_{j}": f.sum()})
    np.savez_compressed(path, **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["512", "colour", "batch"]
    if "512" in which:
        make_512(os.path.join(HERE, "fullsize_512.npz"))
    if "colour" in which:
        make_colour(os.path.join(HERE, "fullsize_colour.npz"))
    if "batch" in which:
        make_batch(os.path.join(HERE, "fullsize_batch.npz"))
