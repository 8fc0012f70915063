"""GPU parity: the HIP path (through the C ABI) against the oracle.

Tolerances:
  * FP64 GPU vs FP64 oracle: 1e-10 max-abs on iterates (same recursion, only
    the summation order inside the filters and the blur differs).
  * FP32 GPU vs FP64 oracle: 1e-5 max-abs on f = Psi z and on z after a fixed
    iteration count (BASELINE tolerance for the forward solve).  Inputs are in
    [0, 1]-scale (clean image + noise).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
import syninputs as SI  # noqa: E402
import paper_2005_09870_amd as P  # noqa: E402

DEV = "cuda"
H = None


def _h():
    global H
    if H is None:
        H = O.symmlet(6)
    return H


def _t(a, dtype):
    return torch.as_tensor(np.array(a, dtype=np.float64), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().double().cpu().numpy()


def _op(pb, dtype):
    if pb.op_identity:
        return P.Operator.identity()
    return P.Operator.from_taps(pb.kt, pb.R, dtype=dtype)


def _problem(n1, n2, C=1, levels=None, op="op1", lam=0.1, seed=0, joint=False, coeff=False):
    case = SI.make_case(n1, n2, C, 6, 4, "const", 0.1, lam, levels=levels, seed=seed)
    L = case.levels
    if coeff:
        rng = np.random.default_rng(seed + 100)
        w = np.log1p(np.exp(rng.normal(-2.0, 0.1, (C, n2, n1))))
    else:
        w = O.expand_level_weights(case.level_w, n1, n2, L, C)
    pb = O.Problem(n1, n2, C, L, h=_h(), op=op, w=w, joint=joint)
    f0 = np.stack([O.apply_H(pb, case.clean[c]) for c in range(C)]) + case.noise
    return pb, f0, case


def _gpu_solve(pb, f0, case, tau, iters, dtype, coeff=False, **kw):
    op = _op(pb, dtype)
    args = dict(level_w=None if coeff else case.level_w,
                coeff_w=_t(pb.w, dtype) if coeff else None, joint=bool(pb.joint))
    args.update(kw)
    return P.pd_solve(_t(f0, dtype), op, _h(), pb.levels, tau, iters, **args)


# ------------------------------------------------------------ building blocks
@pytest.mark.parametrize("shape,levels", [((64, 64), 6), ((96, 160), 5), ((512, 512), 9), ((32, 64), 2)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fwt_matches_oracle(shape, levels, dtype):
    rng = np.random.default_rng(10)
    x = rng.standard_normal((2,) + shape)
    c = _np(P.pd_fwt(_t(x, dtype), _h(), levels))
    ref = O.fwt(x, levels, _h())
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert np.abs(c - ref).max() < tol * max(1.0, np.abs(ref).max())
    back = _np(P.pd_fwt(_t(ref, dtype), _h(), levels, inverse=True))
    assert np.abs(back - x).max() < tol * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("shape", [(64, 64), (96, 160), (40, 24)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_blur_matches_oracle(shape, dtype):
    n2, n1 = shape
    kt, R = O.op1_profiles(n2)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((1, n2, n1))
    op = P.Operator.from_taps(kt, R, dtype=dtype)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for tr in (False, True):
        got = _np(P.pd_apply_op(_t(x, dtype), op, transpose=tr))
        ref = O.blur(x[0], kt, R, transpose=tr)
        assert np.abs(got[0] - ref).max() < tol


# ----------------------------------------------------------------- solver ---
def test_solve_fp64_matches_oracle_64():
    """64x64, Operator 1, lambda 0.1, 500 iterations (the small workload), FP64."""
    pb, f0, case = _problem(64, 64, seed=1)
    tau = O.step_size(pb)
    ref = O.fista(pb, f0, tau, 500, log=True)
    out = _gpu_solve(pb, f0, case, tau, 500, torch.float64, stats=True)
    assert np.abs(_np(out["z_cur"]) - ref["z"]).max() < 1e-10
    assert np.abs(_np(out["f"]) - ref["f"]).max() < 1e-10
    st = _np(out["stats"])
    np.testing.assert_allclose(st, ref["log"], rtol=1e-9, atol=1e-12)


def test_solve_fp32_matches_oracle_64():
    """Same workload in FP32 against the FP64 oracle: 1e-5 max-abs."""
    pb, f0, case = _problem(64, 64, seed=1)
    tau = O.step_size(pb)
    ref = O.fista(pb, f0, tau, 500, log=True)
    out = _gpu_solve(pb, f0, case, tau, 500, torch.float32, stats=True)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < 1e-5
    assert np.abs(_np(out["z_cur"]) - ref["z"]).max() < 1e-5
    st = _np(out["stats"])
    np.testing.assert_allclose(st[:, :2], ref["log"][:, :2], rtol=1e-4)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_solve_ragged_nonsquare(dtype, tol):
    """96 x 160 (tiles do not divide the image), 5 levels, 100 iterations."""
    pb, f0, case = _problem(160, 96, seed=2)
    tau = O.step_size(pb)
    ref = O.fista(pb, f0, tau, 100)
    out = _gpu_solve(pb, f0, case, tau, 100, dtype)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < tol
    assert np.abs(_np(out["z_cur"]) - ref["z"]).max() < tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_solve_partial_depth_and_coeff_weights(dtype, tol):
    """3 levels of a 64 x 32 image, per-coefficient weight map."""
    pb, f0, case = _problem(64, 32, levels=3, seed=3, coeff=True)
    tau = O.step_size(pb)
    ref = O.fista(pb, f0, tau, 60)
    out = _gpu_solve(pb, f0, case, tau, 60, dtype, coeff=True)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_solve_joint_colour(dtype, tol):
    """3 channels with joint (group) shrinkage across channels."""
    pb, f0, case = _problem(64, 64, C=3, seed=4, joint=True)
    tau = O.step_size(pb)
    ref = O.fista(pb, f0, tau, 80)
    out = _gpu_solve(pb, f0, case, tau, 80, dtype)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < tol


def test_identity_operator_closed_form():
    """H = Id, tau = 1: the first iterate is the closed-form minimiser."""
    pb, f0, case = _problem(64, 64, op="identity", seed=5)
    c = O.fwt(f0, pb.levels, _h())
    zstar = np.sign(c) * np.maximum(np.abs(c) - pb.w, 0.0)
    scale = max(1.0, float(np.abs(zstar).max()))  # approximation band ~ 2^levels
    for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 4e-7)):
        out = _gpu_solve(pb, f0, case, 1.0, 3, dtype)
        assert np.abs(_np(out["z_cur"]) - zstar).max() < tol * scale


def test_zero_iterations_returns_init():
    pb, f0, case = _problem(64, 64, seed=6)
    out = _gpu_solve(pb, f0, case, 0.5, 0, torch.float64)
    np.testing.assert_allclose(_np(out["f"]), f0, atol=1e-12)
    np.testing.assert_allclose(_np(out["z_cur"]), O.fwt(f0, pb.levels, _h()), atol=1e-12)


def test_resume_is_bitwise():
    """K1 iterations, then K2 more from the returned state with iter_offset=K1,
    equals K1+K2 iterations in one call, bit for bit."""
    pb, f0, case = _problem(64, 64, seed=7)
    tau = O.step_size(pb)
    full = _gpu_solve(pb, f0, case, tau, 37, torch.float32)
    a = _gpu_solve(pb, f0, case, tau, 20, torch.float32, want_f=False)
    b = _gpu_solve(pb, f0, case, tau, 17, torch.float32, z_cur=a["z_cur"], z_prev=a["z_prev"],
                   init=False, iter_offset=20)
    assert torch.equal(full["f"], b["f"])
    assert torch.equal(full["z_prev"], b["z_prev"])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_graph_replay_is_bitwise(dtype):
    """The middle iterations replayed from a captured graph (chunks of 64 that
    read the iteration number from the workspace) equal eager launches bit for
    bit, for a fresh capture, a cache hit and a resumed solve (iter_offset)."""
    pb, f0, case = _problem(96, 64, seed=9)
    tau = O.step_size(pb)
    runs = {}
    try:
        for on in (False, True):
            P.pd_graphs_enable(on)
            # 300 iterations: chunks at 1, 65, 129, 193 (captured: replayed 4 times)
            a = _gpu_solve(pb, f0, case, tau, 300, dtype, stats=True)
            b = _gpu_solve(pb, f0, case, tau, 300, dtype, stats=True)  # second call: cached graph
            c = _gpu_solve(pb, f0, case, tau, 290, dtype, z_cur=a["z_cur"].clone(),
                           z_prev=a["z_prev"].clone(), init=False, iter_offset=300)
            runs[on] = (a, b, c)
    finally:
        P.pd_graphs_enable(True)
    for k in ("f", "z_cur", "z_prev"):
        for r in range(3):
            assert torch.equal(runs[False][r][k], runs[True][r][k]), (k, r)
        assert torch.equal(runs[True][0][k], runs[True][1][k])
    # statistics: FP64 partial sums added atomically (order-dependent rounding)
    for r in range(2):
        np.testing.assert_allclose(_np(runs[True][r]["stats"]), _np(runs[False][r]["stats"]), rtol=1e-12)


def test_nonfinite_is_reported():
    pb, f0, case = _problem(64, 64, seed=8)
    f0 = f0.copy()
    f0[0, 10, 10] = np.nan
    with pytest.raises(P.PDError) as e:
        _gpu_solve(pb, f0, case, 0.5, 3, torch.float32, check_finite=True)
    assert e.value.code == -5


def test_full_size_512_first_iterations():
    """The 512 x 512 workload at full size: 3 iterations element by element."""
    case = SI.case_512()
    pb = O.Problem(512, 512, 1, case.levels, h=_h(),
                   w=O.expand_level_weights(case.level_w, 512, 512, case.levels))
    f0 = O.apply_H(pb, case.clean) + case.noise
    tau = 0.89
    ref = O.fista(pb, f0, tau, 3)
    out = _gpu_solve(pb, f0, case, tau, 3, torch.float32)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < 1e-5


def test_batched_equals_per_image():
    """pd_solve_batched on uneven sizes equals pd_solve per image bit for bit."""
    shapes = [(96, 128), (160, 96), (64, 64)]
    f0s, ops, lws, taus, levels, singles = [], [], [], [], [], []
    for b, (n1, n2) in enumerate(shapes):
        pb, f0, case = _problem(n1, n2, seed=20 + b)
        tau = O.step_size(pb)
        f0t = _t(f0, torch.float32)
        op = _op(pb, torch.float32)
        f0s.append(f0t)
        ops.append(op)
        lws.append(case.level_w)
        taus.append(tau)
        levels.append(pb.levels)
        singles.append(P.pd_solve(f0t, op, _h(), pb.levels, tau, 40, level_w=case.level_w)["f"])
    outs, _ = P.pd_solve_batched(f0s, ops, lws, taus, _h(), levels, 40)
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)


# ------------------------------------------------------------- edge cases ---
@pytest.mark.parametrize("n1,n2,levels", [(2, 2, 1), (4, 4, 2), (8, 8, 3), (16, 8, 3), (32, 4, 2)])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_tiny_shapes(n1, n2, levels, dtype, tol):
    """Images smaller than every tile and than the blur support (the profiles
    wrap around the period several times); the coarse block is the image."""
    pb, f0, case = _problem(n1, n2, levels=levels, seed=40 + n1 + n2)
    tau = O.step_size(pb)
    ref = O.fista(pb, f0, tau, 30)
    out = _gpu_solve(pb, f0, case, tau, 30, dtype)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < tol
    assert np.abs(_np(out["z_cur"]) - ref["z"]).max() < tol


def test_zero_weights_is_plain_gradient_descent():
    """lambda = 0: no shrinkage, the iteration is accelerated gradient descent
    on 1/2 ||H Psi z - f0||^2 (the oracle computes the same recursion)."""
    pb, f0, case = _problem(96, 64, seed=50)
    pb0 = O.Problem(pb.n1, pb.n2, 1, pb.levels, h=_h(), w=np.zeros_like(pb.w))
    tau = O.step_size(pb0)
    ref = O.fista(pb0, f0, tau, 50)
    out = P.pd_solve(_t(f0, torch.float64), _op(pb0, torch.float64), _h(), pb0.levels, tau, 50,
                     level_w=np.zeros(pb0.levels + 1))
    assert np.abs(_np(out["f"]) - ref["f"]).max() < 1e-10


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_batched_marching_blur_mix(dtype):
    """Images at least 128 wide run the batched blur as the two marching
    kernels (ragged strips and row blocks here), narrower ones as the tile
    kernel, in one batch; each equals pd_solve on its own bit for bit, and so
    does a three-channel image."""
    for shapes, C in (([(256, 128), (96, 64), (320, 160), (288, 40)], 1), ([(256, 96), (64, 96)], 3)):
        f0s, ops, lws, _, taus, levels, pbs = _batch_inputs(shapes, C=C, seed=90)
        if dtype == torch.float64:
            f0s = [_t(f0, dtype) for _, f0, _ in pbs]
            ops = [_op(pb, dtype) for pb, _, _ in pbs]
        outs, _ = P.pd_solve_batched(f0s, ops, lws, taus, _h(), levels, 50)
        for b in range(len(shapes)):
            single = P.pd_solve(f0s[b], ops[b], _h(), levels[b], taus[b], 50, level_w=lws[b])["f"]
            assert torch.equal(outs[b], single), (shapes[b], C)


def test_batched_edge_cases():
    """A batch of one image, and a batch mixing an image whose coarse block is
    the whole image (no fine level) with larger ones; equal to pd_solve."""
    for shapes in ([(128, 96)], [(32, 32), (160, 96), (64, 128)]):
        f0s, ops, lws, taus, levels, singles = [], [], [], [], [], []
        for b, (n1, n2) in enumerate(shapes):
            pb, f0, case = _problem(n1, n2, seed=60 + b)
            tau = O.step_size(pb)
            f0t = _t(f0, torch.float32)
            op = _op(pb, torch.float32)
            f0s.append(f0t)
            ops.append(op)
            lws.append(case.level_w)
            taus.append(tau)
            levels.append(pb.levels)
            singles.append(P.pd_solve(f0t, op, _h(), pb.levels, tau, 70, level_w=case.level_w)["f"])
        outs, _ = P.pd_solve_batched(f0s, ops, lws, taus, _h(), levels, 70)
        for a, b in zip(outs, singles):
            assert torch.equal(a, b)


def test_colour_2048_full_size():
    """The largest workload (2048 x 2048 x 3, joint shrinkage, salt-and-pepper
    noise) at full size: 2 iterations against the oracle, every pixel."""
    c = SI.case_colour()
    n = 2048
    pb = O.Problem(n, n, 3, c.levels, h=_h(), w=O.expand_level_weights(c.level_w, n, n, c.levels, 3),
                   joint=True)
    f0 = np.stack([O.apply_H(pb, c.clean[k]) for k in range(3)]) + c.noise
    f0 = np.where(c.sp_mask[None], c.sp_val[None], f0)
    tau = 0.89
    ref = O.fista(pb, f0, tau, 2)
    op = P.Operator.from_taps(pb.kt, pb.R, dtype=torch.float32)
    out = P.pd_solve(_t(f0, torch.float32), op, _h(), c.levels, tau, 2, level_w=c.level_w, joint=True)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < 1e-5


def _batch_inputs(shapes, C=1, seed=70, coeff=False, iters=None):
    f0s, ops, lws, cws, taus, levels, pbs = [], [], [], [], [], [], []
    for b, (n1, n2) in enumerate(shapes):
        pb, f0, case = _problem(n1, n2, C=C, seed=seed + b, coeff=coeff, joint=False)
        f0s.append(_t(f0, torch.float32))
        ops.append(_op(pb, torch.float32))
        lws.append(case.level_w)
        cws.append(_t(pb.w, torch.float32) if coeff else None)
        taus.append(0.8 + 0.02 * b)
        levels.append(pb.levels)
        pbs.append((pb, f0, case))
    return f0s, ops, lws, cws, taus, levels, pbs


def test_batched_graph_replay_is_bitwise():
    """300 iterations (the middle ones replayed from captured graph chunks):
    pd_solve_batched equals itself with graph replay off and pd_solve per image
    bit for bit; the statistics agree to the rounding of their FP64 atomics."""
    shapes = [(96, 128), (160, 96), (64, 64)]
    f0s, ops, lws, _, taus, levels, _ = _batch_inputs(shapes)
    K = 300
    runs = {}
    try:
        for g in (True, False):
            P.pd_graphs_enable(g)
            runs[g] = [P.pd_solve_batched(f0s, ops, lws, taus, _h(), levels, K, stats=True) for _ in range(2)]
    finally:
        P.pd_graphs_enable(True)
    for b in range(len(shapes)):
        single = P.pd_solve(f0s[b], ops[b], _h(), levels[b], taus[b], K, level_w=lws[b], stats=True)
        for g in (True, False):
            for r in range(2):
                assert torch.equal(runs[g][r][0][b], single["f"]), (b, g, r)
                np.testing.assert_allclose(_np(runs[g][r][1][b]), _np(single["stats"]), rtol=1e-12)


def test_batched_weight_maps_and_joint_prox():
    """Per-coefficient weight maps and the joint colour prox in lock-step
    batches: bitwise equal to pd_solve per image, and the joint batch against
    the oracle."""
    shapes = [(96, 64), (64, 128), (32, 32)]
    f0s, ops, lws, cws, taus, levels, _ = _batch_inputs(shapes, coeff=True, seed=80)
    outs, _ = P.pd_solve_batched(f0s, ops, lws, taus, _h(), levels, 60, coeff_ws=cws)
    for b in range(len(shapes)):
        ref = P.pd_solve(f0s[b], ops[b], _h(), levels[b], taus[b], 60, coeff_w=cws[b])["f"]
        assert torch.equal(outs[b], ref), b
    f0s, ops, lws, _, taus, levels, pbs = _batch_inputs(shapes, C=3, seed=90)
    outs, st = P.pd_solve_batched(f0s, ops, lws, taus, _h(), levels, 60, joint=True, stats=True)
    for b in range(len(shapes)):
        ref = P.pd_solve(f0s[b], ops[b], _h(), levels[b], taus[b], 60, level_w=lws[b], joint=True, stats=True)
        assert torch.equal(outs[b], ref["f"]), b
        np.testing.assert_allclose(_np(st[b]), _np(ref["stats"]), rtol=1e-12)
        pb, f0, case = pbs[b]
        pbj = O.Problem(pb.n1, pb.n2, 3, pb.levels, h=_h(), w=pb.w, joint=True)
        orc = O.fista(pbj, f0, taus[b], 60)
        assert np.abs(_np(outs[b]) - orc["f"]).max() < 1e-5
    with pytest.raises(P.PDError) as e:  # every image of a batch takes the same prox kind
        f0m = [f0s[0], f0s[1][:1].contiguous()]
        P.pd_solve_batched(f0m, ops[:2], lws[:2], taus[:2], _h(), levels[:2], 5, joint=True)
    assert e.value.code == -7


@pytest.mark.parametrize("n,levels", [(64, 6), (96, 5)])
def test_joint_prox_single_channel(n, levels):
    """The joint (group) prox with one channel, whose coarse block is done level
    by level before the tail (the joint workgroup keeps the block in its home
    array for the synthesis): against the oracle's joint prox."""
    pb, f0, case = _problem(n, n, C=1, levels=levels, seed=95, joint=True)
    tau = O.step_size(pb)
    ref = O.fista(pb, f0, tau, 30)
    out = _gpu_solve(pb, f0, case, tau, 30, torch.float64)
    assert np.abs(_np(out["f"]) - ref["f"]).max() < 1e-10
    assert np.abs(_np(out["z_cur"]) - ref["z"]).max() < 1e-10


@pytest.mark.parametrize("n1,n2,C,dtype", [(512, 512, 1, torch.float32), (160, 96, 3, torch.float32),
                                            (384, 200, 1, torch.float32), (8, 8, 1, torch.float32),
                                            (256, 136, 2, torch.float64)])
def test_blur_variants_are_bitwise(n1, n2, C, dtype):
    """Every blur variant (fused tile heights 32 and 48, and the two marching
    kernels with 20, 39 and 58 rows per wave) gives the same iterates bit for
    bit (the autotuner's choice never changes results), on widths that are not
    a multiple of any strip and heights shorter than the profile window;
    pd_tune records a variant and reports it."""
    pb, f0, case = _problem(n1, n2, C=C, levels=3 if n1 == 8 else None, seed=97)
    f0t = _t(f0, dtype)
    op = _op(pb, dtype)
    outs = {}
    try:
        for v in P.BLUR_VARIANTS:
            assert P.pd_tune(f0t, op, pb.levels, pin=v) == v
            outs[v] = P.pd_solve(f0t, op, _h(), pb.levels, 0.85, 40, level_w=case.level_w, stats=True)
        for v in P.BLUR_VARIANTS[1:]:
            for k in ("f", "z_cur", "z_prev"):
                assert torch.equal(outs[32][k], outs[v][k]), (v, k)
            np.testing.assert_allclose(_np(outs[32]["stats"]), _np(outs[v]["stats"]), rtol=1e-12)
        chosen = P.pd_tune(f0t, op, pb.levels)
        assert chosen in P.BLUR_VARIANTS
        again = P.pd_solve(f0t, op, _h(), pb.levels, 0.85, 40, level_w=case.level_w)
        assert torch.equal(again["f"], outs[32]["f"])
    finally:
        P.pd_tune(f0t, op, pb.levels, pin=32)
    ref = O.fista(pb, f0, 0.85, 40)
    assert np.abs(_np(outs[1039]["f"]) - ref["f"]).max() < (1e-10 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("n1,n2", [(96, 64), (256, 160)])
def test_blur_variants_reverse_mode_is_bitwise(n1, n2):
    """The reverse mode's accumulation of H Psi v through the blur (the
    marching r kernel's racc path) gives the same gradients bit for bit under
    every variant."""
    pb, f0, case = _problem(n1, n2, seed=98)
    f0t = _t(f0, torch.float32)
    op = _op(pb, torch.float32)
    rng = np.random.default_rng(5)
    gf = torch.tensor(rng.normal(size=f0.shape), dtype=torch.float32, device="cuda")
    outs = {}
    try:
        for v in P.BLUR_VARIANTS:
            P.pd_tune(f0t, op, pb.levels, pin=v)
            outs[v] = P.pd_backward(f0t, op, _h(), pb.levels, 0.85, 25, gf, level_w=case.level_w,
                                    checkpoint_every=10)
    finally:
        P.pd_tune(f0t, op, pb.levels, pin=32)
    for v in P.BLUR_VARIANTS[1:]:
        for a, b in zip(outs[32], outs[v]):
            if a is not None:
                assert torch.equal(a, b), v


@pytest.mark.parametrize("n1,n2,C,levels,coeff", [(512, 512, 1, 9, False), (160, 96, 2, 5, False),
                                                   (256, 128, 1, 3, False), (1024, 64, 1, 6, False),
                                                   (512, 256, 1, 2, False), (512, 512, 1, 9, True),
                                                   (352, 224, 1, 5, True), (320, 256, 2, 6, False),
                                                   (2048, 16, 1, 4, False), (16, 2048, 1, 4, True)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_fused_levels_are_bitwise(n1, n2, C, levels, coeff, dtype):
    """The coarsest fine synthesis levels in one launch (three, or two) and the two
    coarsest fine analysis levels in one launch give the same iterates and,
    statistics aside, bit for bit as one launch per level (on 2048 x 16 the
    fused analysis pair is levels 3 and 4, bands 2 and 1 rows high with level
    4 the last, and its 82-row input region wraps around a 4-row plane; and
    pd_fwt's forward and inverse transforms the same output), with level or
    per-coefficient weights."""
    pb, f0, case = _problem(n1, n2, C=C, levels=levels, seed=99, coeff=coeff)
    f0t = _t(f0, dtype)
    op = _op(pb, dtype)
    cw = _t(pb.w, dtype) if coeff else None
    outs = {}
    try:
        for fuse in (True, False):
            P.pd_fuse_enable(fuse)
            kw = dict(coeff_w=cw) if coeff else dict(level_w=case.level_w)
            outs[fuse] = (P.pd_solve(f0t, op, _h(), pb.levels, 0.85, 30, stats=True, **kw),
                          P.pd_fwt(f0t, _h(), pb.levels, inverse=True),
                          P.pd_fwt(f0t, _h(), pb.levels))
    finally:
        P.pd_fuse_enable(True)
    for k in ("f", "z_cur", "z_prev"):
        assert torch.equal(outs[True][0][k], outs[False][0][k]), k
    np.testing.assert_allclose(_np(outs[True][0]["stats"]), _np(outs[False][0]["stats"]), rtol=1e-12)
    assert torch.equal(outs[True][1], outs[False][1])
    assert torch.equal(outs[True][2], outs[False][2])
    ref = O.fista(pb, f0, 0.85, 30)
    assert np.abs(_np(outs[True][0]["f"]) - ref["f"]).max() < (1e-10 if dtype == torch.float64 else 1e-5)
