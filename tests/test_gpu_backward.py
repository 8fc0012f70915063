"""GPU reverse mode (pd_backward, segment checkpointing) against the oracle's
full-tape reverse pass, which is itself pinned to FP64 central differences.

Tolerances (relative l2 error of each gradient): FP64 1e-9; FP32 1e-4 (the
BASELINE gradient tolerance).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
import syninputs as SI  # noqa: E402
import paper_2005_09870_amd as P  # noqa: E402

DEV = "cuda"


def _t(a, dtype):
    return torch.as_tensor(np.array(a, dtype=np.float64), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(n=32, seed=31, coeff=True):
    c = SI.make_case(n, n, 1, 6, 4, "const", 0.1, 0.1, seed=seed, theta=(-2.0, 0.1))
    kt, R = O.op1_profiles(n)
    h = O.symmlet(6)
    if coeff:
        w = np.log1p(np.exp(c.theta))
    else:
        w = O.expand_level_weights(c.level_w, n, n, c.levels)
    pb = O.Problem(n, n, 1, c.levels, h=h, op=(kt, R), w=w)
    f0 = O.apply_H(pb, c.clean) + c.noise
    return pb, f0, c, h, kt, R


def _oracle_grads(pb, f0, clean, tau, K):
    out = O.fista(pb, f0, tau, K, tape=True)
    fbar = out["f"] - clean
    g0, gw = O.fista_reverse(pb, tau, K, out["tape"], fbar)
    return fbar, g0, gw


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
@pytest.mark.parametrize("K,ce", [(25, 7), (12, 12), (1, 5)])
def test_backward_matches_oracle(dtype, tol, K, ce):
    pb, f0, c, h, kt, R = _case()
    tau = O.step_size(pb)
    fbar, g0, gw = _oracle_grads(pb, f0, c.clean, tau, K)
    op = P.Operator.from_taps(kt, R, dtype=dtype)
    gf0, gww = P.pd_backward(_t(f0, dtype), op, h, pb.levels, tau, K, _t(fbar, dtype),
                             coeff_w=_t(pb.w, dtype), checkpoint_every=ce)
    assert _rel(_np(gf0), g0) < tol
    assert _rel(_np(gww), gw) < tol


def test_backward_level_weights_and_nonsquare():
    """Per-band weights, 48 x 64 image, 4 levels, FP64."""
    c = SI.make_case(64, 48, 1, 6, 4, "const", 0.1, 0.1, seed=33, levels=4)
    kt, R = O.op1_profiles(48)
    h = O.symmlet(6)
    pb = O.Problem(64, 48, 1, 4, h=h, op=(kt, R),
                   w=O.expand_level_weights(c.level_w, 64, 48, 4))
    f0 = O.apply_H(pb, c.clean) + c.noise
    tau = O.step_size(pb)
    fbar, g0, gw = _oracle_grads(pb, f0, c.clean, tau, 15)
    op = P.Operator.from_taps(kt, R, dtype=torch.float64)
    gf0, gww = P.pd_backward(_t(f0, torch.float64), op, h, 4, tau, 15, _t(fbar, torch.float64),
                             level_w=c.level_w, checkpoint_every=4)
    assert _rel(_np(gf0), g0) < 1e-9
    assert _rel(_np(gww), gw) < 1e-9


def test_checkpoint_interval_does_not_change_gradients():
    """The recomputed iterates are bitwise those of the forward pass, so the
    gradients do not depend on the checkpoint interval (bit for bit)."""
    pb, f0, c, h, kt, R = _case(seed=34)
    tau = O.step_size(pb)
    op = P.Operator.from_taps(kt, R, dtype=torch.float32)
    gf = _t(np.random.default_rng(0).standard_normal(f0.shape), torch.float32)
    res = [P.pd_backward(_t(f0, torch.float32), op, h, pb.levels, tau, 20, gf,
                         coeff_w=_t(pb.w, torch.float32), checkpoint_every=ce) for ce in (1, 3, 20, 50)]
    for a in res[1:]:
        assert torch.equal(a[0], res[0][0]) and torch.equal(a[1], res[0][1])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_backward_graph_replay_is_bitwise(dtype):
    """Full segments replayed from one captured graph (the recomputation and
    the adjoint read the iteration number from the workspace) give the same
    gradients, bit for bit, as eager launches.  60 iterations, checkpoint 10:
    six segments, five replayed."""
    pb, f0, c, h, kt, R = _case(n=64, seed=33)
    tau = O.step_size(pb)
    op = P.Operator.from_taps(kt, R, dtype=dtype)
    fbar = np.random.default_rng(34).standard_normal(f0.shape)
    res = {}
    try:
        for on in (False, True):
            P.pd_graphs_enable(on)
            res[on] = P.pd_backward(_t(f0, dtype), op, h, pb.levels, tau, 60, _t(fbar, dtype),
                                    coeff_w=_t(pb.w, dtype), checkpoint_every=10)
    finally:
        P.pd_graphs_enable(True)
    assert torch.equal(res[False][0], res[True][0])
    assert torch.equal(res[False][1], res[True][1])


def test_autograd_function_matches_oracle():
    """torch.autograd through FistaSolve with w = softplus(theta): gradients of
    L = 1/2 ||f - clean||^2 w.r.t. f0 and theta (theta_bar = w_bar sigmoid(theta))."""
    pb, f0, c, h, kt, R = _case(seed=35)
    tau = O.step_size(pb)
    K = 20
    fbar, g0, gw = _oracle_grads(pb, f0, c.clean, tau, K)
    gtheta = gw * (1.0 / (1.0 + np.exp(-c.theta)))
    op = P.Operator.from_taps(kt, R, dtype=torch.float64)
    f0t = _t(f0, torch.float64).requires_grad_(True)
    th = _t(c.theta, torch.float64).requires_grad_(True)
    f = P.solve_autograd(f0t, th, op, h, pb.levels, tau, K, checkpoint_every=6)
    loss = 0.5 * ((f - _t(c.clean, torch.float64)) ** 2).sum()
    loss.backward()
    assert _rel(_np(f0t.grad), g0) < 1e-9
    assert _rel(_np(th.grad), gtheta) < 1e-9


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("K,ce", [(25, 7), (40, 20), (3, 5)])
def test_checkpointed_forward_and_backward_are_bitwise(dtype, K, ce):
    """pd_solve_checkpointed writes the f of pd_solve bit for bit and leaves
    checkpoints from which pd_backward_checkpointed returns pd_backward's
    gradients bit for bit (twice, for two seeds on one workspace)."""
    pb, f0, c, h, kt, R = _case(n=48, seed=33)
    tau = O.step_size(pb)
    op = P.Operator.from_taps(kt, R, dtype=dtype)
    f0t, wt = _t(f0, dtype), _t(pb.w, dtype)
    f_ref = P.pd_solve(f0t, op, h, pb.levels, tau, K, coeff_w=wt)["f"]
    f, ws = P.pd_solve_checkpointed(f0t, op, h, pb.levels, tau, K, coeff_w=wt, checkpoint_every=ce)
    assert torch.equal(f, f_ref)
    for seed in (0, 1):
        fbar = _t(np.random.default_rng(seed).standard_normal(f0.shape), dtype)
        a0, aw = P.pd_backward(f0t, op, h, pb.levels, tau, K, fbar, coeff_w=wt, checkpoint_every=ce)
        b0, bw = P.pd_backward(f0t, op, h, pb.levels, tau, K, fbar, coeff_w=wt, checkpoint_every=ce, ws=ws)
        assert torch.equal(a0, b0) and torch.equal(aw, bw), seed
