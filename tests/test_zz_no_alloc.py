"""pd_solve_noalloc (the entry point for callers that cannot allocate) against
pd_solve on the same inputs: two calls in a row on the library's fixed
scratch, the second on a smaller problem with other options, each equal to
pd_solve (which runs on its own workspace) bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
import syninputs as SI  # noqa: E402
import paper_2005_09870_amd as P  # noqa: E402

DEV = "cuda"


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.array(a, dtype=np.float64), dtype=dtype, device=DEV)


def _inputs(n1, n2, seed, C=1):
    c = SI.make_case(n1, n2, C, 6, 4, "const", 0.1, 0.1, seed=seed)
    pb = O.Problem(n1, n2, C, c.levels, h=O.symmlet(6))
    f0 = np.stack([O.apply_H(pb, c.clean[k]) for k in range(C)]) + c.noise
    return c, _t(f0), P.Operator.op1(n2, dtype=torch.float32, device=DEV)


def test_noalloc_matches_pd_solve_twice():
    h = P.pd_symmlet(6)
    # 1: 512 x 512, 300 iterations (pd_solve replays graph chunks, the allocation-free call launches each)
    c, f0, op = _inputs(512, 512, seed=2)
    K = 300
    ref = P.pd_solve(f0, op, h, c.levels, 0.89, K, level_w=c.level_w, stats=True)
    f = torch.empty_like(f0)
    st = torch.zeros((K, 3), dtype=torch.float64, device=DEV)
    out = P.pd_solve_noalloc(f0, op, h, c.levels, 0.89, K, level_w=c.level_w, f_out=f, stats=st)
    torch.cuda.synchronize()
    for k in ("z_cur", "z_prev"):
        assert torch.equal(out[k], ref[k]), k
    assert torch.equal(f, ref["f"])
    np.testing.assert_allclose(st.cpu().numpy(), ref["stats"].cpu().numpy(), rtol=1e-12)
    # 2: a smaller problem right after (the scratch keeps the first call's contents):
    # 160 x 96 with per-coefficient weights and the finite check
    c2, f02, op2 = _inputs(160, 96, seed=5)
    rng = np.random.default_rng(6)
    w = _t(np.log1p(np.exp(rng.normal(-2.0, 0.1, (1, 96, 160)))))
    K2 = 45
    ref2 = P.pd_solve(f02, op2, h, c2.levels, 0.85, K2, coeff_w=w, stats=True)
    f2 = torch.empty_like(f02)
    st2 = torch.zeros((K2, 3), dtype=torch.float64, device=DEV)
    out2 = P.pd_solve_noalloc(f02, op2, h, c2.levels, 0.85, K2, coeff_w=w, f_out=f2, stats=st2,
                              check_finite=True)
    for k in ("z_cur", "z_prev"):
        assert torch.equal(out2[k], ref2[k]), k
    assert torch.equal(f2, ref2["f"])
    np.testing.assert_allclose(st2.cpu().numpy(), ref2["stats"].cpu().numpy(), rtol=1e-12)
    # and against the oracle (the forward tolerance)
    pb2 = O.Problem(160, 96, 1, c2.levels, h=O.symmlet(6), w=w.double().cpu().numpy())
    orc = O.fista(pb2, f02.double().cpu().numpy(), 0.85, K2)
    assert np.abs(f2.double().cpu().numpy() - orc["f"]).max() < 1e-5


def test_noalloc_rejects_problems_beyond_its_scratch():
    f0 = torch.zeros((1, 2048, 2048), dtype=torch.float32, device=DEV)  # workspace ~ 40 MB > the scratch
    op = P.Operator.op1(2048, dtype=torch.float32, device=DEV)
    with pytest.raises(P.PDError) as e:
        P.pd_solve_noalloc(f0, op, P.pd_symmlet(6), 11, 0.89, 3, level_w=np.zeros(12))
    assert e.value.code == -3
