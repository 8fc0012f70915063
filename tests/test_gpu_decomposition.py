"""GPU parity of Algorithm 1 (Section 3.2; Section 5): pd_decompose against the
dense FP64 oracle on the same expansion.  Both sides threshold in FP64 with
the same rule; Theta~ is compared entry by entry (1e-12 of its largest
magnitude), and the certificate ||Theta - Theta~||_2 <= eta is checked on the
GPU's output with an exact spectral norm.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from oracle import decomposition as D  # noqa: E402
from oracle import product_convolution as PC  # noqa: E402
from oracle import wavelet_domain as W  # noqa: E402
import paper_2005_09870_amd as P  # noqa: E402
from paper_2005_09870_amd import _lib as C  # noqa: E402

DEV = "cuda"
H6 = O.symmlet(6)


def _case(n2, n1, m, R, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((m, 2 * R + 1, 2 * R + 1)) / (2 * R + 1)
    y2, y1 = np.meshgrid(np.arange(n2) / n2, np.arange(n1) / n1, indexing="ij")
    v = np.stack([1.0 + 0.5 * np.cos(2 * np.pi * (a * y1 + b * y2) + c) for a, b, c in rng.uniform(0, 2, (m, 3))])
    return u, v


def _dense(cols: "P.Csr", N: int) -> np.ndarray:
    cp = cols.row_ptr.cpu().numpy()
    r = cols.col.cpu().numpy()
    v = cols.val.cpu().numpy()
    M = np.zeros((N, N))
    for j in range(N):
        M[r[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
    return M


def _gpu(u, v, L, eta, **kw):
    n2, n1 = v.shape[1:]
    op = P.Operator.pc(u, v, dtype=torch.float64, device=DEV)
    return P.pd_decompose(op, H6, L, n2, n1, eta, **kw)


@pytest.mark.parametrize("n2,n1,L,m,R", [(16, 16, 2, 3, 2), (16, 32, 3, 2, 1), (32, 16, 2, 2, 3)])
@pytest.mark.parametrize("eta", [0.0, 1e-2, 0.1])
def test_decompose_matches_oracle(n2, n1, L, m, R, eta):
    u, v = _case(n2, n1, m, R, n1 + 7 * m)
    ref = D.decompose(u, v, L, H6, eta)["theta"]
    cols = _gpu(u, v, L, eta)
    got = _dense(cols, n1 * n2)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    cp = cols.row_ptr.cpu().numpy()
    assert cp[0] == 0 and np.all(np.diff(cp) >= 0) and cp[-1] == cols.nnz
    r = cols.col.cpu().numpy()
    for j in range(0, n1 * n2, 17):
        assert np.all(np.diff(r[cp[j]:cp[j + 1]]) > 0)


def test_exact_operator1_expansion_is_theta():
    """eta = 0 with the full-rank expansion of Operator 1: Theta~ = Psi^* H Psi."""
    n = 16
    kt, R = O.op1_profiles(n)
    u, vr, _ = PC.pc_expansion(kt, R)
    v = PC.rows_to_pixels(vr, n)
    ref = W.theta_dense(O.Problem(n, n, 1, 2, h=H6))
    got = _dense(_gpu(u, v, 2, 0.0), n * n)
    assert np.abs(got - ref).max() < 1e-11


def test_certificate_on_gpu_output():
    n2 = n1 = 32
    L = 3
    u, v = _case(n2, n1, 3, 2, 11)
    theta = D.wavelet_matrix(lambda x: PC.apply_pc(u, v, x), n2, n1, L, H6)
    for eta in (0.02, 0.2):
        got = _dense(_gpu(u, v, L, eta), n1 * n2)
        assert np.linalg.norm(theta - got, 2) <= eta * (1 + 1e-10)


def test_capacity_and_count_only():
    """Too small a capacity is an error with the count reported; a second call
    with room gives the same matrix (the FP64 atomic sums are not bitwise
    reproducible, so the values agree to rounding and an entry that cancels
    may be absent in one call and present, tiny, in the other)."""
    u, v = _case(16, 16, 2, 1, 3)
    full = _gpu(u, v, 2, 0.05)
    with pytest.raises(C.PDError) as e:
        _gpu(u, v, 2, 0.05, capacity=max(full.nnz // 2, 1))
    assert e.value.code == C.PD_ERR_WORKSPACE
    again = _gpu(u, v, 2, 0.05, capacity=full.nnz + 4096)
    a, b = _dense(full, 256), _dense(again, 256)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    assert abs(again.nnz - full.nnz) <= full.nnz // 100


def test_two_accumulator_parts_exact_columns():
    """96 x 256 (N = 24576: two accumulator parts, the second partial), eta = 0:
    sampled columns of Theta~ equal Psi^* H Psi e_mu from the oracle."""
    n2, n1, L = 96, 256, 3
    u, v = _case(n2, n1, 2, 1, 21)
    cols = _gpu(u, v, L, 0.0)
    cp, r, val = (t.cpu().numpy() for t in (cols.row_ptr, cols.col, cols.val))
    N = n1 * n2
    rng = np.random.default_rng(4)
    picks = list(rng.choice(N, 12, replace=False)) + [0, 5, n1 * (n2 // 8) + 3, N - 1]
    for mu in picks:
        e = np.zeros(N)
        e[mu] = 1.0
        ref = O.fwt(PC.apply_pc(u, v, O.ifwt(e.reshape(n2, n1), L, H6)), L, H6).ravel()
        got = np.zeros(N)
        got[r[cp[mu]:cp[mu + 1]]] = val[cp[mu]:cp[mu + 1]]
        assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), mu


def test_single_level_flat_image():
    """levels = 1 on a flat 8 x 32 image (four bands), eta 0 and 0.05."""
    u, v = _case(8, 32, 2, 2, 31)
    for eta in (0.0, 0.05):
        ref = D.decompose(u, v, 1, H6, eta)["theta"]
        got = _dense(_gpu(u, v, 1, eta), 8 * 32)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
