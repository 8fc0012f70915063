"""Host logic of the Theta_L builder (paper_2005_09870_amd.theta): with the
oracle's transforms and blur plugged in as the probe, the probed, shift-filled
matrix must equal the oracle's dense Theta = Psi^* H Psi thresholded at eta,
entry for entry (Section 4.3's Theta_L, here every entry with |value| >= eta).
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from oracle import wavelet_domain as W  # noqa: E402
from paper_2005_09870_amd import solver as S  # noqa: E402
from paper_2005_09870_amd import theta as TH  # noqa: E402


@pytest.mark.parametrize("n1,n2,levels,eta", [(32, 32, 5, 4e-3), (64, 32, 4, 2e-3), (32, 64, 3, 1e-2),
                                               (16, 16, 4, 0.0)])
def test_probed_theta_equals_dense(n1, n2, levels, eta):
    pb = O.Problem(n1, n2, 1, levels, h=O.symmlet(6))
    T = W.theta_dense(pb)

    def apply(x, transpose):
        xs = x.numpy()
        return torch.from_numpy(np.stack([
            O.fwt(O.apply_H(pb, O.ifwt(xs[c], levels, pb.h), transpose=transpose), levels, pb.h)
            for c in range(xs.shape[0])]))

    m = TH.theta_rowblur(S.Operator(1, pb.R, None), pb.h, n1, n2, levels, eta, dtype=torch.float64,
                         device="cpu", apply=apply)
    A = sp.csr_matrix((m.val.numpy(), m.col.numpy(), m.row_ptr.numpy()), shape=T.shape)
    assert A.has_sorted_indices
    ref = np.where(np.abs(T) >= eta, T, 0.0)
    assert A.nnz == int(np.count_nonzero(np.abs(T) >= eta))
    assert np.abs(A.toarray() - ref).max() < 1e-14
