"""Host-side pieces of the adjoint wrapper (CPU only)."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("n,c", [(512, 32), (16, 4), (100, 7), (33, 33)])
def test_bspline_operator_is_the_periodic_cubic_bspline(n, c):
    """The package's control-grid operator equals the input module's independent definition, and every
    row is a positive partition of unity (so a positive theta gives a positive D)."""
    from paper_2312_10316_amd import adjoint
    B = adjoint.bspline_operator(n, c, device="cpu").numpy()
    assert B.shape == (n, c)
    assert np.abs(B - W.bspline_matrix(n, c)).max() <= 1e-15
    assert np.abs(B.sum(axis=1) - 1.0).max() <= 1e-15
    assert B.min() >= 0.0
    # at a node that sits on a control point the weights are 1/6, 2/3, 1/6
    if n % c == 0:
        row = B[0]
        assert np.allclose(sorted(row[row > 0]), [1 / 6, 1 / 6, 2 / 3], rtol=0, atol=1e-15)
