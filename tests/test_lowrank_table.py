"""The low-rank preconditioner's host factor (kp_lowrank_table, no GPU)
against LAPACK's SVD of the Hadamard pseudoinverse built from the library's
closed-form eigenvalues."""

import numpy as np
import pytest


@pytest.mark.parametrize("n,bn,q,bq,r", [(9, "D", 12, "DN", 3), (50, "N", 100, "P", 3),
                                         (64, "D", 64, "D", 2), (20, "N", 30, "P", 2),
                                         (128, "P", 128, "P", 5), (40, "DN", 120, "P", 16),
                                         (7, "P", 5, "N", 5)])
def test_table_is_the_best_rank_r_approximation(n, bn, q, bq, r):
    from paper_2501_03377_amd import kp_basis_1d, kp_lowrank_table
    T = kp_lowrank_table(n, bn, q, bq, r)
    ln, lq = kp_basis_1d(n, bn)[1], kp_basis_1d(q, bq)[1]
    S = ln[:, None] + lq[None, :]
    small = np.abs(S) < 1e-13
    G = np.where(small, 0.0, 1.0 / np.where(small, 1.0, S))
    X, s, Yt = np.linalg.svd(G)
    ref = (X[:, :r] * s[:r]) @ Yt[:r]
    assert T.shape == (q, n)
    assert np.abs(T.T - ref).max() <= 1e-13 * np.abs(ref).max()


def test_table_rejects_bad_input():
    from paper_2501_03377_amd import KpError, kp_lowrank_table
    for args in [(9, "D", 12, "DN", 0), (9, "D", 12, "DN", 17), (5, "D", 4, "N", 5),
                 (2, "D", 12, "DN", 1), (9, 7, 12, "DN", 1)]:
        with pytest.raises(KpError):
            kp_lowrank_table(*args)
