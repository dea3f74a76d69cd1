"""Pins of the oracle's block constants beta = ||B||_2^2 / ||B||_F^2 (Section 2.2, Remark 9)."""
import numpy as np

from paper_2001_04179_amd import workloads as W


def test_closed_forms(oracle_lib):
    rng = np.random.default_rng(0)
    # rank-1 row blocks: ||B||_2 = ||B||_F, beta = 1
    u = rng.standard_normal((12, 1))
    v = rng.standard_normal((1, 9))
    br, bc = oracle_lib.block_betas(u @ v, [0, 4, 12], [0, 3, 9])
    assert np.allclose(br, 1.0, rtol=1e-12) and np.allclose(bc, 1.0, rtol=1e-12)
    # a block with orthogonal rows of equal norm: all singular values equal, beta = 1 / rows
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    A = 3.0 * Q[:, :30]
    br, _ = oracle_lib.block_betas(A, [0, 5, 30], [0, 30])
    assert np.allclose(br, [1 / 5, 1 / 25], rtol=1e-12)
    # B = Q diag(d): beta = max d^2 / sum d^2
    d = np.array([1.0, 2.0, 3.0, 0.5])
    B = Q[:, :4] * d
    _, bc = oracle_lib.block_betas(B, [0, 30], [0, 4])
    assert np.isclose(bc[0], 9.0 / np.sum(d * d), rtol=1e-12)


def test_bounds_of_remark_9(oracle_lib):
    """max 1/|block| <= beta <= 1 for every block (Remark 9), and the SVD gives the same value."""
    S = W.type2(90, 40, rng_seed=4, row_tau=7, col_tau=6)
    br, bc = oracle_lib.block_betas(S.A, S.row_off, S.col_off)
    sizes_r = np.diff(S.row_off)
    sizes_c = np.diff(S.col_off)
    assert np.all(br >= 1.0 / sizes_r - 1e-15) and np.all(br <= 1.0)
    assert np.all(bc >= 1.0 / sizes_c - 1e-15) and np.all(bc <= 1.0)
    for i in range(len(br)):
        B = S.A[S.row_off[i]:S.row_off[i + 1]]
        sv = np.linalg.svd(B, compute_uv=False)
        assert np.isclose(br[i], sv[0] ** 2 / np.sum(sv ** 2), rtol=1e-12)
    assert np.isclose(max(br.max(), bc.max()), 1.0 / S.alpha, rtol=1e-12)
