"""The input generators: shapes, the inconsistency r in null(A^T), A^+ b by projection, beta bounds."""
import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W


def test_contiguous_offsets_last_block_smaller():
    assert W.contiguous_offsets(23, 10).tolist() == [0, 10, 20, 23]
    assert W.contiguous_offsets(20, 10).tolist() == [0, 10, 20]


@pytest.mark.parametrize("make", [
    lambda: W.type2(60, 25, rng_seed=1, noise=0.1, row_tau=7, col_tau=4),
    lambda: W.type2(25, 60, rng_seed=2, noise=0.1, row_tau=7, col_tau=4),
    lambda: W.type1(50, 30, 12, 5.0, rng_seed=3, noise=0.2, row_tau=9, col_tau=5),
    lambda: W.factor_product(70, 40, 15, rng_seed=4, noise=0.1, row_tau=10, col_tau=8, fro2_target=70.0),
])
def test_reference_solution_is_pinv_b(make):
    S = make()
    assert np.linalg.norm(S.x_ref - np.linalg.pinv(S.A) @ S.b) <= 1e-10 * np.linalg.norm(S.x_ref)
    r = S.b - S.A @ S.x_star
    assert np.linalg.norm(S.A.T @ r) <= 1e-10 * np.linalg.norm(S.A) * max(np.linalg.norm(r), 1.0)


def test_noise_ratio_and_normalisation():
    S = W.factor_product(300, 80, 30, rng_seed=5, noise=0.1, row_tau=20, col_tau=8, fro2_target=300.0)
    r = S.b - S.A @ S.x_star
    np.testing.assert_allclose(np.linalg.norm(r), 0.1 * np.linalg.norm(S.A @ S.x_star), rtol=1e-12)
    np.testing.assert_allclose(np.sum(S.A * S.A), 300.0, rtol=1e-12)


def test_beta_bounds():
    """Remark 9: max 1/|block| <= beta_max <= 1 (per row and per column partition)."""
    for seed in range(3):
        S = W.type2(120, 50, rng_seed=seed, row_tau=11, col_tau=6)
        nI = np.diff(S.row_off)
        nJ = np.diff(S.col_off)
        assert (1.0 / nI).max() <= S.beta_row + 1e-15 and S.beta_row <= 1.0 + 1e-15
        assert (1.0 / nJ).max() <= S.beta_col + 1e-15 and S.beta_col <= 1.0 + 1e-15
        assert S.alpha == pytest.approx(1.0 / max(S.beta_row, S.beta_col))


def test_low_precision_rounding_matches_torch():
    import torch
    x = np.random.default_rng(6).standard_normal(10000) * 3.0
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    # float32 first is exact-enough here only where no double rounding occurs; compare on values
    # already representable in float32
    x32 = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(W.round_to_bf16(x32), ref)
    assert np.array_equal(W.round_to_f16(x), x.astype(np.float16).astype(np.float64))


def test_benchmark_configs_shapes():
    S = W.dense_gaussian_1000x100()
    assert S.A.shape == (1000, 100) and len(S.row_off) == 11 and len(S.col_off) == 11 and S.seed == 0
    S = W.rank1500_20000x2000(scale=10)
    assert S.A.shape == (2000, 200)
    assert np.linalg.matrix_rank(S.A) == 150
