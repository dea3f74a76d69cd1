"""Pins of the oracle's random block draw: Philox4x64-10 against NumPy's implementation, the
integer-threshold sampler against the probability law of Algorithm 1, and the block weights
against exact sums."""
import numpy as np
import pytest
from scipy import stats


def test_philox_matches_numpy(oracle_lib):
    """Salmon et al. (SC'11) Philox4x64-10; NumPy's generator advances the counter by one before
    producing each block of four words, so counter c yields NumPy's output for counter c - 1."""
    rng = np.random.default_rng(0)
    for _ in range(300):
        ctr = [int(v) for v in rng.integers(0, 2**64, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**64, size=2, dtype=np.uint64)]
        ctr[0] = max(ctr[0], 1)
        prev = [ctr[0] - 1] + ctr[1:]
        ref = np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array(key, dtype=np.uint64)).random_raw(4)
        assert np.array_equal(oracle_lib.philox4x64_10(ctr, key), ref)


def test_philox_fill_matches_numpy_stream(oracle_lib):
    bg = np.random.Philox(counter=[9, 1, 2, 3], key=[7, 8])
    ref = bg.random_raw(4 * 5000).reshape(5000, 4)
    assert np.array_equal(oracle_lib.philox_fill([10, 1, 2, 3], [7, 8], 5000), ref)


def test_philox_counter_wraps(oracle_lib):
    words = oracle_lib.philox_fill([2**64 - 2, 5, 0, 0], [3, 0], 4)
    assert np.array_equal(words[2], oracle_lib.philox4x64_10([0, 5, 0, 0], [3, 0]))


def test_block_weights_exact_on_integers(oracle_lib):
    """Integer entries make every partial sum exact, so any summation order gives the same bits."""
    rng = np.random.default_rng(1)
    A = rng.integers(-50, 51, size=(37, 23)).astype(np.float64)
    ro = [0, 10, 20, 30, 37]
    co = [0, 5, 6, 20, 23]
    w_row, w_col = oracle_lib.block_weights(A, ro, co)
    exp_row = [np.sum(A[ro[i]:ro[i + 1]] ** 2) for i in range(4)]
    exp_col = [np.sum(A[:, co[j]:co[j + 1]] ** 2) for j in range(4)]
    assert np.array_equal(w_row, exp_row) and np.array_equal(w_col, exp_col)


def test_block_weights_close_on_floats(oracle_lib):
    rng = np.random.default_rng(2)
    A = rng.standard_normal((200, 90))
    ro = list(range(0, 200, 30)) + [200]
    co = list(range(0, 90, 7)) + [90]
    w_row, w_col = oracle_lib.block_weights(A, ro, co)
    exp_row = np.array([np.sum(A[ro[i]:ro[i + 1]] ** 2) for i in range(len(ro) - 1)])
    exp_col = np.array([np.sum(A[:, co[j]:co[j + 1]] ** 2) for j in range(len(co) - 1)])
    np.testing.assert_allclose(w_row, exp_row, rtol=1e-13)
    np.testing.assert_allclose(w_col, exp_col, rtol=1e-13)
    # both partitions cover ||A||_F^2
    np.testing.assert_allclose(w_row.sum(), w_col.sum(), rtol=1e-13)


def test_thresholds_shape(oracle_lib):
    w = np.array([0.5, 0.0, 2.0, 1e-300, 3.5, 0.0])
    T = oracle_lib.thresholds(w)
    assert T[-1] == 2**53
    assert np.all(np.diff(T.astype(np.int64)) >= 0)
    total = w.sum()
    widths = np.diff(np.concatenate([[0], T.astype(np.float64)]))
    assert np.all(np.abs(widths - w / total * 2.0**53) <= 1.0)
    assert widths[1] == 0 and widths[5] == 0


def test_thresholds_reject_bad_weights(oracle_lib):
    for w in ([0.0, 0.0], [1.0, -1.0], [1.0, np.nan], [np.inf, 1.0]):
        with pytest.raises(ValueError):
            oracle_lib.thresholds(np.array(w))


def test_pick_boundaries(oracle_lib):
    """Block j is drawn exactly when T_{j-1} <= d < T_j, d = word >> 11 (strict upper bound)."""
    T = oracle_lib.thresholds(np.array([1.0, 2.0, 0.0, 1.0]))
    for j in range(len(T)):
        lo = 0 if j == 0 else int(T[j - 1])
        hi = int(T[j])
        if hi == lo:  # an empty interval is never drawn
            continue
        assert oracle_lib.pick(T, lo << 11) == j
        assert oracle_lib.pick(T, ((hi - 1) << 11) | 0x7FF) == j
    assert oracle_lib.pick(T, 0) == 0
    assert oracle_lib.pick(T, 2**64 - 1) == 3


def test_sampling_law_chi_square(oracle_lib):
    """10^6 draws: frequencies match w_j / sum(w) (Algorithm 1) for the column and the row draw."""
    w_col = np.array([1.0, 4.0, 0.0, 2.5, 0.5, 7.0])
    w_row = np.array([3.0, 1.0, 1.0, 0.0, 5.0])
    n = 1_000_000
    j, i = oracle_lib.sample_blocks(w_row, w_col, seed=1234, k0=0, count=n)
    for draws, w in ((j, w_col), (i, w_row)):
        counts = np.bincount(draws, minlength=len(w))
        assert np.all(counts[w == 0] == 0)
        p = w / w.sum()
        keep = p > 0
        chi2 = np.sum((counts[keep] - n * p[keep]) ** 2 / (n * p[keep]))
        assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4


def test_column_and_row_draws_independent(oracle_lib):
    """Words 0 and 1 of one Philox output are independent: contingency test on the pair."""
    w = np.ones(4)
    j, i = oracle_lib.sample_blocks(w, w, seed=77, k0=10**9, count=200_000)
    table = np.zeros((4, 4))
    np.add.at(table, (j, i), 1)
    assert stats.chi2_contingency(table)[1] > 1e-4


def test_sample_blocks_matches_solver_trace(oracle_lib):
    from paper_2001_04179_amd import workloads as W
    S = W.type2(120, 40, rng_seed=3, row_tau=12, col_tau=5, seed=42)
    out = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, S.seed, S.b, max_iter=500)
    w_row, w_col = oracle_lib.block_weights(S.A, S.row_off, S.col_off)
    j, i = oracle_lib.sample_blocks(w_row, w_col, S.seed, 0, 500)
    assert np.array_equal(out["j"], j) and np.array_equal(out["i"], i)
    # k0 offsets the counter: iterations 201..500
    j2, i2 = oracle_lib.sample_blocks(w_row, w_col, S.seed, 200, 300)
    assert np.array_equal(j2, j[200:]) and np.array_equal(i2, i[200:])
