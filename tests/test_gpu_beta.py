"""GPU block constants (Gram matrices + power iteration) against the oracle's eigen-solves."""
import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W

from _helpers import to_dev

pytestmark = pytest.mark.gpu

STORE = {"f64": lambda A: A, "f32": W.round_to_f32, "bf16": W.round_to_bf16}

CASES = {
    "type2_ragged": lambda: W.type2(203, 77, rng_seed=5, row_tau=16, col_tau=10),
    "type1": lambda: W.type1(160, 120, 40, 3.0, rng_seed=6, row_tau=20, col_tau=12),
    "wide_blocks": lambda: W.type2(64, 600, rng_seed=7, row_tau=32, col_tau=150),
    "factor": lambda: W.factor_product(300, 90, 30, rng_seed=8, row_tau=25, col_tau=9),
}


@pytest.mark.parametrize("panel", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_block_betas_match_oracle(rebk, oracle_lib, name, panel):
    S = CASES[name]()
    Ast = STORE[panel](S.A)
    sv = rebk.Solver(to_dev(Ast), S.row_off, S.col_off, S.alpha, 0, panel_dtype=panel)
    br, bc, bmax, steps = sv.block_betas(max_steps=20000, rtol=1e-14)
    ref_r, ref_c = oracle_lib.block_betas(Ast, S.row_off, S.col_off)
    assert steps < 20000
    assert np.allclose(br, ref_r, rtol=1e-8, atol=0)
    assert np.allclose(bc, ref_c, rtol=1e-8, atol=0)
    # the Rayleigh quotient never exceeds the largest eigenvalue
    assert np.all(br <= ref_r * (1 + 1e-12)) and np.all(bc <= ref_c * (1 + 1e-12))
    assert np.isclose(bmax, max(ref_r.max(), ref_c.max()), rtol=1e-8)
    assert np.isclose(sv.suggest_alpha(1.75), 1.75 / bmax, rtol=1e-8)
    sv.close()


def test_block_betas_rank_one_and_invalid(rebk):
    rng = np.random.default_rng(1)
    A = np.outer(rng.standard_normal(40), rng.standard_normal(24))
    sv = rebk.Solver(to_dev(A), [0, 10, 40], [0, 8, 24], 1.0, 0)
    br, bc, bmax, _ = sv.block_betas()
    assert np.allclose(br, 1.0, rtol=1e-12) and np.allclose(bc, 1.0, rtol=1e-12)
    with pytest.raises(rebk.RebkError):
        sv.block_betas(max_steps=0)
    sv.close()


def test_block_betas_benchmark_system(rebk, oracle_lib):
    """The 20000 x 2000 rank-1500 system: beta_max agrees with the LAPACK value used for alpha."""
    S = W.rank1500_20000x2000(scale=4)
    sv = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, 0)
    _, _, bmax, steps = sv.block_betas(max_steps=20000, rtol=1e-14)
    assert np.isclose(bmax, 1.0 / S.alpha, rtol=1e-7), (bmax, 1 / S.alpha, steps)
    sv.close()
