"""FP64 refinement around REBK on rounded panels (BF16 / FP16 / FP32) against the oracle.

The GPU solve and the oracle run the same outer steps and the same inner block sequence on the
same stored panel values; x and z must agree to the FP64 parity tolerance, and the refined limit
is A^+ b from an SVD pseudoinverse.
"""
import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W

from _helpers import RTOL_F64, rel, to_dev

pytestmark = pytest.mark.gpu

STORE = {"bf16": W.round_to_bf16, "f16": W.round_to_f16, "f32": W.round_to_f32}

CASES = {
    "over": lambda: W.type2(60, 20, rng_seed=1, noise=0.1, row_tau=10, col_tau=4),
    "under": lambda: W.type2(20, 60, rng_seed=2, noise=0.1, row_tau=4, col_tau=10),
    "rank_deficient": lambda: W.factor_product(50, 40, 10, rng_seed=3, noise=0.1, row_tau=10, col_tau=8),
}


def pinv_solution(A, b):
    return np.linalg.pinv(A, rcond=1e-12) @ b


def refined_pair(rebk, oracle, S, panel, *, inner, outer, x_ref=None, tol=0.0, kernel="auto", grid_wgs=0):
    Ast = STORE[panel](S.A)
    solver = rebk.Solver(to_dev(Ast), S.row_off, S.col_off, S.alpha, 0, panel_dtype=panel)
    out = solver.solve_refined(to_dev(S.A), to_dev(S.b), x_ref=None if x_ref is None else to_dev(x_ref), tol=tol,
                               inner_iters=inner, max_outer=outer, kernel=kernel, grid_wgs=grid_wgs)
    solver.close()
    ref = oracle.rebk_refine(S.A, Ast, S.row_off, S.col_off, S.alpha, 0, S.b, x_ref=x_ref, tol=tol,
                             inner_iters=inner, max_outer=outer)
    return out, ref


@pytest.mark.parametrize("panel", ["bf16", "f16", "f32"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_refined_matches_oracle(rebk, oracle_lib, name, panel):
    S = CASES[name]()
    out, ref = refined_pair(rebk, oracle_lib, S, panel, inner=120, outer=4)
    assert out["result"].iterations == ref["iterations"] == 480
    x, z = out["x"].cpu().numpy(), out["z"].cpu().numpy()
    assert rel(x, ref["x"]) <= RTOL_F64, rel(x, ref["x"])
    assert rel(z, ref["z"]) <= RTOL_F64, rel(z, ref["z"])


@pytest.mark.parametrize("kernel,grid_wgs", [("workgroup", 0), ("grid", 8)])
@pytest.mark.parametrize("name", sorted(CASES))
def test_refined_limit_is_pinv_b(rebk, oracle_lib, name, kernel, grid_wgs):
    S = CASES[name]()
    xp = pinv_solution(S.A, S.b)
    out, ref = refined_pair(rebk, oracle_lib, S, "bf16", inner=400, outer=30, x_ref=xp, tol=1e-12, kernel=kernel,
                            grid_wgs=grid_wgs)
    r = out["result"]
    assert r.status == "ok", out["err_trace"]
    x = out["x"].cpu().numpy()
    assert rel(x, xp) < 1e-12
    # same number of outer steps as the oracle, and the same error history where it is well above
    # rounding
    assert r.iterations == ref["iterations"]
    tr, tro = out["err_trace"], ref["err_trace"]
    assert len(tr) == len(tro)
    big = tro > 1e-9
    assert np.allclose(tr[big], tro[big], rtol=1e-6)
    b_perp = S.b - S.A @ xp
    assert np.linalg.norm(out["z"].cpu().numpy() - b_perp) < 1e-10 * np.linalg.norm(S.b)


def test_refined_residual_rule(rebk, oracle_lib):
    S = CASES["under"]()
    tol = 1e-11
    out, ref = refined_pair(rebk, oracle_lib, S, "f16", inner=300, outer=40, tol=tol)
    assert out["result"].status == "ok"
    x, z = out["x"].cpu().numpy(), out["z"].cpu().numpy()
    f = S.b - z - S.A @ x
    g = S.A.T @ z
    assert np.linalg.norm(f) <= tol * np.linalg.norm(S.b) * (1 + 1e-6)
    assert np.linalg.norm(g) <= tol * np.linalg.norm(S.A) * np.linalg.norm(S.b) * (1 + 1e-6)
    assert out["result"].iterations == ref["iterations"]


def test_refined_underdetermined_rank_deficient_grid(rebk, oracle_lib):
    """The mixed-precision workload's shape, scaled down: A = U V (U 200 x 120, V 120 x 5000),
    20-row and 100-column blocks, BF16 panels on the whole-chip kernel."""
    S = W.factor_product(200, 5000, 120, rng_seed=7, noise=0.1, row_tau=10, col_tau=100)
    out, ref = refined_pair(rebk, oracle_lib, S, "bf16", inner=150, outer=3, kernel="grid")
    assert rel(out["x"].cpu().numpy(), ref["x"]) <= RTOL_F64
    assert rel(out["z"].cpu().numpy(), ref["z"]) <= RTOL_F64


def test_grid_row_slabs_from_hbm(rebk, oracle_lib):
    """FP64 panels too wide for LDS-staged row slabs (157 columns x 64 rows per workgroup, double
    buffered, exceeds 160 KB): the grid kernel reads them from the row panels instead."""
    from _helpers import gpu_vs_oracle
    S = W.type2(512, 40000, rng_seed=8, noise=0.1, row_tau=64, col_tau=16)
    gpu_vs_oracle(rebk, oracle_lib, S, kernel="grid", max_iter=60)


def test_refined_invalid(rebk):
    S = CASES["over"]()
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, 0, panel_dtype="bf16")
    with pytest.raises(rebk.RebkError):
        solver.solve_refined(to_dev(S.A), to_dev(S.b), inner_iters=0)
    with pytest.raises(rebk.RebkError):
        solver.solve_refined(to_dev(S.A), to_dev(S.b), max_outer=-1)
    with pytest.raises(ValueError):
        solver.solve_refined(to_dev(S.A.T.copy()), to_dev(S.b))
    solver.close()


@pytest.fixture(scope="module")
def cfg3():
    return W.rank1200_2000x50000()


@pytest.mark.parametrize("panel", ["bf16", "f16"])
def test_refined_2000x50000_full_shape(rebk, oracle_lib, cfg3, panel):
    """The mixed-precision workload at its real size and blocks (A = U V, 2000 x 50000, rank 1200;
    20 row blocks of 100, 500 column blocks of 100), in the benchmark's launch configuration (the
    whole-chip kernel): two outer steps of 50 inner iterations against the oracle on the same
    stored panels."""
    print(f"case 2000x50000 refined panels={panel}", flush=True)
    out, ref = refined_pair(rebk, oracle_lib, cfg3, panel, inner=50, outer=2, kernel="grid")
    assert out["result"].iterations == ref["iterations"] == 100
    assert rel(out["x"].cpu().numpy(), ref["x"]) <= RTOL_F64, rel(out["x"].cpu().numpy(), ref["x"])
    assert rel(out["z"].cpu().numpy(), ref["z"]) <= RTOL_F64, rel(out["z"].cpu().numpy(), ref["z"])
