"""Pins of the oracle's iterative refinement (augmented least-squares system, Algorithm 1 as the
inner solver on rounded panel values, FP64 residuals and x-updates).

* R1  the refined iterates converge to A^+ b from an SVD pseudoinverse, to 1e-12, although the
      inner iterations run on BF16-rounded values (plain Algorithm 1 on those values stalls near
      the rounding level: the contrast shows what the outer loop adds);
* R2  x stays in range(A^T) (x = x0 + A^T y with the FP64 A), for a rank-deficient A;
* R3  z converges to (I - A A^+) b (the limit of Lemma 6);
* R4  with exact panels, one outer step from x0 = 0, z0 = b is Algorithm 1 itself: the
      correction equations are Algorithm 1's iteration written for dz = z - b (g = -A^T b, f = 0);
* R5  the residual stop rule: without a reference the loop stops once ||b - z - A x|| and
      ||A^T z|| are below tol, and they are.
"""
import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W


def pinv_solution(A, b):
    return np.linalg.pinv(A, rcond=1e-12) @ b


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = {
    "over_full_rank": lambda: W.type2(60, 20, rng_seed=1, noise=0.1, row_tau=10, col_tau=4),
    "under_full_rank": lambda: W.type2(20, 60, rng_seed=2, noise=0.1, row_tau=4, col_tau=10),
    "rank_deficient": lambda: W.factor_product(50, 40, 10, rng_seed=3, noise=0.1, row_tau=10, col_tau=8),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_r1_refined_limit_is_pinv_b(oracle_lib, name):
    S = CASES[name]()
    Ast = W.round_to_bf16(S.A)
    xp = pinv_solution(S.A, S.b)
    out = oracle_lib.rebk_refine(S.A, Ast, S.row_off, S.col_off, S.alpha, 0, S.b, x_ref=xp, tol=1e-12,
                                 inner_iters=400, max_outer=30)
    assert out["status"] == 0, out["err_trace"]
    assert rel(out["x"], xp) < 1e-12
    # the error falls across outer steps
    tr = out["err_trace"]
    assert tr[-1] < tr[0] * 1e-9
    # Algorithm 1 alone on the rounded values stops far short of A^+ b
    plain = oracle_lib.rebk_solve(Ast, S.row_off, S.col_off, S.alpha, 0, S.b, max_iter=out["iterations"], trace=False)
    assert rel(plain["x"], xp) > 1e-5


def test_r2_x_in_row_space(oracle_lib):
    S = CASES["rank_deficient"]()
    Ast = W.round_to_bf16(S.A)
    out = oracle_lib.rebk_refine(S.A, Ast, S.row_off, S.col_off, S.alpha, 0, S.b, inner_iters=200, max_outer=4)
    x = out["x"]
    U, sv, Vt = np.linalg.svd(S.A)
    r = int(np.sum(sv > sv[0] * 1e-12))
    Vr = Vt[:r].T
    assert np.linalg.norm(x - Vr @ (Vr.T @ x)) < 1e-13 * np.linalg.norm(x)
    # the rounded matrix has full rank: its row space is all of R^n, so plain Algorithm 1 on it
    # leaves a component of x outside range(A^T)
    plain = oracle_lib.rebk_solve(Ast, S.row_off, S.col_off, S.alpha, 0, S.b, max_iter=800, trace=False)
    xp = plain["x"]
    assert np.linalg.norm(xp - Vr @ (Vr.T @ xp)) > 1e-6 * np.linalg.norm(xp)


def test_r3_z_converges_to_b_perp(oracle_lib):
    S = CASES["rank_deficient"]()
    Ast = W.round_to_bf16(S.A)
    out = oracle_lib.rebk_refine(S.A, Ast, S.row_off, S.col_off, S.alpha, 0, S.b, x_ref=pinv_solution(S.A, S.b),
                                 tol=1e-12, inner_iters=400, max_outer=30)
    b_perp = S.b - S.A @ pinv_solution(S.A, S.b)
    assert np.linalg.norm(out["z"] - b_perp) < 1e-10 * np.linalg.norm(S.b)


def test_r4_first_outer_step_with_exact_panels_is_algorithm_1(oracle_lib):
    S = CASES["over_full_rank"]()
    K = 37
    out = oracle_lib.rebk_refine(S.A, S.A, S.row_off, S.col_off, S.alpha, 0, S.b, inner_iters=K, max_outer=1)
    plain = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, 0, S.b, max_iter=K, trace=False)
    assert out["iterations"] == K
    assert rel(out["x"], plain["x"]) < 1e-12
    assert rel(out["z"], plain["z"]) < 1e-12


def test_r5_residual_stop_rule(oracle_lib):
    S = CASES["under_full_rank"]()
    Ast = W.round_to_f16(S.A)
    tol = 1e-11
    out = oracle_lib.rebk_refine(S.A, Ast, S.row_off, S.col_off, S.alpha, 0, S.b, tol=tol, inner_iters=300,
                                 max_outer=40)
    assert out["status"] == 0
    f = S.b - out["z"] - S.A @ out["x"]
    g = S.A.T @ out["z"]
    bn, an = np.linalg.norm(S.b), np.linalg.norm(S.A)
    assert np.linalg.norm(f) <= tol * bn * (1 + 1e-6)
    assert np.linalg.norm(g) <= tol * an * bn * (1 + 1e-6)
    assert rel(out["x"], pinv_solution(S.A, S.b)) < 1e-9
