"""The pipelined whole-chip kernel (REBK_KERNEL_PIPE) through the C ABI.

Its iterates are those of Algorithm 1 (Section 2); it forms the block products of the next steps
from x and z two and three iterations old and corrects them with the Gram matrices A A^T and
A^T A, so only the order of the sums differs from the oracle's.  The shared parity cases run it
through tests/test_gpu_parity.py; here: grid sizes, several launches, preparation and release of
the Gram matrices, the error paths, and agreement with the grid kernel at the benchmark's size.
"""
import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W
from tests._helpers import RTOL_F64, gpu_vs_oracle, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg1():
    return W.dense_gaussian_1000x100()


@pytest.mark.parametrize("grid_wgs", [128, 200, 256])
def test_pipe_grid_sizes(rebk, oracle_lib, cfg1, grid_wgs):
    """As many workgroups as broadcast entries (128: every workgroup owns one), an uneven count, and
    more workgroups than entries (those own no entry but still add their partial sums)."""
    print(f"case pipe dense 1000x100 grid_wgs={grid_wgs}", flush=True)
    gpu_vs_oracle(rebk, oracle_lib, cfg1, kernel="pipe", grid_wgs=grid_wgs, max_iter=400)


def test_pipe_grid_beyond_compute_units(rebk, oracle_lib, cfg1):
    """512 workgroups, two per compute unit: either all fit at once and the solve matches the
    oracle (workgroups past the 128 broadcast entries own none), or the launch is refused before
    it starts because they cannot be co-resident (it depends on the kernel's register count)."""
    S = cfg1
    try:
        gpu_vs_oracle(rebk, oracle_lib, S, kernel="pipe", grid_wgs=512, max_iter=300)
    except rebk.RebkError as e:
        assert "co-resident" in str(e)


@pytest.mark.parametrize("panel", ["f32", "bf16", "f16"])
def test_pipe_ragged_low_precision(rebk, oracle_lib, panel):
    """Ragged blocks on 2-byte and 4-byte panels: the Gram matrices are formed from the stored
    values, so the oracle on those values agrees to FP64 rounding."""
    S = W.type2(517, 203, rng_seed=21, noise=0.2, row_tau=50, col_tau=16, alpha_c=1.0, seed=5)
    rnd = {"f32": W.round_to_f32, "bf16": W.round_to_bf16, "f16": W.round_to_f16}[panel]
    print(f"case pipe ragged 517x203 panel={panel}", flush=True)
    gpu_vs_oracle(rebk, oracle_lib, S, kernel="pipe", max_iter=700, panel=panel, A_stored=rnd(S.A))


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_pipe_few_iterations(rebk, oracle_lib, cfg1, K):
    """Runs shorter than the pipeline's depth, with and without a reference (the error of x^K
    then comes three broadcasts after the last step)."""
    S = cfg1
    print(f"case pipe K={K}", flush=True)
    gpu_vs_oracle(rebk, oracle_lib, S, kernel="pipe", max_iter=K)
    out, _ = gpu_vs_oracle(rebk, oracle_lib, S, kernel="pipe", max_iter=K, tol=1e-30)
    r = out["result"]
    assert r.iterations == K and r.status == "not_converged"
    assert abs(r.rel_err - rel(out["x"].cpu().numpy(), S.x_ref)) <= 1e-12


@pytest.mark.parametrize("check_every", [1, 7, 64])
def test_pipe_stop_rule_matches_grid(rebk, cfg1, check_every):
    """The error check every check_every iterations stops where the grid kernel stops, with the
    same returned x (the state of the checked iteration, not a later one)."""
    S = cfg1
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, S.seed)
    res = {}
    for kernel in ("grid", "pipe"):
        out = solver.solve_ex(to_dev(S.b), max_iter=5000, x_ref=to_dev(S.x_ref), tol=1e-6,
                              check_every=check_every, kernel=kernel)
        res[kernel] = out
    solver.close()
    g, p = res["grid"], res["pipe"]
    assert p["result"].status == "ok" and p["result"].kernel == "pipe"
    assert p["result"].iterations == g["result"].iterations
    assert p["result"].iterations % check_every == 0
    assert rel(p["x"].cpu().numpy(), g["x"].cpu().numpy()) <= RTOL_F64
    assert rel(p["z"].cpu().numpy(), g["z"].cpu().numpy()) <= RTOL_F64
    assert abs(p["result"].rel_err - g["result"].rel_err) <= 1e-9 * g["result"].rel_err


def test_pipe_resume_and_residual_mode(rebk, oracle_lib):
    """Several launches: an exact resume at k0 and the residual stop rule (chunks of launches
    that start from the previous x and z)."""
    S = W.type2(300, 80, rng_seed=21, noise=0.3, row_tau=30, col_tau=8, seed=4)
    first, _ = gpu_vs_oracle(rebk, oracle_lib, S, kernel="pipe", max_iter=150)
    second, _ = gpu_vs_oracle(rebk, oracle_lib, S, kernel="pipe", max_iter=250, x0=first["x"].cpu().numpy(),
                              z0=first["z"].cpu().numpy(), k0=150)
    whole = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, S.seed, S.b, max_iter=400)
    assert rel(second["x"].cpu().numpy(), whole["x"]) <= RTOL_F64
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, S.seed)
    out = solver.solve_ex(to_dev(S.b), max_iter=20000, tol=1e-9, check_every=100, kernel="pipe")
    solver.close()
    r = out["result"]
    assert r.status == "ok" and r.iterations % 100 == 0
    ref = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, S.seed, S.b, max_iter=r.iterations)
    assert rel(out["x"].cpu().numpy(), ref["x"]) <= RTOL_F64


def test_pipe_prepare_and_release(rebk, cfg1):
    """rebk_pipe_prepare builds the Gram matrices once; after rebk_pipe_release a solve builds them
    again and gives the same iterates."""
    S = cfg1
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, S.seed)
    assert solver.pipe_prepare() > 0.0
    assert solver.pipe_prepare() == 0.0
    a = solver.solve_ex(to_dev(S.b), max_iter=500, kernel="pipe")["x"].cpu().numpy()
    solver.pipe_release()
    b = solver.solve_ex(to_dev(S.b), max_iter=500, kernel="pipe")["x"].cpu().numpy()
    assert solver.pipe_prepare() == 0.0
    solver.close()
    assert np.array_equal(a, b)


def test_auto_picks_pipe_once_prepared(rebk, oracle_lib, cfg1):
    """AUTO runs the grid kernel until the Gram matrices exist, the pipelined kernel after
    rebk_pipe_prepare (same iterates), and the grid kernel again after rebk_pipe_release; all with
    FP32 panels.  With FP64 panels AUTO stays on the grid kernel (faster there), while an explicit
    pipelined request still runs it."""
    S = cfg1
    A32 = W.round_to_f32(S.A)
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, S.seed, panel_dtype="f32")
    a = solver.solve_ex(to_dev(S.b), max_iter=300)
    assert a["result"].kernel == "grid"
    solver.pipe_prepare()
    b = solver.solve_ex(to_dev(S.b), max_iter=300)
    assert b["result"].kernel == "pipe"
    # the refinement's inner solves stay on the grid kernel
    r = solver.solve_refined(to_dev(S.A), to_dev(S.b), x_ref=to_dev(S.x_ref), tol=1e-9, inner_iters=200)
    assert r["result"].kernel == "grid" and r["result"].status == "ok"
    solver.pipe_release()
    c = solver.solve_ex(to_dev(S.b), max_iter=300)
    solver.close()
    assert c["result"].kernel == "grid"
    ref = oracle_lib.rebk_solve(A32, S.row_off, S.col_off, S.alpha, S.seed, S.b, max_iter=300)
    for o in (a, b, c):
        assert rel(o["x"].cpu().numpy(), ref["x"]) <= RTOL_F64
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, S.seed)
    solver.pipe_prepare()
    d = solver.solve_ex(to_dev(S.b), max_iter=300)
    e = solver.solve_ex(to_dev(S.b), max_iter=300, kernel="pipe")
    solver.close()
    assert d["result"].kernel == "grid" and e["result"].kernel == "pipe"
    ref = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, S.seed, S.b, max_iter=300)
    for o in (d, e):
        assert rel(o["x"].cpu().numpy(), ref["x"]) <= RTOL_F64


def test_pipe_rejections(rebk, cfg1):
    """What the pipelined kernel does not run is an error, never a silent fallback."""
    S = cfg1
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, S.seed)
    # 128 broadcast entries (100 + 10 + 1, rounded up) need at least 128 workgroups
    with pytest.raises(rebk.RebkError, match="invalid"):
        solver.solve_ex(to_dev(S.b), max_iter=10, kernel="pipe", grid_wgs=64)
    # the static workspace runs the workgroup and grid kernels only
    with pytest.raises(rebk.RebkError, match="invalid"):
        solver.solve_ex(to_dev(S.b), max_iter=10, x_ref=to_dev(S.x_ref), kernel="pipe", static_workspace=True)
    # no refinement steps
    with pytest.raises(rebk.RebkError, match="invalid"):
        solver.solve_refined(to_dev(S.A), to_dev(S.b), x_ref=to_dev(S.x_ref), tol=1e-8, kernel="pipe")
    solver.close()
    # blocks of 300 rows: more broadcast entries than the 256 workgroups
    A = np.random.default_rng(3).standard_normal((600, 40))
    T = W.general(A, rng_seed=4, noise=0.1, row_tau=300, col_tau=10, seed=1)
    solver = rebk.Solver(to_dev(T.A), T.row_off, T.col_off, T.alpha, T.seed)
    with pytest.raises(rebk.RebkError, match="invalid"):
        solver.solve_ex(to_dev(T.b), max_iter=10, kernel="pipe")
    solver.close()


def test_pipe_agrees_with_grid_20000x2000(rebk):
    """The benchmark's system and launch (FP32 panels, one workgroup per compute unit): 3000
    iterations of the pipelined and the grid kernel give the same x and z to FP64 rounding."""
    S = W.rank1500_20000x2000()
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, S.seed, panel_dtype="f32")
    print("case pipe vs grid 20000x2000 f32", flush=True)
    g = solver.solve_ex(to_dev(S.b), max_iter=3000, kernel="grid")
    p = solver.solve_ex(to_dev(S.b), max_iter=3000, kernel="pipe")
    solver.close()
    assert p["result"].kernel == "pipe"
    assert rel(p["x"].cpu().numpy(), g["x"].cpu().numpy()) <= RTOL_F64
    assert rel(p["z"].cpu().numpy(), g["z"].cpu().numpy()) <= RTOL_F64
