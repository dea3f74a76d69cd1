"""Teams of workgroups in the batched solve against the oracle.

A team splits one tile of up to 16 right-hand sides of one system over P workgroups, each owning a
slice of the rows and columns, with one reduction in device memory per iteration.  It runs the
same iteration and stop rule as a one-workgroup tile, so every right-hand side still equals the
oracle's run of Algorithm 1 from the system's Philox stream (the block products are summed in
another order: agreement to rounding, not bit for bit).
"""
import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W

from _helpers import RTOL_F64, rel, to_dev
from test_gpu_batch import close, make_batch, oracle_check, small_batch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P", [2, 5, 16])
def test_team_fixed_iterations_match_oracle(rebk, oracle_lib, P):
    """Seven small systems with 1..8 right-hand sides, every one a team of P workgroups (with P = 16
    some workgroups of the narrow systems own no column)."""
    systems = small_batch()
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, max_iter=150, team=P, want_z=True)
    assert out["status"] == "ok"
    assert np.all(out["iterations"] == 150)
    assert np.all(out["team"] == P)
    assert np.array_equal(out["tile"], np.repeat([S.B.shape[0] for S in systems], [S.B.shape[0] for S in systems]))
    oracle_check(oracle_lib, systems, out, out["iterations"])
    close(solvers, batch)


def test_team_tiles_of_sixteen(rebk, oracle_lib):
    """37 right-hand sides of one system: team tiles of 16, 16 and 5."""
    rng = np.random.default_rng(21)
    S = W.batch_system(260, 70, 70, 37, rng, row_tau=16, col_tau=4, sys_id=3)
    solvers, batch = make_batch(rebk, [S])
    out = batch.solve([to_dev(S.B)], max_iter=110, team=4, want_z=True)
    assert out["tile"].tolist() == [16] * 32 + [5] * 5
    assert np.all(out["team"] == 4)
    oracle_check(oracle_lib, [S], out, out["iterations"])
    close(solvers, batch)


def test_team_stops_on_tolerance(rebk, oracle_lib):
    systems = small_batch(seed=12)
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    XR = [to_dev(S.X_ref) for S in systems]
    tol, ce = 1e-8, 4
    out = batch.solve(B, x_ref=XR, max_iter=200000, tol=tol, check_every=ce, team=6, want_z=True)
    assert out["status"] == "ok", out["rhs_status"]
    assert np.all(out["iterations"] % ce == 0)
    assert np.all(out["rel_err"] < tol)
    for s, S in enumerate(systems):
        X = out["x"][s].cpu().numpy()
        for k in range(S.B.shape[0]):
            assert rel(X[k], S.X_ref[k]) < tol
    oracle_check(oracle_lib, systems, out, out["iterations"])
    # the tile stops at the first check where all its right-hand sides are below tol
    q = 0
    for S in systems:
        K = int(out["iterations"][q])
        if K > ce:
            errs = [rel(oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, 0, S.B[k], max_iter=K - ce,
                                              sys=S.sys_id, trace=False)["x"], S.X_ref[k])
                    for k in range(S.B.shape[0])]
            assert max(errs) >= tol * 0.999
        q += S.B.shape[0]
    close(solvers, batch)


def test_team_reports_the_final_check(rebk, oracle_lib):
    """Without a tolerance the error of the last iterate is still reported (check at max_iter)."""
    systems = small_batch(count=3, seed=18)
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    XR = [to_dev(S.X_ref) for S in systems]
    out = batch.solve(B, x_ref=XR, max_iter=77, team=3)
    assert out["status"] == "not_converged"
    q = 0
    for s, S in enumerate(systems):
        X = out["x"][s].cpu().numpy()
        for k in range(S.B.shape[0]):
            want = rel(X[k], S.X_ref[k])
            assert abs(out["rel_err"][q] - want) <= 1e-9 * max(want, 1e-300)
            q += 1
    oracle_check(oracle_lib, systems, out, out["iterations"])
    close(solvers, batch)


@pytest.mark.parametrize("panel,stored", [("f32", W.round_to_f32), ("bf16", W.round_to_bf16), ("f16", W.round_to_f16)])
def test_team_low_precision_panels(rebk, oracle_lib, panel, stored):
    systems = small_batch(count=4, seed=13)
    solvers, batch = make_batch(rebk, systems, panel=panel, stored=stored)
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, max_iter=120, team=3, want_z=True)
    oracle_check(oracle_lib, systems, out, out["iterations"], stored=stored)
    close(solvers, batch)


def test_team_starting_point(rebk, oracle_lib):
    systems = small_batch(count=3, seed=15)
    rng = np.random.default_rng(3)
    solvers, batch = make_batch(rebk, systems)
    x0 = [rng.standard_normal((S.B.shape[0], S.A.shape[0])) @ S.A for S in systems]
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, x0=[to_dev(v) for v in x0], max_iter=70, team=4)
    oracle_check(oracle_lib, systems, out, out["iterations"], x0=x0)
    close(solvers, batch)


def test_team_is_reproducible(rebk):
    """Each reduced value is summed by one workgroup in a fixed order: two runs agree bit for bit."""
    systems = small_batch(count=4, seed=19)
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    a = batch.solve(B, max_iter=95, team=7, want_z=True)
    b = batch.solve(B, max_iter=95, team=7, want_z=True)
    for xa, xb in zip(a["x"] + a["z"], b["x"] + b["z"]):
        assert bool((xa == xb).all())
    close(solvers, batch)


def test_team_chosen_automatically_for_a_heavy_system(rebk, oracle_lib):
    """One system streams far more panel per iteration than the others; after a first solve (one
    workgroup per tile) the second runs it as a team and the others as ordinary tiles."""
    rng = np.random.default_rng(22)
    big = W.batch_system(1200, 3100, 900, 16, rng, sys_id=0)
    small = [W.batch_system(m, n, n, 4, rng, row_tau=16, col_tau=4, sys_id=1 + q)
             for q, (m, n) in enumerate([(120, 40), (90, 60), (200, 30)])]
    systems = [big] + small
    solvers, batch = make_batch(rebk, systems, panel="f32", stored=W.round_to_f32)
    B = [to_dev(S.B) for S in systems]
    first = batch.solve(B, max_iter=60)
    assert np.all(first["team"] == 0)
    second = batch.solve(B, max_iter=60, want_z=True)
    assert np.all(second["team"][:16] > 0) and np.all(second["team"][16:] == 0)
    oracle_check(oracle_lib, systems, second, second["iterations"], stored=W.round_to_f32)
    off = batch.solve(B, max_iter=60, team=-1)
    assert np.all(off["team"] == 0)
    close(solvers, batch)


def test_team_workload_shapes(rebk, oracle_lib):
    """Systems of the batched workload (16 right-hand sides, blocks 64 x 16, FP32 panels) including
    the slowest-converging one, as teams of 64 workgroups, 30 iterations against the oracle."""
    rng = np.random.default_rng(1004)
    shapes = W.batch_shapes(256, rng)
    pick = [215, 155, 0]
    systems = [W.batch_system(m, n, rk, 16, np.random.default_rng([1004, q]), sys_id=q)
               for q, (m, n, rk) in [(q, shapes[q]) for q in pick]]
    solvers, batch = make_batch(rebk, systems, panel="f32", stored=W.round_to_f32)
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, max_iter=30, team=64, want_z=True)
    assert np.all(out["team"] == 64)
    oracle_check(oracle_lib, systems, out, out["iterations"], stored=W.round_to_f32)
    close(solvers, batch)


def test_team_invalid_arguments(rebk):
    systems = small_batch(count=2, seed=17)
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    with pytest.raises(rebk.RebkError):
        batch.solve(B, max_iter=10, team=257)                                  # more than 256 workgroups
    with pytest.raises(rebk.RebkError):
        batch.solve(B, x0=[to_dev(np.zeros((S.B.shape[0], S.A.shape[1]))) for S in systems], max_iter=10,
                    team=2, z0_from_x0=True)                                   # teams start from z0 = b
    out = batch.solve(B, max_iter=10)                                          # the batch still works
    assert out["status"] == "ok"
    close(solvers, batch)
