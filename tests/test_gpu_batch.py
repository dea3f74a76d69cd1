"""Batched solves (many systems, many right-hand sides, one launch) against the oracle.

Every right-hand side of a batch is an independent run of Algorithm 1 on its system, drawing
blocks from the Philox stream of the system's id; the oracle replays each one separately.
"""
import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W

from _helpers import RTOL_F64, rel, to_dev

pytestmark = pytest.mark.gpu


def small_batch(count=7, nrhs=(1, 3, 5, 8, 2, 7, 4), seed=11, min_aspect=2.0, row_tau=16, col_tau=4):
    rng = np.random.default_rng(seed)
    shapes = W.batch_shapes(count, rng, m_range=(40, 300), n_range=(12, 90), min_aspect=min_aspect)
    return [W.batch_system(m, n, rk, nrhs[q % len(nrhs)], rng, row_tau=row_tau, col_tau=col_tau, sys_id=q)
            for q, (m, n, rk) in enumerate(shapes)]


def make_batch(rebk, systems, panel="f64", stored=None):
    solvers = [rebk.Solver(to_dev(S.A if stored is None else stored(S.A)), S.row_off, S.col_off, S.alpha, 0,
                           panel_dtype=panel) for S in systems]
    batch = rebk.Batch(solvers, sys_ids=[S.sys_id for S in systems])
    return solvers, batch


def close(solvers, batch):
    batch.close()
    for sv in solvers:
        sv.close()


def oracle_check(oracle, systems, out, iters_per_rhs, stored=None, rtol=RTOL_F64, x0=None):
    q = 0
    for s, S in enumerate(systems):
        A = S.A if stored is None else stored(S.A)
        X = out["x"][s].cpu().numpy()
        Z = out["z"][s].cpu().numpy() if out["z"] is not None else None
        for k in range(S.B.shape[0]):
            K = int(iters_per_rhs[q])
            ref = oracle.rebk_solve(A, S.row_off, S.col_off, S.alpha, 0, S.B[k], max_iter=K, sys=S.sys_id,
                                    x0=None if x0 is None else x0[s][k], trace=False)
            assert rel(X[k], ref["x"]) <= rtol, f"system {s} rhs {k}: x differs by {rel(X[k], ref['x']):.3e}"
            if Z is not None:
                assert rel(Z[k], ref["z"]) <= rtol, f"system {s} rhs {k}: z differs by {rel(Z[k], ref['z']):.3e}"
            q += 1


@pytest.mark.parametrize("threads,max_tile", [(256, 1), (512, 2), (256, 4), (512, 4)])
def test_batch_fixed_iterations_match_oracle(rebk, oracle_lib, threads, max_tile):
    systems = small_batch()
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, max_iter=150, threads=threads, max_tile=max_tile, want_z=True)
    assert out["status"] == "ok"
    assert np.all(out["iterations"] == 150)
    assert np.all(out["tile"] <= max_tile)
    oracle_check(oracle_lib, systems, out, out["iterations"])
    close(solvers, batch)


def test_batch_narrows_tiles_after_a_solve(rebk, oracle_lib):
    """The first solve uses the widest tiles that fit (widths 4, 2 and 1 in one call, run as
    concurrent kernels); the second knows every system's iteration count, and a system whose tile
    would outlast the average load of a compute unit (7 small systems on a whole chip: the larger
    ones) gets narrower tiles.  Both match the oracle."""
    systems = small_batch()
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    first = batch.solve(B, max_iter=120, threads=512, max_tile=4, xcd_order=1)
    assert set(np.unique(first["tile"]).tolist()) == {1, 2, 4}
    oracle_check(oracle_lib, systems, first, first["iterations"])
    second = batch.solve(B, max_iter=120, threads=512, max_tile=4, xcd_order=1)
    assert np.all(second["tile"] <= first["tile"]) and np.any(second["tile"] < first["tile"])
    oracle_check(oracle_lib, systems, second, second["iterations"])
    close(solvers, batch)


def test_batch_stops_on_tolerance(rebk, oracle_lib):
    systems = small_batch(seed=12)
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    XR = [to_dev(S.X_ref) for S in systems]
    tol, ce = 1e-8, 4
    out = batch.solve(B, x_ref=XR, max_iter=200000, tol=tol, check_every=ce, want_z=True)
    assert out["status"] == "ok", out["rhs_status"]
    assert np.all(out["iterations"] % ce == 0)
    for s, S in enumerate(systems):
        X = out["x"][s].cpu().numpy()
        for k in range(S.B.shape[0]):
            assert rel(X[k], S.X_ref[k]) < tol
    assert np.all(out["rel_err"] < tol)
    oracle_check(oracle_lib, systems, out, out["iterations"])
    # the group of right-hand sides solved together stops at the first check where all are below tol:
    # ce iterations earlier at least one of them was not (oracle, same block sequence)
    q = 0
    for s, S in enumerate(systems):
        K = int(out["iterations"][q])
        tile = int(out["tile"][q])
        if K > ce:
            errs = []
            for k in range(min(tile, S.B.shape[0])):
                ref = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, 0, S.B[k], max_iter=K - ce,
                                            sys=S.sys_id, trace=False)
                errs.append(rel(ref["x"], S.X_ref[k]))
            assert max(errs) >= tol * 0.999
        q += S.B.shape[0]
    close(solvers, batch)


@pytest.mark.parametrize("panel,stored", [("f32", W.round_to_f32), ("bf16", W.round_to_bf16), ("f16", W.round_to_f16)])
def test_batch_low_precision_panels(rebk, oracle_lib, panel, stored):
    systems = small_batch(count=4, seed=13)
    solvers, batch = make_batch(rebk, systems, panel=panel, stored=stored)
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, max_iter=120, want_z=True)
    oracle_check(oracle_lib, systems, out, out["iterations"], stored=stored)
    close(solvers, batch)


def test_batch_order_does_not_change_results(rebk):
    """Task order alone leaves every result bit-identical (two fresh batches, so both solves use
    the same tile widths: a later solve may narrow tiles, which sums in another order)."""
    systems = small_batch(seed=14)
    solvers, batch = make_batch(rebk, systems)
    solvers2, batch2 = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    a = batch.solve(B, max_iter=90, xcd_order=1, max_tile=4)
    b = batch2.solve(B, max_iter=90, xcd_order=0, max_tile=4)
    assert np.array_equal(a["tile"], b["tile"])
    for xa, xb in zip(a["x"], b["x"]):
        assert bool((xa == xb).all())
    close(solvers, batch)
    close(solvers2, batch2)


def test_batch_starting_point_and_sys_ids(rebk, oracle_lib):
    systems = small_batch(count=3, seed=15)
    rng = np.random.default_rng(3)
    for q, S in enumerate(systems):
        S.sys_id = 1000 + 7 * q
    solvers, batch = make_batch(rebk, systems)
    # x0 in range(A^T), as Theorem 7 asks
    x0 = [rng.standard_normal((S.B.shape[0], S.A.shape[0])) @ S.A for S in systems]
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, x0=[to_dev(v) for v in x0], max_iter=70)
    oracle_check(oracle_lib, systems, out, out["iterations"], x0=x0)
    close(solvers, batch)


def test_batch_autotune_then_solve(rebk, oracle_lib):
    systems = small_batch(count=5, seed=16)
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    cfg = batch.autotune(B, probe_iters=16)
    assert cfg["threads"] in (256, 512, 1024) and cfg["max_tile"] in (1, 2, 4) and cfg["xcd_order"] in (0, 1)
    assert cfg["ms"] > 0
    out = batch.solve(B, max_iter=60)
    oracle_check(oracle_lib, systems, out, out["iterations"])
    close(solvers, batch)


def test_batch_invalid_arguments(rebk):
    systems = small_batch(count=2, seed=17)
    solvers, batch = make_batch(rebk, systems)
    B = [to_dev(S.B) for S in systems]
    with pytest.raises(rebk.RebkError):
        batch.solve(B, max_iter=0)
    with pytest.raises(rebk.RebkError):
        batch.solve(B, max_iter=10, tol=1e-6)          # a tolerance needs x_ref
    with pytest.raises(rebk.RebkError):
        batch.solve(B, max_iter=10, threads=384)
    with pytest.raises(rebk.RebkError):
        batch.solve(B, max_iter=10, max_tile=8)
    with pytest.raises(rebk.RebkError):
        batch.solve(B, max_iter=10, lds_budget=256)    # no system fits
    other = rebk.Solver(to_dev(systems[0].A), systems[0].row_off, systems[0].col_off, systems[0].alpha, 0,
                        panel_dtype="f32")
    with pytest.raises(rebk.RebkError):
        rebk.Batch([solvers[0], other])                # mixed panel types
    other.close()
    close(solvers, batch)


def test_batch_cfg_shapes_prefix(rebk, oracle_lib):
    """The batched workload's own shapes (m up to 8000, n up to 2000, 16 right-hand sides, blocks
    64 x 16): a few of its systems for 40 iterations, every right-hand side against the oracle."""
    rng = np.random.default_rng(1004)
    shapes = W.batch_shapes(256, rng)
    pick = [0, 1, 3, 4]  # full rank over/underdetermined and a rank-deficient one
    systems = [W.batch_system(m, n, rk, 16, np.random.default_rng([1004, q]), sys_id=q)
               for q, (m, n, rk) in [(q, shapes[q]) for q in pick]]
    solvers, batch = make_batch(rebk, systems, panel="f32", stored=W.round_to_f32)
    B = [to_dev(S.B) for S in systems]
    out = batch.solve(B, max_iter=40)
    oracle_check(oracle_lib, systems, out, out["iterations"], stored=W.round_to_f32)
    close(solvers, batch)
