"""Shared test helpers: moving inputs to the device and comparing a GPU solve with the oracle."""
from __future__ import annotations

import numpy as np

# FP64 iterates: relative difference allowed between the GPU solve and the oracle at the same
# iteration (the two sum in different orders; the block sequence is identical).
RTOL_F64 = 1e-10


def to_dev(a, dtype=None):
    import torch
    dtype = dtype or torch.float64
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gpu_vs_oracle(rebk, oracle, S, *, kernel="auto", max_iter=2000, tol=0.0, panel="f64", A_stored=None,
                  x0=None, z0=None, k0=0, check_every=1, grid_wgs=0, rtol=RTOL_F64):
    """Solve S on the GPU (with index trace) and replay the same iterations in the oracle.

    A_stored is the matrix as the panels store it (rounded for low-precision panels); the oracle
    runs on it, in FP64.  Returns (gpu_output, oracle_output)."""
    A_used = S.A if A_stored is None else A_stored
    solver = rebk.Solver(to_dev(A_used), S.row_off, S.col_off, S.alpha, S.seed, panel_dtype=panel)
    out = solver.solve_ex(to_dev(S.b), x0=None if x0 is None else to_dev(x0), z0=None if z0 is None else to_dev(z0),
                          k0=k0, max_iter=max_iter, x_ref=to_dev(S.x_ref) if tol > 0 else None, tol=tol,
                          check_every=check_every, trace=True, kernel=kernel, grid_wgs=grid_wgs)
    K = out["result"].iterations
    assert K >= 1
    ref = oracle.rebk_solve(A_used, S.row_off, S.col_off, S.alpha, S.seed, S.b, x0=x0, z0=z0, k0=k0, max_iter=K)
    j = out["j"].cpu().numpy()
    i = out["i"].cpu().numpy()
    assert np.array_equal(j, ref["j"]), "column-block sequence differs from the oracle"
    assert np.array_equal(i, ref["i"]), "row-block sequence differs from the oracle"
    x = out["x"].cpu().numpy()
    z = out["z"].cpu().numpy()
    assert rel(x, ref["x"]) <= rtol, f"x differs from the oracle by {rel(x, ref['x']):.3e}"
    assert rel(z, ref["z"]) <= rtol, f"z differs from the oracle by {rel(z, ref['z']):.3e}"
    solver.close()
    return out, ref
