"""P8: the oracle reproduces the paper's own iteration counts (Tables 1 and 2) in distribution.

The paper's MATLAB random streams cannot be reproduced, so the check is statistical: on freshly
drawn matrices of the printed shapes, the stepsize c / beta_max lands near the printed alpha and
the mean iteration count over 10 trials lands near the printed ITER (Section 3 protocol)."""
import json
import os

import numpy as np
import pytest

from paper_2001_04179_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("row", GOLDEN["rows"], ids=[r["cite"] for r in GOLDEN["rows"]])
def test_paper_iteration_counts(oracle_lib, row):
    iters, alphas = [], []
    for trial in range(10):
        if row["type"] == 1:
            S = W.type1(row["m"], row["n"], row["rank"], row["kappa"], rng_seed=500 + trial, noise=0.1,
                        row_tau=10, col_tau=10, alpha_c=row["alpha_mult"], seed=trial)
        else:
            S = W.type2(row["m"], row["n"], rng_seed=600 + trial, noise=0.1, row_tau=10, col_tau=10,
                        alpha_c=row["alpha_mult"], seed=trial)
        tol = 1e-5 / np.linalg.norm(S.x_ref)  # the paper stops on the absolute error 1e-5
        out = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, S.seed, S.b, max_iter=200000,
                                    x_ref=S.x_ref, tol=tol, trace=False)
        assert out["status"] == 0
        iters.append(out["iterations"])
        alphas.append(S.alpha)
    assert abs(np.mean(alphas) / row["alpha"] - 1.0) < 0.08, np.mean(alphas)
    assert abs(np.mean(iters) / row["iter"] - 1.0) < 0.25, np.mean(iters)
