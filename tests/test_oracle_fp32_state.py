"""Why the iterates stay in FP64: the all-FP32 form of Algorithm 1 stalls above 1e-6.

On the 20000 x 2000 rank-1500 workload scaled down tenfold in every dimension (2000 x 200, rank
150, 200-row / 20-column blocks), REBK with FP64 iterates on the FP32 values of A reaches relative
error 1e-6 against A^+ b; the same iteration with every vector and operation in FP32 (same blocks,
same stepsize) bottoms out several times above 1e-6 and then drifts upward, because rounding
errors outside range(A^T) are never removed by the x-steps (Theorem 7's hypothesis on x).
"""
import numpy as np

import oracle
from paper_2001_04179_amd import workloads as W


def test_all_fp32_iteration_stalls_above_1e6():
    S = W.rank1500_20000x2000(scale=10)
    A32 = W.round_to_f32(S.A)
    ref = oracle.rebk_solve(A32, S.row_off, S.col_off, S.alpha, S.seed, S.b, max_iter=60000, x_ref=S.x_ref,
                            tol=1e-6, trace=False)
    assert ref["status"] == 0 and ref["err"] < 1e-6          # FP64 iterates reach the tolerance
    k = ref["iterations"]
    f32 = oracle.rebk_f32state(S.A, S.row_off, S.col_off, S.alpha, S.seed, S.b, S.x_ref, max_iter=2 * k,
                               every=500)
    err = f32["err"]
    assert err.min() > 2e-6                                  # the FP32 form never gets there
    assert err[-1] > 1.5 * err.min()                         # and drifts away from its best
