"""Pins of the warm-start network oracle (oracle/mlp_oracle.py).

* M1  every gradient matches central finite differences of the loss (FP64, tiny network);
* M2  x0 = A^T y lies in range(A^T) for any parameters (Theorem 7's hypothesis on x0);
* M3  the first Adam step moves every parameter by lr * g / (|g| + eps) (bias corrections cancel);
* M4  with half-precision rounding the gradients stay within the rounding level of the exact ones,
      and the residual scale is a power of two that does not change the exact gradients.
"""
import numpy as np

from oracle import mlp_oracle as M


def tiny(rng, in_dim=12, hidden=6, out_dim=12, n=5, batch=7):
    A = rng.standard_normal((out_dim, n))
    params = M.init_params(in_dim, hidden, out_dim, rng)
    for k in ("c1", "c2", "c3"):
        params[k] = 0.1 * rng.standard_normal(params[k].shape)
    B = rng.standard_normal((batch, in_dim))
    Xt = rng.standard_normal((batch, n))
    return params, A, B, Xt


def test_m1_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params, A, B, Xt = tiny(rng)
    osc = 0.3
    _, g = M.loss_and_grads(params, B, A, Xt, out_scale=osc)
    h = 1e-6
    for k in M.PARAMS:
        P = params[k]
        fd = np.zeros_like(P)
        for idx in np.ndindex(P.shape):
            old = P[idx]
            P[idx] = old + h
            lp, _ = M.loss_and_grads(params, B, A, Xt, out_scale=osc)
            P[idx] = old - h
            lm, _ = M.loss_and_grads(params, B, A, Xt, out_scale=osc)
            P[idx] = old
            fd[idx] = (lp - lm) / (2 * h)
        assert np.allclose(g[k], fd, rtol=1e-5, atol=1e-8), k


def test_m2_x0_in_row_space():
    rng = np.random.default_rng(1)
    U = rng.standard_normal((12, 3))
    A = U @ rng.standard_normal((3, 5))          # rank 3
    params = M.init_params(12, 6, 12, rng)
    B = rng.standard_normal((4, 12))
    x0 = M.forward(params, B, A)["x0"]
    _, sv, Vt = np.linalg.svd(A)
    V = Vt[:3].T
    assert np.linalg.norm(x0 - (x0 @ V) @ V.T) < 1e-12 * np.linalg.norm(x0)


def test_m3_first_adam_step():
    rng = np.random.default_rng(2)
    params, A, B, Xt = tiny(rng)
    _, g = M.loss_and_grads(params, B, A, Xt)
    lr, eps = 1e-3, 1e-8
    new = M.adam_step(params, g, {}, lr, eps=eps)
    for k in M.PARAMS:
        assert np.allclose(params[k] - new[k], lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-12, atol=1e-15), k


def test_m4_half_precision_rounding_and_scale():
    rng = np.random.default_rng(3)
    params = M.init_params(64, 32, 64, rng)
    A = rng.standard_normal((64, 16))
    B = rng.standard_normal((8, 64))
    Xt = rng.standard_normal((8, 16))
    l0, g0 = M.loss_and_grads(params, B, A, Xt)
    l1, g1 = M.loss_and_grads(params, B, A, Xt, round16=True)
    assert abs(l1 - l0) < 1e-2 * l0
    for k in M.PARAMS:
        assert np.linalg.norm(g1[k] - g0[k]) < 2e-2 * np.linalg.norm(g0[k]), k
    R = rng.standard_normal((5, 3)) * 1e-3
    s = M.residual_scale(R)
    assert s == 2.0 ** round(np.log2(s)) and 4.0 <= np.max(np.abs(s * R)) <= 8.0
