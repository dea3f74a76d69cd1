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


# --- Adam over several steps, against closed forms of its moment recursions ------------------------
#
# For a gradient sequence g_1, g_2, ... the first moment is m_t = (1 - b1) sum_s b1^(t-s) g_s and the
# second v_t = (1 - b2) sum_s b2^(t-s) g_s^2.  For the sequences below those sums have closed forms,
# derived by hand, that do not restate the recursion: a wrong decay, a swapped b1/b2, a bias
# correction with the wrong power of t, or a moment that is not carried from step to step changes
# the steps these formulas predict.

def _scalar_params(value):
    return {k: np.array([value]) for k in M.PARAMS}


def _run_adam(grads_seq, lr, b1, b2, eps, p0=0.5):
    params, state, traj = _scalar_params(p0), {}, []
    for g in grads_seq:
        params = M.adam_step(params, {k: np.array([g]) for k in M.PARAMS}, state, lr, beta1=b1, beta2=b2, eps=eps)
        traj.append(float(params["W1"][0]))
    return traj


def test_m5_adam_constant_gradient():
    """Constant g: m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so every bias-corrected step is
    lr g / (|g| + eps), at every t (not only the first)."""
    lr, b1, b2, eps, g = 1e-2, 0.8, 0.95, 1e-3, -0.37
    traj = _run_adam([g] * 6, lr, b1, b2, eps)
    for t, p in enumerate(traj, start=1):
        assert abs(p - (0.5 - t * lr * g / (abs(g) + eps))) < 1e-14, t


def test_m5_adam_alternating_gradient():
    """g_t = (-1)^(t+1) c: sum_s b1^(t-s) (-1)^(s+1) = (-1)^(t+1) (1 - (-b1)^t) / (1 + b1), and the
    second moment sees the constant c^2, so the bias-corrected step is
    lr (-1)^(t+1) c (1 - b1)(1 - (-b1)^t) / ((1 + b1)(1 - b1^t)) / (|c| + eps)."""
    lr, b1, b2, eps, c = 1e-2, 0.8, 0.95, 1e-4, 0.6
    T = 5
    traj = _run_adam([(-1) ** (t + 1) * c for t in range(1, T + 1)], lr, b1, b2, eps)
    p = 0.5
    for t in range(1, T + 1):
        mh = (-1) ** (t + 1) * c * (1 - b1) * (1 - (-b1) ** t) / ((1 + b1) * (1 - b1 ** t))
        p -= lr * mh / (abs(c) + eps)
        assert abs(traj[t - 1] - p) < 1e-14, t
    # a hand value of the two-step case: with b1 = 0.8, mh_2 = -c (0.2)(0.36) / (1.8 * 0.36) = -c/9,
    # so the second step moves the parameter up by lr (c/9) / (c + eps)
    step2 = traj[1] - traj[0]
    assert abs(step2 - lr * c * (0.2 * 0.36) / (1.8 * 0.36) / (c + eps)) < 1e-15


def test_m5_adam_geometric_gradient():
    """g_t = c r^t: sum_s b^(t-s) r^s = r (r^t - b^t) / (r - b), so
    m_t = (1 - b1) c r (r^t - b1^t) / (r - b1),  v_t = (1 - b2) c^2 r^2 (r^2t - b2^t) / (r^2 - b2);
    both moments and both bias corrections enter each step with distinct b1, b2."""
    lr, b1, b2, eps, c, r = 1e-2, 0.8, 0.95, 1e-6, 1.3, 0.5
    T = 6
    traj = _run_adam([c * r ** t for t in range(1, T + 1)], lr, b1, b2, eps)
    p = 0.5
    for t in range(1, T + 1):
        m = (1 - b1) * c * r * (r ** t - b1 ** t) / (r - b1)
        v = (1 - b2) * c * c * r * r * (r ** (2 * t) - b2 ** t) / (r * r - b2)
        p -= lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        assert abs(traj[t - 1] - p) < 1e-13, t


# --- inference ------------------------------------------------------------------------------------

def test_m6_inference_start_point():
    """With W3 = 0 the output is the bias: y = c3 exactly, so with c3 = e_i the start point is
    out_scale times row i of A (a transposed or rounded A fails); x0 stays in range(A^T) for any
    parameters; and inference uses the unrounded A while training rounds it."""
    rng = np.random.default_rng(7)
    m, n = 12, 5
    A = rng.standard_normal((m, n)) * (1 + 1e-4 * rng.standard_normal((m, n)))
    params = M.init_params(16, 8, m, rng)
    params["W3"] = np.zeros_like(params["W3"])
    B = rng.standard_normal((3, 16))
    for i in (0, 7, 11):
        params["c3"] = np.eye(m)[i]
        out = M.infer(params, B, A, out_scale=0.25)
        assert np.array_equal(out["y"], np.tile(np.eye(m)[i], (3, 1)))
        assert np.array_equal(out["x0"], np.tile(0.25 * A[i], (3, 1)))
    U = rng.standard_normal((m, 3))
    A2 = U @ rng.standard_normal((3, n))
    params = M.init_params(16, 8, m, rng)
    x0 = M.infer(params, B, A2, out_scale=0.3)["x0"]
    _, _, Vt = np.linalg.svd(A2)
    V = Vt[:3].T
    assert np.linalg.norm(x0 - (x0 @ V) @ V.T) < 1e-13 * np.linalg.norm(x0)
    # training forward rounds A to half precision, inference does not
    f = M.forward(params, B, A, round16=True, out_scale=0.3)
    g = M.infer(params, B, A, out_scale=0.3)
    assert np.allclose(g["x0"], 0.3 * (g["y"] @ A), rtol=0, atol=1e-14)
    assert not np.allclose(f["x0"], g["x0"], rtol=1e-9, atol=0)
