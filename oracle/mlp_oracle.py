"""FP64 CPU oracle of the learned warm start (TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may use this
module; it shares no code with the GPU library.

The warm start feeds REBK (Du, Si, Sun, arXiv:2001.04179, Algorithm 1) a starting point
x0 = A^T y in range(A^T) -- the hypothesis of Theorem 7 -- with y produced from b by a small
network, and z0 = b - A x0 (in b + range(A), the other hypothesis).  The network and its
training objective are defined here in plain numpy:

  h1 = relu(W1 b + c1),  h2 = relu(W2 h1 + c2),  y = W3 h2 + c3,  x0 = out_scale A^T y
  loss = 1 / (2 batch) * sum over the batch of ||x0 - x_target||^2
(out_scale a fixed constant, 1/sqrt(m) by default, so that y is of order one)

At inference (``infer``) y is left unrounded and x0 = out_scale A^T y is formed from the FP64 A,
so that x0 lies in range(A^T) to FP64 rounding.

The backward pass of that composition and the Adam update (Kingma and Ba, ICLR 2015):
  m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
  p -= lr * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).

Batches are rows: B is batch x in_dim, Y batch x out_dim, X batch x n.  Weights are row-major
(W1: hidden x in_dim, W2: hidden x hidden, W3: out_dim x hidden).

``round16=True`` rounds to IEEE half precision at the points where the GPU stores half
precision (the inputs, the weight copies, A, the activations h1, h2, y, the scaled residual and
the back-propagated signals), with every product and sum still in FP64: the GPU, which
accumulates in FP32, must then agree to FP32 rounding.  The residual is scaled by a power of two
s (chosen from its largest magnitude, as on the GPU) before that rounding, and the gradients
divided by s afterwards; without rounding the scaling changes nothing.
"""
from __future__ import annotations

import numpy as np

PARAMS = ("W1", "c1", "W2", "c2", "W3", "c3")


def to_half(a):
    """Round to IEEE binary16 (round to nearest even), returned as FP64."""
    return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def residual_scale(R, target_log2=3):
    """Power of two s with max|s R| in [2^(target-1), 2^target] (1 if R = 0)."""
    mx = float(np.max(np.abs(R))) if R.size else 0.0
    if not (mx > 0.0) or not np.isfinite(mx):
        return 1.0
    e = int(np.ceil(np.log2(mx)))
    return float(2.0 ** (target_log2 - e))


def forward(params, B, A, round16=False, out_scale=1.0):
    """Activations of the network for the batch B (rows) and x0 = out_scale A^T y (rows of Y A)."""
    r = to_half if round16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, c1, W2, c2, W3, c3 = (np.asarray(params[k], dtype=np.float64) for k in PARAMS)
    Bq = r(B)
    h1 = r(np.maximum(Bq @ r(W1).T + c1, 0.0))
    h2 = r(np.maximum(h1 @ r(W2).T + c2, 0.0))
    y = h2 @ r(W3).T + c3
    yq = r(y)
    x0 = out_scale * (yq @ r(A))
    return {"B": Bq, "h1": h1, "h2": h2, "y": y, "yq": yq, "x0": x0}


def infer(params, B, A, out_scale=1.0):
    """Inference start point: the network in half-precision storage as in ``forward(round16=True)``,
    but y kept unrounded and x0 = out_scale A^T y formed from the unrounded FP64 A.  A product with
    a rounded A would leave x0 slightly outside range(A^T), a component the x-steps of REBK never
    remove (they only add rows of A); Theorem 7 needs x0 in range(A^T)."""
    f = forward(params, B, A, round16=True, out_scale=out_scale)
    y = f["y"]
    return {"y": y, "x0": x0_of_y(y, A, out_scale)}


def x0_of_y(Y, A, out_scale=1.0):
    """Rows x0 = out_scale A^T y for the rows y of Y, in FP64 (A: m x n, Y: batch x m)."""
    return out_scale * (np.asarray(Y, dtype=np.float64) @ np.asarray(A, dtype=np.float64))


def loss_and_grads(params, B, A, Xt, round16=False, out_scale=1.0):
    """Loss and gradients of every parameter (FP64; see the module header for round16)."""
    r = to_half if round16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, c1, W2, c2, W3, c3 = (np.asarray(params[k], dtype=np.float64) for k in PARAMS)
    f = forward(params, B, A, round16, out_scale)
    batch = B.shape[0]
    R = f["x0"] - Xt
    loss = float(np.sum(R * R)) / (2.0 * batch)
    s = residual_scale(R) if round16 else 1.0
    Aq = r(A)
    dY = r((r(s * R)) @ Aq.T)                       # s * dL/dy * batch / out_scale
    gW3 = dY.T @ f["h2"]
    gc3 = dY.sum(axis=0)
    dH2 = r((dY @ r(W3)) * (f["h2"] > 0))
    gW2 = dH2.T @ f["h1"]
    gc2 = dH2.sum(axis=0)
    dH1 = r((dH2 @ r(W2)) * (f["h1"] > 0))
    gW1 = dH1.T @ f["B"]
    gc1 = dH1.sum(axis=0)
    k = out_scale / (s * batch)
    grads = {"W1": gW1 * k, "c1": gc1 * k, "W2": gW2 * k, "c2": gc2 * k, "W3": gW3 * k, "c3": gc3 * k}
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of every parameter; state holds m, v (dicts) and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for k in PARAMS:
        g = np.asarray(grads[k], dtype=np.float64)
        m = beta1 * state.setdefault("m", {}).get(k, np.zeros_like(g)) + (1.0 - beta1) * g
        v = beta2 * state.setdefault("v", {}).get(k, np.zeros_like(g)) + (1.0 - beta2) * g * g
        state["m"][k], state["v"][k] = m, v
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        out[k] = np.asarray(params[k], dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return out


def init_params(in_dim, hidden, out_dim, rng):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (for tests)."""
    def u(o, i):
        b = 1.0 / np.sqrt(i)
        return rng.uniform(-b, b, size=(o, i))
    return {"W1": u(hidden, in_dim), "c1": np.zeros(hidden), "W2": u(hidden, hidden), "c2": np.zeros(hidden),
            "W3": u(out_dim, hidden), "c3": np.zeros(out_dim)}
