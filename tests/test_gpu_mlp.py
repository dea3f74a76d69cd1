"""Learned warm start: the network's GPU kernels against the FP64 oracle, training, and REBK from
the network's start point against the oracle.

Forward and gradients are compared with the oracle evaluated with half-precision rounding at the
points where the GPU stores half precision; the GPU accumulates in FP32, so a value that lands
next to a half-precision rounding boundary may round the other way: the bar is a few half-precision
units (2^-11) in norm.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2001_04179_amd import workloads as W

from _helpers import RTOL_F64, rel, to_dev

pytestmark = pytest.mark.gpu

HALF_ULP = 2.0 ** -11


def setup(rebk, in_dim=128, hidden=64, m=128, n=64, batch=64, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    params = M.init_params(in_dim, hidden, m, rng)
    for k in ("c1", "c2", "c3"):
        params[k] = 0.05 * rng.standard_normal(params[k].shape)
    params = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}  # FP32-exact values
    B = rng.standard_normal((batch, in_dim))
    Xt = rng.standard_normal((batch, n))
    net = rebk.WarmStart(to_dev(A), in_dim, hidden, max_batch=batch)
    net.set_params(params)
    return net, A, params, B, Xt


def test_forward_matches_oracle(rebk):
    net, A, params, B, Xt = setup(rebk)
    X0, Y = net.forward(to_dev(B), want_y=True)
    ref = M.forward(params, B, A, round16=True, out_scale=net.out_scale)
    Yg = Y.cpu().numpy()
    assert rel(Yg, ref["y"]) < 4 * HALF_ULP
    # inference forms x0 = out_scale A^T y in FP64 from the FP64 A
    assert rel(X0.cpu().numpy(), net.out_scale * (Yg @ A)) < 1e-12
    assert rel(X0.cpu().numpy(), ref["x0"]) < 8 * HALF_ULP
    net.close()


def test_gradients_match_oracle(rebk):
    net, A, params, B, Xt = setup(rebk, seed=1)
    loss = net.grad(to_dev(B), to_dev(Xt))
    g = net.grads()
    ref_loss, ref = M.loss_and_grads(params, B, A, Xt, round16=True, out_scale=net.out_scale)
    assert abs(loss - ref_loss) < 8 * HALF_ULP * ref_loss
    for k in M.PARAMS:
        assert rel(g[k], ref[k]) < 8 * HALF_ULP, (k, rel(g[k], ref[k]))
    # and within the half-precision level of the exact FP64 gradients
    _, exact = M.loss_and_grads(params, B, A, Xt, out_scale=net.out_scale)
    for k in M.PARAMS:
        assert rel(g[k], exact[k]) < 3e-2, k
    net.close()


def test_adam_step_matches_oracle(rebk):
    net, A, params, B, Xt = setup(rebk, seed=2)
    net.grad(to_dev(B), to_dev(Xt))
    g = {k: v.astype(np.float64) for k, v in net.grads().items()}
    lr = 1e-3
    net.adam(lr)
    got = net.params()
    want = M.adam_step(params, g, {}, lr)
    for k in M.PARAMS:
        assert rel(got[k], want[k]) < 1e-6, k
    net.close()


def test_adam_several_steps_match_oracle(rebk):
    """Four Adam steps with different batches (so different gradients) and non-default decays: the
    moments carried between steps and the bias corrections at t = 2..4 are compared, not only the
    first step's lr sign(g)."""
    net, A, params, B, Xt = setup(rebk, seed=6)
    rng = np.random.default_rng(60)
    lr, b1, b2, eps = 2e-3, 0.8, 0.95, 1e-7
    state = {}
    want = {k: v.copy() for k, v in params.items()}
    for step in range(4):
        Bs = B if step == 0 else rng.standard_normal(B.shape)
        Xs = Xt if step == 0 else rng.standard_normal(Xt.shape)
        net.grad(to_dev(Bs), to_dev(Xs))
        g = {k: v.astype(np.float64) for k, v in net.grads().items()}
        net.adam(lr, b1, b2, eps)
        want = M.adam_step(want, g, state, lr, beta1=b1, beta2=b2, eps=eps)
        got = net.params()
        for k in M.PARAMS:
            assert rel(got[k], want[k]) < 1e-6, (step, k, rel(got[k], want[k]))
        # each step really moved the parameters by about lr (not a no-op)
        assert np.max(np.abs(got["W1"] - params["W1"])) > 0.5 * lr
    net.close()


def test_inference_matches_oracle(rebk):
    """rebk_mlp_forward against the oracle's inference: y within a few half-precision units, and
    x0 = out_scale A^T y formed in FP64 from the FP64 A (tight against the oracle's product of the
    GPU's y, and at the half-precision level against the oracle's own y)."""
    net, A, params, B, Xt = setup(rebk, seed=8)
    X0, Y = net.forward(to_dev(B), want_y=True)
    ref = M.infer(params, B, A, out_scale=net.out_scale)
    Yg, Xg = Y.cpu().numpy(), X0.cpu().numpy()
    assert rel(Yg, ref["y"]) < 4 * HALF_ULP
    assert rel(Xg, M.x0_of_y(Yg, A, net.out_scale)) < 1e-13
    assert rel(Xg, ref["x0"]) < 4 * HALF_ULP
    net.close()


def test_full_size_network_matches_oracle(rebk):
    """The warm-start workload's network at its real dimensions, 8192 -> 512 -> 512 -> 8192 with A
    8192 x 1024 (rank 768), one batch of 64: inference, gradients and one Adam step against the
    oracle."""
    rng = np.random.default_rng(11)
    m, n, in_dim, hidden, batch = 8192, 1024, 8192, 512, 64
    A = (rng.standard_normal((m, 768)) @ rng.standard_normal((768, n))) / np.sqrt(768)
    params = M.init_params(in_dim, hidden, m, rng)
    for k in ("c1", "c2", "c3"):
        params[k] = 0.05 * rng.standard_normal(params[k].shape)
    params = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    B = A @ rng.standard_normal((n, batch)) / np.sqrt(n)
    B = np.ascontiguousarray(B.T)
    Xt = np.ascontiguousarray((np.linalg.lstsq(A, B.T, rcond=None)[0]).T)
    net = rebk.WarmStart(to_dev(A), in_dim, hidden, max_batch=batch)
    net.set_params(params)
    X0, Y = net.forward(to_dev(B), want_y=True)
    ref = M.infer(params, B, A, out_scale=net.out_scale)
    assert rel(Y.cpu().numpy(), ref["y"]) < 4 * HALF_ULP
    assert rel(X0.cpu().numpy(), ref["x0"]) < 4 * HALF_ULP
    loss = net.grad(to_dev(B), to_dev(Xt))
    g = net.grads()
    ref_loss, rg = M.loss_and_grads(params, B, A, Xt, round16=True, out_scale=net.out_scale)
    assert abs(loss - ref_loss) < 8 * HALF_ULP * ref_loss
    for k in M.PARAMS:
        assert rel(g[k], rg[k]) < 8 * HALF_ULP, (k, rel(g[k], rg[k]))
    net.adam(1e-3)
    want = M.adam_step(params, {k: v.astype(np.float64) for k, v in g.items()}, {}, 1e-3)
    got = net.params()
    for k in M.PARAMS:
        assert rel(got[k], want[k]) < 1e-6, k
    net.close()


def test_training_reduces_the_loss(rebk):
    """The targets are a linear function of the inputs (x = P b for a fixed P); 300 Adam steps."""
    rng = np.random.default_rng(3)
    in_dim, hidden, m, n, batch = 128, 128, 128, 64, 128
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    P = rng.standard_normal((n, in_dim)) / np.sqrt(in_dim)
    B = rng.standard_normal((batch, in_dim))
    Xt = B @ P.T
    net = rebk.WarmStart(to_dev(A), in_dim, hidden, max_batch=batch, seed=5)
    Bd, Xd = to_dev(B), to_dev(Xt)
    first = net.train_step(Bd, Xd, lr=3e-3)
    for _ in range(300):
        last = net.train_step(Bd, Xd, lr=3e-3)
    assert last < 0.1 * first, (first, last)
    net.close()


def test_warm_started_solve_matches_oracle(rebk, oracle_lib):
    """REBK from x0 (here: the network's x0 = A^T y, or a good start near A^+ b) and z0 = b - A x0,
    computed in the batched kernel, equals the oracle run from the same start; a start with
    ||b - A x0|| >= ||b|| falls back to x0 = 0, z0 = b, on both sides."""
    rng = np.random.default_rng(4)
    m, n, batch = 256, 64, 64
    S = W.type2(m, n, rng_seed=9, noise=0.05, row_tau=32, col_tau=8)
    Bmat = np.stack([S.A @ rng.standard_normal(n) + 0.0 for _ in range(batch)])
    net = rebk.WarmStart(to_dev(S.A), m, 64, max_batch=batch, seed=1)
    x_net = net.forward(to_dev(Bmat)).cpu().numpy()
    pinv = np.linalg.pinv(S.A)
    x0 = x_net.copy()
    x0[batch // 2:] = Bmat[batch // 2:] @ pinv.T + 0.01 * x_net[batch // 2:]   # good starts
    solver = rebk.Solver(to_dev(S.A), S.row_off, S.col_off, S.alpha, 0)
    batch_solver = rebk.Batch([solver], sys_ids=[0])
    K = 80
    out = batch_solver.solve([to_dev(Bmat)], x0=[to_dev(x0)], max_iter=K, z0_from_x0=True, want_z=True)
    X = out["x"][0].cpu().numpy()
    used = []
    for k in list(range(6)) + list(range(batch // 2, batch // 2 + 6)):
        z0 = Bmat[k] - S.A @ x0[k]
        warm = np.dot(z0, z0) < np.dot(Bmat[k], Bmat[k])
        used.append(warm)
        ref = oracle_lib.rebk_solve(S.A, S.row_off, S.col_off, S.alpha, 0, Bmat[k], x0=x0[k] if warm else None,
                                    z0=z0 if warm else None, max_iter=K, trace=False)
        assert rel(X[k], ref["x"]) <= RTOL_F64, k
    assert any(used) and not all(used)   # both branches exercised
    # the network's x0 lies in range(A^T)
    _, sv, Vt = np.linalg.svd(S.A, full_matrices=False)
    assert np.linalg.norm(x_net - (x_net @ Vt.T) @ Vt) < 1e-13 * np.linalg.norm(x_net)
    batch_solver.close()
    solver.close()
    net.close()


def test_invalid(rebk):
    rng = np.random.default_rng(0)
    A = to_dev(rng.standard_normal((128, 64)))
    with pytest.raises(rebk.RebkError):
        rebk.WarmStart(A, 100, 64)          # not a multiple of 64
    net = rebk.WarmStart(A, 128, 64, max_batch=128)
    with pytest.raises(rebk.RebkError):
        net.forward(to_dev(rng.standard_normal((32, 128))))   # batch not a multiple of 64
    with pytest.raises(rebk.RebkError):
        net.adam(1e-3)                       # no gradients yet
    net.close()
