"""What the learned warm start gains (Section 2.2: a start x0 in ran(A^T) with z0 = b - A x0 keeps
the convergence guarantee of Theorem 7).

A network trained on REBK-generated pairs (b, x) for a low-rank system of the warm-start workload's
shape, scaled down four times (2048 x 256, rank 192, right-hand sides b = A x(theta) + r with r
orthogonal to ran(A)), starts REBK on held-out right-hand sides.  The warm-started solves must reach
relative error 1e-6 against A^+ b in fewer iterations on average than the plain start x0 = 0, z0 = b;
a warm solve that does not converge is redone from the plain start (the fallback), and every final
solution is checked against A^+ b.  The iteration count of the training targets is chosen on a slice
of the training right-hand sides, never on the held-out ones.
"""
import math

import numpy as np
import pytest
import torch

from paper_2001_04179_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-6


def test_warm_start_needs_fewer_iterations(rebk):
    print("case warm-start gain 2048x256 rank 192", flush=True)
    P = W.warmstart_problem(n_train=16384, n_eval=512, m=2048, n=256, rank=192, row_tau=16, col_tau=4)
    A_d, ro, co, alpha = P["A_dev"], P["row_off"], P["col_off"], P["alpha"]
    m, n = A_d.shape
    solver = rebk.Solver(A_d, ro, co, alpha, 0, panel_dtype="f32")
    batch = rebk.Batch([solver], sys_ids=[0])
    net = None
    try:
        Btr, Xtr_ref = P["B_train"], P["X_train_ref"]
        Bev, Xev = P["B_eval"], P["X_eval_ref"]

        cold = batch.solve([Bev], x_ref=[Xev], max_iter=2_000_000, tol=TOL, check_every=16)
        assert np.all(cold["rhs_status"] == 0) and np.all(cold["rel_err"] <= TOL)
        print(f"plain: mean {cold['iterations'].mean():.0f} iterations", flush=True)

        # training targets: REBK for the iteration count that brings a slice of the training
        # right-hand sides to 1e-3
        probe = batch.solve([Btr[:256].contiguous()], x_ref=[Xtr_ref[:256].contiguous()], max_iter=2_000_000,
                            tol=1e-3, check_every=16)
        K_gen = int(probe["iterations"].max())
        Xtr = batch.solve([Btr], max_iter=K_gen)["x"][0]
        print(f"targets: {K_gen} iterations", flush=True)

        bs = 256
        b_scale = 1.0 / float(Btr.pow(2).mean().sqrt())
        net = rebk.WarmStart(A_d, m, 256, max_batch=bs, seed=7)
        nb = Btr.shape[0] // bs
        epochs = 20
        total = epochs * nb
        lr0, lr_min = 1e-3, 1e-5
        gen = torch.Generator(device="cpu").manual_seed(11)
        step = 0
        first = last = None
        for ep in range(epochs):
            perm = torch.randperm(nb * bs, generator=gen).to(A_d.device)
            loss = 0.0
            for q in range(nb):
                lr = lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * step / total))
                step += 1
                idx = perm[q * bs:(q + 1) * bs]
                loss += net.train_step(Btr[idx].contiguous(), Xtr[idx].contiguous(), lr=lr, b_scale=b_scale)
            first = loss / nb if first is None else first
            last = loss / nb
        print(f"training: loss {first:.3e} -> {last:.3e}", flush=True)
        assert last < first

        X0 = torch.cat([net.forward(Bev[q:q + bs].contiguous(), b_scale=b_scale) for q in range(0, Bev.shape[0], bs)])
        # Theorem 7's hypothesis: x0 lies in ran(A^T) (the network's output is A^T y)
        U, s, Vt = np.linalg.svd(P["A"], full_matrices=False)
        Q = Vt[s > 1e-10 * s[0]].T
        X0h = X0.cpu().numpy()
        assert np.linalg.norm(X0h - (X0h @ Q) @ Q.T) <= 1e-10 * np.linalg.norm(X0h)

        warm = batch.solve([Bev], x_ref=[Xev], x0=[X0], max_iter=int(2 * cold["iterations"].max()), tol=TOL,
                           check_every=16, z0_from_x0=True)
        x_warm = warm["x"][0].clone()
        failed = np.nonzero(warm["rhs_status"] != 0)[0]
        if failed.size:  # the fallback: those right-hand sides from the plain start
            idx = torch.from_numpy(failed).to(A_d.device)
            redo = batch.solve([Bev[idx].contiguous()], x_ref=[Xev[idx].contiguous()], max_iter=2_000_000, tol=TOL,
                               check_every=16)
            assert np.all(redo["rhs_status"] == 0)
            x_warm[idx] = redo["x"][0]
        err = ((x_warm - Xev).norm(dim=1) / Xev.norm(dim=1)).cpu().numpy()
        assert np.all(err <= TOL)
        err_cold = ((cold["x"][0] - Xev).norm(dim=1) / Xev.norm(dim=1)).cpu().numpy()
        assert np.all(err_cold <= TOL)

        ok = warm["rhs_status"] == 0
        warm_mean = float(warm["iterations"][ok].mean()) if ok.any() else float("inf")
        print(f"warm: mean {warm_mean:.0f} iterations ({failed.size} fell back); plain "
              f"{cold['iterations'].mean():.0f}", flush=True)
        assert failed.size <= Bev.shape[0] // 20
        assert warm_mean < float(cold["iterations"].mean())
    finally:
        if net is not None:
            net.close()
        batch.close()
        solver.close()
