"""Seeded synthetic inputs shaped like the paper's test problems (NumPy, FP64, host memory).

This module only builds inputs: matrices, right-hand sides, partitions, the reference solution
A^+ b and a stepsize.  It holds none of the iteration's arithmetic and serves the tests, the
benchmark and the oracle runs alike.

* Section 3 builds inconsistent systems b = A x + r with x ~ N(0, I) and r in null(A^T); the
  scale of r is not stated there, so it is a parameter (``noise`` = ||r|| / ||A x||).
* Type I matrices are U D V^T with orthonormal U (m x r), V (n x r) from QR of Gaussian
  matrices and D uniform in (1, kappa); Type II matrices are dense N(0, 1) (Section 3.1).
* A^+ b is formed by projection, never by an iterative solve: with r orthogonal to range(A),
  A^+ b = P x where P projects onto range(A^T).
* The stepsize default is alpha = c / beta_max, beta_max = max over blocks of
  ||B||_2^2 / ||B||_F^2 (Section 2.2, Remark 9), computed here with LAPACK.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class System:
    A: np.ndarray            # m x n, FP64, row-major
    b: np.ndarray            # m
    x_star: np.ndarray       # n, the generating vector
    x_ref: np.ndarray        # n, A^+ b
    row_off: np.ndarray      # s + 1
    col_off: np.ndarray      # t + 1
    alpha: float
    seed: int                # Philox seed of the block sampler
    beta_row: float = 0.0
    beta_col: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.A.shape


def contiguous_offsets(total: int, tau: int) -> np.ndarray:
    """[0, tau, 2 tau, ..., total]: equal blocks of tau with a smaller last block (Section 3)."""
    off = list(range(0, total, tau)) + [total]
    return np.asarray(off, dtype=np.int64)


def orthonormal(M: np.ndarray) -> np.ndarray:
    q, _ = np.linalg.qr(M, mode="reduced")
    return q


def beta_max(A: np.ndarray, row_off, col_off):
    """(beta_max over row blocks, beta_max over column blocks): max ||B||_2^2 / ||B||_F^2."""
    def ratio(B):
        g = B @ B.T if B.shape[0] <= B.shape[1] else B.T @ B
        tr = np.trace(g)
        if not tr > 0.0:
            return 0.0  # a zero block is never drawn and does not bound the stepsize
        lam = np.linalg.eigvalsh(g)[-1]
        return float(lam / tr)
    br = max(ratio(A[row_off[i]:row_off[i + 1], :]) for i in range(len(row_off) - 1))
    bc = max(ratio(A[:, col_off[j]:col_off[j + 1]]) for j in range(len(col_off) - 1))
    return br, bc


def rhs_in_range_plus_noise(A, x_star, Q_range, noise, rng, g=None):
    """b = A x* + r with r = (I - Q Q^T) g scaled to ||r|| = noise ||A x*|| (Q: basis of range(A))."""
    Ax = A @ x_star
    if noise <= 0.0 or Q_range.shape[1] >= A.shape[0]:
        return Ax.copy(), np.zeros_like(Ax)
    if g is None:
        g = rng.standard_normal(A.shape[0])
    r = g - Q_range @ (Q_range.T @ g)
    r *= noise * np.linalg.norm(Ax) / np.linalg.norm(r)
    return Ax + r, r


def _finish(A, x_star, Q_range, Q_rowsp, noise, rng, row_tau, col_tau, alpha_c, seed, meta, row_off=None,
            col_off=None):
    m, n = A.shape
    b, r = rhs_in_range_plus_noise(A, x_star, Q_range, noise, rng)
    x_ref = Q_rowsp @ (Q_rowsp.T @ x_star) if Q_rowsp is not None else x_star.copy()
    ro = contiguous_offsets(m, row_tau) if row_off is None else np.asarray(row_off, dtype=np.int64)
    co = contiguous_offsets(n, col_tau) if col_off is None else np.asarray(col_off, dtype=np.int64)
    br, bc = beta_max(A, ro, co)
    alpha = alpha_c / max(br, bc)
    meta = dict(meta)
    meta["noise"] = noise
    meta["r_norm"] = float(np.linalg.norm(r))
    return System(A=np.ascontiguousarray(A), b=b, x_star=x_star, x_ref=x_ref, row_off=ro, col_off=co, alpha=alpha,
                  seed=seed, beta_row=br, beta_col=bc, meta=meta)


def type2(m, n, *, rng_seed=0, noise=0.1, row_tau=10, col_tau=10, alpha_c=1.0, seed=0) -> System:
    """Type II: A = randn(m, n) (Section 3.1); full rank almost surely."""
    rng = np.random.default_rng(rng_seed)
    A = rng.standard_normal((m, n))
    x_star = rng.standard_normal(n)
    if m >= n:
        Q_range, Q_rowsp = orthonormal(A), None          # full column rank: A^+ b = x*
    else:
        Q_range, Q_rowsp = np.eye(m), orthonormal(A.T)   # full row rank: consistent
    return _finish(A, x_star, Q_range, Q_rowsp, noise, rng, row_tau, col_tau, alpha_c, seed,
                   {"kind": "type2", "m": m, "n": n})


def type1(m, n, r, kappa, *, rng_seed=0, noise=0.1, row_tau=10, col_tau=10, alpha_c=1.0, seed=0) -> System:
    """Type I: A = U D V^T, U, V orthonormal (QR of Gaussians), D ~ U(1, kappa) (Section 3.1)."""
    rng = np.random.default_rng(rng_seed)
    U = orthonormal(rng.standard_normal((m, r)))
    V = orthonormal(rng.standard_normal((n, r)))
    D = 1.0 + (kappa - 1.0) * rng.random(r)
    A = (U * D) @ V.T
    x_star = rng.standard_normal(n)
    return _finish(A, x_star, U, V, noise, rng, row_tau, col_tau, alpha_c, seed,
                   {"kind": "type1", "m": m, "n": n, "rank": r, "kappa": kappa})


def factor_product(m, n, r, *, rng_seed=0, noise=0.1, row_tau=10, col_tau=10, alpha_c=1.0, seed=0,
                   fro2_target: Optional[float] = None) -> System:
    """Rank-r factor product A = c U V with Gaussian U (m x r), V (r x n); optional scaling so that
    ||A||_F^2 = fro2_target.  range(A) = range(U), range(A^T) = range(V^T)."""
    rng = np.random.default_rng(rng_seed)
    U = rng.standard_normal((m, r))
    V = rng.standard_normal((r, n))
    A = U @ V
    if fro2_target is not None:
        A *= np.sqrt(fro2_target / np.sum(A * A))
    x_star = rng.standard_normal(n)
    Q_range = orthonormal(U)
    Q_rowsp = orthonormal(V.T)
    return _finish(A, x_star, Q_range, Q_rowsp, noise, rng, row_tau, col_tau, alpha_c, seed,
                   {"kind": "factor", "m": m, "n": n, "rank": r})


def general(A: np.ndarray, *, rng_seed=0, noise=0.1, row_off=None, col_off=None, row_tau=1, col_tau=1,
            alpha_c=1.0, seed=0, x_star=None) -> System:
    """Any (small) A: range bases from an SVD.  For tests on tiny or degenerate matrices."""
    rng = np.random.default_rng(rng_seed)
    m, n = A.shape
    if x_star is None:
        x_star = rng.standard_normal(n)
    U, sv, Vt = np.linalg.svd(A, full_matrices=False)
    rank = int(np.sum(sv > sv[0] * max(m, n) * np.finfo(float).eps)) if sv.size and sv[0] > 0 else 0
    Q_range, Q_rowsp = U[:, :rank], Vt[:rank].T
    return _finish(A, x_star, Q_range, Q_rowsp, noise, rng, row_tau, col_tau, alpha_c, seed,
                   {"kind": "general", "m": m, "n": n, "rank": rank}, row_off=row_off, col_off=col_off)


# ---------------------------------------------------------------------------------------------
# The benchmark configurations

def dense_gaussian_1000x100(rng_seed=1001, seed=0) -> System:
    """A 1000 x 100 dense N(0,1) (full column rank), x* ~ N(0,1), r in null(A^T) with
    ||r|| = 0.1 ||A x*||; 10 row blocks of 100 rows and 10 column blocks of 10 columns;
    alpha = 1 / beta_max (Remark 9); x0 = 0, z0 = b; Philox seed 0."""
    return type2(1000, 100, rng_seed=rng_seed, noise=0.1, row_tau=100, col_tau=10, alpha_c=1.0, seed=seed)


def rank1500_20000x2000(rng_seed=1002, seed=0, scale: int = 1) -> System:
    """Rank-deficient overdetermined A = c U V (U 20000 x 1500, V 1500 x 2000, N(0,1)),
    ||A||_F^2 = m; b = A x* + r, r in null(A^T), ||r|| = 0.1 ||A x*||; 100 row blocks of 200
    rows, 100 column blocks of 20 columns; alpha = 1 / beta_max.  ``scale`` > 1 divides every
    dimension (not the block sizes) for quick tests."""
    m, n, r = 20000 // scale, 2000 // scale, 1500 // scale
    return factor_product(m, n, r, rng_seed=rng_seed, noise=0.1, row_tau=200, col_tau=20, alpha_c=1.0, seed=seed,
                          fro2_target=float(m))


def rank1200_2000x50000(rng_seed=1003, seed=0, scale: int = 1) -> System:
    """Underdetermined rank-deficient A = U V (U 2000 x 1200, V 1200 x 50000, N(0,1), not
    normalised); b = A x* + r, r in null(A^T) with ||r|| = 0.1 ||A x*||; 20 row blocks of 100
    rows, 500 column blocks of 100 columns; alpha = 1 / beta_max.  ``scale`` > 1 divides the
    dimensions (not the block sizes)."""
    m, n, r = 2000 // scale, 50000 // scale, 1200 // scale
    return factor_product(m, n, r, rng_seed=rng_seed, noise=0.1, row_tau=100, col_tau=100, alpha_c=1.0, seed=seed)


def warmstart_problem(n_train=65536, n_eval=4096, rng_seed=1005, m=8192, n=1024, rank=768, n_basis=8, n_freq=16,
                      noise=0.05, row_tau=64, col_tau=16, device="cuda", chunk=8192):
    """The learned-warm-start workload.  A = U V / sqrt(rank) (U m x rank, V rank x n, N(0,1));
    right-hand sides b = A x(theta) + r with theta ~ U[-1, 1]^8, x(theta) = sum_k theta_k phi_k over
    fixed smooth bases phi_k(t) = sum_{f=1}^{16} a_kf cos(pi f t + psi_kf) on 1024 points of [0, 1]
    (a_kf ~ N(0, 1/f^2), psi_kf ~ U[0, 2 pi)), r = (I - P_range(A)) g scaled to 0.05 ||A x||;
    references x_ref = P_range(A^T) x(theta) = A^+ b.  The factorisations run on the host (numpy,
    seed rng_seed); the right-hand sides are generated on the device in chunks with a seeded
    torch generator (inputs only).  Returns a dict of device tensors and host metadata."""
    import torch
    rng = np.random.default_rng(rng_seed)
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((rank, n))
    A = (U @ V) / np.sqrt(rank)
    Qu = orthonormal(U)
    Qv = orthonormal(V.T)
    t = np.linspace(0.0, 1.0, n)
    f = np.arange(1, n_freq + 1)
    a = rng.standard_normal((n_basis, n_freq)) / f
    psi = rng.uniform(0.0, 2.0 * np.pi, (n_basis, n_freq))
    Phi = np.einsum("kf,kft->kt", a, np.cos(np.pi * f[None, :, None] * t[None, None, :] + psi[:, :, None]))
    ro = contiguous_offsets(m, row_tau)
    co = contiguous_offsets(n, col_tau)
    br, bc = beta_max(A, ro, co)
    dev = torch.device(device)
    A_d = torch.from_numpy(A).to(dev)
    Qu_d, Qv_d, Phi_d = (torch.from_numpy(v).to(dev) for v in (Qu, Qv, Phi))
    gen = torch.Generator(device=dev).manual_seed(rng_seed)

    def rhs(N):
        B = torch.empty((N, m), dtype=torch.float64, device=dev)
        X = torch.empty((N, n), dtype=torch.float64, device=dev)
        for c0 in range(0, N, chunk):
            c1 = min(N, c0 + chunk)
            theta = torch.rand((c1 - c0, n_basis), generator=gen, device=dev, dtype=torch.float64) * 2.0 - 1.0
            Xs = theta @ Phi_d
            AX = Xs @ A_d.T
            G = torch.randn((c1 - c0, m), generator=gen, device=dev, dtype=torch.float64)
            Rn = G - (G @ Qu_d) @ Qu_d.T
            Rn *= (noise * AX.norm(dim=1) / Rn.norm(dim=1)).unsqueeze(1)
            B[c0:c1] = AX + Rn
            X[c0:c1] = (Xs @ Qv_d) @ Qv_d.T
        return B, X

    B_tr, X_tr = rhs(n_train)
    B_ev, X_ev = rhs(n_eval)
    return {"A": A, "A_dev": A_d, "row_off": ro, "col_off": co, "alpha": 1.0 / max(br, bc), "beta_row": br,
            "beta_col": bc, "B_train": B_tr, "X_train_ref": X_tr, "B_eval": B_ev, "X_eval_ref": X_ev,
            "rank": rank}


@dataclass
class BatchSystem:
    """One system of a batch with several right-hand sides (rows of B, X_ref)."""
    A: np.ndarray            # m x n
    B: np.ndarray            # nrhs x m
    X_star: np.ndarray       # nrhs x n
    X_ref: np.ndarray        # nrhs x n, A^+ b for every right-hand side
    row_off: np.ndarray
    col_off: np.ndarray
    alpha: float
    sys_id: int
    rank: int
    beta_row: float = 0.0
    beta_col: float = 0.0

    @property
    def shape(self):
        return self.A.shape


def _spd_solve(G: np.ndarray, R: np.ndarray) -> np.ndarray:
    from scipy.linalg import cho_factor, cho_solve
    return cho_solve(cho_factor(G, lower=False, check_finite=False), R, check_finite=False)


def batch_system(m: int, n: int, rank: Optional[int], nrhs: int, rng: np.random.Generator, *, noise=0.05,
                 row_tau=64, col_tau=16, alpha_c=1.0, sys_id=0) -> BatchSystem:
    """Dense N(0, 1) A (m x n) or, with ``rank``, the factor product U V / sqrt(rank) (U m x rank,
    V rank x n, N(0, 1)).  Right-hand sides b = A x* + r, x* ~ N(0, I), r = (I - P_range(A)) g
    scaled to ||r|| = noise ||A x*|| (r = 0 where null(A^T) = {0}); x_ref = P_range(A^T) x*.
    The projections use Cholesky factors of the Gram matrices of full-rank factors, so a system of
    a few thousand rows and columns is built in a fraction of a second."""
    X = rng.standard_normal((nrhs, n))
    if rank is None:
        A = rng.standard_normal((m, n))
        if m >= n:          # full column rank: range(A^T) = R^n, x_ref = x*
            AX = X @ A.T
            Gm = rng.standard_normal((nrhs, m))
            Rn = Gm - (_spd_solve(A.T @ A, (Gm @ A).T).T @ A.T)
            X_ref = X.copy()
        else:               # full row rank: null(A^T) = {0}, consistent; x_ref = A^T (A A^T)^-1 A x*
            AX = X @ A.T
            Rn = np.zeros((nrhs, m))
            X_ref = _spd_solve(A @ A.T, AX.T).T @ A
        r_rank = min(m, n)
    else:
        U = rng.standard_normal((m, rank))
        V = rng.standard_normal((rank, n))
        A = (U @ V) / np.sqrt(rank)
        AX = X @ A.T
        Gm = rng.standard_normal((nrhs, m))
        Rn = Gm - (_spd_solve(U.T @ U, (Gm @ U).T).T @ U.T)     # (I - U (U^T U)^-1 U^T) g
        X_ref = _spd_solve(V @ V.T, (X @ V.T).T).T @ V           # V^T (V V^T)^-1 V x*
        r_rank = rank
    B = AX.copy()
    for k in range(nrhs):
        rn = np.linalg.norm(Rn[k])
        if noise > 0.0 and rn > 0.0:
            B[k] += Rn[k] * (noise * np.linalg.norm(AX[k]) / rn)
    ro = contiguous_offsets(m, row_tau)
    co = contiguous_offsets(n, col_tau)
    br, bc = beta_max(A, ro, co)
    return BatchSystem(A=np.ascontiguousarray(A), B=np.ascontiguousarray(B), X_star=X,
                       X_ref=np.ascontiguousarray(X_ref), row_off=ro, col_off=co, alpha=alpha_c / max(br, bc),
                       sys_id=sys_id, rank=r_rank, beta_row=br, beta_col=bc)


def batch_shapes(count: int, rng: np.random.Generator, m_range=(500, 8000), n_range=(100, 2000),
                 min_aspect=4.0, rank_every=4):
    """Shapes of a batch: m, n uniform in their ranges, redrawn until max/min >= min_aspect (a
    near-square Gaussian system is so ill-conditioned that the method needs millions of
    iterations); odd-indexed systems are transposed (m < n, half the batch underdetermined); every
    rank_every-th system (index rank_every-1, 2 rank_every-1, ...) has rank floor(min(m, n) / 2)."""
    shapes = []
    while len(shapes) < count:
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        if max(m, n) < min_aspect * min(m, n):
            continue
        idx = len(shapes)
        if idx % 2 == 1:
            m, n = n, m
        rank = min(m, n) // 2 if (rank_every and idx % rank_every == rank_every - 1) else None
        shapes.append((m, n, rank))
    return shapes


def batch_256_dense(rng_seed=1004, count=256, nrhs=16, m_range=(500, 8000), n_range=(100, 2000), min_aspect=4.0,
                    noise=0.05, row_tau=64, col_tau=16, workers=1):
    """The batched workload: 256 dense Gaussian systems with m in [500, 8000] and n in [100, 2000]
    (aspect ratio at least 4, odd ones transposed, every fourth of rank min(m, n)/2), 16
    right-hand sides each with noise ratio 0.05, blocks of 64 rows and 16 columns, alpha =
    1 / beta_max per system, Philox system id = index, seed 0.  ``workers`` > 1 builds the
    systems in that many processes (same values)."""
    shapes = batch_shapes(count, np.random.default_rng(rng_seed), m_range, n_range, min_aspect)
    args = [(rng_seed, q, m, n, rk, nrhs, noise, row_tau, col_tau) for q, (m, n, rk) in enumerate(shapes)]
    # one BLAS thread per system whatever the worker count; workers are threads: the random fills and BLAS calls release the GIL and nothing is copied
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        if workers > 1:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=workers) as ex:
                return list(ex.map(_batch_member, args))
        return [_batch_member(a) for a in args]


def _batch_member(args) -> BatchSystem:
    """System q of a batch, from its own generator seeded with (rng_seed, q): any subset of a batch
    can be rebuilt, in any order or in parallel (random values identical, BLAS-computed ones equal
    up to rounding)."""
    rng_seed, q, m, n, rk, nrhs, noise, row_tau, col_tau = args
    rng = np.random.default_rng([rng_seed, q])
    return batch_system(m, n, rk, nrhs, rng, noise=noise, row_tau=row_tau, col_tau=col_tau, sys_id=q)


def round_to_bf16(A: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64.

    Values are first rounded to 8 significant bits on the FP64 bit pattern (ties to even), which
    is exact for normal bfloat16 numbers; the input range here is far from bfloat16's limits."""
    a = np.ascontiguousarray(A, dtype=np.float64)
    bits = a.view(np.uint64)
    drop = np.uint64(52 - 7)
    lsb = (bits >> drop) & np.uint64(1)
    rounded = (bits + (np.uint64(1) << (drop - np.uint64(1))) - np.uint64(1) + lsb) & ~((np.uint64(1) << drop) - np.uint64(1))
    return rounded.view(np.float64).copy()


def round_to_f16(A: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest IEEE half (ties to even), returned as FP64 (NumPy's cast)."""
    return np.asarray(A, dtype=np.float64).astype(np.float16).astype(np.float64)


def round_to_f32(A: np.ndarray) -> np.ndarray:
    return np.asarray(A, dtype=np.float64).astype(np.float32).astype(np.float64)
