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
        lam = np.linalg.eigvalsh(g)[-1]
        return float(lam / np.trace(g))
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
