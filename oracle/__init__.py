"""FP64 CPU oracle for the randomized extended block Kaczmarz method.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import this package.  It shares no code with the GPU library under
``paper_2001_04179_amd`` and never imports it.

The arithmetic lives in ``rebk_oracle.c`` (plain loops, FP64, compiled with
``-ffp-contract=off``); this module only builds it and marshals numpy arrays.
It follows Du, Si and Sun, arXiv:2001.04179, Section 2, Algorithm 1; the
fixed choices the paper leaves open (summation order of the block weights,
the integer-threshold block draw, the Philox counter layout) are stated in the
C file's header.  Philox4x64-10 follows Salmon et al., SC'11.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rebk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_SRC_OMP = os.path.join(_HERE, "rebk_oracle_omp.c")
_SRC_F32 = os.path.join(_HERE, "rebk_oracle_f32state.c")
_LIB_OMP = os.path.join(_HERE, "liboracle_variants.so")

_lib = None
_lib_omp = None


def _stale(lib, srcs):
    return not os.path.exists(lib) or any(os.path.getmtime(lib) < os.path.getmtime(s) for s in srcs)


def build(force: bool = True) -> str:
    """Compile ``rebk_oracle.c`` into ``liboracle.so`` with gcc (no FMA contraction), and two
    variants of the iteration that reuse its Philox and draws -- the OpenMP timing variant
    (``rebk_oracle_omp.c``) and the all-FP32 form (``rebk_oracle_f32state.c``) -- into
    ``liboracle_variants.so``."""
    flags = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
    if force or _stale(_LIB, [_SRC]):
        tmp = _LIB + ".tmp"
        subprocess.check_call(flags + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    if force or _stale(_LIB_OMP, [_SRC, _SRC_OMP, _SRC_F32]):
        tmp = _LIB_OMP + ".tmp"
        subprocess.check_call(flags + ["-fopenmp", "-o", tmp, _SRC_OMP, _SRC_F32, _SRC, "-lm"])
        os.replace(tmp, _LIB_OMP)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    U64 = ctypes.c_uint64
    lib.oracle_philox4x64_10.argtypes = [P, P, P]
    lib.oracle_philox4x64_10.restype = None
    lib.oracle_block_weights.argtypes = [P, I64, I64, I64, P, I64, P, I64, P, P]
    lib.oracle_block_weights.restype = None
    lib.oracle_thresholds.argtypes = [P, I64, P]
    lib.oracle_thresholds.restype = ctypes.c_int
    lib.oracle_pick.argtypes = [P, I64, U64]
    lib.oracle_pick.restype = I64
    lib.oracle_rebk_solve.argtypes = [P, I64, I64, I64, P, I64, P, I64, ctypes.c_double, U64, U64,
                                      P, P, P, I64, I64, P, ctypes.c_double, P, P, P, P, P, P]
    lib.oracle_rebk_solve.restype = ctypes.c_int
    lib.oracle_rebk_refine.argtypes = [P, P, I64, I64, I64, P, I64, P, I64, ctypes.c_double, U64, U64,
                                       P, P, P, ctypes.c_double, I64, I64, P, P, P, P, P, P]
    lib.oracle_rebk_refine.restype = ctypes.c_int
    lib.oracle_philox_fill.argtypes = [P, P, I64, P]
    lib.oracle_philox_fill.restype = None
    lib.oracle_sample_blocks.argtypes = [P, I64, P, I64, U64, U64, I64, I64, P, P]
    lib.oracle_sample_blocks.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def philox4x64_10(counter, key) -> np.ndarray:
    """Philox4x64-10 of one (counter[4], key[2]) pair -> 4 uint64 words."""
    lib = _load()
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.oracle_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_fill(counter, key, count) -> np.ndarray:
    """Philox4x64-10 words for counters (c0+q, c1, c2, c3), q < count: array of shape (count, 4)."""
    lib = _load()
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros((int(count), 4), dtype=np.uint64)
    lib.oracle_philox_fill(_ptr(c), _ptr(k), int(count), _ptr(out))
    return out


def sample_blocks(w_row, w_col, seed, k0, count, sys=0):
    """0-based (j, i) block draws of iterations k0+1 .. k0+count from the block weights."""
    lib = _load()
    wr, wc = _f64(w_row), _f64(w_col)
    j = np.zeros(int(count), dtype=np.int32)
    i = np.zeros(int(count), dtype=np.int32)
    st = lib.oracle_sample_blocks(_ptr(wr), len(wr), _ptr(wc), len(wc), ctypes.c_uint64(int(seed)),
                                  ctypes.c_uint64(int(sys)), int(k0), int(count), _ptr(j), _ptr(i))
    if st != 0:
        raise ValueError("block weights must be non-negative with a positive finite sum")
    return j, i


def block_weights(A, row_off, col_off):
    """(w_row[s], w_col[t]): squared Frobenius norms of the row and column blocks."""
    lib = _load()
    A = _f64(A)
    m, n = A.shape
    ro, co = _i64(row_off), _i64(col_off)
    s, t = len(ro) - 1, len(co) - 1
    w_row = np.zeros(s)
    w_col = np.zeros(t)
    lib.oracle_block_weights(_ptr(A), m, n, n, _ptr(ro), s, _ptr(co), t, _ptr(w_row), _ptr(w_col))
    return w_row, w_col


def thresholds(w) -> np.ndarray:
    """Cumulative 53-bit integer thresholds for drawing block j with probability w_j / sum(w)."""
    lib = _load()
    w = _f64(w)
    T = np.zeros(len(w), dtype=np.uint64)
    if lib.oracle_thresholds(_ptr(w), len(w), _ptr(T)) != 0:
        raise ValueError("block weights must be non-negative with a positive finite sum")
    return T


def pick(T, word) -> int:
    """Block drawn by one 64-bit Philox word against thresholds T."""
    lib = _load()
    T = np.ascontiguousarray(T, dtype=np.uint64)
    return int(lib.oracle_pick(_ptr(T), len(T), ctypes.c_uint64(int(word))))


def rebk_solve(A, row_off, col_off, alpha, seed, b, *, x0=None, z0=None, k0=0, max_iter=1000,
               x_ref=None, tol=0.0, sys=0, trace=True):
    """Run Algorithm 1 for iterations k0+1 .. k0+max_iter (stopping early on tol if x_ref is given).

    Returns a dict with x, z, iterations, err (relative error to x_ref, or -1), status
    (0 stopped/ran, 1 tol not met, -1 invalid) and, with ``trace``, the 0-based block
    indices j (column blocks) and i (row blocks) drawn at each iteration.
    """
    lib = _load()
    A = _f64(A)
    m, n = A.shape
    ro, co = _i64(row_off), _i64(col_off)
    s, t = len(ro) - 1, len(co) - 1
    b = _f64(b)
    x0 = _f64(x0)
    z0 = _f64(z0)
    x_ref = _f64(x_ref)
    x = np.zeros(n)
    z = np.zeros(m)
    jt = np.zeros(max(max_iter, 1), dtype=np.int32) if trace else None
    it = np.zeros(max(max_iter, 1), dtype=np.int32) if trace else None
    iters = np.zeros(1, dtype=np.int64)
    err = np.zeros(1)
    st = lib.oracle_rebk_solve(_ptr(A), m, n, n, _ptr(ro), s, _ptr(co), t, float(alpha),
                               ctypes.c_uint64(int(seed)), ctypes.c_uint64(int(sys)),
                               _ptr(b), _ptr(x0), _ptr(z0), int(k0), int(max_iter),
                               _ptr(x_ref), float(tol), _ptr(x), _ptr(z), _ptr(jt), _ptr(it),
                               _ptr(iters), _ptr(err))
    if st < 0:
        raise ValueError("invalid REBK input")
    k = int(iters[0])
    out = {"x": x, "z": z, "iterations": k, "err": float(err[0]), "status": int(st)}
    if trace:
        out["j"] = jt[:k].copy()
        out["i"] = it[:k].copy()
    return out


def _load_omp():
    global _lib_omp
    if _lib_omp is not None:
        return _lib_omp
    if _stale(_LIB_OMP, [_SRC, _SRC_OMP, _SRC_F32]):
        build(force=False)
    lib = ctypes.CDLL(_LIB_OMP)
    P, I64, U64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    lib.oracle_rebk_solve_omp.argtypes = [P, I64, I64, I64, P, I64, P, I64, ctypes.c_double, U64, U64, P, I64, P, P]
    lib.oracle_rebk_solve_omp.restype = ctypes.c_int
    lib.oracle_omp_threads.argtypes = []
    lib.oracle_omp_threads.restype = ctypes.c_int
    lib.oracle_rebk_f32state.argtypes = [P, I64, I64, P, I64, P, I64, ctypes.c_double, U64, P, P, I64, I64, P, P]
    lib.oracle_rebk_f32state.restype = ctypes.c_int
    _lib_omp = lib
    return lib


def omp_threads() -> int:
    """Threads the OpenMP variant uses (OMP_NUM_THREADS, else the cores OpenMP sees)."""
    return int(_load_omp().oracle_omp_threads())


def rebk_solve_omp(A, row_off, col_off, alpha, seed, b, *, max_iter=1000, sys=0):
    """Algorithm 1 from x0 = 0, z0 = b for exactly max_iter iterations with the block products on
    OpenMP threads (timing baseline only; the plain oracle is the parity reference).  Returns
    dict(x, z)."""
    lib = _load_omp()
    A = _f64(A)
    m, n = A.shape
    ro, co = _i64(row_off), _i64(col_off)
    b = _f64(b)
    x = np.zeros(n)
    z = np.zeros(m)
    st = lib.oracle_rebk_solve_omp(_ptr(A), m, n, n, _ptr(ro), len(ro) - 1, _ptr(co), len(co) - 1, float(alpha),
                                   ctypes.c_uint64(int(seed)), ctypes.c_uint64(int(sys)), _ptr(b), int(max_iter),
                                   _ptr(x), _ptr(z))
    if st < 0:
        raise ValueError("invalid REBK input")
    return {"x": x, "z": z}


def rebk_f32state(A, row_off, col_off, alpha, seed, b, x_ref, *, max_iter=1000, every=100):
    """Algorithm 1 from x0 = 0, z0 = b with every vector and every operation in FP32 on the FP32
    values of A (the all-FP32 form; a measurement aid, not a parity reference).  Returns dict(x
    (FP32), err: the relative error to x_ref every `every` iterations and at the end)."""
    lib = _load_omp()
    A32 = np.ascontiguousarray(A, dtype=np.float32)
    m, n = A32.shape
    ro, co = _i64(row_off), _i64(col_off)
    b32 = np.ascontiguousarray(b, dtype=np.float32)
    xr = _f64(x_ref)
    nerr = (int(max_iter) + int(every) - 1) // int(every) + 1
    err = np.full(nerr, np.nan)
    x = np.zeros(n, dtype=np.float32)
    st = lib.oracle_rebk_f32state(_ptr(A32), m, n, _ptr(ro), len(ro) - 1, _ptr(co), len(co) - 1, float(alpha),
                                  ctypes.c_uint64(int(seed)), _ptr(b32), _ptr(xr), int(max_iter), int(every),
                                  _ptr(err), _ptr(x))
    if st < 0:
        raise ValueError("invalid REBK input")
    return {"x": x, "err": err[~np.isnan(err)]}


def rebk_refine(A, A_stored, row_off, col_off, alpha, seed, b, *, x0=None, x_ref=None, tol=0.0, inner_iters=100,
                max_outer=10, sys=0):
    """FP64 iterative refinement of the augmented least-squares system with Algorithm 1 as the
    inner solver on A_stored (the stored panel values), residuals and x-updates on A.

    Returns dict(x, z, err_trace (one entry per tested outer step), outer, iterations, err, status
    (0 stopped on tol, 1 max_outer reached))."""
    lib = _load()
    A = _f64(A)
    Ast = _f64(A_stored)
    m, n = A.shape
    if Ast.shape != A.shape:
        raise ValueError("A_stored must have A's shape")
    ro, co = _i64(row_off), _i64(col_off)
    s, t = len(ro) - 1, len(co) - 1
    b = _f64(b)
    x0 = _f64(x0)
    x_ref = _f64(x_ref)
    x = np.zeros(n)
    z = np.zeros(m)
    trace = np.full(int(max_outer) + 1, np.nan)
    outer = np.zeros(1, dtype=np.int64)
    iters = np.zeros(1, dtype=np.int64)
    err = np.zeros(1)
    st = lib.oracle_rebk_refine(_ptr(A), _ptr(Ast), m, n, n, _ptr(ro), s, _ptr(co), t, float(alpha),
                                ctypes.c_uint64(int(seed)), ctypes.c_uint64(int(sys)), _ptr(b), _ptr(x0),
                                _ptr(x_ref), float(tol), int(inner_iters), int(max_outer), _ptr(x), _ptr(z),
                                _ptr(trace), _ptr(outer), _ptr(iters), _ptr(err))
    if st < 0:
        raise ValueError("invalid refinement input")
    tested = int(outer[0]) + 1
    return {"x": x, "z": z, "err_trace": trace[:tested], "outer": int(outer[0]), "iterations": int(iters[0]),
            "err": float(err[0]), "status": int(st)}



def block_betas(A, row_off, col_off):
    """Block constants of Section 2.2: beta = ||B||_2^2 / ||B||_F^2 for every row block
    A[I_i, :] and column block A[:, J_j], from the largest eigenvalue of the Gram matrix of the
    block's shorter side (LAPACK, FP64) over its trace.  Returns (beta_row, beta_col)."""
    A = _f64(A)

    def beta(B):
        G = B @ B.T if B.shape[0] <= B.shape[1] else B.T @ B
        tr = float(np.trace(G))
        return float(np.linalg.eigvalsh(G)[-1]) / tr if tr > 0 else 0.0

    ro, co = _i64(row_off), _i64(col_off)
    br = np.array([beta(A[ro[i]:ro[i + 1], :]) for i in range(len(ro) - 1)])
    bc = np.array([beta(A[:, co[j]:co[j + 1]]) for j in range(len(co) - 1)])
    return br, bc
