"""REBK on MI355X: Python binding of ``librebk.so``.

Randomized extended block Kaczmarz (Du, Si, Sun, arXiv:2001.04179, Section 2, Algorithm 1) for
the minimum-norm least-squares solution A^+ b.  Every step of the method runs in the HIP
library; this module only marshals arguments.  PyTorch supplies device memory and the stream.
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N

__all__ = ["Solver", "SolveResult", "Batch", "WarmStart", "philox4x64_10", "contiguous_offsets", "RebkError",
           "version"]

RebkError = N.RebkError


def version() -> str:
    return N.load().rebk_version().decode()


def contiguous_offsets(total: int, tau: int) -> np.ndarray:
    """Offsets of the contiguous partition into blocks of size tau, the last one smaller
    (Section 3): [0, tau, 2 tau, ..., total]."""
    if total <= 0 or tau <= 0:
        raise ValueError("total and tau must be positive")
    off = list(range(0, total, tau)) + [total]
    return np.asarray(off, dtype=np.int64)


@dataclass
class SolveResult:
    status: str
    code: int
    kernel: str
    iterations: int
    rel_err: float
    time_ms: float


def _dev_ptr(t: Optional[torch.Tensor], n: int, name: str, dtype=torch.float64):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor with {n} entries")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# Library objects still open when the interpreter exits are closed by an exit handler, while the HIP
# runtime is intact: batches first (they refer to solvers), then networks, then solvers.  Finalizers
# make no library call once the interpreter is shutting down.
_OPEN = {"batch": weakref.WeakSet(), "net": weakref.WeakSet(), "solver": weakref.WeakSet()}


@atexit.register
def _close_all():
    for kind in ("batch", "net", "solver"):
        for obj in list(_OPEN[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _finalize(obj, _is_finalizing=sys.is_finalizing):
    if _is_finalizing():
        return
    try:
        obj.close()
    except Exception:
        pass


class Solver:
    """``rebk_create`` on a CUDA tensor A (m x n, float64 or float32, row-major).

    row_offsets / col_offsets: the contiguous partitions (s+1 and t+1 offsets).  panel_dtype
    chooses the stored precision of the dual panel layout ("f64", "f32", "bf16", "f16").
    """

    def __init__(self, A: torch.Tensor, row_offsets: Sequence[int], col_offsets: Sequence[int],
                 alpha: float, seed: int = 0, panel_dtype: str = "f64"):
        lib = N.load()
        if A.dim() != 2 or not A.is_cuda or A.dtype not in (torch.float64, torch.float32):
            raise ValueError("A must be a 2-D CUDA float64/float32 tensor")
        if A.stride(1) != 1:
            raise ValueError("A must be row-major with unit column stride")
        if panel_dtype not in N.DTYPES:
            raise ValueError(f"panel_dtype must be one of {sorted(N.DTYPES)}")
        self.m, self.n = int(A.shape[0]), int(A.shape[1])
        ro = np.ascontiguousarray(row_offsets, dtype=np.int64)
        co = np.ascontiguousarray(col_offsets, dtype=np.int64)
        self.row_offsets, self.col_offsets = ro, co
        self.s, self.t = len(ro) - 1, len(co) - 1
        self.alpha, self.seed, self.panel_dtype = float(alpha), int(seed), panel_dtype
        h = ctypes.c_void_p()
        a_dt = N.F64_T if A.dtype == torch.float64 else N.F32_T
        code = lib.rebk_create(ctypes.byref(h), ctypes.c_void_p(A.data_ptr()), a_dt, N.DTYPES[panel_dtype],
                               self.m, self.n, int(A.stride(0)),
                               ro.ctypes.data_as(ctypes.c_void_p), self.s,
                               co.ctypes.data_as(ctypes.c_void_p), self.t,
                               self.alpha, ctypes.c_uint64(self.seed), _stream_ptr())
        N.check(code, "rebk_create")
        self._h = h
        self.device = A.device
        _OPEN["solver"].add(self)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            N.load().rebk_destroy(self._h)
            self._h = ctypes.c_void_p()

    def pipe_prepare(self) -> float:
        """``rebk_pipe_prepare``: build the pipelined kernel's Gram matrices now; returns the build
        time in ms (0 when already built)."""
        ms = ctypes.c_double(0.0)
        N.check(N.load().rebk_pipe_prepare(self._h, ctypes.byref(ms)), "rebk_pipe_prepare")
        return ms.value

    def pipe_release(self):
        """``rebk_pipe_release``: free the pipelined kernel's Gram matrices."""
        N.load().rebk_pipe_release(self._h)

    def __del__(self, _fin=_finalize):  # bound at definition: module globals are gone at shutdown
        _fin(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ queries
    def weights(self):
        w_row = np.zeros(self.s)
        w_col = np.zeros(self.t)
        N.check(N.load().rebk_get_weights(self._h, w_row.ctypes.data_as(ctypes.c_void_p),
                                          w_col.ctypes.data_as(ctypes.c_void_p)), "rebk_get_weights")
        return w_row, w_col

    def thresholds(self):
        T_row = np.zeros(self.s, dtype=np.uint64)
        T_col = np.zeros(self.t, dtype=np.uint64)
        N.check(N.load().rebk_get_thresholds(self._h, T_row.ctypes.data_as(ctypes.c_void_p),
                                             T_col.ctypes.data_as(ctypes.c_void_p)), "rebk_get_thresholds")
        return T_row, T_col

    def info(self):
        vals = [ctypes.c_int64() for _ in range(6)]
        N.check(N.load().rebk_get_info(self._h, *[ctypes.byref(v) for v in vals]), "rebk_get_info")
        keys = ["m", "n", "s", "t", "max_row_block", "max_col_block"]
        return {k: v.value for k, v in zip(keys, vals)}

    def sample_blocks(self, k0: int, count: int, system: int = 0):
        """Device sampler: 0-based (j, i) of iterations k0+1 .. k0+count, as int32 CUDA tensors."""
        j = torch.empty(count, dtype=torch.int32, device=self.device)
        i = torch.empty(count, dtype=torch.int32, device=self.device)
        N.check(N.load().rebk_sample_blocks(self._h, ctypes.c_uint64(system), int(k0), int(count),
                                            ctypes.c_void_p(j.data_ptr()), ctypes.c_void_p(i.data_ptr())),
                "rebk_sample_blocks")
        return j, i

    # ------------------------------------------------------------------ solves
    def solve(self, b: torch.Tensor, x0: Optional[torch.Tensor] = None, tol: float = 1e-6,
              max_iter: int = 100000):
        """``rebk_solve``: residual stop rule, z^0 = b.  Returns (x, SolveResult)."""
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        res = N.Result()
        code = N.load().rebk_solve(self._h, _dev_ptr(b, self.m, "b"), _dev_ptr(x0, self.n, "x0"),
                                   _dev_ptr(x, self.n, "x"), float(tol), int(max_iter), ctypes.byref(res))
        N.check(code, "rebk_solve")
        return x, self._result(res)

    def solve_ex(self, b: torch.Tensor, *, x0=None, z0=None, k0: int = 0, max_iter: int = 100000,
                 x_ref=None, tol: float = 0.0, check_every: int = 0, trace: bool = False,
                 kernel: str = "auto", grid_wgs: int = 0, x_out=None, z_out=None, static_workspace: bool = False):
        """``rebk_solve_ex`` (``rebk_solve_ex_static`` with static_workspace: the library allocates
        nothing; pass x_out / z_out to allocate nothing here either).  Returns dict(x, z, result, j,
        i) (j, i: traces when requested)."""
        x = x_out if x_out is not None else torch.empty(self.n, dtype=torch.float64, device=self.device)
        z = z_out if z_out is not None else torch.empty(self.m, dtype=torch.float64, device=self.device)
        tj = ti = None
        if trace:
            tj = torch.full((max_iter,), -1, dtype=torch.int32, device=self.device)
            ti = torch.full((max_iter,), -1, dtype=torch.int32, device=self.device)
        o = N.SolveOpts()
        o.b_dev = _dev_ptr(b, self.m, "b")
        o.x0_dev = _dev_ptr(x0, self.n, "x0")
        o.z0_dev = _dev_ptr(z0, self.m, "z0")
        o.k0 = int(k0)
        o.max_iter = int(max_iter)
        o.x_ref_dev = _dev_ptr(x_ref, self.n, "x_ref")
        o.tol = float(tol)
        o.check_every = int(check_every)
        o.x_out_dev = _dev_ptr(x, self.n, "x_out")
        o.z_out_dev = _dev_ptr(z, self.m, "z_out")
        o.trace_j_dev = _dev_ptr(tj, max_iter, "trace_j", torch.int32)
        o.trace_i_dev = _dev_ptr(ti, max_iter, "trace_i", torch.int32)
        o.kernel = N.KERNELS[kernel]
        o.grid_wgs = int(grid_wgs)
        res = N.Result()
        fn = "rebk_solve_ex_static" if static_workspace else "rebk_solve_ex"
        code = getattr(N.load(), fn)(self._h, ctypes.byref(o), ctypes.byref(res))
        N.check(code, fn)
        r = self._result(res)
        out = {"x": x, "z": z, "result": r}
        if trace:
            out["j"] = tj[: r.iterations]
            out["i"] = ti[: r.iterations]
        return out

    def block_betas(self, max_steps: int = 5000, rtol: float = 1e-13):
        """``rebk_block_betas``: (beta_row (s,), beta_col (t,), beta_max, steps) of the stored panels."""
        br = np.zeros(self.s)
        bc = np.zeros(self.t)
        bm = ctypes.c_double()
        steps = ctypes.c_int32()
        N.check(N.load().rebk_block_betas(self._h, int(max_steps), float(rtol), br.ctypes.data_as(ctypes.c_void_p),
                                          bc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(bm), ctypes.byref(steps)),
                "rebk_block_betas")
        return br, bc, float(bm.value), int(steps.value)

    def suggest_alpha(self, c: float = 1.0, **kw) -> float:
        """alpha = c / beta_max (Remark 9: c = 1 is the paper's default; any 0 < c < 2 converges)."""
        return float(c) / self.block_betas(**kw)[2]

    def solve_refined(self, A64: torch.Tensor, b: torch.Tensor, *, x0=None, x_ref=None, tol: float = 1e-10,
                      inner_iters: int = 1000, max_outer: int = 20, kernel: str = "auto", grid_wgs: int = 0,
                      x_out=None, z_out=None):
        """``rebk_solve_refined``: FP64 refinement of the augmented system around REBK on this
        solver's panels.  A64 is the FP64 matrix (CUDA, row-major).  Returns dict(x, z, result,
        err_trace (numpy, one entry per tested outer step))."""
        if not (A64.is_cuda and A64.dtype == torch.float64 and A64.dim() == 2 and A64.stride(1) == 1
                and tuple(A64.shape) == (self.m, self.n)):
            raise ValueError("A64 must be a row-major CUDA float64 tensor of the solver's shape")
        x = x_out if x_out is not None else torch.empty(self.n, dtype=torch.float64, device=self.device)
        z = z_out if z_out is not None else torch.empty(self.m, dtype=torch.float64, device=self.device)
        trace = np.full(int(max_outer) + 1, np.nan)
        o = N.RefineOpts()
        o.A_dev = ctypes.c_void_p(A64.data_ptr())
        o.lda = int(A64.stride(0))
        o.b_dev = _dev_ptr(b, self.m, "b")
        o.x0_dev = _dev_ptr(x0, self.n, "x0")
        o.x_ref_dev = _dev_ptr(x_ref, self.n, "x_ref")
        o.tol = float(tol)
        o.inner_iters = int(inner_iters)
        o.max_outer = int(max_outer)
        o.kernel = N.KERNELS[kernel]
        o.grid_wgs = int(grid_wgs)
        o.x_out_dev = _dev_ptr(x, self.n, "x_out")
        o.z_out_dev = _dev_ptr(z, self.m, "z_out")
        o.err_trace = trace.ctypes.data_as(ctypes.c_void_p)
        res = N.Result()
        code = N.load().rebk_solve_refined(self._h, ctypes.byref(o), ctypes.byref(res))
        N.check(code, "rebk_solve_refined")
        r = self._result(res)
        return {"x": x, "z": z, "result": r, "err_trace": trace[~np.isnan(trace)]}

    @staticmethod
    def _result(res: "N.Result") -> SolveResult:
        return SolveResult(status=N.STATUS_NAMES.get(res.status, str(res.status)), code=int(res.status),
                           kernel=N.KERNEL_NAMES.get(res.kernel, str(res.kernel)), iterations=int(res.iterations),
                           rel_err=float(res.rel_err), time_ms=float(res.time_ms))


class Batch:
    """``rebk_batch_create`` over existing solvers (same panel type): independent systems, each
    with several right-hand sides, solved in one launch.  System s draws its blocks from the
    Philox stream of ``sys_ids[s]`` (default s).  Close the batch before its solvers."""

    def __init__(self, solvers: Sequence[Solver], sys_ids: Optional[Sequence[int]] = None):
        lib = N.load()
        self.solvers = list(solvers)
        self.nsys = len(self.solvers)
        hs = (ctypes.c_void_p * self.nsys)(*[sv._h.value for sv in self.solvers])
        ids = None
        if sys_ids is not None:
            self._ids = (ctypes.c_uint64 * self.nsys)(*[int(v) for v in sys_ids])
            ids = ctypes.cast(self._ids, ctypes.c_void_p)
        b = ctypes.c_void_p()
        N.check(lib.rebk_batch_create(ctypes.byref(b), self.nsys, ctypes.cast(hs, ctypes.c_void_p), ids,
                                      _stream_ptr()), "rebk_batch_create")
        self._b = b
        _OPEN["batch"].add(self)

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            N.load().rebk_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self, _fin=_finalize):  # bound at definition: module globals are gone at shutdown
        _fin(self)

    def _opts(self, B, x_ref, x0, x_out, z_out, max_iter, tol, check_every, threads, lds_budget, max_tile,
              xcd_order, z0_from_x0=False, team=0):
        """B[s]: (nrhs_s, m_s) float64 CUDA tensors; x_ref / x0 (optional) and x_out: (nrhs_s, n_s)."""
        if len(B) != self.nsys:
            raise ValueError("one right-hand-side matrix per system")
        keep = []

        def ptrs(lst, rows, cols_of, name, optional_entries=False):
            if lst is None:
                return None
            arr = (ctypes.c_void_p * self.nsys)()
            for s, t in enumerate(lst):
                if t is None and optional_entries:
                    arr[s] = None
                    continue
                shape = (rows[s], cols_of(s))
                if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
                    raise ValueError(f"{name}[{s}] must be a contiguous CUDA float64 tensor of shape {shape}")
                arr[s] = t.data_ptr()
            keep.append(arr)
            return ctypes.cast(arr, ctypes.c_void_p)

        nrhs = [int(b.shape[0]) for b in B]
        nr = (ctypes.c_int32 * self.nsys)(*nrhs)
        keep.append(nr)
        o = N.BatchOpts()
        o.nrhs = ctypes.cast(nr, ctypes.c_void_p)
        o.b_dev = ptrs(B, nrhs, lambda s: self.solvers[s].m, "B")
        o.x0_dev = ptrs(x0, nrhs, lambda s: self.solvers[s].n, "x0", True)
        o.x_ref_dev = ptrs(x_ref, nrhs, lambda s: self.solvers[s].n, "x_ref")
        o.x_out_dev = ptrs(x_out, nrhs, lambda s: self.solvers[s].n, "x_out")
        o.z_out_dev = ptrs(z_out, nrhs, lambda s: self.solvers[s].m, "z_out")
        o.max_iter = int(max_iter)
        o.tol = float(tol)
        o.check_every = int(check_every)
        o.threads = int(threads)
        o.lds_budget = int(lds_budget)
        o.max_tile = int(max_tile)
        o.xcd_order = int(xcd_order)
        o.z0_from_x0 = 1 if z0_from_x0 else 0
        o.team = int(team)
        return o, nrhs, keep

    def solve(self, B, *, x_ref=None, x0=None, max_iter: int = 100000, tol: float = 0.0, check_every: int = 0,
              threads: int = 0, lds_budget: int = 0, max_tile: int = 0, xcd_order: int = -1, want_z: bool = False,
              z0_from_x0: bool = False, team: int = 0):
        """``rebk_batch_solve``.  Returns dict(x=[...], z=[...] or None, iterations, rel_err, status, tile,
        team (numpy arrays over all right-hand sides, system after system), time_ms, code).  team: 0
        automatic, -1 never, P > 0 every system in teams of P workgroups."""
        dev = self.solvers[0].device
        x_out = [torch.empty((int(b.shape[0]), sv.n), dtype=torch.float64, device=dev)
                 for b, sv in zip(B, self.solvers)]
        z_out = ([torch.empty((int(b.shape[0]), sv.m), dtype=torch.float64, device=dev)
                  for b, sv in zip(B, self.solvers)] if want_z else None)
        o, nrhs, keep = self._opts(B, x_ref, x0, x_out, z_out, max_iter, tol, check_every, threads, lds_budget,
                                   max_tile, xcd_order, z0_from_x0, team)
        total = sum(nrhs)
        res = (N.BatchRhs * total)()
        ms = ctypes.c_double(0.0)
        code = N.load().rebk_batch_solve(self._b, ctypes.byref(o), ctypes.cast(res, ctypes.c_void_p),
                                         ctypes.byref(ms))
        N.check(code, "rebk_batch_solve")
        del keep
        return {
            "x": x_out, "z": z_out, "code": code, "status": N.STATUS_NAMES.get(code, str(code)),
            "time_ms": float(ms.value),
            "iterations": np.array([r.iterations for r in res], dtype=np.int64),
            "rel_err": np.array([r.rel_err for r in res]),
            "rhs_status": np.array([r.status for r in res], dtype=np.int32),
            "tile": np.array([r.tile for r in res], dtype=np.int32),
            "team": np.array([r.team for r in res], dtype=np.int32),
        }

    def autotune(self, B, *, x_ref=None, probe_iters: int = 64):
        """``rebk_batch_autotune``: returns dict(threads, lds_budget, max_tile, xcd_order, ms)."""
        dev = self.solvers[0].device
        x_out = [torch.empty((int(b.shape[0]), sv.n), dtype=torch.float64, device=dev)
                 for b, sv in zip(B, self.solvers)]
        o, _, keep = self._opts(B, x_ref, None, x_out, None, probe_iters, 0.0, 0, 0, 0, 0, -1)
        th, ld, tl, xo = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        N.check(N.load().rebk_batch_autotune(self._b, ctypes.byref(o), int(probe_iters), ctypes.byref(th),
                                             ctypes.byref(ld), ctypes.byref(tl), ctypes.byref(xo), ctypes.byref(ms)),
                "rebk_batch_autotune")
        del keep
        return {"threads": th.value, "lds_budget": ld.value, "max_tile": tl.value, "xcd_order": xo.value,
                "ms": ms.value}


class WarmStart:
    """``rebk_mlp_*``: the learned warm start network in_dim -> hidden -> hidden -> m for A (m x n,
    CUDA float64).  forward(B) gives rows x0 = out_scale A^T y (out_scale defaults to 1/sqrt(m));
    grad / adam / train_step train it."""

    NAMES = ("W1", "c1", "W2", "c2", "W3", "c3")

    def __init__(self, A: torch.Tensor, in_dim: int, hidden: int = 512, max_batch: int = 256, seed: int = 0,
                 out_scale: Optional[float] = None):
        if not (A.is_cuda and A.dtype == torch.float64 and A.dim() == 2 and A.is_contiguous()):
            raise ValueError("A must be a contiguous CUDA float64 matrix")
        self.m, self.n = int(A.shape[0]), int(A.shape[1])
        self.in_dim, self.hidden, self.max_batch = int(in_dim), int(hidden), int(max_batch)
        self.device = A.device
        self.out_scale = float(out_scale) if out_scale is not None else 1.0 / np.sqrt(self.m)
        w = ctypes.c_void_p()
        N.check(N.load().rebk_mlp_create(ctypes.byref(w), self.in_dim, self.hidden, ctypes.c_void_p(A.data_ptr()),
                                         self.m, self.n, self.out_scale, self.max_batch, ctypes.c_uint64(int(seed)),
                                         _stream_ptr()),
                "rebk_mlp_create")
        self._w = w
        _OPEN["net"].add(self)

    def shapes(self):
        h, i, m = self.hidden, self.in_dim, self.m
        return {"W1": (h, i), "c1": (h,), "W2": (h, h), "c2": (h,), "W3": (m, h), "c3": (m,)}

    def close(self):
        if getattr(self, "_w", None) and self._w.value:
            N.load().rebk_mlp_destroy(self._w)
            self._w = ctypes.c_void_p()

    def __del__(self, _fin=_finalize):  # bound at definition: module globals are gone at shutdown
        _fin(self)

    def set_params(self, params: dict):
        arrs = [np.ascontiguousarray(params[k], dtype=np.float32) if k in params else None for k in self.NAMES]
        for k, a in zip(self.NAMES, arrs):
            if a is not None and a.shape != self.shapes()[k]:
                raise ValueError(f"{k} must have shape {self.shapes()[k]}")
        ptrs = [a.ctypes.data_as(ctypes.c_void_p) if a is not None else None for a in arrs]
        N.check(N.load().rebk_mlp_set_params(self._w, *ptrs), "rebk_mlp_set_params")

    def _get(self, fn, where):
        out = {k: np.zeros(s, dtype=np.float32) for k, s in self.shapes().items()}
        N.check(fn(self._w, *[out[k].ctypes.data_as(ctypes.c_void_p) for k in self.NAMES]), where)
        return out

    def params(self):
        return self._get(N.load().rebk_mlp_get_params, "rebk_mlp_get_params")

    def grads(self):
        return self._get(N.load().rebk_mlp_get_grads, "rebk_mlp_get_grads")

    def _batch(self, B):
        if not (B.is_cuda and B.dtype == torch.float64 and B.is_contiguous() and B.dim() == 2
                and B.shape[1] == self.in_dim):
            raise ValueError("B must be a contiguous CUDA float64 (batch, in_dim) tensor")
        return int(B.shape[0])

    def forward(self, B: torch.Tensor, b_scale: float = 1.0, want_y: bool = False):
        batch = self._batch(B)
        X0 = torch.empty((batch, self.n), dtype=torch.float64, device=self.device)
        Y = torch.empty((batch, self.m), dtype=torch.float64, device=self.device) if want_y else None
        N.check(N.load().rebk_mlp_forward(self._w, ctypes.c_void_p(B.data_ptr()), batch, float(b_scale),
                                          ctypes.c_void_p(X0.data_ptr()),
                                          ctypes.c_void_p(Y.data_ptr()) if Y is not None else None),
                "rebk_mlp_forward")
        return (X0, Y) if want_y else X0

    def grad(self, B: torch.Tensor, Xt: torch.Tensor, b_scale: float = 1.0) -> float:
        batch = self._batch(B)
        if not (Xt.is_cuda and Xt.dtype == torch.float64 and Xt.is_contiguous() and tuple(Xt.shape) == (batch, self.n)):
            raise ValueError("Xt must be a contiguous CUDA float64 (batch, n) tensor")
        loss = ctypes.c_double()
        N.check(N.load().rebk_mlp_grad(self._w, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(Xt.data_ptr()), batch,
                                       float(b_scale), ctypes.byref(loss)), "rebk_mlp_grad")
        return float(loss.value)

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        N.check(N.load().rebk_mlp_adam(self._w, float(lr), float(beta1), float(beta2), float(eps)), "rebk_mlp_adam")

    def train_step(self, B: torch.Tensor, Xt: torch.Tensor, lr: float, b_scale: float = 1.0) -> float:
        batch = self._batch(B)
        loss = ctypes.c_double()
        N.check(N.load().rebk_mlp_train_step(self._w, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(Xt.data_ptr()),
                                             batch, float(b_scale), float(lr), ctypes.byref(loss)),
                "rebk_mlp_train_step")
        return float(loss.value)


def philox4x64_10(counter: Sequence[int], key: Sequence[int], count: int, device="cuda") -> torch.Tensor:
    """Device Philox4x64-10 words for counters (c0+q, c1, c2, c3), q < count: uint64 as int64 (count, 4)."""
    out = torch.empty((count, 4), dtype=torch.int64, device=device)
    c = [ctypes.c_uint64(int(v)) for v in counter]
    k = [ctypes.c_uint64(int(v)) for v in key]
    N.check(N.load().rebk_philox4x64_10(*c, *k, int(count), ctypes.c_void_p(out.data_ptr()), _stream_ptr()),
            "rebk_philox4x64_10")
    return out
