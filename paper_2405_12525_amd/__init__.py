"""MI355X level-blocked matrix power kernel (Python binding of libmpk.so).

Computes y_k = A^k x for k = 1..p (all powers kept) for a CSR matrix A, as
in Lacey et al., "Cache Blocking of Distributed-Memory Parallel Matrix Power
Kernels": the level-blocked kernel (Sec. "RACE Applied to the Matrix Power
Kernel"; localLBMPK of Alg. 2 on one process) and its p x SpMV baseline
(Alg. 1 without halo exchange), plus the Chebyshev-style three-term
recurrence of Eq. (anderson_spmv).  Every step runs in the HIP kernels of
libmpk.so; this module only marshals arguments.  PyTorch supplies device
memory and streams.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi
from ._capi import (MPK_DEVICE_CURRENT, MPK_DEVICE_NONE, MPK_ORDER_ORIGINAL, MPK_ORDER_PLAN,
                    MPK_REORDER_BFS, MPK_REORDER_NONE, MPK_REORDER_SUBLEVELS, MPK_ROOT_AUTO, MPK_SCHED_DIAG, MPK_SCHED_POWERS,
                    MPK_SCHED_STEPS, MPK_SCHED_WAVE, MPK_SCHED_XCD, MPKError, check)

__all__ = ["Plan", "MPKError", "version", "MPK_ORDER_ORIGINAL", "MPK_ORDER_PLAN",
           "MPK_REORDER_BFS", "MPK_REORDER_NONE", "MPK_REORDER_SUBLEVELS", "MPK_ROOT_AUTO", "MPK_SCHED_STEPS", "MPK_SCHED_WAVE", "MPK_SCHED_DIAG",
           "MPK_SCHED_POWERS", "MPK_SCHED_XCD", "use_torch_allocator", "MPK_DEVICE_NONE", "MPK_DEVICE_CURRENT", "chebyshev_coefficients",
           "cheb_time_coefficients",
           "flops", "lib", "probe_load", "probe_load_xcd"]

_SCHED = {"steps": MPK_SCHED_STEPS, "wave": MPK_SCHED_WAVE, "diag": MPK_SCHED_DIAG,
          "powers": MPK_SCHED_POWERS, "xcd": MPK_SCHED_XCD}


def lib():
    return _capi.load()


def version() -> str:
    return lib().mpk_version().decode()


def chebyshev_coefficients(p: int):
    """Coefficients of v_1 = H v_0, v_{k+1} = 2 H v_k - v_{k-1} for mpk_run_recur."""
    a = np.full(p, 2.0)
    a[0] = 1.0
    g = np.full(p, -1.0)
    g[0] = 0.0
    return a, np.zeros(p), g


def cheb_time_coefficients(M: int, dt: float):
    """alpha, beta, gamma (M each) and the weights wa, wb (M + 1 each) of one
    Chebyshev time step exp(-i dt H) (mpk_cheb_time_coefficients)."""
    L = lib()
    a, b, g = np.empty(M), np.empty(M), np.empty(M)
    wa, wb = np.empty(M + 1), np.empty(M + 1)
    check(L.mpk_cheb_time_coefficients(int(M), float(dt), a.ctypes.data, b.ctypes.data,
                                       g.ctypes.data, wa.ctypes.data, wb.ctypes.data))
    return a, b, g, wa, wb


def flops(nnz: int, n: int, p: int, nrhs: int, recur: bool = False) -> float:
    """2 flops per nonzero and right-hand side per power (plus the recurrence update)."""
    f = 2.0 * nnz * nrhs * p
    if recur:
        f += 2.0 * n * nrhs * max(0, p - 1)
    return f


def probe_load(buf, passes: int = 1, workgroups: int = 2048, sink=None, stream=None):
    """Launch the load-only bandwidth probe over a float64 device tensor."""
    torch = _torch()
    if buf.dtype != torch.float64 or not buf.is_contiguous() or not buf.is_cuda:
        raise TypeError("buf must be a contiguous float64 device tensor")
    if sink is None:
        sink = torch.empty(workgroups, dtype=torch.float64, device=buf.device)
    check(lib().mpk_probe_load(ctypes.c_void_p(buf.data_ptr()), buf.numel(), int(passes),
                               int(workgroups), ctypes.c_void_p(sink.data_ptr()),
                               _stream_handle(stream)))
    return sink


def probe_load_xcd(buf, regions: int = 8, passes: int = 1, workgroups: int = 2048, sink=None,
                   xcc=None, stream=None):
    """XCD-local load probe (mpk_probe_load_xcd): each workgroup reads the
    part of buf belonging to the XCD it runs on.  Returns (sink, xcc)."""
    torch = _torch()
    if buf.dtype != torch.float64 or not buf.is_contiguous() or not buf.is_cuda:
        raise TypeError("buf must be a contiguous float64 device tensor")
    if sink is None:
        sink = torch.empty(workgroups, dtype=torch.float64, device=buf.device)
    if xcc is None:
        xcc = torch.empty(workgroups, dtype=torch.int32, device=buf.device)
    check(lib().mpk_probe_load_xcd(ctypes.c_void_p(buf.data_ptr()), buf.numel(), int(regions),
                                   int(passes), int(workgroups), ctypes.c_void_p(sink.data_ptr()),
                                   ctypes.c_void_p(xcc.data_ptr()), _stream_handle(stream)))
    return sink, xcc


def _torch():
    import torch
    return torch


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_hooks = None                       # the installed callbacks (kept alive here)
allocator_stats = {"allocs": 0, "frees": 0, "bytes": 0}


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device allocations (plan data, schedules,
    workspaces) through PyTorch's caching allocator (mpk_set_allocator);
    enable=False restores hipMalloc / hipFree.  Buffers keep the free function
    they were allocated with."""
    global _hooks
    if not enable:
        check(lib().mpk_set_allocator(None, None, None))
        return
    torch = _torch()

    def _alloc(nbytes, ctx):
        try:
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device())
        except Exception:
            return None
        allocator_stats["allocs"] += 1
        allocator_stats["bytes"] += int(nbytes)
        return ptr

    def _free(ptr, ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)
            allocator_stats["frees"] += 1

    hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    check(lib().mpk_set_allocator(ctypes.cast(hooks[0], ctypes.c_void_p),
                                  ctypes.cast(hooks[1], ctypes.c_void_p), None))
    # earlier hooks stay referenced: buffers allocated with them free through them
    _hooks = (hooks, _hooks)


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _vec_check(t, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.shape[0] != n:
        raise ValueError(f"{name} has {t.shape[0]} rows, expected {n}")


class Plan:
    """A preprocessed matrix resident on one device (or host-only).

    ``A`` is any object with ``n``, ``rowptr`` (int32), ``col`` (int32) and
    ``val`` (float64) attributes, e.g. :class:`workloads.CSR`.  When they are
    device tensors the plan is built on the device (mpk_plan_device).
    """

    def __init__(self, A, value_bits: int = 64, reorder: str = "bfs", order: str = "original",
                 root=0, device=MPK_DEVICE_CURRENT, l2_bytes: int = 0, mall_bytes: int = 0,
                 min_group_rows: int = 0, sublevel_root: int = MPK_ROOT_AUTO):
        """reorder: "bfs" (levels from `root`, or root="peripheral"), "none"
        (the caller's order) or "sublevels" (BFS levels, each ordered by the
        distance from `sublevel_root`, -1 = automatic).  l2_bytes /
        mall_bytes / min_group_rows: planner budgets (0 = defaults)."""
        L = lib()
        self._lib = L
        self._h = ctypes.c_void_p()
        on_device = getattr(A.rowptr, "is_cuda", False)
        if on_device:
            torch = _torch()
            rowptr, col, val = A.rowptr, A.col, A.val
            for t, dt, name in ((rowptr, torch.int32, "rowptr"), (col, torch.int32, "col"),
                                (val, torch.float64, "val")):
                if t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
                    raise TypeError(f"{name} must be a contiguous {dt} device tensor")
            nnz = int(col.numel())
            csr = _capi.CSRStruct(int(A.n), nnz, rowptr.data_ptr(),
                                  col.data_ptr() if nnz else None, val.data_ptr() if nnz else None)
        else:
            rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int32)
            col = np.ascontiguousarray(A.col, dtype=np.int32)
            val = None if A.val is None else np.ascontiguousarray(A.val, dtype=np.float64)
            csr = _capi.CSRStruct(int(A.n), int(rowptr[-1]) if rowptr.size else 0,
                                  rowptr.ctypes.data, col.ctypes.data if col.size else None,
                                  val.ctypes.data if (val is not None and val.size) else None)
        opts = _capi.PlanOpts()
        L.mpk_plan_opts_default(ctypes.byref(opts))
        opts.value_bits = int(value_bits)
        opts.reorder = {"bfs": MPK_REORDER_BFS, "none": MPK_REORDER_NONE,
                        "sublevels": MPK_REORDER_SUBLEVELS}[reorder]
        opts.order = {"original": MPK_ORDER_ORIGINAL, "plan": MPK_ORDER_PLAN}[order]
        opts.root = -1 if root == "peripheral" else int(root)   # MPK_ROOT_PERIPHERAL
        opts.l2_bytes = int(l2_bytes)
        opts.mall_bytes = int(mall_bytes)
        opts.min_group_rows = int(min_group_rows)
        opts.sublevel_root = int(sublevel_root)
        if device is None or device == "none":
            device = MPK_DEVICE_NONE
        opts.device = int(device)
        make = L.mpk_plan_device if on_device else L.mpk_plan
        check(make(ctypes.byref(csr), ctypes.byref(opts), ctypes.byref(self._h)))
        self.n = int(A.n)
        self.nnz = int(csr.nnz)
        self.order = order
        self.host_only = opts.device == MPK_DEVICE_NONE
        self._tune = self.default_tune()
        self._tune["cache_bytes"] = self.info()["mall_bytes"]   # the plan's budget C

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.mpk_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ queries
    def info(self) -> dict:
        i = _capi.PlanInfo()
        check(self._lib.mpk_plan_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _capi.PlanInfo._fields_}

    def levels(self):
        """(level_ptr, perm) with perm[new] = old."""
        nl = self.info()["n_levels"]
        lp = np.zeros(nl + 1, dtype=np.int32)
        perm = np.zeros(self.n, dtype=np.int32)
        check(self._lib.mpk_plan_levels(self._h, lp.ctypes.data, perm.ctypes.data))
        return lp, perm

    def schedule(self, p: int) -> dict:
        si = _capi.SchedInfo()
        check(self._lib.mpk_plan_schedule(self._h, int(p), ctypes.byref(si), None, None, None,
                                          None, None, None))
        nc, nt = si.n_chunks, si.n_tasks
        cp = np.zeros(nc + 1, np.int32)
        cg = np.zeros(nc, np.int32)
        lo = np.zeros(nc, np.int32)
        hi = np.zeros(nc, np.int32)
        tasks = np.zeros(2 * nt, np.int32)
        sp = np.zeros(si.n_steps + 1, np.int32)
        check(self._lib.mpk_plan_schedule(self._h, int(p), ctypes.byref(si), cp.ctypes.data,
                                          cg.ctypes.data, lo.ctypes.data, hi.ctypes.data,
                                          tasks.ctypes.data, sp.ctypes.data))
        d = {f: getattr(si, f) for f, _ in _capi.SchedInfo._fields_}
        d.update(chunk_ptr=cp, chunk_group=cg, dep_lo=lo, dep_hi=hi, tasks=tasks.reshape(-1, 2),
                 step_ptr=sp)
        if si.n_deps > 0:
            dp = np.zeros(nc + 1, np.int32)
            di = np.zeros(si.n_deps, np.int32)
            cx = np.zeros(nc, np.int32)
            ro = np.zeros(nc, np.int32)
            qp = np.zeros(si.n_queues + 1, np.int32)
            check(self._lib.mpk_plan_schedule_xcd(self._h, int(p), dp.ctypes.data, di.ctypes.data,
                                                  cx.ctypes.data, ro.ctypes.data, qp.ctypes.data))
            d.update(dep_ptr=dp, dep_idx=di, chunk_xcd=cx, remote_out=ro, qptr=qp)
        return d

    # ------------------------------------------------------------ tuning
    @staticmethod
    def default_tune() -> dict:
        t = _capi.Tune()
        lib().mpk_tune_default(ctypes.byref(t))
        d = {f: getattr(t, f) for f, _ in _capi.Tune._fields_}
        d["schedule"] = {v: k for k, v in _SCHED.items()}[d["schedule"]]
        return d

    def tune(self, **kw) -> dict:
        d = dict(self._tune)
        for k, v in kw.items():
            if k not in d:
                raise KeyError(k)
            d[k] = v
        t = _capi.Tune()
        for f, _ in _capi.Tune._fields_:
            v = d[f]
            if f == "schedule" and isinstance(v, str):
                v = _SCHED[v]
            setattr(t, f, v)
        check(self._lib.mpk_plan_tune(self._h, ctypes.byref(t)))
        self._tune = d
        return dict(d)

    @property
    def tuning(self) -> dict:
        return dict(self._tune)

    def autotune(self, x, p: int, Y=None, reps: int = 3, force: bool = False, recur: bool = False,
                 stream=None) -> dict:
        """Time the candidate tunings for (p, nrhs) and keep the fastest
        (mpk_plan_autotune).  recur: False = the plain run, True = the
        recurrence, 2 = the weighted sums of run_poly.  Y is scratch.  Returns
        the tuning plus "ms"."""
        R, Y = self._prep(x, p, Y)
        t = _capi.Tune()
        ms = ctypes.c_double(0.0)
        check(self._lib.mpk_plan_autotune(self._h, ctypes.c_void_p(x.data_ptr()), int(p), R,
                                          ctypes.c_void_p(Y.data_ptr()), int(reps), int(force),
                                          int(recur), _stream_handle(stream), ctypes.byref(t),
                                          ctypes.byref(ms)))
        d = {f: getattr(t, f) for f, _ in _capi.Tune._fields_}
        d["schedule"] = {v: k for k, v in _SCHED.items()}[d["schedule"]]
        self._tune = {k: v for k, v in d.items()}
        out = dict(d)
        out["ms"] = ms.value
        return out

    def capture(self, x, p: int, Y=None, alpha=None, beta=None, gamma=None) -> "Graph":
        """Capture one run (mpk_graph_capture) for repeated launches with the
        same tensors; recurrence when alpha is given."""
        R, Y = self._prep(x, p, Y)
        keep = []
        ptrs = [None, None, None]
        if alpha is not None:
            for i, c in enumerate((alpha, beta, gamma)):
                a = np.ascontiguousarray(c, dtype=np.float64)
                if a.shape != (p,):
                    raise ValueError("coefficient arrays must have length p")
                keep.append(a)
                ptrs[i] = ctypes.c_void_p(a.ctypes.data)
        h = ctypes.c_void_p()
        check(self._lib.mpk_graph_capture(self._h, ctypes.c_void_p(x.data_ptr()), int(p), R,
                                          ptrs[0], ptrs[1], ptrs[2],
                                          ctypes.c_void_p(Y.data_ptr()), ctypes.byref(h)))
        return Graph(h, self, (x, Y))

    def capture_time_step(self, psi, dt: float, M: int, out=None, baseline: bool = False) -> "Graph":
        """Capture one Chebyshev time step psi -> out (mpk_graph_capture_time_step);
        Graph.launch() returns out.  Scratch for the ring and the sums is
        allocated here and kept by the graph."""
        torch = _torch()
        _vec_check(psi, self.n, "psi")
        if psi.dim() != 2 or psi.shape[1] % 2:
            raise ValueError("psi must be (n, 2m): real and imaginary columns")
        R = int(psi.shape[1])
        if out is None:
            out = torch.empty_like(psi)
        acc = torch.empty((2, self.n, R), dtype=torch.float64, device=psi.device)
        work = torch.empty((2, self.n, R), dtype=torch.float64, device=psi.device)
        h = ctypes.c_void_p()
        check(self._lib.mpk_graph_capture_time_step(
            self._h, ctypes.c_void_p(psi.data_ptr()), R, float(dt), int(M), int(bool(baseline)),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(acc.data_ptr()),
            ctypes.c_void_p(work.data_ptr()), ctypes.byref(h)))
        return Graph(h, self, (psi, out, acc, work))

    # ------------------------------------------------------------ runs
    def _prep(self, x, p, Y):
        torch = _torch()
        _vec_check(x, self.n, "x")
        R = 1 if x.dim() == 1 else int(x.shape[1])
        if Y is None:
            Y = torch.empty((p, self.n, R), dtype=torch.float64, device=x.device)
        else:
            if tuple(Y.shape) != (p, self.n, R) and tuple(Y.shape) != (p, self.n) or \
                    Y.numel() != p * self.n * R:
                raise ValueError("Y must have shape (p, n, nrhs)")
            if Y.dtype != torch.float64 or not Y.is_contiguous() or not Y.is_cuda:
                raise TypeError("Y must be a contiguous float64 device tensor")
        return R, Y

    def prepare(self, ps, rhs=range(1, 17)):
        """Build and upload ahead of time the schedules, slice tables and
        workspace that runs with each p in ps and each R in rhs fetch on
        first use, so that those runs do no host planning."""
        ps = [int(ps)] if isinstance(ps, (int, np.integer)) else [int(p) for p in ps]
        rhs = [int(rhs)] if isinstance(rhs, (int, np.integer)) else [int(r) for r in rhs]
        for p in ps:
            for R in rhs:
                check(self._lib.mpk_plan_prepare(self._h, p, R))

    def run(self, x, p: int, Y=None, stream=None):
        """Level-blocked MPK: returns Y with Y[k-1] = A^k x."""
        R, Y = self._prep(x, p, Y)
        check(self._lib.mpk_run(self._h, ctypes.c_void_p(x.data_ptr()), int(p), R,
                                ctypes.c_void_p(Y.data_ptr()), _stream_handle(stream)))
        return Y

    def run_noalloc(self, x, p: int, Y, status=None, stream=None):
        """mpk_run_noalloc: the level-blocked run with the library's static
        device workspace; allocates nothing (Y must be given, and (p, nrhs)
        prepared).  status: optional int32 tensor (device or pinned host)
        that receives 0, or 1 when a dependency wait hit its limit."""
        R, Y = self._prep(x, p, Y)
        sp = None
        if status is not None:
            torch = _torch()
            if status.dtype != torch.int32 or status.numel() < 1:
                raise TypeError("status must be an int32 tensor")
            sp = ctypes.c_void_p(status.data_ptr())
        check(self._lib.mpk_run_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), int(p), R,
                                        ctypes.c_void_p(Y.data_ptr()), sp,
                                        _stream_handle(stream)))
        return Y

    def run_baseline(self, x, p: int, Y=None, stream=None):
        """p back-to-back SpMVs (one launch per power); bit-identical to run()."""
        R, Y = self._prep(x, p, Y)
        check(self._lib.mpk_run_baseline(self._h, ctypes.c_void_p(x.data_ptr()), int(p), R,
                                         ctypes.c_void_p(Y.data_ptr()), _stream_handle(stream)))
        return Y

    def _coefs(self, alpha, beta, gamma):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        g = np.ascontiguousarray(gamma, dtype=np.float64)
        if not (a.size == b.size == g.size) or a.size < 1:
            raise ValueError("alpha, beta, gamma must have the same length p >= 1")
        return a, b, g

    def run_recur(self, x, alpha, beta, gamma, Y=None, stream=None):
        """Three-term recurrence y_{j+1} = alpha_j A y_j + beta_j y_j + gamma_j y_{j-1}."""
        a, b, g = self._coefs(alpha, beta, gamma)
        p = a.size
        R, Y = self._prep(x, p, Y)
        check(self._lib.mpk_run_recur(self._h, ctypes.c_void_p(x.data_ptr()), p, R,
                                      a.ctypes.data, b.ctypes.data, g.ctypes.data,
                                      ctypes.c_void_p(Y.data_ptr()), _stream_handle(stream)))
        return Y

    def run_baseline_recur(self, x, alpha, beta, gamma, Y=None, stream=None):
        a, b, g = self._coefs(alpha, beta, gamma)
        p = a.size
        R, Y = self._prep(x, p, Y)
        check(self._lib.mpk_run_baseline_recur(self._h, ctypes.c_void_p(x.data_ptr()), p, R,
                                               a.ctypes.data, b.ctypes.data, g.ctypes.data,
                                               ctypes.c_void_p(Y.data_ptr()),
                                               _stream_handle(stream)))
        return Y

    def _poly(self, fn, x, wa, wb, alpha, beta, gamma, acc, work, stream):
        torch = _torch()
        _vec_check(x, self.n, "x")
        R = 1 if x.dim() == 1 else int(x.shape[1])
        wa = np.ascontiguousarray(wa, dtype=np.float64)
        p = wa.size - 1
        if p < 1:
            raise ValueError("wa needs p + 1 >= 2 weights")
        if wb is not None:
            wb = np.ascontiguousarray(wb, dtype=np.float64)
            if wb.size != p + 1:
                raise ValueError("wa and wb must have the same length")
        if alpha is None and beta is None and gamma is None:
            ptrs = (None, None, None)
        else:
            a, b, g = self._coefs(alpha, beta, gamma)
            if a.size != p:
                raise ValueError("alpha, beta, gamma need p = len(wa) - 1 values")
            ptrs = (a.ctypes.data, b.ctypes.data, g.ctypes.data)
        nsum = 1 if wb is None else 2

        def buf(t, k, name):
            if t is None:
                return torch.empty((k, self.n, R), dtype=torch.float64, device=x.device)
            if t.numel() != k * self.n * R or t.dtype != torch.float64 or \
                    not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float64 device tensor of "
                                 f"{k} x n x nrhs values")
            return t
        acc = buf(acc, nsum, "acc")
        work = buf(work, 2, "work")
        check(fn(self._h, ctypes.c_void_p(x.data_ptr()), p, R, *ptrs, wa.ctypes.data,
                 None if wb is None else wb.ctypes.data, ctypes.c_void_p(acc.data_ptr()),
                 ctypes.c_void_p(work.data_ptr()), _stream_handle(stream)))
        return acc, work

    def run_poly(self, x, wa, wb=None, alpha=None, beta=None, gamma=None, acc=None, work=None,
                 stream=None):
        """Weighted sums acc[0] = sum_k wa[k] y_k (and acc[1] with wb), k = 0..p
        with p = len(wa) - 1, y_0 = x and y_k the recurrence (plain powers when
        alpha, beta, gamma are None), level-blocked, keeping only a ring of
        two vectors (mpk_run_poly).  Returns (acc, work); work[(k-1) % 2]
        holds y_k for k = p-1, p."""
        return self._poly(self._lib.mpk_run_poly, x, wa, wb, alpha, beta, gamma, acc, work,
                          stream)

    def run_baseline_poly(self, x, wa, wb=None, alpha=None, beta=None, gamma=None, acc=None,
                          work=None, stream=None):
        """The same sums with one p x SpMV launch per power (mpk_run_baseline_poly)."""
        return self._poly(self._lib.mpk_run_baseline_poly, x, wa, wb, alpha, beta, gamma, acc,
                          work, stream)

    def cheb_time_step(self, psi, dt: float, M: int, out=None, baseline: bool = False,
                       stream=None):
        """One Chebyshev time step psi -> exp(-i dt H) psi for a matrix whose
        spectrum lies in [-1, 1].  psi: (n, 2m) float64, column 2j the real
        and 2j+1 the imaginary part of state j.  Returns the stepped states
        in the same layout (mpk_run_poly + mpk_combine_complex)."""
        torch = _torch()
        _vec_check(psi, self.n, "psi")
        if psi.dim() != 2 or psi.shape[1] % 2:
            raise ValueError("psi must be (n, 2m): real and imaginary columns")
        R = int(psi.shape[1])
        al, be, ga, wa, wb = cheb_time_coefficients(M, dt)
        run = self.run_baseline_poly if baseline else self.run_poly
        acc, work = run(psi, wa, wb, al, be, ga, stream=stream)
        out = self.combine_complex(acc, out, stream=stream)
        if stream is not None:
            # the temporaries stay reserved until the work queued on `stream` is done
            acc.record_stream(stream)
            work.record_stream(stream)
        return out

    def combine_complex(self, acc, out=None, stream=None):
        """Complex states from the two sums of run_poly (mpk_combine_complex):
        acc (2, n, 2m) -> out (n, 2m) with column pairs (real, imaginary)."""
        torch = _torch()
        if acc.dim() != 3 or acc.shape[0] != 2 or acc.shape[1] != self.n or \
                acc.dtype != torch.float64 or not acc.is_contiguous() or not acc.is_cuda:
            raise ValueError("acc must be a contiguous float64 device tensor (2, n, nrhs)")
        R = int(acc.shape[2])
        if out is None:
            out = torch.empty((self.n, R), dtype=torch.float64, device=acc.device)
        elif out.numel() != self.n * R or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of n x nrhs values")
        check(self._lib.mpk_combine_complex(self._h, ctypes.c_void_p(acc.data_ptr()), R,
                                            ctypes.c_void_p(out.data_ptr()),
                                            _stream_handle(stream)))
        return out

    def permute(self, v, to_plan: bool, out=None, stream=None):
        """Convert (nvec, n, R) / (n, R) / (n,) blocks between numberings."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(v)
        if v.dim() == 1:
            nvec, R = 1, 1
        elif v.dim() == 2:
            nvec, R = 1, int(v.shape[1])
        else:
            nvec, R = int(v.shape[0]), int(v.shape[2])
        if v.dtype != torch.float64 or not v.is_contiguous() or out.shape != v.shape:
            raise ValueError("permute needs contiguous float64 tensors of equal shape")
        check(self._lib.mpk_permute(self._h, 1 if to_plan else 0, ctypes.c_void_p(v.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), nvec, R,
                                    _stream_handle(stream)))
        return out

    def sync(self):
        """Wait for this plan's runs; raises MPKError(MPK_ETIMEOUT) on a failed wait."""
        check(self._lib.mpk_plan_sync(self._h))

    def run_status(self, out, stream=None):
        """Enqueue on `stream` a copy of the failure word of this plan's runs
        issued there since the last call (mpk_run_status) into out[0]: an
        int32 tensor in device memory or pinned host memory.  0 = all
        completed, 1 = a wait hit its limit (those outputs are invalid)."""
        torch = _torch()
        if out.dtype != torch.int32 or out.numel() < 1:
            raise TypeError("out must be an int32 tensor with at least one element")
        if not (out.is_cuda or out.is_pinned()):
            raise TypeError("out must be device memory or pinned host memory")
        check(self._lib.mpk_run_status(self._h, _stream_handle(stream),
                                       ctypes.c_void_p(out.data_ptr())))
        return out


class Graph:
    """A captured level-blocked run (mpk_graph_*).  Keeps its plan and
    tensors alive; launches must not overlap; close() before the plan."""

    def __init__(self, handle, plan, tensors):
        self._h = handle
        self._plan = plan
        self._tensors = tensors
        self._lib = lib()

    def launch(self, stream=None):
        check(self._lib.mpk_graph_launch(self._h, _stream_handle(stream)))
        return self._tensors[1]

    def close(self):
        if self._h:
            self._lib.mpk_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
