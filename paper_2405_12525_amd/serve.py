"""Continuous-batching request loop over device-resident plans.

Requests ask for the powers (or a Chebyshev recurrence) of one of the
matrices whose plans the server holds on the device.  They arrive over time;
the loop admits them as stream slots and memory free up:

* requests for the same matrix and kind that are waiting together form one
  batch: their right-hand sides are stacked (at most 16 columns) and the
  batch runs p = max p_i powers.  Every column is computed exactly as if it
  ran alone (the kernels' per-column arithmetic does not depend on the
  right-hand-side count) and powers are prefix-consistent, so request i takes
  the first p_i powers of its own columns;
* a Chebyshev time step (kind "time_step": one step exp(-i dt H) psi with
  M = p terms, psi as real and imaginary column pairs) batches only with
  steps of the same dt and M, since those fix the weights; each request
  takes its own columns of the stepped states;
* batches for different matrices run concurrently on separate HIP streams,
  at most max_inflight_per_matrix batches of one matrix at a time (by
  default one), so that requests arriving for a busy matrix wait together
  and leave as one larger batch instead of taking every stream; with lanes,
  each matrix runs on a fixed stream (Server.size_lanes gives the largest
  matrices a stream each and lets the small ones share one, so that their
  short batches do not wait behind long ones);
* each plan runs its batches through the level-blocked kernels or, where
  the caller found them faster for that matrix (use_baseline), through the
  p x SpMV kernels: the results are the same bit for bit.  Plans served
  through the level-blocked kernels are set to take tasks from the shared
  counter (tune dynamic_tickets = 1): their runs share the device with other
  batches, and the fixed task order needs every workgroup of a launch
  resident, which other kernels delay, while with the counter a task waits
  only on tasks that running workgroups hold;
* a batch is admitted only while the device memory held by running batches
  (stacked inputs plus outputs) stays within the budget;
* each batch's device status (mpk_run_status, copied into pinned host memory
  on the batch's stream) is read when the batch completes and before any of
  its outputs is handed out: a batch whose dependency wait hit its limit
  delivers nothing, and its requests are reported as failed.

All arithmetic runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import MPKError, Plan, chebyshev_coefficients, flops, _torch
from ._capi import MPK_ETIMEOUT

MAX_RHS = 16


@dataclasses.dataclass
class Request:
    id: int
    arrival: float            # seconds from the start of serving
    matrix: int               # index into the server's plans
    p: int
    x: object                 # device tensor (n, R), float64
    kind: str = "powers"      # "powers", "chebyshev" or "time_step"
    dt: float = 0.0           # time step (kind "time_step"; p is the expansion order M)

    @property
    def R(self) -> int:
        return 1 if self.x.dim() == 1 else int(self.x.shape[1])


@dataclasses.dataclass
class Result:
    id: int
    Y: object                 # device tensor view (p, n, R); (n, R) for a time step
    arrival: float
    start: float              # batch launch time
    done: float               # completion observed by the loop
    batch_size: int
    error: Optional[str] = None   # the batch failed on the device (Y is None)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def batch_bytes(n: int, p: int, R: int, kind: str = "powers") -> int:
    """Device bytes a batch holds while running: stacked x plus Y, or for a
    time step x, the stepped states, the two sums and the two-vector ring."""
    return 8 * n * R * (6 if kind == "time_step" else p + 1)


def _same_batch(a: Request, b: Request) -> bool:
    if a.kind != b.kind:
        return False
    return a.kind != "time_step" or (a.p == b.p and a.dt == b.dt)


def form_batch(queue: collections.deque, max_rhs: int = MAX_RHS) -> List[Request]:
    """Take the head request and then later ones of the same kind, in arrival
    order, while the stacked right-hand sides fit max_rhs."""
    head = queue[0]
    batch, total = [], 0
    keep = collections.deque()
    while queue:
        r = queue.popleft()
        if _same_batch(r, head) and total + r.R <= max_rhs:
            batch.append(r)
            total += r.R
        else:
            keep.append(r)
    queue.extend(keep)
    return batch


class Server:
    """Holds plans on the device and serves request streams.

    Streams that share a hardware queue run in that queue's order, so a
    short batch waits for a long one queued before it on another stream.
    HIP maps a process's streams onto GPU_MAX_HW_QUEUES queues (4 unless set
    in the environment before HIP starts), the default stream included: give
    the process more queues than n_streams.  A level-blocked batch holds its
    persistent workgroups for its whole run; two long ones can fill the
    device, and batches on other streams then wait for them.

    plans: one Plan per matrix (device plans, already tuned as wished; a
        plan served through the level-blocked kernels is set to
        dynamic_tickets = 1 here, so tune it with that set, e.g.
        P.tune(dynamic_tickets=1) before P.autotune, which then keeps it).
    n_streams: batches that may run at once.
    mem_budget: bytes of batch memory (inputs plus outputs) in flight.
    """

    def __init__(self, plans: Sequence[Plan], n_streams: int = 4,
                 mem_budget: Optional[int] = None, max_rhs: int = MAX_RHS,
                 max_inflight_per_matrix: int = 1,
                 use_baseline: Optional[Sequence[bool]] = None,
                 lanes: Optional[Sequence[int]] = None):
        torch = _torch()
        self.plans = list(plans)
        self.lanes = None if lanes is None else [int(v) for v in lanes]
        if self.lanes is not None and (len(self.lanes) != len(self.plans) or
                                       not all(0 <= v < max(1, int(n_streams)) for v in self.lanes)):
            raise ValueError("lanes needs one stream index in [0, n_streams) per plan")
        self.max_inflight_per_matrix = max(1, int(max_inflight_per_matrix))
        self.use_baseline = [False] * len(self.plans) if use_baseline is None \
            else [bool(b) for b in use_baseline]
        if len(self.use_baseline) != len(self.plans):
            raise ValueError("use_baseline needs one entry per plan")
        for P, base in zip(self.plans, self.use_baseline):
            if not base and P.n > 0 and not P.tuning["dynamic_tickets"]:
                P.tune(dynamic_tickets=1)
        self.max_rhs = int(max_rhs)
        if not 1 <= self.max_rhs <= MAX_RHS:
            raise ValueError("max_rhs must be in [1, 16]")
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info()
            mem_budget = int(free * 0.6)
        self.mem_budget = int(mem_budget)
        self.streams = [torch.cuda.Stream() for _ in range(max(1, int(n_streams)))]
        # per-stream device status of the batch last launched there, written by
        # the stream itself into pinned host memory (mpk_run_status)
        self._status = [torch.zeros(1, dtype=torch.int32, pin_memory=True)
                        for _ in self.streams]
        # per-stream buffers reused by serve(keep=False): stacked inputs, outputs
        self._stage = [None] * len(self.streams)
        self._out = [None] * len(self.streams)

    def prepare(self, max_p: int, rhs=range(1, MAX_RHS + 1)) -> None:
        """Build ahead of time what batches of up to max_p powers and any
        stacked right-hand-side count in rhs fetch on first use (schedules,
        slice tables, workspaces; mpk_plan_prepare).  Otherwise the first
        batch of each new shape plans and uploads on the host while the loop
        waits, and every batch in flight is observed late."""
        for P, base in zip(self.plans, self.use_baseline):
            if P.n > 0:
                P.prepare([1] if base else range(1, int(max_p) + 1), rhs)

    @staticmethod
    def size_lanes(plans: Sequence[Plan], n_streams: int) -> List[int]:
        """Stream per matrix: the n_streams - 1 largest matrices (by stored
        entries) get a stream each and the others share the last one, so a
        small matrix's short batches never queue behind a large matrix's
        long ones on a stream (nor on the hardware queue it maps to, when
        n_streams does not exceed the device's hardware queues)."""
        n_streams = max(1, int(n_streams))
        order = sorted(range(len(plans)), key=lambda m: -plans[m].nnz)
        lanes = [n_streams - 1] * len(plans)
        for rank, m in enumerate(order[:n_streams - 1]):
            lanes[m] = rank
        return lanes

    def _scratch(self, store: list, si: int, numel: int, device):
        """Stream si's reusable buffer of at least numel doubles.  Only the
        batch on that stream uses it, and a stream is handed out again only
        once its batch has finished, so no copy is in flight when it is
        reused or grown."""
        torch = _torch()
        b = store[si]
        if b is None or b.numel() < numel:
            store[si] = None
            with torch.cuda.stream(self.streams[si]):
                b = torch.empty(numel, dtype=torch.float64, device=device)
            store[si] = b
        return b[:numel]

    # one batch on stream si; keep=False takes the stacked inputs and the
    # outputs from the stream's reused buffers instead of new allocations
    def _launch(self, batch: List[Request], si: int, keep: bool):
        torch = _torch()
        stream = self.streams[si]
        P = self.plans[batch[0].matrix]
        p = max(r.p for r in batch)
        kind = batch[0].kind
        with torch.cuda.stream(stream):
            xs = [r.x.reshape(P.n, -1) for r in batch]
            R = sum(int(x.shape[1]) for x in xs)
            dev = xs[0].device
            if len(xs) == 1:
                X = xs[0]
            elif keep:
                X = torch.cat(xs, dim=1).contiguous()
            else:
                X = torch.cat(xs, dim=1,
                              out=self._scratch(self._stage, si, P.n * R, dev).view(P.n, R))
            Yo = None
            if not keep:
                nvec = 1 if kind == "time_step" else p
                Yo = self._scratch(self._out, si, nvec * P.n * R, dev)
                Yo = Yo.view(P.n, R) if kind == "time_step" else Yo.view(p, P.n, R)
            base = self.use_baseline[batch[0].matrix]
            if kind == "chebyshev":
                run = P.run_baseline_recur if base else P.run_recur
                Y = run(X, *chebyshev_coefficients(p), Y=Yo, stream=stream)
            elif kind == "time_step":
                Y = P.cheb_time_step(X, batch[0].dt, p, out=Yo, stream=stream, baseline=base)
            else:
                Y = (P.run_baseline if base else P.run)(X, p, Y=Yo, stream=stream)
            # the batch's failure word, ready when the event below completes
            P.run_status(self._status[si], stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return Y, ev, p

    def serve(self, requests: Sequence[Request], realtime: bool = True,
              keep: bool = True,
              on_result: Optional[Callable[[Request, object], None]] = None,
              raise_on_error: bool = True) -> List[Result]:
        """Serve the requests (sorted by arrival); returns results by id.

        realtime=True replays the arrival times against the wall clock;
        realtime=False makes every request available at once (saturation).
        keep=False drops each output once its batch has finished (Result.Y is
        None): for measuring streams whose outputs would not fit at once.
        The batches then write into one output buffer per stream, reused and
        kept for the server's lifetime, so that the device allocator does not
        fill with freed outputs of every size.
        on_result(request, Y) is called when a request's batch has finished,
        with the request's own output view; with keep=False the view is only
        valid during the call.
        A batch whose run failed on the device (a dependency wait hit its
        limit) hands out nothing: on_result is not called for its requests and
        their Results carry `error` and no output.  The other batches are
        unaffected.  raise_on_error=True then raises MPKError(MPK_ETIMEOUT)
        once the stream has been served."""
        torch = _torch()
        for r in requests:
            if not 0 <= r.matrix < len(self.plans):
                raise ValueError(f"request {r.id}: no matrix {r.matrix}")
            if r.R > self.max_rhs or r.p < 1:
                raise ValueError(f"request {r.id}: bad p or R")
            if r.kind not in ("powers", "chebyshev", "time_step"):
                raise ValueError(f"request {r.id}: unknown kind {r.kind}")
            if r.kind == "time_step" and r.R % 2:
                raise ValueError(f"request {r.id}: a time step needs real and imaginary columns")
            need = batch_bytes(self.plans[r.matrix].n, r.p, r.R, r.kind)
            if need > self.mem_budget:
                raise ValueError(f"request {r.id} needs {need} bytes, above the budget")
        order = sorted(requests, key=lambda r: r.arrival)
        pending: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
        free_streams = list(range(len(self.streams)))
        running = []   # (stream index, event, batch, Y, p, bytes, start)
        results: Dict[int, Result] = {}
        in_use = 0
        i = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while len(results) < len(order):
            now = time.perf_counter() - t0
            while i < len(order) and (not realtime or order[i].arrival <= now):
                pending[order[i].matrix].append(order[i])
                i += 1
            # completions
            still = []
            for item in running:
                si, ev, batch, Y, p, nbytes, start = item
                if ev.query():
                    done = time.perf_counter() - t0
                    failed = int(self._status[si][0]) != 0
                    c0 = 0
                    for r in batch:
                        arr = r.arrival if realtime else 0.0
                        if failed:
                            results[r.id] = Result(r.id, None, arr, start, done, len(batch),
                                                   error="a dependency wait hit its limit")
                            continue
                        if r.kind == "time_step":
                            view = Y[:, c0:c0 + r.R]
                        else:
                            view = Y[:r.p, :, c0:c0 + r.R]
                        c0 += r.R
                        if on_result is not None:
                            on_result(r, view)
                        results[r.id] = Result(r.id, view if keep else None, arr, start, done,
                                               len(batch))
                    in_use -= nbytes
                    free_streams.append(si)
                else:
                    still.append(item)
            running = still
            # dispatch: oldest waiting request first, while slots and memory
            # allow, skipping matrices that already have their batches in flight
            while free_streams:
                busy = collections.Counter(item[2][0].matrix for item in running)
                heads = [(q[0].arrival, m) for m, q in pending.items()
                         if q and busy[m] < self.max_inflight_per_matrix and
                         (self.lanes is None or self.lanes[m] in free_streams)]
                if not heads:
                    break
                _, m = min(heads)
                q = pending[m]
                batch = form_batch(q, self.max_rhs)
                p = max(r.p for r in batch)
                nbytes = batch_bytes(self.plans[m].n, p, sum(r.R for r in batch), batch[0].kind)
                if in_use + nbytes > self.mem_budget and running:
                    for r in reversed(batch):
                        q.appendleft(r)
                    break
                if self.lanes is None:
                    si = free_streams.pop()
                else:
                    si = self.lanes[m]
                    free_streams.remove(si)
                start = time.perf_counter() - t0
                Y, ev, p = self._launch(batch, si, keep)
                in_use += nbytes
                running.append((si, ev, batch, Y, p, nbytes, start))
            # idle until the next arrival or a completion can be observed
            now = time.perf_counter() - t0
            if not (i < len(order) and order[i].arrival <= now):
                wait = 20e-6 if running else (order[i].arrival - now if i < len(order) else 0.0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        failed = [i for i, r in results.items() if r.error is not None]
        for P in self.plans:
            try:
                P.sync()
            except MPKError as e:
                # a failed run is already reported per batch above
                if e.status != MPK_ETIMEOUT or not failed:
                    raise
        out = [results[r.id] for r in sorted(requests, key=lambda r: r.id)]
        if failed and raise_on_error:
            raise MPKError(MPK_ETIMEOUT, f"{len(failed)} requests failed on the device "
                                         f"(first ids {sorted(failed)[:8]}); nothing was "
                                         "delivered for them")
        return out


def summarize(results: Sequence[Result], requests: Sequence[Request], plans: Sequence[Plan]) -> dict:
    """Latency percentiles, throughput and delivered Gflop/s of a served stream."""
    results = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in results])
    by_id = {r.id: r for r in requests}
    fl = 0.0
    for res in results:
        rq = by_id[res.id]
        P = plans[rq.matrix]
        fl += flops(P.nnz, P.n, rq.p, rq.R, recur=rq.kind != "powers")
        if rq.kind == "time_step":   # the weighted sums and the complex combination
            fl += 2.0 * P.n * rq.R * (rq.p + 1) + P.n * rq.R
    first = min(r.arrival for r in results)
    last = max(r.done for r in results)
    span = max(last - first, 1e-9)
    # where the latency goes: waiting for a stream and memory (arrival to
    # launch) and the batch's time from launch to observed completion
    wait = np.array([r.start - r.arrival for r in results])
    run = np.array([r.done - r.start for r in results])
    mat = np.array([by_id[r.id].matrix for r in results])
    by_matrix = {}
    for m in sorted(set(mat.tolist())):
        sel = mat == m
        lm = lat[sel]
        by_matrix[m] = {"n": plans[m].n, "requests": int(lm.size),
                        "p50_ms": float(np.percentile(lm, 50) * 1e3),
                        "p99_ms": float(np.percentile(lm, 99) * 1e3),
                        "queue_p99_ms": float(np.percentile(wait[sel], 99) * 1e3),
                        "device_p50_ms": float(np.percentile(run[sel], 50) * 1e3),
                        "device_p99_ms": float(np.percentile(run[sel], 99) * 1e3)}
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "queue_p50_ms": float(np.percentile(wait, 50) * 1e3),
            "queue_p99_ms": float(np.percentile(wait, 99) * 1e3),
            "device_p50_ms": float(np.percentile(run, 50) * 1e3),
            "device_p99_ms": float(np.percentile(run, 99) * 1e3),
            "throughput_rps": len(results) / span, "gflops": fl / span / 1e9,
            "mean_batch": float(np.mean([r.batch_size for r in results])), "span_s": span,
            "by_matrix": by_matrix}
