"""Continuous-batching solve server over the HEC / ILU / Krylov library.

Requests (a sparse system A x = b each, of any size) arrive over time. The
server keeps up to ``slots`` of them in flight at once, each on its own HIP
stream, with its HEC matrix, ILU factor, level schedule and Krylov workspace
resident in HBM for the duration of its solve. A request is admitted in arrival
order as soon as a slot is free and its estimated device footprint fits in the
remaining memory budget (so the head of the queue can never be starved by later,
smaller requests). Once its handles are built, the reservation becomes what the
library reports they hold (hec_footprint) plus the Krylov workspace the solve
adds, and the difference goes back to the budget; after the solve the library's
figure (workspace included) is recorded. Admitted requests run concurrently: their kernels overlap on
the device, and the host side of one request's setup (symbolic ILU, level
schedules) runs while others compute, since every library call releases the
Python interpreter lock.

Small systems (n <= batch_max_n, when batching is on) take another route: a
slot prepares the system (HEC matrix, factor, level schedules, right-hand side)
and hands it to the batcher, which solves the prepared small systems in one
persistent launch replayed from a hipGraph (gmres_solve_batched), one workgroup
per system. Once a system is ready the batcher holds the launch for more, for as
long as about batch_target systems take to arrive at the recent hand-over rate
(an exponential average), at most batch_wait, and not at all when fewer than one
more system is expected within batch_wait: at a high arrival rate launches fill
up, at a low one a system does not wait for company that is not coming. The slot
is free again as soon as it has handed the system over.

Each result is independent of what else is in flight: every kernel's reduction
order depends only on the request's own size, and a batched system is solved by
its own workgroup, so a request solved alone and in a mix gives bit-identical
solutions (on the same route).

Latency of a request = time from its arrival to its solution in host memory.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import hec


@dataclass
class Request:
    rid: int
    A: object                 # CSR (n, Ap, Aj, Ax)
    b: np.ndarray
    precision: int = 0        # 0 FP64, 1 mixed (FP32 storage + FP64 refinement)
    rtol: float = 1e-8
    arrival: float = 0.0      # seconds after the start of the run


@dataclass
class Result:
    rid: int
    x: np.ndarray
    info: dict
    n: int
    footprint: int
    arrival: float
    admitted: float
    done: float
    slot: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def workspace_bytes(n: int, restart: int = 30, precision: int = 0) -> int:
    """Upper estimate of the Krylov workspace a GMRES solve adds to the matrix handle:
    V (m+1 vectors, padded) and Z (m vectors), work vectors, FP32 copies in mixed precision."""
    f64 = 8
    ws_b = (2 * restart + 1) * (n + 2048) * f64 + 16 * n * f64
    if precision:
        ws_b += (2 * restart + 1) * (n + 2048) * 4 + 4 * n * 4
    return ws_b + (1 << 20)


def footprint_bytes(n: int, nnz: int, restart: int = 30, precision: int = 0, nnz_lu: int | None = None) -> int:
    """Upper estimate of the device memory one request holds while it is solved, for
    admission before its handles exist (the library reports the real figure once they
    do; the serving tests check that it never exceeds this).

    HEC matrix (ELL slab + remainder, up to 1.3x padding), ILU factor, its level-ordered
    triangle plans (up to 1.3x padding) and, on a 3D grid, the wavefront plans (packed
    coefficients with the tiles' skew, face buffers), the Krylov workspace; FP32 copies
    in mixed precision.
    """
    nnz_lu = nnz if nnz_lu is None else nnz_lu
    f64 = 8
    hec_b = int(1.3 * nnz) * (4 + f64) + 8 * n
    ilu_b = nnz_lu * (4 + f64) + 16 * n
    lev_b = 2 * (int(1.3 * nnz_lu) * (4 + f64) + 32 * n)
    grid_b = 2 * 4 * int(1.5 * n) * f64 + 4 * int(1.5 * n) * f64
    if precision:
        hec_b += int(1.3 * nnz) * 4
        ilu_b += nnz_lu * 4
        lev_b += int(1.3 * nnz_lu) * 4
        grid_b += 2 * 4 * int(1.5 * n) * 4 + 4 * int(1.5 * n) * 4
    return hec_b + ilu_b + lev_b + grid_b + workspace_bytes(n, restart, precision) + (1 << 20)


@dataclass
class Server:
    slots: int = 8
    mem_budget: int = 64 << 30
    restart: int = 30
    batch_max_n: int = 0          # 0: no batching; else systems with n <= batch_max_n are batched
    batch_capacity: int = 256     # systems per batched launch
    batch_wait: float = 0.002     # longest hold of a batched launch for more systems (seconds)
    batch_target: int = 16        # systems a hold waits for at the recent hand-over rate
    results: list = field(default_factory=list)

    def __post_init__(self):
        self._cv = threading.Condition()
        self._queue: deque = deque()
        self._free_mem = self.mem_budget
        self._inflight = 0
        self._closed = False
        self._batchq: deque = deque()   # prepared small systems, in hand-over order
        self._workers_done = False
        self._streams: list = []        # kept alive until every handle made on them is destroyed
        self.peak_mem = 0               # largest reservation in flight (estimates, then library figures)
        self.peak_reported = 0          # largest sum of library-reported footprints in flight
        self._reported = 0
        self.reported: dict = {}        # rid -> library-reported device bytes after the solve
        self._small_rate = 0.0          # exponential average of small-system hand-overs per second
        self._last_small = None
        self.peak_inflight = 0
        self.batches: list = []         # sizes of the batched launches
        self.errors: list = []

    # ------------------------------------------------------------ admission
    def _admit(self):
        """Blocks until the head of the queue fits; returns it (or None when closed and empty)."""
        with self._cv:
            while True:
                if self._queue:
                    req, fp = self._queue[0]
                    if fp <= self._free_mem or self._inflight == 0:
                        self._queue.popleft()
                        self._free_mem -= fp
                        self._inflight += 1
                        used = self.mem_budget - self._free_mem
                        self.peak_mem = max(self.peak_mem, used)
                        self.peak_inflight = max(self.peak_inflight, self._inflight)
                        self._cv.notify_all()
                        return req, fp
                elif self._closed:
                    return None
                self._cv.wait()

    def _release(self, fp, reported=0):
        with self._cv:
            self._free_mem += fp
            self._reported -= reported
            self._inflight -= 1
            self._cv.notify_all()

    def _settle(self, fp, handles_bytes, n, precision):
        """After setup: the reservation becomes the library's figure for the handles plus the
        workspace estimate (never more than admitted: the estimate is an upper bound).
        Returns the new reservation."""
        new = min(fp, handles_bytes + workspace_bytes(n, self.restart, precision))
        with self._cv:
            self._free_mem += fp - new
            self._reported += handles_bytes
            self.peak_reported = max(self.peak_reported, self._reported)
            self._cv.notify_all()
        return new

    def _record(self, rid, fp_bytes, handles_bytes):
        """After the solve: the library's figure with the workspace."""
        with self._cv:
            self.reported[rid] = fp_bytes
            self._reported += fp_bytes - handles_bytes
            self.peak_reported = max(self.peak_reported, self._reported)

    def submit(self, req: Request):
        fp = footprint_bytes(req.A.n, req.A.nnz, self.restart, req.precision)
        with self._cv:
            self._queue.append((req, fp))
            self._cv.notify_all()

    def close(self):
        with self._cv:
            self._closed = True
            self._cv.notify_all()

    # ------------------------------------------------------------ workers
    def _worker(self, slot: int, t0: float):
        import torch
        stream = torch.cuda.Stream()
        with self._cv:
            self._streams.append(stream)
        while True:
            item = self._admit()
            if item is None:
                return
            req, fp = item
            t_adm = time.perf_counter() - t0
            if self.batch_max_n and req.A.n <= self.batch_max_n:
                self._prepare_small(req, fp, t_adm, slot, stream)
                continue
            hb = 0
            try:
                with torch.cuda.stream(stream):
                    keep = req.precision == 1
                    M = hec.hec_from_csr(req.A, keep_f32=keep, stream=stream)
                    F = hec.ilu_factor(req.A, k=0, keep_f32=keep, stream=stream)
                    lv = hec.level_schedule(F, stream=stream)
                    hb = hec.footprint(M, F, lv)
                    fp = self._settle(fp, hb, req.A.n, req.precision)
                    bd = torch.from_numpy(req.b).to("cuda", non_blocking=False)
                    x = torch.empty_like(bd)
                    info = hec.gmres_solve(M, F, lv, bd, x, restart=self.restart, rtol=req.rtol,
                                           precision=req.precision, stream=stream, check=False)
                    xh = x.cpu().numpy()
                    stream.synchronize()
                    fb = hec.footprint(M, F, lv)
                    self._record(req.rid, fb, hb)
                    hb = fb
                    del bd, x
                    lv.close(); F.close(); M.close()
                    stream.synchronize()
                t_done = time.perf_counter() - t0
                res = Result(req.rid, xh, info, req.A.n, fp, req.arrival, t_adm, t_done, slot)
                with self._cv:
                    self.results.append(res)
            except Exception as e:  # recorded, the server keeps serving
                with self._cv:
                    self.errors.append((req.rid, repr(e)))
            finally:
                self._release(fp, hb)

    # ------------------------------------------------------------ small systems
    def _prepare_small(self, req, fp, t_adm, slot, stream):
        import torch
        try:
            with torch.cuda.stream(stream):
                keep = req.precision == 1
                M = hec.hec_from_csr(req.A, keep_f32=keep, stream=stream)
                F = hec.ilu_factor(req.A, k=0, keep_f32=keep, stream=stream)
                lv = hec.level_schedule(F, stream=stream)
                hb = hec.footprint(M, F, lv)  # the batch context holds the Krylov workspace
                bd = torch.from_numpy(req.b).to("cuda", non_blocking=False)
                x = torch.empty_like(bd)
                stream.synchronize()
        except Exception as e:
            with self._cv:
                self.errors.append((req.rid, repr(e)))
            self._release(fp)
            return
        with self._cv:
            now = time.perf_counter()
            if self._last_small is not None:  # recent hand-over rate (exponential average over ~8)
                gap = max(now - self._last_small, 1e-6)
                self._small_rate = 0.875 * self._small_rate + 0.125 / gap
            self._last_small = now
            new = min(fp, hb)
            self._free_mem += fp - new
            self._reported += hb
            self.reported[req.rid] = hb
            self.peak_reported = max(self.peak_reported, self._reported)
            self._batchq.append((req, new, t_adm, slot, M, F, lv, bd, x, hb))
            self._cv.notify_all()

    def _take_batch(self):
        """Blocks for the next group of prepared systems with one (precision, rtol)."""
        with self._cv:
            while not self._batchq:
                if self._workers_done:
                    return None
                self._cv.wait()
            # hold for about batch_target systems at the recent hand-over rate, at most
            # batch_wait; not at all when fewer than one more is expected within batch_wait
            hold = self.batch_wait
            if self._small_rate > 0:
                hold = min(hold, self.batch_target / self._small_rate)
                if self._small_rate * self.batch_wait < 1.0:
                    hold = 0.0
            deadline = time.perf_counter() + hold
            while len(self._batchq) < min(self.batch_capacity, self.batch_target) and not self._workers_done:
                left = deadline - time.perf_counter()
                if left <= 0:
                    break
                self._cv.wait(left)
            key = (self._batchq[0][0].precision, self._batchq[0][0].rtol)
            group, rest = [], deque()
            while self._batchq:
                it = self._batchq.popleft()
                if len(group) < self.batch_capacity and (it[0].precision, it[0].rtol) == key:
                    group.append(it)
                else:
                    rest.append(it)
            self._batchq = rest
            return group

    def _batcher(self, t0: float):
        contexts = {}
        while True:
            group = self._take_batch()
            if group is None:
                break
            prec, rtol = group[0][0].precision, group[0][0].rtol
            try:
                if prec not in contexts:
                    contexts[prec] = hec.Batch(self.batch_capacity, self.restart, self.batch_max_n)
                infos = hec.gmres_solve_batched(contexts[prec], [(it[4], it[5], it[6], it[7], it[8]) for it in group],
                                                rtol=rtol, precision=prec, check=False)
                xs = [it[8].cpu().numpy() for it in group]
                t_done = time.perf_counter() - t0
                with self._cv:
                    self.batches.append(len(group))
                    for it, info, xh in zip(group, infos, xs):
                        req, fp, t_adm, slot = it[:4]
                        self.results.append(Result(req.rid, xh, info, req.A.n, fp, req.arrival, t_adm, t_done, slot))
            except Exception as e:
                with self._cv:
                    for it in group:
                        self.errors.append((it[0].rid, repr(e)))
            finally:
                for it in group:
                    for h in (it[6], it[5], it[4]):
                        h.close()
                    self._release(it[1], it[9])
        for B in contexts.values():
            B.close()

    def run(self, source, t0: float | None = None):
        """Serve requests from ``source`` (an iterable of Request, in arrival order):
        each is submitted when its arrival time is reached. Returns the results."""
        t0 = time.perf_counter() if t0 is None else t0
        workers = [threading.Thread(target=self._worker, args=(s, t0), daemon=True) for s in range(self.slots)]
        batcher = None
        if self.batch_max_n:
            batcher = threading.Thread(target=self._batcher, args=(t0,), daemon=True)
            batcher.start()
        for w in workers:
            w.start()
        for req in source:
            delay = req.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            self.submit(req)
        self.close()
        for w in workers:
            w.join()
        with self._cv:
            self._workers_done = True
            self._cv.notify_all()
        if batcher is not None:
            batcher.join()
        return self.results


def latency_stats(results):
    lat = np.array([r.latency for r in results]) * 1e3
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}
