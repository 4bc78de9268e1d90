"""Continuous-batching solve server over the HEC / ILU / Krylov library.

Requests (a sparse system A x = b each, of any size) arrive over time. The
server keeps up to ``slots`` of them in flight at once, each on its own HIP
stream, with its HEC matrix, ILU factor, level schedule and Krylov workspace
resident in HBM for the duration of its solve. A request is admitted in arrival
order as soon as a slot is free and its estimated device footprint fits in the
remaining memory budget (so the head of the queue can never be starved by later,
smaller requests). Admitted requests run concurrently: their kernels overlap on
the device, and the host side of one request's setup (symbolic ILU, level
schedules) runs while others compute, since every library call releases the
Python interpreter lock.

Each result is independent of what else is in flight: every kernel's reduction
order depends only on the request's own size, so a request solved alone and in
a mix gives bit-identical solutions.

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


def footprint_bytes(n: int, nnz: int, restart: int = 30, precision: int = 0, nnz_lu: int | None = None) -> int:
    """Upper estimate of the device memory one request holds while it is solved.

    HEC matrix (ELL slab + remainder, up to 1.3x padding), ILU factor and its two
    level-ordered triangle copies, Krylov workspace V (m+1 vectors) and Z (m
    vectors), work vectors; FP32 copies in mixed precision.
    """
    nnz_lu = nnz if nnz_lu is None else nnz_lu
    f64 = 8
    hec_b = int(1.3 * nnz) * (4 + f64) + 8 * n
    ilu_b = nnz_lu * (4 + f64) + 16 * n
    lev_b = 2 * (int(1.3 * nnz_lu) * (4 + f64) + 32 * n)
    ws_b = (2 * restart + 1) * n * f64 + 16 * n * f64
    if precision:
        hec_b += int(1.3 * nnz) * 4
        ilu_b += nnz_lu * 4
        lev_b += int(1.3 * nnz_lu) * 4
        ws_b += (2 * restart + 1) * n * 4 + 4 * n * 4
    return hec_b + ilu_b + lev_b + ws_b + (1 << 20)


@dataclass
class Server:
    slots: int = 8
    mem_budget: int = 64 << 30
    restart: int = 30
    results: list = field(default_factory=list)

    def __post_init__(self):
        self._cv = threading.Condition()
        self._queue: deque = deque()
        self._free_mem = self.mem_budget
        self._inflight = 0
        self._closed = False
        self.peak_mem = 0
        self.peak_inflight = 0
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

    def _release(self, fp):
        with self._cv:
            self._free_mem += fp
            self._inflight -= 1
            self._cv.notify_all()

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
        while True:
            item = self._admit()
            if item is None:
                return
            req, fp = item
            t_adm = time.perf_counter() - t0
            try:
                with torch.cuda.stream(stream):
                    keep = req.precision == 1
                    M = hec.hec_from_csr(req.A, keep_f32=keep, stream=stream)
                    F = hec.ilu_factor(req.A, k=0, keep_f32=keep, stream=stream)
                    lv = hec.level_schedule(F, stream=stream)
                    bd = torch.from_numpy(req.b).to("cuda", non_blocking=False)
                    x = torch.empty_like(bd)
                    info = hec.gmres_solve(M, F, lv, bd, x, restart=self.restart, rtol=req.rtol,
                                           precision=req.precision, stream=stream, check=False)
                    xh = x.cpu().numpy()
                    stream.synchronize()
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
                self._release(fp)

    def run(self, source, t0: float | None = None):
        """Serve requests from ``source`` (an iterable of Request, in arrival order):
        each is submitted when its arrival time is reached. Returns the results."""
        t0 = time.perf_counter() if t0 is None else t0
        workers = [threading.Thread(target=self._worker, args=(s, t0), daemon=True) for s in range(self.slots)]
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
        return self.results


def latency_stats(results):
    lat = np.array([r.latency for r in results]) * 1e3
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}
