"""Continuous-batching request loop for sequences of dual systems.

A request is a sequence of dual systems A x_j = b_j, A^H x~_j = b~_j with one
matrix (the sequence setting of the paper's problem statement, solved with
recycling between its systems).  The server admits requests in arrival order
as soon as a slot and enough device memory are free; every admitted request
runs on its own HIP stream with its own solver handle, so that its matrix,
recycle space and workspace stay on the device between its systems and the
kernels of several requests overlap on the GPU.  Each request's arithmetic
depends only on its own handle, so its results are the same alone and in the
mix.

The scheduler is plain Python threads: the solves run inside librbicg.so (the
ctypes calls release the interpreter lock), the threads only hand out work.
With ``batched=True`` every admitted request's handle is attached to one
rbicg batch, so the iteration kernels of all requests that are iterating run
in one set of launches (continuous batching at the launch level); results are
bitwise those of the unbatched handles.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import workloads as wl


@dataclass
class RequestResult:
    rid: int
    arrival: float
    admitted: float
    finished: float
    edge: int
    nsys: int
    stats: List[dict] = field(default_factory=list)
    solutions: Optional[list] = None   # per system (x, x~) host arrays, when kept

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def request_bytes(req: wl.Request, prec: str = "mixed", s: int = 40) -> int:
    """Device memory a request holds while it runs: two sliced-ELL matrices
    (7-point stencil, int32 index + value), the handle's vectors, recycle
    bases and cycle rings (float storage plus FP64 outer vectors in the
    FP32-inner mode), with 10% headroom."""
    n = req.edge ** 3
    ld = (n + 255) // 256 * 256
    vb = 4 if prec == "mixed" else 8
    mat = 2 * 7 * n * (4 + 8 + (4 if prec == "mixed" else 0))
    vecs = ld * vb * (12 + 16 * req.k + 4 * (2 * s + 1))
    extra = ld * 8 * 8 if prec == "mixed" else 0
    rhs = 4 * n * 8
    return int(1.1 * (mat + vecs + extra + rhs))


class Server:
    """Admits requests (in arrival order) into at most ``slots`` concurrent
    slots while their device memory fits ``hbm_budget`` bytes; ``execute``
    runs one request (default: GPU solve of its sequence) and returns its
    per-system stats and, optionally, solutions."""

    def __init__(self, slots: int = 4, hbm_budget: Optional[int] = None, prec: str = "mixed",
                 tol: float = 1e-8, inner_tol: float = 1e-5, s: int = 40,
                 keep_solutions: bool = False,
                 execute: Optional[Callable] = None, batched: bool = False,
                 window_us: float = 50.0, batch_max_rows: int = 262144,
                 tune_cache: Optional[str] = None, graphs: bool = False):
        self.slots = slots
        # launch shapes from the autotuner's JSON cache (paper_1010_0762_amd/
        # tune.py) for request shapes it holds; the automatic grid otherwise
        self.tune_cache = tune_cache
        # requests of at most batch_max_rows unknowns go through the batch;
        # larger ones fill the GPU on their own and keep their own launches
        # (in one batch stream their long chunks would hold up the small ones)
        self.batch_max_rows = batch_max_rows
        # continuous batching: the admitted requests' iteration chunks go
        # through one rbicg batch (one set of launches for all of them)
        self.batch = None
        if batched:
            from .solver import Batch
            self.batch = Batch(max_slots=min(16, slots), window_us=window_us, graphs=graphs)
        self.prec = prec
        self.tol = tol
        self.inner_tol = inner_tol
        self.s = s
        self.keep = keep_solutions
        if hbm_budget is None:
            hbm_budget = self._free_device_memory()
        self.budget = int(hbm_budget)
        self.execute = execute or self._execute_gpu

    @staticmethod
    def _free_device_memory() -> int:
        import torch
        free, _ = torch.cuda.mem_get_info()
        return int(0.8 * free)

    # ------------------------------------------------------------ execution
    def prepare(self, requests: List[wl.Request]) -> None:
        """Assemble every request's matrix on the host ahead of the replay (a
        request arrives with its problem data)."""
        self._csr = {r.rid: wl.convdiff(r.edge, 3, r.beta) for r in requests}

    def _execute_gpu(self, req: wl.Request):
        import torch
        from ._lib import RBiCGError
        from .solver import DeviceMatrix, Solver
        stream = torch.cuda.Stream()
        cache = getattr(self, "_csr", None)
        A = cache.pop(req.rid) if cache and req.rid in cache else wl.convdiff(req.edge, 3, req.beta)
        M = S = None
        try:
            with torch.cuda.stream(stream):
                M = DeviceMatrix(A)
                # FP64 RBiCG restarts a stalled recycled solve without recycling
                # (stall guard; plain Algorithm 2 diverges on some of the larger
                # strongly convective systems)
                shape = {}
                if self.tune_cache is not None:
                    from . import tune
                    hit = tune.lookup(M, k=req.k, s=self.s, prec=self.prec, cache=self.tune_cache)
                    if hit:
                        shape = {"blocks": hit["blocks"], "chunk": hit["chunk"]}
                S = Solver(M, k=req.k, s=self.s, prec=self.prec, inner_tol=self.inner_tol,
                           max_outer=30, stream=stream, stall_window=4 if self.prec == "f64" else 0,
                           batch=self.batch if A.n <= self.batch_max_rows else None, **shape)
                stats, sols = [], []
                for j in range(req.nsys):
                    b, bt = wl.request_rhs(req, j)
                    bd = torch.as_tensor(b, device="cuda")
                    btd = torch.as_tensor(bt, device="cuda")
                    if j:
                        S.update_recycle()
                    try:
                        x, xt, st = S.solve(bd, btd, tol=self.tol)
                    except RBiCGError as e:  # a failed system is reported, not fatal
                        x, xt, st = None, None, {"status": e.code, "iters": 0,
                                                 "relres": float("nan"),
                                                 "relres_dual": float("nan")}
                    stats.append(st)
                    if self.keep:
                        sols.append(None if x is None else (x.cpu().numpy(), xt.cpu().numpy()))
                stream.synchronize()
        finally:
            # the handle before the matrix it was created on
            if S is not None:
                S.close()
            if M is not None:
                M.close()
        return stats, (sols if self.keep else None)

    # ------------------------------------------------------------ scheduling
    def run(self, requests: List[wl.Request], time_scale: float = 1.0) -> List[RequestResult]:
        """Replay the trace: request r becomes available at r.arrival *
        time_scale seconds after the start.  Returns one result per request
        (in request order)."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        need = {r.rid: request_bytes(r, self.prec, self.s) for r in reqs}
        for r in reqs:
            if need[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs {need[r.rid]} bytes, more than the "
                                 f"budget {self.budget}")
        cv = threading.Condition()
        state = {"used": 0, "active": 0, "next": 0, "error": None}
        results = {}
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def worker():
            while True:
                with cv:
                    while True:
                        if state["error"] is not None or state["next"] >= len(reqs):
                            return
                        r = reqs[state["next"]]
                        wait = r.arrival * time_scale - now()
                        fits = state["used"] + need[r.rid] <= self.budget
                        if wait <= 0 and fits:
                            break
                        cv.wait(timeout=max(0.0005, wait) if wait > 0 else 0.01)
                    state["next"] += 1
                    state["used"] += need[r.rid]
                    state["active"] += 1
                admitted = now()
                try:
                    stats, sols = self.execute(r)
                except Exception as e:  # surfaced to the caller
                    with cv:
                        state["error"] = e
                        cv.notify_all()
                    return
                finished = now()
                with cv:
                    state["used"] -= need[r.rid]
                    state["active"] -= 1
                    results[r.rid] = RequestResult(r.rid, r.arrival * time_scale, admitted,
                                                   finished, r.edge, r.nsys, stats, sols)
                    cv.notify_all()

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if state["error"] is not None:
            raise state["error"]
        return [results[r.rid] for r in requests]


def latency_summary(results: List[RequestResult]) -> dict:
    lat = np.asarray([r.latency for r in results])
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    nsys = sum(r.nsys for r in results)
    return {"requests": len(results), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "makespan_s": float(span), "requests_per_s": len(results) / span,
            "dual_solves_per_s": nsys / span,
            "all_converged": all(st["status"] == 0 for r in results for st in r.stats)}
