"""Autotuner for the iteration-kernel launch shape, with a JSON cache.

Two launch parameters of a handle decide how the rows of an iteration map
onto the GPU and how often the host looks at the stopping test:
  blocks  iteration-kernel blocks of 1024 threads (rows per block n/blocks,
          one to eight rows per thread), automatic by default;
  chunk   iterations launched between two reads of the stopping test.
``autotune`` times a short recycled solve (two cycles of s iterations, the
same kernels and cycle-end work as a real solve) for each candidate pair on
the matrix in question and keeps the fastest per iteration.  Results go to a
JSON cache keyed by device, problem size, vector type and recycle sizes, so
a server tunes a problem shape once (``lookup`` reads the cache without
timing anything).  The choice changes speed only: every candidate solves the
same pair, though the reduction order of the block partial sums, and with it
the rounding, depends on the number of blocks.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Tuple

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rbicg", "tune.json")
ROWS_PER_BLOCK = 1024 * 8   # most rows one 1024-thread block covers


def cache_path(path: Optional[str] = None) -> str:
    return path or os.environ.get("RBICG_TUNE_CACHE") or DEFAULT_CACHE


def key(device: str, n: int, nnz: int, prec: str, k: int, s: int) -> str:
    return f"{device}|n={n}|nnz={nnz}|{prec}|k={k}|s={s}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    p = cache_path(path)
    try:
        with open(p) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(entry_key: str, entry: dict, path: Optional[str] = None) -> None:
    """Add one entry (merged with what the file holds; written atomically)."""
    p = cache_path(path)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    data = load_cache(p)
    data[entry_key] = entry
    tmp = p + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def candidates(n: int, blocks: Iterable[int] = (0, 64, 128, 256, 512, 1024),
               chunks: Iterable[int] = (4, 8, 16)) -> List[Tuple[int, int]]:
    """(blocks, chunk) pairs valid for n rows (blocks 0 = automatic)."""
    least = max(1, -(-n // ROWS_PER_BLOCK))
    most = max(1, -(-n // 1024))          # more blocks than this leave blocks without rows
    bl = sorted({b for b in blocks if b == 0 or least <= b <= min(most, 4096)})
    return [(b, c) for b in bl for c in chunks]


def pick(times: Dict[Tuple[int, int], float]) -> Tuple[int, int]:
    """The fastest candidate; ties go to the automatic grid, then fewer
    blocks, then the larger chunk (fewer host reads)."""
    return min(times, key=lambda bc: (times[bc], bc[0] != 0, bc[0], -bc[1]))


def autotune(A, *, k: int = 20, s: int = 40, prec: str = "f64", cache: Optional[str] = None,
             cands: Optional[List[Tuple[int, int]]] = None, repeats: int = 2, refresh: bool = False,
             measure: Optional[Callable[[int, int], float]] = None) -> dict:
    """Best (blocks, chunk) for the handle shape (A, k, s, prec).  A: host
    CSR or DeviceMatrix.  The cached entry is returned when present (unless
    refresh).  measure(blocks, chunk) -> seconds per iteration replaces the
    GPU timing (for tests of the selection and the cache)."""
    n, nnz, device = _shape(A, measure is not None)
    ek = key(device, n, nnz, prec, k, s)
    if not refresh:
        hit = load_cache(cache).get(ek)
        if hit is not None:
            return dict(hit, cached=True)
    cands = cands or candidates(n)
    meas = measure or _gpu_measure(A, k, s, prec)
    times = {}
    for bc in cands:
        times[bc] = min(meas(*bc) for _ in range(max(1, repeats)))
    b, c = pick(times)
    entry = {"blocks": int(b), "chunk": int(c), "us_per_iter": round(times[(b, c)] * 1e6, 3),
             "auto_us_per_iter": round(min(t for (bb, _), t in times.items() if bb == 0) * 1e6, 3)
             if any(bb == 0 for bb, _ in times) else None,
             "candidates": {f"{bb},{cc}": round(t * 1e6, 3) for (bb, cc), t in sorted(times.items())}}
    store(ek, entry, cache)
    return dict(entry, cached=False)


def lookup(A, *, k: int = 20, s: int = 40, prec: str = "f64", cache: Optional[str] = None,
           device: Optional[str] = None) -> Optional[dict]:
    """The cached entry for the handle shape, or None (nothing is timed)."""
    n, nnz, dev = _shape(A, device is not None)
    return load_cache(cache).get(key(device or dev, n, nnz, prec, k, s))


def _shape(A, no_device: bool):
    if hasattr(A, "info") and callable(A.info):           # DeviceMatrix
        inf = A.info()
        n, nnz = int(inf["n"]), int(inf["nnz"])
    elif hasattr(A, "rowptr"):
        n, nnz = int(A.n), int(A.rowptr[-1])
    else:
        n, nnz = int(A.shape[0]), int(A.nnz)
    device = "cpu"
    if not no_device:
        import torch
        device = torch.cuda.get_device_name(0).replace("|", "/")
    return n, nnz, device


def _gpu_measure(A, k, s, prec):
    """Seconds per iteration of a two-cycle solve with the given launch shape
    that recycles the space of a first, untimed one (a fixed random pair,
    tolerance out of reach so that every candidate runs the same number of
    iterations, with the cycle-end updates)."""
    import torch
    from .solver import DeviceMatrix, Solver
    M = A if hasattr(A, "info") and callable(A.info) else DeviceMatrix(A)
    dtype = torch.complex128 if prec == "c128" else torch.float64
    g = torch.Generator(device="cuda").manual_seed(1234)
    b = torch.randn(M.n, dtype=torch.float64, device="cuda", generator=g).to(dtype)
    bt = torch.randn(M.n, dtype=torch.float64, device="cuda", generator=g).to(dtype)

    def measure(blocks, chunk):
        S = Solver(M, k=k, s=s, maxit=2 * s, prec=prec, blocks=blocks, chunk=chunk)
        try:
            x, xt = torch.zeros_like(b), torch.zeros_like(bt)
            S.solve(b, bt, x, xt, tol=1e-30)          # warm-up: first launches, a cycle space
            x.zero_(); xt.zero_()
            S.update_recycle()                         # the timed solve recycles it
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st = S.solve(b, bt, x, xt, tol=1e-30)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / max(1, st["iters"])
        finally:
            S.close()
    return measure
