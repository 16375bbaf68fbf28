"""IRKA (Algorithm 3, E = I) driven by the library's shifted dual solves.

Each IRKA step solves the r shifted dual pairs (sigma_i I - A) v_i = b,
(sigma_i I - A)^H w_i = c with rbicg_solve_shifted (all shifts in one batch,
sharing one recycle space that the shift of smallest modulus rebuilds every
step, so step m+1 recycles what step m learnt), forms the reduced pencil
A_r = W^H A V, E_r = W^H V and b_r, c_r with rbicg_project on the device, and
takes the new shifts as the mirror images of the reduced poles from the host
QZ (rbicg_host_eig).  The previous step's solutions are the initial guesses of
the next step's solves (each new shift takes the solution of the nearest old
shift).  Stops when the relative change of the shifts is below tol (Sec. 6.2
uses 1e-6).  Argument marshalling and the r x r bookkeeping only; every n-sized
operation runs in librbicg.so.
"""
from __future__ import annotations

import ctypes as ct
import time
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import _lib


def ordered(sig) -> np.ndarray:
    """Shifts sorted by real part, then imaginary part (rounded, so that the
    two members of a conjugate pair computed with rounding stay adjacent)."""
    sig = np.asarray(sig, dtype=np.complex128)
    return sig[np.lexsort((np.round(sig.imag, 12), np.round(sig.real, 12)))]


def pencil_eigvals(Ar: np.ndarray, Er: np.ndarray) -> np.ndarray:
    """Eigenvalues of A_r w = lambda E_r w by the library's host QZ."""
    m = Ar.shape[0]
    lib = _lib.load()
    P = np.ascontiguousarray(Ar.T).reshape(-1)   # column-major
    Q = np.ascontiguousarray(Er.T).reshape(-1)
    lam = np.zeros(m, np.complex128)
    rc = lib.rbicg_host_eig(m, P.view(np.float64).ctypes.data_as(_lib._DP),
                            Q.view(np.float64).ctypes.data_as(_lib._DP),
                            lam.view(np.float64).ctypes.data_as(_lib._DP), None, None)
    _lib.check(rc, "rbicg_host_eig")
    return lam


@dataclass
class IrkaRun:
    shifts: List[np.ndarray] = field(default_factory=list)   # shifts solved at each step
    changes: List[float] = field(default_factory=list)
    iters: List[List[int]] = field(default_factory=list)     # per step, per shift
    step_ms: List[float] = field(default_factory=list)
    steps: int = 0
    converged: bool = False
    all_solved: bool = True
    Ar: np.ndarray = None
    Er: np.ndarray = None
    br: np.ndarray = None
    cr: np.ndarray = None


def irka(S, b, c, sigma0, tol=1e-6, maxit=50, solve_tol=1e-10) -> IrkaRun:
    """S: a complex (prec="c128") Solver on A, whose one recycle space all
    shifts share (the second strategy of Sec. 5.2), or a list of r such
    Solvers on one DeviceMatrix, solver i keeping the recycle space of shift
    slot i from one IRKA step to the next (the first strategy; the r solves
    of a step run concurrently on the solvers' streams).  b, c: complex CUDA
    n-vectors; sigma0: initial shifts (closed under conjugation for real A,
    b, c)."""
    import torch
    sig = ordered(sigma0)
    r = len(sig)
    per_shift = isinstance(S, (list, tuple))
    if per_shift and len(S) != r:
        raise ValueError("one solver per shift expected")
    S0 = S[0] if per_shift else S
    X = torch.zeros((r, S0.n), dtype=torch.complex128, device="cuda")
    Xt = torch.zeros_like(X)
    pool = None
    if per_shift:
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=r)
    run = IrkaRun()

    def solve_all(sig, X, Xt):
        if not per_shift:
            return S.solve_shifted(sig, b, c, X, Xt, tol=solve_tol)

        def one(i):
            xi, xti, st = S[i].solve_shifted(sig[i:i + 1], b, c, X[i:i + 1], Xt[i:i + 1],
                                             tol=solve_tol, update_from=0)
            return st[0]
        sts = list(pool.map(one, range(r)))
        return X, Xt, sts

    for step in range(maxit):
        t0 = time.perf_counter()
        X, Xt, sts = solve_all(sig, X, Xt)
        Ar, Er, br, cr = S0.project(X, Xt, b, c)
        run.step_ms.append((time.perf_counter() - t0) * 1e3)
        run.shifts.append(sig.copy())
        run.iters.append([st["iters"] for st in sts])
        run.all_solved &= all(st["status"] == 0 for st in sts)
        run.Ar, run.Er, run.br, run.cr = Ar, Er, br, cr
        run.steps = step + 1
        new = ordered(-pencil_eigvals(Ar, Er))
        change = float(np.max(np.abs(new - sig) / np.abs(sig)))
        run.changes.append(change)
        if change < tol:
            run.converged = True
            break
        # warm start: each new shift starts from the solution of the nearest old one
        near = [int(np.argmin(np.abs(sig - s))) for s in new]
        idx = torch.as_tensor(near, device="cuda")
        X = X.index_select(0, idx).contiguous()
        Xt = Xt.index_select(0, idx).contiguous()
        if per_shift:
            torch.cuda.synchronize()  # the solvers' own streams read X next
        sig = new
    if pool is not None:
        pool.shutdown()
    return run
