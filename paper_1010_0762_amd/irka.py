"""IRKA (Algorithm 3) driven by the library's dual solves.

irka (E = I):
Each IRKA step solves the r shifted dual pairs (sigma_i I - A) v_i = b,
(sigma_i I - A)^H w_i = c with rbicg_solve_shifted (all shifts in one batch,
sharing one recycle space that the shift of smallest modulus rebuilds every
step, so step m+1 recycles what step m learnt), forms the reduced pencil
A_r = W^H A V, E_r = W^H V and b_r, c_r with rbicg_project on the device, and
takes the new shifts as the mirror images of the reduced poles from the host
QZ (rbicg_host_eig).  The previous step's solutions are the initial guesses of
the next step's solves (each new shift takes the solution of the nearest old
shift).  Stops when the relative change of the shifts is below tol (Sec. 6.2
uses 1e-6).

irka_pencil (E != I): every shift slot solves with its own pencil matrix
sigma_i E - A, formed on the device by rbicg_matrix_pencil (see there).

Argument marshalling and the r x r bookkeeping only; every n-sized operation
runs in librbicg.so.
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


def irka_pencil(A, E, b, c, sigma0, *, k=20, s=40, tol=1e-6, maxit=50, solve_tol=1e-10,
                recycle="per_shift", pick_tol=0.5) -> IrkaRun:
    """IRKA for the model G(s) = c^H (s E - A)^{-1} b with E != I (Algorithm
    3; Sec. 5.2 notes that most model-reduction problems have E != I).

    A, E: DeviceMatrix objects on one sparsity pattern (E given on A's
    pattern); b, c: complex CUDA n-vectors; sigma0: initial shifts.  Every
    shift slot i owns a complex pencil matrix sigma_i E - A (rbicg_matrix_pencil,
    values rewritten on the device at each step) and a solver handle on it.
    recycle:
      "per_shift" -- the first strategy of Sec. 5.2: slot i recycles the space
                     its own solve built at the previous step (the r solves
                     of a step run concurrently on the slots' streams);
      "pool"      -- the third strategy: the i-th solve of step m+1 takes the
                     recycle space of the system, among the shifts of step m
                     and the shifts 1..i-1 of step m+1, whose shift is
                     relatively closest to its own (if within pick_tol); the
                     solves of a step then run one after another;
      "none"      -- k = 0.
    A_r = W^H A V and E_r = W^H E V come from rbicg_project on A and on E.
    Initial guesses: the previous solution of the nearest old shift."""
    import torch
    from .solver import DeviceMatrix, Solver
    if recycle not in ("per_shift", "pool", "none"):
        raise ValueError(f"unknown recycling strategy {recycle!r}")
    sig = ordered(sigma0)
    r = len(sig)
    kk = 0 if recycle == "none" else k
    streams = [torch.cuda.Stream() for _ in range(r)]
    torch.cuda.synchronize()
    P = [DeviceMatrix.pencil(A, E, sig[i], -1.0, stream=streams[i]) for i in range(r)]
    torch.cuda.synchronize()
    S = [Solver(P[i], k=kk, s=s, prec="c128", stream=streams[i]) for i in range(r)]
    SA = Solver(A, k=0, s=s, prec="c128")
    SE = Solver(E, k=0, s=s, prec="c128")
    X = torch.zeros((r, A.n), dtype=torch.complex128, device="cuda")
    Xt = torch.zeros_like(X)
    pool = None
    if recycle == "per_shift":
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=r)
    run = IrkaRun()
    prev_sig = None   # shifts whose systems built the slots' current spaces
    try:
        for step in range(maxit):
            t0 = time.perf_counter()
            # every slot's previous work (solves, recycle updates) is done
            # before its pencil's values change
            torch.cuda.synchronize()
            for i in range(r):
                DeviceMatrix.pencil(A, E, sig[i], -1.0, out=P[i], stream=streams[i])

            def one(i):
                with torch.cuda.stream(streams[i]):
                    if step > 0 and kk > 0:
                        S[i].update_recycle(P[i])   # C = (sigma_i E - A) U
                    x, xt, st = S[i].solve(b, c, X[i], Xt[i], tol=solve_tol)
                    return st

            if recycle == "per_shift":
                sts = list(pool.map(one, range(r)))
            elif recycle == "pool":
                sts = []
                built = []   # (shift, slot) of the spaces available to this step
                if prev_sig is not None:
                    built = [(prev_sig[j], j) for j in range(r)]
                for i in range(r):
                    took = False
                    if built and kk > 0:
                        rel = [abs(sg - sig[i]) / abs(sig[i]) for sg, _ in built]
                        j = int(np.argmin(rel))
                        src = built[j][1]
                        if rel[j] <= pick_tol and src != i:
                            # that system's space, installed for slot i's
                            # matrix (C = (sigma_i E - A) U, Sec. 4.3)
                            streams[src].synchronize()
                            U, Ut, _, _ = S[src].get_recycle(next=True, kcap=kk)
                            if U.shape[1] == 0:
                                U, Ut, _, _ = S[src].get_recycle(next=False, kcap=kk)
                            S[i].set_recycle(U, Ut)
                            took = True
                    with torch.cuda.stream(streams[i]):
                        if step > 0 and kk > 0 and not took:
                            S[i].update_recycle(P[i])
                        x, xt, st = S[i].solve(b, c, X[i], Xt[i], tol=solve_tol)
                    sts.append(st)
                    streams[i].synchronize()
                    built = [bs for bs in built if bs[1] != i] + [(sig[i], i)]
            else:
                sts = [one(i) for i in range(r)]
            torch.cuda.synchronize()
            Ar, _, br, cr = SA.project(X, Xt, b, c)
            Er, _ = SE.project(X, Xt)
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
            near = [int(np.argmin(np.abs(sig - z))) for z in new]
            idx = torch.as_tensor(near, device="cuda")
            X = X.index_select(0, idx).contiguous()
            Xt = Xt.index_select(0, idx).contiguous()
            prev_sig = sig
            sig = new
    finally:
        if pool is not None:
            pool.shutdown()
        torch.cuda.synchronize()
        for h in S + [SA, SE]:
            h.close()
        for m in P:
            m.close()
    return run
