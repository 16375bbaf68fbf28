"""Drivers on top of the single-pair oracle solver.

  rbicg_sequence -- a sequence of dual pairs (eq. initialSys): the final U_j,
                    U~_j of system j become U, U~ of system j+1, whose C, C~ are
                    recomputed with the new matrix and biorthogonalized
                    (Sec. 4.3, last paragraph).
  shifted_pairs  -- pairs (sigma I - A) x = b, (sigma I - A)^H x~ = c of IRKA
                    (Algorithm 3, steps 2-3) for several shifts sharing one
                    recycle space U, U~; each shift gets its own C_sigma =
                    (sigma I - A) U biorthogonalized on its own.  For E = I the
                    shifted matrices share A's eigenvectors, which is why one U
                    can serve all shifts (reading; the paper recycles per shift).
  mixed_refine   -- FP64 iterative refinement around an RBiCG inner solve that
                    stores vectors and matrix values in FP32 (not in the paper).
  bilinear       -- u^H A^{-1} w from one dual solve with the correction term
                    x~^H r (error r~^H A^{-1} r, quadratic in the residuals).
  rbicg_restart_on_stall -- not in the paper: Algorithm 2 with the opt-in
                    stall stop of ``rbicg``; a stalled recycled run is
                    followed by a fresh run from the initial guesses without
                    the recycle space.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .krylov import rbicg, as_csr, SolveResult, _dot
from . import recycle as rc


def rbicg_restart_on_stall(A, b, bt, x=None, xt=None, U=None, Ut=None, C=None, Ct=None,
                           tol=1e-8, maxit=1000, s=40, k=None, update=True, seed=0,
                           max_restarts=2, svd_tol=1e-2, stall_window=4) -> SolveResult:
    """Restart without recycling after a stall (a heuristic of this
    implementation, not part of the paper).  An oblique projector I - C C~^H
    with nearly orthogonal C and C~ can keep a recycled iteration from
    converging on strongly non-normal operators.  First ``rbicg`` runs with
    ``stall_window`` (it stops with status "stalled" when the smallest
    cycle-end residual has not halved over that many cycles); then, if it
    stalled and a restart is left, a second ``rbicg`` runs from the initial
    guesses x, x~ with no recycle space (its cycles build a new one) and the
    remaining iteration budget.  Iteration counts and logs accumulate; the
    stall counts as one of the ``max_restarts``.  Returns a SolveResult whose
    ``restarts`` includes the stall restart."""
    A = as_csr(A)
    first = rbicg(A, b, bt, x, xt, U, Ut, C, Ct, tol=tol, maxit=maxit, s=s, k=k, update=update,
                  seed=seed, max_restarts=max_restarts, svd_tol=svd_tol,
                  stall_window=stall_window)
    if first.status != "stalled":
        return first
    if max_restarts < 1 or first.iters >= maxit:
        first.status = "maxit"
        return first
    kk = k if k is not None else (U.shape[1] if U is not None else None)
    second = rbicg(A, b, bt, x, xt, None, None, None, None, tol=tol, maxit=maxit - first.iters,
                   s=s, k=kk, update=update, seed=seed + first.reseeds,
                   max_restarts=max_restarts - 1, svd_tol=svd_tol)
    second.iters += first.iters
    second.restarts += 1
    second.reseeds += first.reseeds
    second.log = {key: np.concatenate([np.asarray(first.log[key]), np.asarray(second.log[key])])
                  for key in second.log}
    second.stalled_at = first.iters
    return second


def rbicg_sequence(mats, bs, bts, k, s, tol, maxit=5000, x0s=None, xt0s=None,
                   update=True, svd_tol=1e-2, seed=0, max_restarts=2,
                   U0=None, Ut0=None, stall_window=None, pencil_setup="explicit"):
    """Solve the dual pairs in order, recycling between them.  With k=0 (or
    update=False and no U0) this is plain BiCG on every pair.  With
    ``stall_window`` every pair goes through ``rbicg_restart_on_stall``
    instead of plain ``rbicg``.
    Returns (results, (U, U~)) with the recycle space left after the last pair."""
    U, Ut = U0, Ut0
    out = []
    for j, A in enumerate(mats):
        A = as_csr(A)
        AH = A.conj().T.tocsr()
        C = Ct = None
        if U is not None and U.shape[1] > 0 and k > 0:
            U, Ut, C, Ct = rc.biorthogonalize(A, AH, U, Ut, svd_tol)
            if C is None:
                U = Ut = None
        x0 = None if x0s is None else x0s[j]
        xt0 = None if xt0s is None else xt0s[j]
        kw = dict(tol=tol, maxit=maxit, s=s, k=k, update=(update and k > 0), seed=seed,
                  max_restarts=max_restarts, svd_tol=svd_tol)
        if pencil_setup != "explicit":
            kw["pencil_setup"] = pencil_setup
        if stall_window:
            res = rbicg_restart_on_stall(A, bs[j], bts[j], x0, xt0, U, Ut, C, Ct,
                                         stall_window=stall_window, **kw)
        else:
            res = rbicg(A, bs[j], bts[j], x0, xt0, U, Ut, C, Ct, **kw)
        out.append(res)
        U, Ut = res.U_next, res.Ut_next
    return out, (U, Ut)


def shifted_matrix(A, sigma):
    A = as_csr(A)
    n = A.shape[0]
    return (sigma * sp.identity(n, dtype=np.complex128, format="csr") - A).tocsr()


def shifted_pairs(A, b, c, sigmas, U=None, Ut=None, k=20, s=40, tol=1e-8,
                  maxit=5000, x0s=None, xt0s=None, update_from=None,
                  svd_tol=1e-2, seed=0):
    """One IRKA-style sweep: for each shift sigma_i solve
    (sigma_i I - A) x_i = b and (sigma_i I - A)^H x~_i = c with RBiCG, all
    shifts sharing the recycle space (U, U~).  The recycle space for the next
    sweep comes from the cycle data of shift index ``update_from`` (default: the
    shift of smallest modulus; reading, since the paper recycles only for the
    small shifts).  Returns (results, (U_next, U~_next))."""
    A = as_csr(A)
    if update_from is None:
        update_from = int(np.argmin(np.abs(np.asarray(sigmas))))
    out = []
    Unext = Utnext = None
    for i, sg in enumerate(sigmas):
        M = shifted_matrix(A, sg)
        MH = M.conj().T.tocsr()
        Ui = Uti = C = Ct = None
        if U is not None and U.shape[1] > 0:
            Ui, Uti, C, Ct = rc.biorthogonalize(M, MH, U.astype(np.complex128),
                                                Ut.astype(np.complex128), svd_tol)
            if C is None:
                Ui = Uti = None
        x0 = None if x0s is None else x0s[i]
        xt0 = None if xt0s is None else xt0s[i]
        res = rbicg(M, b.astype(np.complex128), c.astype(np.complex128), x0, xt0,
                    Ui, Uti, C, Ct, tol=tol, maxit=maxit, s=s, k=k,
                    update=(i == update_from), seed=seed, svd_tol=svd_tol)
        out.append(res)
        if i == update_from:
            Unext, Utnext = res.U_next, res.Ut_next
    if Unext is None:
        Unext, Utnext = U, Ut
    return out, (Unext, Utnext)


# No-progress window of the FP32 inner solve, in cycles (reading for FP32
# storage): BiCG's residual norms are not monotone and plateau for a few
# cycles on convection-dominated operators before dropping again.
FP32_NOPROGRESS_CYCLES = 6


def _f32(v):
    return np.asarray(v).astype(np.float32)


def rbicg_fp32_inner(A32, AH32, b, bt, U, Ut, C, Ct, tol, maxit, s, k, update,
                     svd_tol=1e-2, A64=None, AH64=None):
    """RBiCG with FP32 storage: matrix values and every n-vector are float32;
    each element operation is evaluated in float64 and rounded once when stored;
    all inner products and norms accumulate in float64.  Starts from x = x~ = 0.
    With a recycle space, r and r~ are re-projected in every iteration (see
    the loop).
    The recycle space (U, C, ...) is given in FP64 and used through FP32
    copies; the cycle update works in FP64 on the FP64 matrix (A64) from the
    FP32-stored Lanczos vectors.  Returns (d, d~, iters, cycle state)."""
    from .krylov import _CycleState
    n = A32.shape[0]
    f64 = np.float64
    kc = 0 if U is None else U.shape[1]
    U32, Ut32 = (_f32(U), _f32(Ut)) if kc else (None, None)
    C32, Ct32 = (_f32(C), _f32(Ct)) if kc else (None, None)
    A64e = A32.astype(f64)
    AH64e = AH32.astype(f64)
    r = _f32(b); rt = _f32(bt)        # r_{-1} with x_{-1} = 0
    x = np.zeros(n, np.float32); xt = np.zeros(n, np.float32)
    if kc:
        g = Ct32.astype(f64).T @ r.astype(f64)
        x = _f32(x.astype(f64) + U32.astype(f64) @ g)
        r = _f32(r.astype(f64) - C32.astype(f64) @ g)
        gt = C32.astype(f64).T @ rt.astype(f64)
        xt = _f32(xt.astype(f64) + Ut32.astype(f64) @ gt)
        rt = _f32(rt.astype(f64) - Ct32.astype(f64) @ gt)
    bn = np.linalg.norm(b); btn = np.linalg.norm(bt)
    cyc = _CycleState(U if kc else None, Ut if kc else None, k, s, True, svd_tol)
    p = np.zeros(n, np.float32); pt = np.zeros(n, np.float32)
    beta = 0.0
    zeta_c = np.zeros(kc); zetat_c = np.zeros(kc)
    rho = float(rt.astype(f64) @ r.astype(f64))
    rn = np.linalg.norm(r.astype(f64)); rtn = np.linalg.norm(rt.astype(f64))
    V, Vt, ca, cb, cr = [], [], [], [], []
    # relative residual max(||r||/||b||, ||r~||/||b~||) by iteration, for the
    # stagnation stop below
    hist = [max(rn / bn, rtn / btn)]
    best = [hist[0]]     # smallest cycle-end value of hist so far, by cycle
    diverged = False
    it = 0
    while it < maxit and not (rn <= tol * bn and rtn <= tol * btn):
        it += 1
        p = _f32(r.astype(f64) + beta * p.astype(f64))
        pt = _f32(rt.astype(f64) + beta * pt.astype(f64))
        z = _f32(A64e @ p.astype(f64))
        zt = _f32(AH64e @ pt.astype(f64))
        if kc:
            zeta = Ct32.astype(f64).T @ z.astype(f64)
            zetat = C32.astype(f64).T @ zt.astype(f64)
            q = _f32(z.astype(f64) - C32.astype(f64) @ zeta)
            qt = _f32(zt.astype(f64) - Ct32.astype(f64) @ zetat)
        else:
            q, qt = z, zt
        sigma = float(pt.astype(f64) @ q.astype(f64))
        if sigma == 0.0 or not np.isfinite(sigma):
            diverged = True      # breakdown in float storage: treated as divergence
            break
        alpha = rho / sigma
        if kc:
            zeta_c += alpha * zeta
            zetat_c += alpha * zetat
        if update:
            v = r.astype(f64) / rn
            V.append(v); Vt.append(rt.astype(f64) / float(v @ rt.astype(f64)))
            ca.append(alpha); cb.append(beta); cr.append(rn)
        if kc:
            # Re-projection (reading for FP32 storage, not in the paper): in
            # exact arithmetic C~^H r = 0 and C^H r~ = 0 (Sec. 3.1), so
            # r <- r - C (C~^H r) together with zeta_c <- zeta_c - C~^H r
            # changes nothing; in float storage the rounding of every update
            # feeds C~^H r, which the oblique projector amplifies until the
            # iteration stagnates.  Done on r_{i-1} once per iteration.
            g = Ct32.astype(f64).T @ r.astype(f64)
            gt = C32.astype(f64).T @ rt.astype(f64)
            r = _f32(r.astype(f64) - C32.astype(f64) @ g)
            rt = _f32(rt.astype(f64) - Ct32.astype(f64) @ gt)
            zeta_c -= g
            zetat_c -= gt
        x = _f32(x.astype(f64) + alpha * p.astype(f64))
        xt = _f32(xt.astype(f64) + alpha * pt.astype(f64))
        r = _f32(r.astype(f64) - alpha * q.astype(f64))
        rt = _f32(rt.astype(f64) - alpha * qt.astype(f64))
        rho_new = float(rt.astype(f64) @ r.astype(f64))
        rn = np.linalg.norm(r.astype(f64)); rtn = np.linalg.norm(rt.astype(f64))
        if rho_new == 0.0 or not (np.isfinite(rho_new) and np.isfinite(rn) and np.isfinite(rtn)):
            diverged = True
            break
        if update and len(V) == s:
            cyc.update(A64, AH64, V, Vt, np.asarray(ca), np.asarray(cb), np.asarray(cr))
            V, Vt, ca, cb, cr = [], [], [], [], []
        if rn <= tol * bn and rtn <= tol * btn:
            break
        hist.append(max(rn / bn, rtn / btn))
        # Cycle-end guards (reading for FP32 storage, not in the paper):
        #  stagnation -- float storage (behind the oblique projector when a
        #    recycle space is in use) limits the attainable residual to about
        #    the inner tolerance; once below sqrt(tol), a cycle that does not
        #    halve the residual returns the iterate and lets the FP64 outer
        #    loop go on;
        #  no progress -- float rounding can keep the iteration from
        #    converging where FP64 converges (ill-conditioned deflation with
        #    some recycle spaces; plain BiCG on strongly non-normal operators):
        #    when the best cycle-end residual has not halved over the last six
        #    cycles, stop; above sqrt(tol) the solve counts as diverged (the
        #    outer loop discards it, drops the recycle space and takes its next
        #    inner solve in FP64), else as stagnated.
        if it % s == 0 and it >= s:
            c = it // s
            best.append(min(best[-1], hist[it]))
            if hist[it] <= np.sqrt(tol) and hist[it] >= 0.5 * hist[it - s]:
                break
            if c >= FP32_NOPROGRESS_CYCLES and best[c] >= 0.5 * best[c - FP32_NOPROGRESS_CYCLES]:
                if best[c] > np.sqrt(tol):
                    diverged = True
                break
        beta = rho_new / rho
        rho = rho_new
    d = x.astype(f64)
    dt_ = xt.astype(f64)
    if kc:
        d = d - U @ zeta_c
        dt_ = dt_ - Ut @ zetat_c
    return d, dt_, it, cyc, diverged


# unit roundoff of IEEE binary32
EPS32 = 2.0 ** -24


def mixed_svd_tol(svd_tol, inner_tol):
    """Cosine cut of the biorthogonalization in FP32-inner mode (reading, not
    in the paper): float rounding inside the projected iteration is amplified
    by ||I - C C~^H|| <= 1 + 1/tau, so the attainable inner residual is about
    eps32 / tau; keeping it ten times below the inner tolerance needs
    tau >= 10 eps32 / inner_tol."""
    return max(svd_tol, 10.0 * EPS32 / inner_tol)


def mixed_refine(A, b, bt, U=None, Ut=None, k=30, s=40, tol=1e-10,
                 inner_tol=1e-5, max_outer=30, maxit_inner=5000, svd_tol=1e-2,
                 update=True):
    """FP64 iterative refinement with an FP32-storage RBiCG inner solver.
    Outer: r = b - A x, r~ = b~ - A^H x~ in FP64; stop when both relative true
    residuals are <= tol; otherwise solve A d = r, A^H d~ = r~ to inner_tol
    relative with the FP32 inner RBiCG and update x += d, x~ += d~ in FP64.
    The recycle space carries over between outer steps (the latest cycle's
    space when one completed), biorthogonalized with the cut of
    mixed_svd_tol.  Safeguards (readings): an inner solve stopped as diverging
    is discarded and the next outer step solves in FP64 (plain BiCG); a
    correction that raises max(||r||/||b||, ||r~||/||b~||) is taken back
    (x -= d, x~ -= d~); either way the recycle space is dropped.
    Returns (x, x~, info, (U, U~))."""
    A = as_csr(A).astype(np.float64)
    AH = A.T.tocsr()
    A32 = A.astype(np.float32)
    AH32 = AH.astype(np.float32)
    tau = mixed_svd_tol(svd_tol, inner_tol)
    escalate = False     # next inner solve in FP64 (after a diverged FP32 one)
    fp64_inner = 0
    n = A.shape[0]
    x = np.zeros(n); xt = np.zeros(n)
    bn = np.linalg.norm(b); btn = np.linalg.norm(bt)
    bn = bn if bn > 0 else 1.0
    btn = btn if btn > 0 else 1.0
    inner_total = 0
    outer = 0
    prev = None          # residual measure before the last applied correction
    last = None          # the last applied correction (d, d~)
    while True:
        r = b - A @ x
        rt = bt - AH @ xt
        rel, relt = np.linalg.norm(r) / bn, np.linalg.norm(rt) / btn
        if last is not None and max(rel, relt) > prev:
            x = x - last[0]
            xt = xt - last[1]
            U = Ut = None
            r = b - A @ x
            rt = bt - AH @ xt
            rel, relt = np.linalg.norm(r) / bn, np.linalg.norm(rt) / btn
        last = None
        if (rel <= tol and relt <= tol) or outer >= max_outer:
            break
        if escalate:
            # FP64 inner solve (plain BiCG, Algorithm 1) for this outer step
            res = rbicg(A, r, rt, tol=inner_tol, maxit=maxit_inner, k=0, update=False)
            inner_total += res.iters
            outer += 1
            fp64_inner += 1
            escalate = False
            prev = max(rel, relt)
            last = (res.x, res.xt)
            x = x + res.x
            xt = xt + res.xt
            continue
        C = Ct = None
        if U is not None and U.shape[1] > 0:
            U, Ut, C, Ct = rc.biorthogonalize(A, AH, U, Ut, tau)
            if C is None:
                U = Ut = None
        d, dt_, it, cyc, diverged = rbicg_fp32_inner(A32, AH32, r, rt, U, Ut, C, Ct, inner_tol,
                                                     maxit_inner, s, k, update, tau, A, AH)
        inner_total += it
        outer += 1
        if diverged:
            U = Ut = None
            escalate = True
            continue
        prev = max(rel, relt)
        last = (d, dt_)
        x = x + d
        xt = xt + dt_
        if cyc.Uj is not None and cyc.Uj.shape[1] > 0:
            U, Ut = cyc.Uj, cyc.Utj
    info = {"outer": outer, "inner_iters": inner_total, "relres": rel, "relres_dual": relt,
            "fp64_inner": fp64_inner}
    return x, xt, info, (U, Ut)


def bilinear(A, u, w, tol=1e-8, maxit=5000, U=None, Ut=None, C=None, Ct=None, s=40,
             k=None, update=False):
    """u^H A^{-1} w (Sec. 1): solve A x = w and A^H x~ = u with RBiCG and return
    u^H x + x~^H r with the true residual r = w - A x.  Since
    u^H A^{-1} w = u^H x + x~^H r + r~^H A^{-1} r, the error is r~^H A^{-1} r,
    bounded by ||r~|| ||A^{-1}|| ||r||.  Returns (value, ||r|| * ||r~||, result)."""
    A = as_csr(A)
    res = rbicg(A, w, u, None, None, U, Ut, C, Ct, tol=tol, maxit=maxit, s=s, k=k,
                update=update)
    r = w - A @ res.x
    rt = u - A.conj().T @ res.xt
    val = _dot(u, res.x) + _dot(res.xt, r)
    return val, float(np.linalg.norm(r) * np.linalg.norm(rt)), res
