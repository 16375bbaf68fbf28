"""BiCG (Algorithm 1) and RBiCG (Algorithm 2) for one dual pair, oracle side.

Everything is FP64 (complex128 when any input is complex) and follows the
algorithms step by step, with these readings of points the paper leaves open:
  * inner product (a, b) = a^H b;
  * the stopping test is relative: ||r|| <= tol*||b|| and ||r~|| <= tol*||b~||
    (if b~ = 0, ||r~_{-1}|| replaces ||b~||);
  * zeta_c and zeta~_c start at zero;
  * rho' = (r~_i, r_i) is always formed before the stopping test, so a cycle
    that ends on the converging iteration still has everything it needs;
  * after the final correction x -= U zeta_c the true residuals are checked,
    and if either fails the solve restarts from the current iterates (at most
    ``max_restarts`` times; iteration counts accumulate);
  * re-seed (Algorithm 1 step 2 / Algorithm 2 step 3): if
    |(r_0, r~_0)| <= 1e-14 ||r_0|| ||r~_0||, x~_{-1} is replaced by the
    SplitMix64 vector of ``rng.reseed_vector`` (at most 3 times);
  * breakdown (|(p~, q)| or |rho| vanishing, or a NaN) stops with
    status "breakdown"; no look-ahead.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .rng import reseed_vector
from . import recycle as rc
from . import sec44 as s44


def as_csr(A):
    """scipy CSR from a scipy matrix, a dense array, or any object with
    n/rowptr/colind/vals attributes."""
    if sp.issparse(A):
        return A.tocsr()
    if isinstance(A, np.ndarray):
        return sp.csr_matrix(A)
    return sp.csr_matrix((np.asarray(A.vals), np.asarray(A.colind), np.asarray(A.rowptr)),
                         shape=(A.n, A.n))


def _hop(A):
    return A.conj().T.tocsr()


def _dot(a, b):
    """(a, b) = a^H b."""
    return np.vdot(a, b)


@dataclass
class SolveResult:
    x: np.ndarray
    xt: np.ndarray
    iters: int
    status: str                       # "ok", "maxit", "breakdown", "stalled"
    relres: float = np.nan            # true ||b - A x|| / ||b||
    relres_dual: float = np.nan
    restarts: int = 0
    cycles: int = 0
    reseeds: int = 0
    U_next: Optional[np.ndarray] = None
    Ut_next: Optional[np.ndarray] = None
    log: dict = field(default_factory=dict)
    history: list = field(default_factory=list)
    lanczos: dict = field(default_factory=dict)
    pencils: list = field(default_factory=list)


def _refnorms(b, bt, r_m1, rt_m1):
    bn = np.linalg.norm(b)
    btn = np.linalg.norm(bt)
    if bn == 0.0:
        bn = np.linalg.norm(r_m1) or 1.0
    if btn == 0.0:
        btn = np.linalg.norm(rt_m1) or 1.0
    return bn, btn


def bicg(A, b, bt, x=None, xt=None, tol=1e-8, maxit=1000, seed=0,
         keep_history=False) -> SolveResult:
    """Algorithm 1 (BiCG) with the relative stopping test."""
    A = as_csr(A)
    AH = _hop(A)
    dt = np.result_type(A.dtype, b.dtype, bt.dtype, np.float64)
    n = A.shape[0]
    x = np.zeros(n, dt) if x is None else np.array(x, dtype=dt)
    xt = np.zeros(n, dt) if xt is None else np.array(xt, dtype=dt)
    b = b.astype(dt); bt = bt.astype(dt)
    # step 1
    r = b - A @ x
    rt = bt - AH @ xt
    # step 2
    reseeds = 0
    while (abs(_dot(rt, r)) <= 1e-14 * np.linalg.norm(r) * np.linalg.norm(rt)
           and np.linalg.norm(r) > 0 and reseeds < 3):
        xt = reseed_vector(seed + reseeds, n, np.iscomplexobj(xt)).astype(dt)
        rt = bt - AH @ xt
        reseeds += 1
    bn, btn = _refnorms(b, bt, r, rt)
    # step 3
    p = np.zeros(n, dt)
    pt = np.zeros(n, dt)
    beta = dt.type(0)
    rho = _dot(rt, r)
    res = SolveResult(x, xt, 0, "maxit", reseeds=reseeds)
    lg = {"alpha": [], "beta": [], "rnorm": [np.linalg.norm(r)], "rtnorm": [np.linalg.norm(rt)],
          "rho": [rho]}
    if np.linalg.norm(r) <= tol * bn and np.linalg.norm(rt) <= tol * btn:
        res.status = "ok"
    else:
        # step 4
        for i in range(1, maxit + 1):
            p = r + beta * p
            pt = rt + np.conj(beta) * pt
            q = A @ p
            qt = AH @ pt
            sigma = _dot(pt, q)
            if sigma == 0 or not np.isfinite(sigma):
                res.status = "breakdown"; res.iters = i; break
            alpha = rho / sigma
            x = x + alpha * p
            xt = xt + np.conj(alpha) * pt
            r = r - alpha * q
            rt = rt - np.conj(alpha) * qt
            rho_new = _dot(rt, r)
            rn, rtn = np.linalg.norm(r), np.linalg.norm(rt)
            lg["alpha"].append(alpha); lg["rnorm"].append(rn); lg["rtnorm"].append(rtn)
            lg["rho"].append(rho_new)
            if keep_history:
                res.history.append(x.copy())
            res.iters = i
            if rn <= tol * bn and rtn <= tol * btn:
                res.status = "ok"; break
            if rho_new == 0 or not np.isfinite(rho_new):
                res.status = "breakdown"; break
            beta = rho_new / rho
            lg["beta"].append(beta)
            rho = rho_new
    res.x, res.xt = x, xt
    res.log = {k: np.asarray(v) for k, v in lg.items()}
    res.relres = np.linalg.norm(b - A @ x) / bn
    res.relres_dual = np.linalg.norm(bt - AH @ xt) / btn
    return res


class _CycleState:
    """Recycle-space update state carried across the cycles of one solve."""

    def __init__(self, U, Ut, k, s, real_problem, svd_tol, setup="explicit", Ct=None):
        self.U, self.Ut = U, Ut            # current system's recycle space
        self.Ct = Ct                        # C~ = A^H U~ of that space
        self.Uj = None                      # U_j, U~_j of the last completed cycle
        self.Utj = None
        self.k, self.s = k, s
        self.real = real_problem
        self.svd_tol = svd_tol
        self.cycles = 0
        if setup not in ("explicit", "recurrence"):
            raise ValueError(f"unknown pencil set-up {setup!r}")
        self.setup = setup
        # Sec. 4.4 state: blocks carried to the next cycle and the run they
        # belong to (a restart starts a new Lanczos process)
        self.blocks = None
        self.blocks_run = None
        self.pencils = []                   # per cycle of the recurrence set-up: case, P, Q (+ inputs)
        self.keep_bases = False

    def update(self, A, AH, V, Vt, alpha, beta_prev, rnorm, rec=None):
        """End of a cycle: V, Vt are the s Lanczos vectors of the cycle;
        alpha, beta_prev (beta_{i-1}), rnorm (||r_{i-1}||) the cycle's scalars.
        ``rec`` (recurrence set-up) carries what Sec. 4.4 needs beyond them:
        run, rn_end, beta_end, the restrictions zeta_i, zeta~_i of the cycle
        and the one before, the dual scale factors, v~_{js+1}, and the previous
        cycle's last alpha, ||r|| and v~."""
        V = np.stack(V, axis=1)
        Vt = np.stack(Vt, axis=1)
        have_prev = self.Uj is not None
        have_sys = self.U is not None and self.U.shape[1] > 0
        if self.setup == "recurrence" and rec is not None:
            done = self._update_sec44(A, AH, V, Vt, alpha, beta_prev, rnorm, rec,
                                      have_prev, have_sys)
            if done:
                self.cycles += 1
                return
        if not have_prev and not have_sys:
            # first cycle of the first system: eigenvectors of T (Sec. 4.2)
            T = rc.t_from_scalars(alpha, beta_prev, rnorm)
            W, Wt, _ = rc.first_cycle_eigvecs(T, self.k, self.real)
            Uj = V @ W
            Utj = Vt @ Wt
        else:
            Uprev = self.Uj if have_prev else self.U
            Utprev = self.Utj if have_prev else self.Ut
            Phi = np.concatenate([Uprev, V], axis=1)
            Phit = np.concatenate([Utprev, Vt], axis=1)
            P, Q, _, _ = rc.harmonic_pencils(A, AH, Phi, Phit)
            W, Wt, _ = rc.pencil_eigvecs(P, Q, self.k, self.real)
            Uj = Phi @ W
            Utj = Phit @ Wt
        m = min(Uj.shape[1], Utj.shape[1])
        Uj, Utj = Uj[:, :m], Utj[:, :m]
        if m > 0:
            Uj, Utj, _, _ = rc.biorthogonalize(A, AH, Uj, Utj, self.svd_tol)
        self.Uj, self.Utj = Uj, Utj
        self.blocks = None
        self.cycles += 1

    def _keep(self, case, P, Q, Phi, Phit, X, YtU, B, Bt, G, Gt):
        d = {"case": case, "P": P, "Q": Q}
        if self.keep_bases:
            d.update(Phi=Phi, Phit=Phit, X=X, YtU=YtU, B=B, Bt=Bt, G=G, Gt=Gt)
        self.pencils.append(d)

    def _update_sec44(self, A, AH, V, Vt, alpha, beta_prev, rnorm, rec, have_prev, have_sys):
        """The cycle update with the pencil set up by the recurrences of
        Sec. 4.4 (module sec44).  Returns False when they do not apply (the
        first cycle of a restarted run that carries a cycle space: its Lanczos
        vectors are not biorthogonal to the earlier cycles' spaces)."""
        s = self.s
        run = rec["run"]
        first_of_run = rec["alpha_before"] is None
        G, Gt = s44.gamma_blocks(alpha, beta_prev, rnorm, rec["rn_end"], rec["beta_end"],
                                 rec["alpha_before"], rec["rnorm_before"])
        kC = self.U.shape[1] if have_sys else 0
        if kC:
            B, Bt = s44.b_blocks(rec["zeta"], rec["zetat"], rec["zeta_before"], rec["zetat_before"],
                                 beta_prev, 1.0 / np.asarray(rnorm), rec["vtscale"])
        else:
            B = np.zeros((0, s)); Bt = np.zeros((0, s))
        if not have_prev and not have_sys:
            case = "T"
            T = rc.t_from_scalars(alpha, beta_prev, rnorm)
            W, Wt, _ = rc.first_cycle_eigvecs(T, self.k, self.real)
            Phi, Phit = V, Vt
            X = s44.empty_blocks(s, G.dtype)
        elif not have_prev and first_of_run:
            case = "first"
            CtU = self.Ct.conj().T @ self.U
            VtU = np.concatenate([Vt, rec["vt_end"][:, None]], axis=1).conj().T @ self.U
            P, Q = s44.pencil_first_cycle(CtU, VtU, B, Bt, G, Gt)
            W, Wt, _ = rc.pencil_eigvecs(P, Q, self.k, self.real)
            Phi = np.concatenate([self.U, V], axis=1)
            Phit = np.concatenate([self.Ut, Vt], axis=1)
            X = s44.system_start_blocks(CtU, s)
            self._keep(case, P, Q, Phi, Phit, X, VtU, B, Bt, G, Gt)
        elif have_prev and self.blocks is not None and self.blocks_run == run and not first_of_run:
            case = "general"
            Ups_t = np.concatenate([rec["vt_before"][:, None], Vt, rec["vt_end"][:, None]], axis=1)
            YtU = Ups_t.conj().T @ self.Uj
            P, Q = s44.pencil_general(self.blocks, YtU, B, Bt, G, Gt)
            W, Wt, _ = rc.pencil_eigvecs(P, Q, self.k, self.real)
            Phi = np.concatenate([self.Uj, V], axis=1)
            Phit = np.concatenate([self.Utj, Vt], axis=1)
            X = self.blocks
            self._keep(case, P, Q, Phi, Phit, X, YtU, B, Bt, G, Gt)
        else:
            return False
        m = min(W.shape[1], Wt.shape[1])
        W, Wt = W[:, :m], Wt[:, :m]
        if m > 0:
            TU, TUt = rc.biorth_transforms(A, AH, Phi @ W, Phit @ Wt, self.svd_tol)
        else:
            TU = np.zeros((0, 0)); TUt = np.zeros((0, 0))
        WN, WtM = W @ TU, Wt @ TUt
        self.Uj, self.Utj = Phi @ WN, Phit @ WtM
        self.blocks = s44.next_blocks(X, WN, WtM, B, Bt, G, Gt)
        self.blocks_run = run
        return True


def rbicg(A, b, bt, x=None, xt=None, U=None, Ut=None, C=None, Ct=None,
          tol=1e-8, maxit=1000, s=40, k=None, update=True, seed=0,
          max_restarts=2, svd_tol=1e-2, keep_history=False,
          keep_lanczos=False, stall_window=None, pencil_setup="explicit") -> SolveResult:
    """Algorithm 2 (RBiCG) for one dual pair with a fixed recycle space U, U~
    (C = A U, C~ = A^H U~, C~^H C = I required), plus the cycle-wise update of
    Sec. 4 producing the recycle space for the next system (``U_next``).

    With an empty recycle space and ``update=False`` this is bitwise Algorithm 1:
    the projection steps are skipped and every other operation is the same.

    ``stall_window`` (default None: off, plain Algorithm 2) is an opt-in stop
    that is not part of the paper: with a recycle space in use, at every cycle
    end (i mod s = 0) the smallest cycle-end value of
    max(||r||/||b||, ||r~||/||b~||) so far is compared with the one
    ``stall_window`` cycles earlier; if it has not halved, the iteration stops
    with status "stalled" (iterates as they are, no final correction, no
    restart).  ``drivers.rbicg_restart_on_stall`` builds the restart on it.

    ``pencil_setup``: "explicit" (default) forms the harmonic Ritz pencil from
    the explicit products A Phi_j, A^H Phi~_j (its plain definition);
    "recurrence" sets it up by the recurrences of Sec. 4.4 (module sec44),
    which are exact in exact arithmetic; the first cycle of a restarted run
    with a carried cycle space falls back to the explicit products.
    """
    A = as_csr(A)
    AH = _hop(A)
    dt = np.result_type(A.dtype, b.dtype, bt.dtype, np.float64,
                        *([U.dtype] if U is not None else []))
    n = A.shape[0]
    kc = 0 if U is None else U.shape[1]
    if kc and (C is None or Ct is None):
        raise ValueError("C and C~ must be given with U")
    x = np.zeros(n, dt) if x is None else np.array(x, dtype=dt)
    xt = np.zeros(n, dt) if xt is None else np.array(xt, dtype=dt)
    b = b.astype(dt); bt = bt.astype(dt)
    kk = k if k is not None else max(kc, 1)
    real_problem = not np.iscomplexobj(np.zeros(0, dt))
    cyc = _CycleState(U if kc else None, Ut if kc else None, kk, s, real_problem, svd_tol,
                      setup=pencil_setup, Ct=Ct if kc else None)
    cyc.keep_bases = keep_lanczos
    rec_on = pencil_setup == "recurrence" and update
    res = SolveResult(x, xt, 0, "maxit")
    lg = {"alpha": [], "beta": [], "rnorm": [], "rtnorm": [], "rho": []}
    lz = {"V": [], "Vt": []}
    total = 0
    restarts = 0
    reseeds = 0
    bn = btn = None
    while True:
        # steps 1-2: eq. minusXR
        r_m1 = b - A @ x
        rt_m1 = bt - AH @ xt
        if kc:
            g = Ct.conj().T @ r_m1
            x0 = x + U @ g
            r = r_m1 - C @ g
        else:
            x0, r = x, r_m1
        def _dual_init(xt_):
            rt_m1_ = bt - AH @ xt_
            if kc:
                gt_ = C.conj().T @ rt_m1_
                return rt_m1_, xt_ + Ut @ gt_, rt_m1_ - Ct @ gt_
            return rt_m1_, xt_, rt_m1_
        rt_m1, xt0, rt = _dual_init(xt)
        # step 3: re-seed
        while (abs(_dot(rt, r)) <= 1e-14 * np.linalg.norm(r) * np.linalg.norm(rt)
               and np.linalg.norm(r) > 0 and reseeds < 3):
            xt = reseed_vector(seed + reseeds, n, np.iscomplexobj(xt)).astype(dt)
            rt_m1, xt0, rt = _dual_init(xt)
            reseeds += 1
        x, xt = x0, xt0
        if bn is None:
            bn, btn = _refnorms(b, bt, r_m1, rt_m1)
        # step 4
        p = np.zeros(n, dt)
        pt = np.zeros(n, dt)
        beta = dt.type(0)
        zeta_c = np.zeros(kc, dt)
        zetat_c = np.zeros(kc, dt)
        rho = _dot(rt, r)
        rn, rtn = np.linalg.norm(r), np.linalg.norm(rt)
        V, Vt, c_alpha, c_beta, c_rn = [], [], [], [], []
        # Sec. 4.4 data: restrictions and dual scales of the cycle, and the
        # previous cycle's last values (none at the start of a run)
        c_zeta, c_zetat, c_vts = [], [], []
        before = {"alpha_before": None, "rnorm_before": None, "zeta_before": None,
                  "zetat_before": None, "vt_before": None}
        converged = rn <= tol * bn and rtn <= tol * btn
        status = "ok" if converged else "maxit"
        # cycle-end values of max(||r||/||b||, ||r~||/||b~||), smallest so far
        best = [max(rn / bn, rtn / btn)]
        i = 0
        while not converged and total < maxit:
            i += 1
            total += 1
            # step 5
            p = r + beta * p
            pt = rt + np.conj(beta) * pt
            z = A @ p
            zt = AH @ pt
            if kc:
                zeta = Ct.conj().T @ z          # C^ = C~
                zetat = C.conj().T @ zt         # C-check = C
                q = z - C @ zeta
                qt = zt - Ct @ zetat
            else:
                q, qt = z, zt
            sigma = _dot(pt, q)
            if sigma == 0 or not np.isfinite(sigma):
                status = "breakdown"; break
            alpha = rho / sigma
            if kc:
                zeta_c = zeta_c + alpha * zeta
                zetat_c = zetat_c + np.conj(alpha) * zetat
            if update:
                v = r / rn
                V.append(v)
                vts = 1.0 / _dot(v, rt)
                Vt.append(rt * vts)
                c_alpha.append(alpha); c_beta.append(beta); c_rn.append(rn)
                if rec_on:
                    c_vts.append(vts)
                    if kc:
                        c_zeta.append(zeta); c_zetat.append(zetat)
            if keep_lanczos:
                v = r / rn
                lz["V"].append(v); lz["Vt"].append(rt / _dot(v, rt))
            x = x + alpha * p
            xt = xt + np.conj(alpha) * pt
            r = r - alpha * q
            rt = rt - np.conj(alpha) * qt
            rho_new = _dot(rt, r)
            rn, rtn = np.linalg.norm(r), np.linalg.norm(rt)
            lg["alpha"].append(alpha); lg["beta"].append(beta); lg["rnorm"].append(rn)
            lg["rtnorm"].append(rtn); lg["rho"].append(rho_new)
            if keep_history:
                res.history.append(x.copy())
            converged = rn <= tol * bn and rtn <= tol * btn
            if update and len(V) == s:
                rec = None
                if rec_on:
                    v_end = r / rn
                    rec = dict(before, run=restarts, rn_end=rn, beta_end=rho_new / rho,
                               zeta=c_zeta, zetat=c_zetat, vtscale=np.asarray(c_vts),
                               vt_end=rt / _dot(v_end, rt))
                    before = {"alpha_before": c_alpha[-1], "rnorm_before": c_rn[-1],
                              "zeta_before": c_zeta[-1] if kc else None,
                              "zetat_before": c_zetat[-1] if kc else None,
                              "vt_before": Vt[-1]}
                cyc.update(A, AH, V, Vt, np.asarray(c_alpha), np.asarray(c_beta),
                           np.asarray(c_rn), rec)
                V, Vt, c_alpha, c_beta, c_rn = [], [], [], [], []
                c_zeta, c_zetat, c_vts = [], [], []
            if converged:
                status = "ok"; break
            if rho_new == 0 or not np.isfinite(rho_new):
                status = "breakdown"; break
            if stall_window and kc and i % s == 0:
                # opt-in stop (not in the paper; see the docstring)
                c = i // s
                best.append(min(best[-1], max(rn / bn, rtn / btn)))
                if c >= stall_window and best[c] >= 0.5 * best[c - stall_window]:
                    status = "stalled"; break
            beta = rho_new / rho
            rho = rho_new
        if status == "stalled":
            break
        # step 7
        if kc:
            x = x - U @ zeta_c
            xt = xt - Ut @ zetat_c
        # true residual check (reading) and restart
        tr = np.linalg.norm(b - A @ x)
        trt = np.linalg.norm(bt - AH @ xt)
        if status == "ok" and (tr > tol * bn or trt > tol * btn) and restarts < max_restarts \
                and total < maxit:
            restarts += 1
            continue
        if status == "ok" and (tr > tol * bn or trt > tol * btn):
            status = "maxit"
        break
    res.x, res.xt = x, xt
    res.iters = total
    res.status = status
    res.relres = np.linalg.norm(b - A @ x) / bn
    res.relres_dual = np.linalg.norm(bt - AH @ xt) / btn
    res.restarts = restarts
    res.reseeds = reseeds
    res.cycles = cyc.cycles
    if cyc.Uj is not None and cyc.Uj.shape[1] > 0:
        res.U_next, res.Ut_next = cyc.Uj, cyc.Utj
    else:
        res.U_next, res.Ut_next = U, Ut
    res.log = {kname: np.asarray(v) for kname, v in lg.items()}
    res.pencils = cyc.pencils
    res.lanczos = lz
    return res
