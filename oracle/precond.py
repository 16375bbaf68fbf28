"""Split ILU(0) preconditioning in red-black ordering -- TEST INFRASTRUCTURE.

Only tests/, the package smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

The experiments of Sec. 6 split-precondition every system with an incomplete
LU factorization (ILUT / ILUTP) and recycle spaces of the preconditioned
systems.  Reading: the threshold and pivoting variants are tied to MATLAB's
implementation; the no-fill factorization ILU(0) is used here, on the
red-black ordering of the unknowns (red first), for matrices whose
off-diagonal graph is two-colourable (the 5- and 7-point stencils of the
convection-diffusion problems).  With P the red-black permutation and
P A P^T = L U + R the ILU(0) factorization, the dual pair
    A x = b,   A^H x~ = b~
becomes the split-preconditioned pair
    A^ y = L^{-1} P b,   A^^H y~ = U^{-H} P b~,   A^ = L^{-1} P A P^T U^{-1},
    x = P^T U^{-1} y,    x~ = P^T L^{-H} y~.
In red-black ordering A^ is block diagonal, [[I, 0], [0, M_B]] (the pins
check this on the explicit product), so the red part of y is the red part of
the preconditioned right-hand side and RBiCG runs on the black block M_B,
whose recycle spaces are those of the preconditioned systems.  Stopping is on
the preconditioned (black) residual.
"""
from __future__ import annotations

from collections import deque

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import as_csr, rbicg
from . import recycle as rc


def two_coloring(A) -> np.ndarray:
    """0 (red) / 1 (black) per unknown by breadth-first search over the
    off-diagonal graph of A + A^T, each component starting red at its lowest
    index; ValueError if an off-diagonal entry joins two unknowns of one
    colour."""
    A = as_csr(A)
    n = A.shape[0]
    G = (abs(A) + abs(A).T).tocsr()
    col = -np.ones(n, dtype=np.int64)
    for s in range(n):
        if col[s] >= 0:
            continue
        col[s] = 0
        q = deque([s])
        while q:
            i = q.popleft()
            for j in G.indices[G.indptr[i]:G.indptr[i + 1]]:
                if j == i:
                    continue
                if col[j] < 0:
                    col[j] = 1 - col[i]
                    q.append(j)
                elif col[j] == col[i]:
                    raise ValueError("the off-diagonal graph is not two-colourable")
    return col


def rb_permutation(color) -> np.ndarray:
    """perm[new] = old: the red unknowns in ascending order, then the black."""
    color = np.asarray(color)
    return np.concatenate([np.flatnonzero(color == 0), np.flatnonzero(color == 1)])


def ilu0(M):
    """ILU(0) of a square sparse matrix by the row-wise (IKJ) elimination
    restricted to the pattern of M: returns (L unit lower, U upper) with
    (L U)_ij = M_ij on the pattern.  Plain loops (small matrices only)."""
    M = as_csr(M).astype(np.complex128)
    M.sort_indices()
    n = M.shape[0]
    ptr, idx = M.indptr, M.indices
    val = M.data.copy()
    pos = [dict(zip(idx[ptr[i]:ptr[i + 1]], range(ptr[i], ptr[i + 1]))) for i in range(n)]
    for i in range(n):
        for p in range(ptr[i], ptr[i + 1]):
            k = idx[p]
            if k >= i:
                break
            val[p] /= val[pos[k][k]]
            for q in range(ptr[k], ptr[k + 1]):
                j = idx[q]
                if j > k and j in pos[i]:
                    val[pos[i][j]] -= val[p] * val[q]
    F = sp.csr_matrix((val, idx.copy(), ptr.copy()), shape=(n, n))
    L = (sp.tril(F, -1) + sp.identity(n, format="csr")).tocsr()
    U = sp.triu(F).tocsr()
    return L, U


class SplitSystem:
    """The split-preconditioned form of one matrix."""

    def __init__(self, A):
        A = as_csr(A).astype(np.complex128)
        self.n = A.shape[0]
        self.color = two_coloring(A)
        self.perm = rb_permutation(self.color)
        self.nr = int(np.sum(self.color == 0))
        P = sp.csr_matrix((np.ones(self.n), (np.arange(self.n), self.perm)), shape=(self.n, self.n))
        self.P = P
        self.At = (P @ A @ P.T).tocsr()
        self.L, self.U = ilu0(self.At)

    def operator(self) -> np.ndarray:
        """A^ = L^{-1} P A P^T U^{-1} as a dense array (small n)."""
        Ad = self.At.toarray()
        X = spla.spsolve_triangular(self.L.tocsr(), Ad, lower=True)
        return spla.spsolve_triangular(self.U.T.tocsr(), X.T, lower=True).T

    def black_block(self) -> sp.csr_matrix:
        return sp.csr_matrix(self.operator()[self.nr:, self.nr:])

    def rhs(self, b, bt):
        """(L^{-1} P b, U^{-H} P b~)."""
        bh = spla.spsolve_triangular(self.L.tocsr(), self.P @ np.asarray(b, np.complex128), lower=True)
        ch = spla.spsolve_triangular(self.U.conj().T.tocsr(), self.P @ np.asarray(bt, np.complex128),
                                     lower=True)
        return bh, ch

    def solution(self, y, yt):
        """(P^T U^{-1} y, P^T L^{-H} y~)."""
        x = spla.spsolve_triangular(self.U.tocsr(), np.asarray(y, np.complex128), lower=False)
        xt = spla.spsolve_triangular(self.L.conj().T.tocsr(), np.asarray(yt, np.complex128), lower=False)
        return self.P.T @ x, self.P.T @ xt


def rbicg_split_sequence(mats, bs, bts, k, s, tol, maxit=5000, update=True, svd_tol=1e-2,
                         seed=0, max_restarts=2, real=True):
    """The dual pairs in order, each split-preconditioned by its own RB
    ILU(0), RBiCG on the black blocks with the recycle space carried between
    them (built for the preconditioned operators).  Zero initial guesses.
    Returns (solutions [(x, x~)], results of the black solves)."""
    U = Ut = None
    sols, out = [], []
    for j, A in enumerate(mats):
        ss = SplitSystem(A)
        MB = ss.black_block()
        if real:
            MB = MB.real.tocsr()
        MBH = MB.conj().T.tocsr()
        bh, ch = ss.rhs(bs[j], bts[j])
        bB, cB = bh[ss.nr:], ch[ss.nr:]
        if real:
            bB, cB = bB.real, cB.real
        C = Ct = None
        if U is not None and U.shape[1] > 0 and k > 0:
            U, Ut, C, Ct = rc.biorthogonalize(MB, MBH, U, Ut, svd_tol)
            if C is None:
                U = Ut = None
        res = rbicg(MB, bB, cB, None, None, U, Ut, C, Ct, tol=tol, maxit=maxit, s=s, k=k,
                    update=(update and k > 0), seed=seed, max_restarts=max_restarts,
                    svd_tol=svd_tol)
        y = np.concatenate([bh[:ss.nr], res.x])
        yt = np.concatenate([ch[:ss.nr], res.xt])
        x, xt = ss.solution(y, yt)
        if real:
            x, xt = x.real, xt.real
        sols.append((x, xt))
        out.append(res)
        U, Ut = res.U_next, res.Ut_next
    return sols, out


# ---------------------------------------------------------------- ILUT
# General split preconditioning (Sec. 6 uses ILUT / ILUTP): the dual-threshold
# incomplete factorization ILUT(tau, p) by row-wise (IKJ) elimination.
# Reading (the paper's experiments use MATLAB's ILU with a drop tolerance and
# give no more): row-wise (IKJ) elimination without pivoting, with the drop
# rule scaled as MATLAB's: when the elimination of row i reaches column k < i,
# the entry w_k (before division by the pivot u_kk) is dropped if
# |w_k| < tau ||A(:, k)||_2, and a dropped multiplier updates nothing; after
# the elimination an entry w_j, j > i, is dropped if |w_j| < tau ||A(:, j)||_2;
# the diagonal is never dropped.  Afterwards at most p entries (the largest in
# modulus, ties by column) are kept in the L part and in the U part besides
# the diagonal (p = None: no count limit).  tau = 0 and p = None give the
# complete LU factorization (no pivoting).


def ilut(A, tau, p=None):
    """ILUT(tau, p) of a square sparse matrix: (L unit lower, U upper) as
    scipy CSR (complex128).  Plain loops over a dictionary working row, for
    small matrices (the pins and parity cases)."""
    import heapq
    A = as_csr(A).astype(np.complex128)
    A.sort_indices()
    n = A.shape[0]
    cn = np.sqrt(np.asarray(abs(A).power(2).sum(axis=0)).ravel())   # column norms
    Lrows, Urows = [], []   # per row: dict col -> value (U includes the diagonal)
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        w = dict(zip(A.indices[lo:hi].tolist(), A.data[lo:hi].tolist()))
        heap = [j for j in w if j < i]
        heapq.heapify(heap)
        seen = set(heap)
        lpart = {}
        while heap:
            k = heapq.heappop(heap)
            wk = w.pop(k)
            if abs(wk) < tau * cn[k]:
                continue                      # dropped multiplier
            wk = wk / Urows[k][k]
            lpart[k] = wk
            for j, ukj in Urows[k].items():
                if j <= k:
                    continue
                w[j] = w.get(j, 0.0) - wk * ukj
                if j < i and j not in seen:
                    seen.add(j)
                    heapq.heappush(heap, j)
        # finished row: drop small entries (never the diagonal), keep the p largest
        lkeep = lpart
        ukeep = {j: v for j, v in w.items() if j > i and abs(v) >= tau * cn[j]}
        if p is not None:
            lkeep = dict(sorted(lkeep.items(), key=lambda t: (-abs(t[1]), t[0]))[:p])
            ukeep = dict(sorted(ukeep.items(), key=lambda t: (-abs(t[1]), t[0]))[:p])
        d = w.get(i, 0.0)
        if d == 0:
            raise ZeroDivisionError(f"ILUT: zero pivot in row {i}")
        ukeep[i] = d
        Lrows.append(lkeep)
        Urows.append(ukeep)

    def to_csr(rows, unit):
        r, c, v = [], [], []
        for i, row in enumerate(rows):
            for j in sorted(row):
                r.append(i); c.append(j); v.append(row[j])
            if unit:
                r.append(i); c.append(i); v.append(1.0)
        M = sp.csr_matrix((np.asarray(v, np.complex128), (r, c)), shape=(n, n))
        M.sort_indices()
        return M
    return to_csr(Lrows, True), to_csr(Urows, False)


# ---------------------------------------------------------------- ILUTP
# ILUT with column pivoting (Sec. 6.2 preconditions with ILUTP).  Reading
# (the paper gives no details): the column-pivoting variant of ILUT.  Columns
# are tracked in a position list perm (position -> original column, initially
# the identity); row i works in original column indices.  Its lower part is
# the columns already pivotal for rows 0..i-1, eliminated in that pivot order
# with the drop rule of ILUT (|w_c| < tau ||A(:, c)||_2 before division by the
# pivot: dropped, no update); after the elimination the remaining entries are
# dropped when |w_c| < tau ||A(:, c)||_2, except the entry of column perm[i]
# (the unpivoted diagonal).  Among the kept remaining entries the largest in
# modulus (ties: the smallest position) becomes the pivot when its modulus
# times permtol exceeds that of column perm[i]; then the positions of the two
# columns are swapped.  At most p off-pivot entries are then kept in the L and
# U parts (largest modulus, ties by position).  With Q the permutation matrix
# of perm ((A Q)(:, j) = A(:, perm[j])), A Q = L U + E.  permtol = 0 never
# pivots (ILUT); tau = 0, permtol = 1 is LU with complete row-wise column
# partial pivoting.


def ilutp(A, tau, p=None, permtol=1.0):
    """ILUTP(tau, p, permtol): (L unit lower, U upper, perm) with
    A[:, perm] ~ L U; L and U in pivot-position numbering (scipy CSR,
    complex128).  Plain loops over a dictionary working row (small n)."""
    import heapq
    A = as_csr(A).astype(np.complex128)
    A.sort_indices()
    n = A.shape[0]
    cn = np.sqrt(np.asarray(abs(A).power(2).sum(axis=0)).ravel())
    perm = list(range(n))       # position -> original column
    pos = list(range(n))        # original column -> position
    Lrows, Urows = [], []       # L: {position k < i: value}; U: {original column: value}
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        w = dict(zip(A.indices[lo:hi].tolist(), A.data[lo:hi].tolist()))
        heap = [pos[c] for c in w if pos[c] < i]
        heapq.heapify(heap)
        seen = set(heap)
        lpart = {}
        while heap:
            k = heapq.heappop(heap)
            c = perm[k]
            wk = w.pop(c)
            if abs(wk) < tau * cn[c]:
                continue                      # dropped multiplier
            wk = wk / Urows[k][c]
            lpart[k] = wk
            for c2, ukc in Urows[k].items():
                if c2 == c:
                    continue
                w[c2] = w.get(c2, 0.0) - wk * ukc
                k2 = pos[c2]
                if k2 < i and k2 not in seen:
                    seen.add(k2)
                    heapq.heappush(heap, k2)
        dcol = perm[i]
        upart = {c: v for c, v in w.items() if pos[c] >= i and (c == dcol or abs(v) >= tau * cn[c])}
        # pivot: the largest kept entry, ties by position
        best = dcol
        bmod = abs(upart.get(dcol, 0.0))
        for c, v in upart.items():
            if abs(v) > bmod or (abs(v) == bmod and pos[c] < pos[best]):
                best, bmod = c, abs(v)
        if best != dcol and bmod * permtol > abs(upart.get(dcol, 0.0)):
            j = pos[best]
            perm[i], perm[j] = best, dcol
            pos[best], pos[dcol] = i, j
            dcol = best
        d = upart.pop(dcol, 0.0)
        if d == 0:
            raise ZeroDivisionError(f"ILUTP: zero pivot in row {i}")
        lkeep, ukeep = lpart, upart
        if p is not None:
            lkeep = dict(sorted(lkeep.items(), key=lambda t: (-abs(t[1]), t[0]))[:p])
            ukeep = dict(sorted(ukeep.items(), key=lambda t: (-abs(t[1]), pos[t[0]]))[:p])
        ukeep[dcol] = d
        Lrows.append(lkeep)
        Urows.append(ukeep)
    r, c, v = [], [], []
    for i, row in enumerate(Lrows):
        for k, val in row.items():
            r.append(i); c.append(k); v.append(val)
        r.append(i); c.append(i); v.append(1.0)
    L = sp.csr_matrix((np.asarray(v, np.complex128), (r, c)), shape=(n, n))
    r, c, v = [], [], []
    for i, row in enumerate(Urows):
        for col, val in row.items():
            r.append(i); c.append(pos[col]); v.append(val)
    U = sp.csr_matrix((np.asarray(v, np.complex128), (r, c)), shape=(n, n))
    L.sort_indices()
    U.sort_indices()
    return L, U, np.asarray(perm, dtype=np.int64)


class IlutpSystem:
    """Split preconditioning by ILUTP factors, A Q = L U + E:
        A^ y = L^{-1} b,   A^^H y~ = U^{-H} Q^T b~,   A^ = L^{-1} A Q U^{-1},
        x = Q U^{-1} y,    x~ = L^{-H} y~."""

    def __init__(self, A, tau, p=None, permtol=1.0):
        self.A = as_csr(A).astype(np.complex128)
        self.n = self.A.shape[0]
        self.L, self.U, self.perm = ilutp(self.A, tau, p, permtol)

    def operator(self) -> sp.csr_matrix:
        """A^ = L^{-1} (A Q) U^{-1}, formed explicitly (dense, small n)."""
        AQ = self.A[:, self.perm].toarray()
        X = spla.spsolve_triangular(self.L.tocsr(), AQ, lower=True)
        Y = spla.spsolve_triangular(self.U.T.tocsr(), X.T, lower=True).T
        return sp.csr_matrix(Y)

    def rhs(self, b, bt):
        bh = spla.spsolve_triangular(self.L.tocsr(), np.asarray(b, np.complex128), lower=True)
        qt = np.asarray(bt, np.complex128)[self.perm]            # Q^T b~
        ch = spla.spsolve_triangular(self.U.conj().T.tocsr(), qt, lower=True)
        return bh, ch

    def solution(self, y, yt):
        t = spla.spsolve_triangular(self.U.tocsr(), np.asarray(y, np.complex128), lower=False)
        x = np.empty_like(t)
        x[self.perm] = t                                          # Q t
        xt = spla.spsolve_triangular(self.L.conj().T.tocsr(), np.asarray(yt, np.complex128), lower=False)
        return x, xt


class IlutSystem:
    """Split preconditioning of one matrix by its ILUT factors (no
    reordering): the dual pair A x = b, A^H x~ = b~ becomes
        A^ y = L^{-1} b,   A^^H y~ = U^{-H} b~,   A^ = L^{-1} A U^{-1},
        x = U^{-1} y,      x~ = L^{-H} y~."""

    def __init__(self, A, tau, p=None):
        self.A = as_csr(A).astype(np.complex128)
        self.n = self.A.shape[0]
        self.L, self.U = ilut(self.A, tau, p)

    def operator(self) -> sp.csr_matrix:
        """A^ = L^{-1} A U^{-1}, formed explicitly (dense, small n): the plain
        definition of the operator RBiCG iterates with."""
        Ad = self.A.toarray()
        X = spla.spsolve_triangular(self.L.tocsr(), Ad, lower=True)              # L^{-1} A
        Y = spla.spsolve_triangular(self.U.T.tocsr(), X.T, lower=True).T         # (L^{-1} A) U^{-1}
        return sp.csr_matrix(Y)

    def rhs(self, b, bt):
        bh = spla.spsolve_triangular(self.L.tocsr(), np.asarray(b, np.complex128), lower=True)
        ch = spla.spsolve_triangular(self.U.conj().T.tocsr(), np.asarray(bt, np.complex128), lower=True)
        return bh, ch

    def solution(self, y, yt):
        x = spla.spsolve_triangular(self.U.tocsr(), np.asarray(y, np.complex128), lower=False)
        xt = spla.spsolve_triangular(self.L.conj().T.tocsr(), np.asarray(yt, np.complex128), lower=False)
        return x, xt


def rbicg_ilut_sequence(mats, bs, bts, k, s, tol, tau, p=None, maxit=5000, update=True,
                        svd_tol=1e-2, seed=0, max_restarts=2, real=True, permtol=None):
    """The dual pairs in order, each split-preconditioned by its own
    ILUT(tau, p) (ILUTP(tau, p, permtol) when permtol is given), RBiCG on the
    preconditioned operators with the recycle space carried between them.
    Zero initial guesses; stopping on the preconditioned residuals.  Returns
    (solutions [(x, x~)], results)."""
    U = Ut = None
    sols, out = [], []
    for j, A in enumerate(mats):
        ss = IlutSystem(A, tau, p) if permtol is None else IlutpSystem(A, tau, p, permtol)
        M = ss.operator()
        if real:
            M = M.real.tocsr()
        MH = M.conj().T.tocsr()
        bh, ch = ss.rhs(bs[j], bts[j])
        if real:
            bh, ch = bh.real, ch.real
        C = Ct = None
        if U is not None and U.shape[1] > 0 and k > 0:
            U, Ut, C, Ct = rc.biorthogonalize(M, MH, U, Ut, svd_tol)
            if C is None:
                U = Ut = None
        res = rbicg(M, bh, ch, None, None, U, Ut, C, Ct, tol=tol, maxit=maxit, s=s, k=k,
                    update=(update and k > 0), seed=seed, max_restarts=max_restarts,
                    svd_tol=svd_tol)
        res.k_used = 0 if U is None else U.shape[1]   # recycle dimension the solve started with
        x, xt = ss.solution(res.x, res.xt)
        if real:
            x, xt = x.real, xt.real
        sols.append((x, xt))
        out.append(res)
        U, Ut = res.U_next, res.Ut_next
    return sols, out
