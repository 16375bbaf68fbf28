"""Seeded synthetic inputs for the recycling-BiCG solvers.

This module only builds problem data: sparse operators in CSR form, right-hand
sides, shift schedules and request traces.  It holds none of the solver's
arithmetic, so both the HIP path and the CPU checker can draw their inputs from
it without sharing any solver code.

The operators stand in for the paper's test problems (convection-diffusion in
Sec. 6.1; the rail heat-transfer model in Sec. 6.2, which is a symmetric
negative definite system used through shifted pairs (sigma I - A)).  The
paper's own coefficient field and the rail matrices are not reproduced; the
recipes below use the same structure (stencil, size, sign and spectrum class).

All randomness comes from ``numpy.random.default_rng(BASE_SEED + cfg)``, with
draws in the order: b, then b~, then any per-system draws.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 10100762


@dataclass
class CSR:
    """Compressed sparse row matrix with int32 indices (row pointers and column
    indices) and float64 values."""
    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=self.vals.dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.colind] = self.vals
        return d


def _assemble(n: int, rows: List[np.ndarray], cols: List[np.ndarray],
              vals: List[np.ndarray]) -> CSR:
    """Sort (row, col) triplets into CSR order; no duplicates are produced by
    the stencil builders below."""
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(vals).astype(np.float64)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    counts = np.bincount(r, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    assert rowptr[-1] < 2**31
    return CSR(n, rowptr.astype(np.int32), c.astype(np.int32), v)


def _stencil(dims: Sequence[int], diag: float, lower: Sequence[float],
             upper: Sequence[float]) -> CSR:
    """Constant-coefficient (2d+1)-point stencil on a tensor grid with
    homogeneous Dirichlet boundaries eliminated.  Unknowns are ordered
    lexicographically with the first axis fastest.  ``lower[a]`` couples a point
    to its neighbour at index-1 along axis a, ``upper[a]`` to index+1."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    strides = np.cumprod((1,) + dims[:-1])
    rows, cols, vals = [idx], [idx], [np.full(n, diag)]
    for a, d in enumerate(dims):
        m = coords[a] > 0
        rows.append(idx[m]); cols.append(idx[m] - strides[a])
        vals.append(np.full(int(m.sum()), lower[a]))
        m = coords[a] < d - 1
        rows.append(idx[m]); cols.append(idx[m] + strides[a])
        vals.append(np.full(int(m.sum()), upper[a]))
    return _assemble(n, rows, cols, vals)


def convdiff(N: int, dim: int, beta: Sequence[float]) -> CSR:
    """-Laplace(u) + beta . grad(u) on the unit square/cube, N interior points
    per axis, h = 1/(N+1), first-order upwind convection (backward difference
    for a positive velocity component, forward for a negative one), unscaled
    1/h^2 and 1/h terms, Dirichlet zero boundary eliminated."""
    h = 1.0 / (N + 1)
    beta = [float(b) for b in beta]
    assert len(beta) == dim
    diag = 2.0 * dim / h**2 + sum(abs(b) for b in beta) / h
    lower = [-1.0 / h**2 - max(b, 0.0) / h for b in beta]
    upper = [-1.0 / h**2 - max(-b, 0.0) / h for b in beta]
    return _stencil([N] * dim, diag, lower, upper)


def jump_convdiff2d(N: int = 63, contrast: float = 1e3, tiles: int = 4,
                    beta: Sequence[float] = (50.0, 25.0)) -> CSR:
    """-(a u_x)_x - (a u_y)_y + beta . grad(u) on the unit square, N x N
    interior points (default h = 1/64, n = 3969, the grid of the 2D experiment
    of Sec. 6.1), central differences for the convection (as there), and a
    piecewise-constant diffusion coefficient a = contrast on the tiles x tiles
    checkerboard's even cells and 1 on the odd ones (the paper's coefficient is
    given only in a figure; this is a synthetic stand-in with the same kind of
    jumps).  Face coefficients are harmonic means of the two cell-centre
    values; Dirichlet zero boundary eliminated; unknowns x-fastest."""
    h = 1.0 / (N + 1)
    n = N * N
    x = (np.arange(N) + 1) * h

    def a(px, py):
        ix = np.minimum((px * tiles).astype(np.int64), tiles - 1)
        iy = np.minimum((py * tiles).astype(np.int64), tiles - 1)
        return np.where((ix + iy) % 2 == 0, contrast, 1.0)

    X, Y = np.meshgrid(x, x, indexing="xy")     # X[j, i] = x_i, Y[j, i] = y_j
    X, Y = X.ravel(), Y.ravel()
    ac = a(X, Y)

    def face(dx, dy):
        an = a(X + dx, Y + dy)
        return 2.0 * ac * an / (ac + an)

    aw, ae, as_, an_ = face(-h, 0.0), face(h, 0.0), face(0.0, -h), face(0.0, h)
    idx = np.arange(n, dtype=np.int64)
    i, j = idx % N, idx // N
    bx, by = float(beta[0]), float(beta[1])
    rows, cols, vals = [idx], [idx], [(aw + ae + as_ + an_) / h**2]
    for m, off, v in ((i > 0, -1, -aw / h**2 - bx / (2 * h)), (i < N - 1, 1, -ae / h**2 + bx / (2 * h)),
                      (j > 0, -N, -as_ / h**2 - by / (2 * h)), (j < N - 1, N, -an_ / h**2 + by / (2 * h))):
        rows.append(idx[m]); cols.append(idx[m] + off); vals.append(v[m])
    return _assemble(n, rows, cols, vals)


def aniso_diffusion(N: int, kappa: Sequence[float] = (1.0, 0.1, 0.01),
                    shift: float = 0.1) -> CSR:
    """A = -L_kappa - shift*I with L_kappa the 7-point SPD operator
    -(kappa_x u_xx + kappa_y u_yy + kappa_z u_zz), h = 1/(N+1).  A is symmetric
    negative definite, like the rail model's A."""
    h = 1.0 / (N + 1)
    k = [float(v) for v in kappa]
    diag = -(2.0 * sum(k) / h**2) - shift
    off = [ki / h**2 for ki in k]
    return _stencil([N, N, N], diag, off, off)


# ----------------------------------------------------------------------------
# the five workload recipes
# ----------------------------------------------------------------------------

@dataclass
class DualSequence:
    """A sequence of dual systems A_j x = b_j, A_j^H x~ = b~_j."""
    name: str
    mats: List[CSR]
    b: List[np.ndarray]
    bt: List[np.ndarray]
    k: int
    s: int
    tol: float
    extra: dict = field(default_factory=dict)


def cfg1_sequence(nsys: int = 5) -> DualSequence:
    """2D convection-diffusion, 32x32 interior grid (n=1024), 5-point upwind,
    beta_j = (1+0.05j)(10,5); b, b~ ~ U[0,1] drawn once; k=10, s=40, tol 1e-8."""
    rng = np.random.default_rng(BASE_SEED + 1)
    n = 32 * 32
    b = rng.uniform(0.0, 1.0, n)
    bt = rng.uniform(0.0, 1.0, n)
    mats = [convdiff(32, 2, [(1 + 0.05 * j) * 10.0, (1 + 0.05 * j) * 5.0])
            for j in range(nsys)]
    return DualSequence("convdiff2d_32", mats, [b] * nsys, [bt] * nsys, 10, 40, 1e-8)


def cfg2_sequence(nsys: int = 10, N: int = 64) -> DualSequence:
    """3D convection-diffusion 7-point upwind on N^3 (default 64^3, n=262144),
    beta_j = (20,10,5)(1+0.02j); b, b~ ~ N(0,1) drawn once; k=20, s=40, tol 1e-8."""
    rng = np.random.default_rng(BASE_SEED + 2)
    n = N ** 3
    b = rng.standard_normal(n)
    bt = rng.standard_normal(n)
    mats = [convdiff(N, 3, [20.0 * (1 + 0.02 * j), 10.0 * (1 + 0.02 * j),
                            5.0 * (1 + 0.02 * j)]) for j in range(nsys)]
    return DualSequence(f"convdiff3d_{N}", mats, [b] * nsys, [bt] * nsys, 20, 40, 1e-8)


def ilut2d_sequence(nsys: int = 4, N: int = 40, repeat: bool = False) -> DualSequence:
    """Split-ILUT cases: 2D convection-diffusion 5-point upwind on N x N
    (default n=1600); beta_j = (40(1+0.03j), 20(1-0.02j)), or beta = (40, 20)
    for every system when repeat (the same pair solved nsys times, as in the
    2D experiment of Sec. 6.1); a fresh N(0,1) pair b_j, b~_j per system (one
    pair when repeat); k=5, s=10 (k=10, s=20 when repeat), tol 1e-8.  The drop
    tolerance goes in extra["droptol"] (0.2: a weaker factorization than the
    paper's 0.05, so that these small systems take several cycles)."""
    rng = np.random.default_rng(BASE_SEED + 6)
    n = N * N
    if repeat:
        b, bt = rng.standard_normal(n), rng.standard_normal(n)
        A = convdiff(N, 2, [40.0, 20.0])
        return DualSequence(f"ilut_convdiff2d_{N}_repeat", [A] * nsys, [b] * nsys, [bt] * nsys,
                            10, 20, 1e-8, {"droptol": 0.2})
    bs = [rng.standard_normal(n) for _ in range(nsys)]
    bts = [rng.standard_normal(n) for _ in range(nsys)]
    mats = [convdiff(N, 2, [40.0 * (1 + 0.03 * j), 20.0 * (1 - 0.02 * j)]) for j in range(nsys)]
    return DualSequence(f"ilut_convdiff2d_{N}", mats, bs, bts, 5, 10, 1e-8, {"droptol": 0.2})


def irka_problem(N: int = 48, r: int = 8, eps: float = 0.3):
    """IRKA (Algorithm 3, E = I) on A = -L_kappa - 0.1 I (N^3, symmetric
    negative definite like the rail model's A): input b ~ N(0,1), output
    c = b + eps g with g ~ N(0,1) (a nearly collocated SISO pair), r initial
    shifts logarithmically spaced on [1, 1e4].  Returns (A, b, c, sigma0)."""
    rng = np.random.default_rng(BASE_SEED + 6)
    A = aniso_diffusion(N)
    n = N ** 3
    b = rng.standard_normal(n)
    c = b + eps * rng.standard_normal(n)
    return A, b, c, np.logspace(0.0, 4.0, r).astype(np.complex128)


def mass_like(N: int) -> CSR:
    """An SPD matrix on the 7-point pattern of an N^3 grid: 0.6 on the
    diagonal, 1/12 for each of the six neighbours (strictly diagonally
    dominant), standing in for a finite-element mass matrix E."""
    return _stencil([N, N, N], 0.6, [1.0 / 12] * 3, [1.0 / 12] * 3)


def irka_problem_e(N: int = 48, r: int = 8, eps: float = 0.3):
    """IRKA with E != I (the model E x' = A x + b v, y = c^* x of Sec. 5): A
    as in irka_problem, E = mass_like(N) on A's sparsity pattern, b, c and
    the initial shifts as in irka_problem.  Returns (A, E, b, c, sigma0)."""
    A, b, c, s0 = irka_problem(N, r, eps)
    return A, mass_like(N), b, c, s0


def cfg3_shifts(nsweeps: int = 6, N: int = 48):
    """Shifted pairs (sigma I - A) x = b, (sigma I - A)^H x~ = c with
    A = -L_kappa - 0.1 I on N^3 (default 48^3, n=110592).  Per sweep 8 shifts in
    4 conjugate pairs: sweep 0 has Re = 0.5*100^(m/3), Im = +-5(m+1), m=0..3;
    each later sweep multiplies every pair by (1+0.05u), u ~ U[-1,1], clipped to
    Re in [0.5,50], |Im| <= 20.  b, c ~ N(0,1) real, fixed over sweeps.
    Returns (A, b, c, sweeps) with sweeps a list of complex arrays of length 8
    ordered [s0, conj(s0), s1, conj(s1), ...]."""
    rng = np.random.default_rng(BASE_SEED + 3)
    A = aniso_diffusion(N)
    n = N ** 3
    b = rng.standard_normal(n)
    c = rng.standard_normal(n)
    base = np.array([0.5 * 100.0 ** (m / 3.0) + 1j * 5.0 * (m + 1) for m in range(4)])
    sweeps = []
    cur = base.copy()
    for sw in range(nsweeps):
        if sw > 0:
            u = rng.uniform(-1.0, 1.0, 4)
            cur = cur * (1.0 + 0.05 * u)
            cur = np.clip(cur.real, 0.5, 50.0) + 1j * np.clip(cur.imag, -20.0, 20.0)
        sig = np.empty(8, dtype=np.complex128)
        sig[0::2] = cur
        sig[1::2] = np.conj(cur)
        sweeps.append(sig)
    return A, b, c, sweeps


def cfg4_sequence(nsys: int = 8, N: int = 128) -> DualSequence:
    """3D convection-diffusion 7-point upwind on N^3 (default 128^3, n=2097152),
    beta = (50,25,10), 8 systems with the same A and a fresh N(0,1) pair of
    right-hand sides per system; k=30, s=40; FP64 outer tolerance 1e-10 on the
    true residual, inner tolerance 1e-5."""
    rng = np.random.default_rng(BASE_SEED + 4)
    n = N ** 3
    A = convdiff(N, 3, [50.0, 25.0, 10.0])
    bs, bts = [], []
    for _ in range(nsys):
        bs.append(rng.standard_normal(n))
        bts.append(rng.standard_normal(n))
    return DualSequence(f"convdiff3d_{N}_mixed", [A] * nsys, bs, bts, 30, 40, 1e-10,
                        extra={"inner_tol": 1e-5})


@dataclass
class Request:
    rid: int
    arrival: float
    edge: int
    beta: Tuple[float, float, float]
    nsys: int
    k: int
    seed: int


def cfg5_trace(nreq: int = 400, lam: float = 50.0,
               edges: Sequence[int] = (32, 48, 64, 96, 128)) -> List[Request]:
    """Poisson stream (rate lam req/s) of requests; each is a sequence of 4..12
    dual systems of 3D convection-diffusion with grid edge uniform in ``edges``,
    beta ~ U[1,50]^3, k in {10,20}; the matrix is fixed per request and each
    system gets a fresh N(0,1) right-hand-side pair (drawn from the request's own
    seed by :func:`request_rhs`)."""
    rng = np.random.default_rng(BASE_SEED + 5)
    t = 0.0
    out = []
    for rid in range(nreq):
        t += rng.exponential(1.0 / lam)
        edge = int(rng.choice(np.asarray(edges)))
        beta = tuple(float(v) for v in rng.uniform(1.0, 50.0, 3))
        nsys = int(rng.integers(4, 13))
        k = int(rng.choice([10, 20]))
        out.append(Request(rid, t, edge, beta, nsys, k, BASE_SEED + 1000 + rid))
    return out


def request_rhs(req: Request, j: int) -> Tuple[np.ndarray, np.ndarray]:
    """Right-hand-side pair of system j of a request."""
    rng = np.random.default_rng([req.seed, j])
    n = req.edge ** 3
    return rng.standard_normal(n), rng.standard_normal(n)


def random_sparse(n: int, per_row: int, seed: int, diag_shift: float = 0.0,
                  complex_vals: bool = False) -> CSR:
    """Random nonsymmetric sparse matrix with ``per_row`` off-diagonal entries
    per row (distinct columns, no self loop), a diagonal entry, and values
    ~ N(0,1) (complex if asked); ``diag_shift`` is added to the diagonal."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        others = np.setdiff1d(rng.choice(n, size=min(per_row + 1, n), replace=False), [i])[:per_row]
        cs = np.concatenate([[i], others])
        rows.append(np.full(len(cs), i)); cols.append(cs)
        v = rng.standard_normal(len(cs))
        if complex_vals:
            v = v + 1j * rng.standard_normal(len(cs))
        v[0] += diag_shift
        vals.append(v)
    r = np.concatenate(rows); c = np.concatenate(cols); v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rowptr[1:])
    return CSR(n, rowptr.astype(np.int32), c.astype(np.int32), v)


def csr_from_dense(D: np.ndarray, drop: float = 0.0) -> CSR:
    """CSR of a dense matrix, keeping entries with |d| > drop."""
    n = D.shape[0]
    mask = np.abs(D) > drop
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), D[rows, cols].copy())


def sine_modes(N: int, dim: int, k: int) -> np.ndarray:
    """The k lowest Dirichlet sine modes of the unit square/cube grid with edge
    N (lexicographic order, x fastest), as an n x k float64 array with unit
    2-norm columns.  Modes are ordered by (a^2 + b^2 + c^2, a, b, c) over the
    wave numbers (a, b, c) >= 1.  A deterministic smooth basis to install as
    an externally supplied recycle space (U = U~) at any problem size."""
    ax = np.arange(1, N + 1) / (N + 1.0)
    m = min(N, k)
    waves = sorted((sum(c * c for c in w), w)
                   for w in (tuple(c + 1 for c in t) for t in np.ndindex(*([m] * dim))))[:k]
    if len(waves) < k:
        raise ValueError("k exceeds the number of grid modes")
    out = np.empty((N ** dim, k))
    for j, (_, w) in enumerate(waves):
        comps = [np.sin(np.pi * w[d] * ax) for d in range(dim)]
        v = comps[dim - 1]
        for d in range(dim - 2, -1, -1):
            v = np.kron(v, comps[d])
        out[:, j] = v / np.linalg.norm(v)
    return out
