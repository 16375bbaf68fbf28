"""Pins of the oracle's split ILU(0) preconditioning in red-black ordering
(oracle/precond.py) against facts fixed independently of its code:
  - ILU(0) of a tridiagonal matrix is the exact LU factorization (no fill);
  - ILU(0) reproduces the matrix on its pattern, (L U)_ij = M_ij;
  - in red-black ordering the split-preconditioned operator is block
    diagonal with an identity red block, and its black block is the Schur
    complement right-scaled by the kept pivots,
    M_B = (D_B - A_BR D_R^{-1} A_RB) diag(...)^{-1};
  - the back-transformed solutions solve the original dual pair."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle.precond import SplitSystem, ilu0, rbicg_split_sequence, two_coloring
import oracle.precond as pc
from paper_1010_0762_amd import workloads as wl


def test_ilu0_of_tridiagonal_is_exact_lu():
    rng = np.random.default_rng(1)
    n = 30
    T = sp.diags([rng.uniform(-1, 0, n - 1), rng.uniform(3, 4, n), rng.uniform(-1, 0, n - 1)],
                 [-1, 0, 1]).tocsr()
    L, U = ilu0(T)
    assert np.abs((L @ U - T).toarray()).max() <= 1e-13


def test_ilu0_matches_matrix_on_pattern():
    A = wl.convdiff(5, 3, [20.0, 10.0, 5.0])
    ss = SplitSystem(A)
    LU = (ss.L @ ss.U).tocsr()
    At = ss.At.tocoo()
    err = max(abs(LU[i, j] - v) for i, j, v in zip(At.row, At.col, At.data))
    assert err <= 1e-12 * np.abs(At.data).max()
    # outside the pattern the product differs (the dropped fill)
    D = (LU - ss.At).toarray()
    assert np.abs(D).max() > 1e-6


def test_two_coloring_and_rejection():
    A = wl.convdiff(4, 2, [1.0, 1.0])
    col = two_coloring(A)
    Ac = A if not hasattr(A, "rowptr") else sp.csr_matrix((A.vals, A.colind, A.rowptr))
    r, c = Ac.nonzero()
    off = r != c
    assert np.all(col[r[off]] != col[c[off]])
    tri = sp.csr_matrix(np.array([[2.0, 1, 1], [1, 2, 1], [1, 1, 2]]))
    with pytest.raises(ValueError):
        two_coloring(tri)


def test_operator_block_structure_and_schur_block():
    A = wl.convdiff(5, 3, [20.0, 10.0, 5.0])
    ss = SplitSystem(A)
    Ah = ss.operator()
    nr = ss.nr
    assert np.abs(Ah[:nr, :nr] - np.eye(nr)).max() <= 1e-13
    assert np.abs(Ah[:nr, nr:]).max() <= 1e-13 and np.abs(Ah[nr:, :nr]).max() <= 1e-13
    # closed form from the blocks of P A P^T
    At = ss.At.toarray()
    dR = np.diag(At)[:nr]
    ABR, ARB, DB = At[nr:, :nr], At[:nr, nr:], np.diag(np.diag(At)[nr:])
    S = DB - ABR @ np.diag(1.0 / dR) @ ARB
    MB = S @ np.diag(1.0 / np.diag(S))
    assert np.abs(Ah[nr:, nr:] - MB).max() <= 1e-12 * np.abs(MB).max()


def test_split_sequence_solves_the_original_pairs():
    rng = np.random.default_rng(4)
    N = 8
    mats = [wl.convdiff(N, 3, [20.0 * (1 + 0.02 * j), 10.0, 5.0]) for j in range(3)]
    b, bt = rng.standard_normal(N ** 3), rng.standard_normal(N ** 3)
    sols, res = rbicg_split_sequence(mats, [b] * 3, [bt] * 3, k=6, s=20, tol=1e-10)
    for A, (x, xt), r in zip(mats, sols, res):
        As = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n))
        assert r.status == "ok"
        assert np.linalg.norm(b - As @ x) <= 1e-7 * np.linalg.norm(b)
        assert np.linalg.norm(bt - As.T @ xt) <= 1e-7 * np.linalg.norm(bt)
    # the preconditioned black systems converge faster than plain BiCG on A
    plain = oracle.bicg(mats[0], b, bt, tol=1e-10, maxit=5000)
    assert res[0].iters < plain.iters


def test_split_solve_complex_pair():
    """Complex values (a missing conjugation in a dual transform fails here)."""
    rng = np.random.default_rng(6)
    A = wl.convdiff(6, 3, [20.0, 10.0, 5.0])
    As = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n)).astype(np.complex128)
    As = (As + 1j * sp.diags(rng.uniform(1.0, 5.0, A.n)) +
          1j * 0.3 * sp.csr_matrix((rng.uniform(-1, 1, A.nnz), A.colind, A.rowptr),
                                   shape=(A.n, A.n))).tocsr()
    b = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    bt = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    sols, res = rbicg_split_sequence([As], [b], [bt], k=0, s=20, tol=1e-11, real=False)
    x, xt = sols[0]
    assert res[0].status == "ok"
    assert np.linalg.norm(b - As @ x) <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm(bt - As.conj().T @ xt) <= 1e-8 * np.linalg.norm(bt)


# ------------------------------------------------------------ ILUT (general)
def _rand_dd(n, seed, cplx=False):
    A = wl.random_sparse(n, 5, seed, diag_shift=12.0, complex_vals=cplx)
    return sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(n, n))


@pytest.mark.parametrize("cplx", [False, True])
def test_ilut_without_dropping_is_lu(cplx):
    """tau = 0, no count limit: the complete LU factorization without
    pivoting, which is unique: L unit lower, U upper, L U = A."""
    A = _rand_dd(60, 3, cplx)
    L, U = pc.ilut(A, 0.0)
    assert sp.triu(L, 1).nnz == 0 and sp.tril(U, -1).nnz == 0
    assert np.allclose(L.diagonal(), 1.0)
    assert np.abs((L @ U - A).toarray()).max() <= 1e-12 * abs(A).max()


def test_ilut_drop_rule_hand_example():
    """A = [[4, 1, 0], [1, 4, 1], [2, 1, 4]] worked by hand; column norms
    ||A(:,0)|| = sqrt(21) = 4.583, ||A(:,1)|| = sqrt(18) = 4.243,
    ||A(:,2)|| = sqrt(17) = 4.123.
    tau = 0.2 (thresholds 0.917, 0.849, 0.825): row 1 keeps w_0 = 1
    (l_10 = 0.25), w_1 = 4 - 0.25 = 3.75, keeps w_2 = 1; row 2 keeps w_0 = 2
    (l_20 = 0.5), then w_1 = 1 - 0.5 = 0.5 < 0.849 is dropped (no update), so
    u_22 = 4.  tau = 0.25 (thresholds 1.146, 1.061, 1.031): row 1 drops w_0 = 1
    and the U entry w_2 = 1, so u_11 = 4 and u_12 = 0; row 2 as before."""
    A = sp.csr_matrix(np.array([[4.0, 1.0, 0.0], [1.0, 4.0, 1.0], [2.0, 1.0, 4.0]]))
    L, U = pc.ilut(A, 0.2)
    assert np.allclose(L.toarray().real, [[1, 0, 0], [0.25, 1, 0], [0.5, 0, 1]])
    assert np.allclose(U.toarray().real, [[4, 1, 0], [0, 3.75, 1], [0, 0, 4]])
    L, U = pc.ilut(A, 0.25)
    assert np.allclose(L.toarray().real, [[1, 0, 0], [0, 1, 0], [0.5, 0, 1]])
    assert np.allclose(U.toarray().real, [[4, 0, 0], [0, 4, 0], [0, 0, 4]])


def test_ilut_limits():
    """Huge tau: only the diagonal survives (L = I, U = diag A); p = 1: at
    most one off-diagonal entry per row in each factor, the largest; no
    fill on a tridiagonal matrix: ILUT = LU for every tau below the
    entries' scale."""
    A = _rand_dd(40, 9)
    L, U = pc.ilut(A, 1e12)
    assert (L - sp.identity(40)).nnz == 0 or np.abs((L - sp.identity(40)).toarray()).max() == 0
    assert np.allclose(U.toarray(), np.diag(A.diagonal()))
    L, U = pc.ilut(A, 0.0, p=1)
    assert max(np.diff(sp.tril(L, -1).tocsr().indptr)) <= 1
    assert max(np.diff(sp.triu(U, 1).tocsr().indptr)) <= 1
    T = sp.diags([np.full(29, -1.0), np.full(30, 4.0), np.full(29, -2.0)], [-1, 0, 1], format="csr")
    L, U = pc.ilut(T, 1e-3)
    assert np.abs((L @ U - T).toarray()).max() <= 1e-13


def test_ilut_split_system_solves_original_pair():
    """The split-preconditioned pair recovers the original solutions: with
    tau = 0 the operator L^{-1} A U^{-1} is the identity (one iteration), and
    for tau = 0.05 RBiCG on it gives x, x~ with small original residuals."""
    A = wl.convdiff(16, 2, (10.0, 5.0))
    As = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n))
    rng = np.random.default_rng(4)
    b, bt = rng.uniform(size=A.n), rng.uniform(size=A.n)
    ss = pc.IlutSystem(A, 0.0)
    assert np.abs(ss.operator().toarray() - np.eye(A.n)).max() <= 1e-10
    sols, res = pc.rbicg_ilut_sequence([A], [b], [bt], 0, 40, 1e-10, tau=0.05, update=False)
    x, xt = sols[0]
    assert np.linalg.norm(b - As @ x) / np.linalg.norm(b) <= 1e-8
    assert np.linalg.norm(bt - As.T @ xt) / np.linalg.norm(bt) <= 1e-8
    assert res[0].iters < 40


# ------------------------------------------------------------ ILUTP
def test_ilutp_without_pivot_tolerance_is_ilut():
    """permtol = 0 never pivots: the factors are ILUT's and perm is the
    identity."""
    A = _rand_dd(50, 5)
    for tau in (0.0, 0.05):
        L, U = pc.ilut(A, tau)
        Lp, Up, perm = pc.ilutp(A, tau, permtol=0.0)
        assert np.array_equal(perm, np.arange(50))
        assert abs(Lp - L).max() == 0 and abs(Up - U).max() == 0


def test_ilutp_complete_pivoted_lu():
    """tau = 0, permtol = 1: A Q = L U exactly (no dropping) and every row of
    U has its largest entry on the diagonal (the pivot is the largest entry
    of the row left after the elimination); on a matrix whose diagonal is
    small the columns are really permuted."""
    rng = np.random.default_rng(8)
    n = 40
    A = sp.random(n, n, density=0.15, random_state=3, data_rvs=rng.standard_normal) + sp.eye(n) * 0.01
    A = sp.csr_matrix(A + sp.diags(rng.standard_normal(n - 1) * 3, 1))
    L, U, perm = pc.ilutp(A, 0.0, permtol=1.0)
    assert sorted(perm.tolist()) == list(range(n)) and not np.array_equal(perm, np.arange(n))
    AQ = A.toarray()[:, perm]
    assert np.abs((L @ U).toarray() - AQ).max() <= 1e-10 * np.abs(AQ).max()
    Ud = U.toarray()
    for i in range(n):
        assert abs(Ud[i, i]) >= np.abs(Ud[i, i + 1:]).max(initial=0.0) - 1e-14
    assert sp.triu(L, 1).nnz == 0 and sp.tril(U, -1).nnz == 0


def test_ilutp_hand_example():
    """A = [[1, 4, 0], [2, 1, 3], [0, 5, 1]], tau = 0, permtol = 1, worked by
    hand: row 0 pivots on column 1 (4 > 1); row 1 eliminates with l = 1/4,
    leaving 1.75 in column 0 and 3 in column 2, and pivots on column 2; row 2
    eliminates with 5/4 and 1/3, leaving -1.25 - 1.75/3 = -11/6 in column 0.
    perm = [1, 2, 0]."""
    A = sp.csr_matrix(np.array([[1.0, 4.0, 0.0], [2.0, 1.0, 3.0], [0.0, 5.0, 1.0]]))
    L, U, perm = pc.ilutp(A, 0.0, permtol=1.0)
    assert perm.tolist() == [1, 2, 0]
    assert np.allclose(L.toarray().real, [[1, 0, 0], [0.25, 1, 0], [1.25, 1 / 3, 1]])
    assert np.allclose(U.toarray().real, [[4, 0, 1], [0, 3, 1.75], [0, 0, -11 / 6]])


def test_ilutp_zero_diagonal_where_ilut_fails():
    """[[0, 1], [1, 0]]: ILUT meets a zero pivot; ILUTP swaps the columns
    (perm = [1, 0], L = U = I)."""
    A = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
    with pytest.raises(ZeroDivisionError):
        pc.ilut(A, 0.0)
    L, U, perm = pc.ilutp(A, 0.0, permtol=1.0)
    assert perm.tolist() == [1, 0]
    assert np.allclose(L.toarray(), np.eye(2)) and np.allclose(U.toarray(), np.eye(2))


def test_ilutp_split_system_solves_original_pair():
    """A row-permuted convection-diffusion matrix (most diagonal entries
    zero): ILUTP(0.05) split preconditioning, RBiCG on the preconditioned pair,
    and the transforms recover x, x~ with small original residuals; with
    tau = 0 the preconditioned operator is the identity."""
    A0 = wl.convdiff(10, 2, (10.0, 5.0))
    As = sp.csr_matrix((A0.vals, A0.colind, A0.rowptr), shape=(A0.n, A0.n))
    rng = np.random.default_rng(6)
    rows = rng.permutation(A0.n)
    Ap = sp.csr_matrix(As[rows])
    assert (Ap.diagonal() == 0).sum() > A0.n // 2
    ss = pc.IlutpSystem(Ap, 0.0, permtol=1.0)
    assert np.abs(ss.operator().toarray() - np.eye(A0.n)).max() <= 1e-9
    b, bt = rng.standard_normal(A0.n), rng.standard_normal(A0.n)
    sols, res = pc.rbicg_ilut_sequence([Ap], [b], [bt], 0, 40, 1e-10, tau=0.05, permtol=1.0,
                                       update=False)
    x, xt = sols[0]
    assert res[0].status == "ok"
    assert np.linalg.norm(b - Ap @ x) / np.linalg.norm(b) <= 1e-8
    assert np.linalg.norm(bt - Ap.T @ xt) / np.linalg.norm(bt) <= 1e-8
