"""CPU checks of the library's host ILUT factorization and level schedules
(rbicg_host_ilut, rbicg_host_levels; the factorization rbicg_ilut_create
uploads) against the oracle's ILUT, which is pinned in test_precond_cpu.py.
No GPU call is made."""
import ctypes as ct

import numpy as np
import pytest
import scipy.sparse as sp

import oracle.precond as pc
from paper_1010_0762_amd import _lib
from paper_1010_0762_amd import workloads as wl


def _p(a):
    return ct.c_void_p(a.ctypes.data)


def _host_ilut(A, tau, p, permtol=0.0, with_perm=False):
    lib = _lib.load()
    A = sp.csr_matrix(A).astype(np.complex128)
    A.sort_indices()
    n = A.shape[0]
    rp = np.ascontiguousarray(A.indptr, np.int32)
    ci = np.ascontiguousarray(A.indices, np.int32)
    v = np.ascontiguousarray(A.data).view(np.float64).copy()
    nnz = (ct.c_int64 * 2)()
    pp = -1 if p is None else p
    rc = lib.rbicg_host_ilut(n, _p(rp), _p(ci), _lib.dptr(v), tau, pp, permtol, nnz, None, None,
                             None, None, None, None, None)
    assert rc == 0, _lib.last_error()
    Lrp = np.zeros(n + 1, np.int32); Lci = np.zeros(max(nnz[0], 1), np.int32)
    Lv = np.zeros(2 * max(nnz[0], 1))
    Urp = np.zeros(n + 1, np.int32); Uci = np.zeros(max(nnz[1], 1), np.int32)
    Uv = np.zeros(2 * max(nnz[1], 1))
    perm = np.zeros(n, np.int32)
    rc = lib.rbicg_host_ilut(n, _p(rp), _p(ci), _lib.dptr(v), tau, pp, permtol, nnz, _p(Lrp),
                             _p(Lci), _lib.dptr(Lv), _p(Urp), _p(Uci), _lib.dptr(Uv), _p(perm))
    assert rc == 0
    L = sp.csr_matrix((Lv.view(np.complex128)[:nnz[0]], Lci[:nnz[0]], Lrp), shape=(n, n))
    U = sp.csr_matrix((Uv.view(np.complex128)[:nnz[1]], Uci[:nnz[1]], Urp), shape=(n, n))
    L = L + sp.identity(n, dtype=np.complex128, format="csr")
    return (L, U, perm) if with_perm else (L, U)


def _mats():
    cd = wl.convdiff(24, 2, (10.0, 5.0))
    yield "convdiff2d", sp.csr_matrix((cd.vals, cd.colind, cd.rowptr), shape=(cd.n, cd.n))
    for cplx in (False, True):
        A = wl.random_sparse(300, 6, 11 + cplx, diag_shift=12.0, complex_vals=cplx)
        yield f"random_{'c' if cplx else 'r'}", sp.csr_matrix((A.vals, A.colind, A.rowptr),
                                                              shape=(A.n, A.n))


@pytest.mark.parametrize("tau,p", [(0.0, None), (0.01, None), (0.05, None), (0.05, 3), (0.2, 1)])
def test_host_ilut_matches_oracle(tau, p):
    """Same pattern, values within 1e-12 relative, for real and complex
    matrices with and without dropping and count limits."""
    for name, A in _mats():
        Lo, Uo = pc.ilut(A, tau, p)
        Lh, Uh = _host_ilut(A, tau, p)
        for F, G in ((Lh, Lo), (Uh, Uo)):
            F, G = F.tocsr(), G.tocsr()
            F.sort_indices(); G.sort_indices()
            assert np.array_equal(F.indptr, G.indptr), name
            assert np.array_equal(F.indices, G.indices), name
            assert np.abs(F.data - G.data).max() <= 1e-12 * np.abs(G.data).max(), name


@pytest.mark.parametrize("tau,p,permtol", [(0.0, None, 1.0), (0.05, None, 1.0), (0.05, 3, 0.5),
                                            (0.01, None, 0.1)])
def test_host_ilutp_matches_oracle(tau, p, permtol):
    """ILUTP: the same permutation, pattern and values (1e-12) as the
    oracle's, on the drop/limit cases and on a row-permuted operator whose
    diagonal is mostly zero (pivoting needed)."""
    cd = wl.convdiff(12, 2, (10.0, 5.0))
    As = sp.csr_matrix((cd.vals, cd.colind, cd.rowptr), shape=(cd.n, cd.n))
    rows = np.random.default_rng(3).permutation(cd.n)
    cases = list(_mats()) + [("rowperm", sp.csr_matrix(As[rows]))]
    for name, A in cases:
        Lo, Uo, po = pc.ilutp(A, tau, p, permtol)
        Lh, Uh, ph = _host_ilut(A, tau, p, permtol, with_perm=True)
        assert np.array_equal(po, ph), name
        for F, G in ((Lh, Lo), (Uh, Uo)):
            F, G = F.tocsr(), G.tocsr()
            F.sort_indices(); G.sort_indices()
            assert np.array_equal(F.indptr, G.indptr), name
            assert np.array_equal(F.indices, G.indices), name
            assert np.abs(F.data - G.data).max() <= 1e-12 * np.abs(G.data).max(), name
    assert not np.array_equal(ph, np.arange(len(ph)))   # the row-permuted case pivots


def test_host_ilut_rejects_zero_pivot():
    A = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
    with pytest.raises(AssertionError):
        _host_ilut(A, 0.0, None)
    assert "pivot" in _lib.last_error()


def _levels(T, lower, pad=64):
    lib = _lib.load()
    T = sp.csr_matrix(T)
    n = T.shape[0]
    rp = np.ascontiguousarray(T.indptr, np.int32)
    ci = np.ascontiguousarray(T.indices, np.int32)
    ln = ct.c_int64()
    nl = lib.rbicg_host_levels(n, _p(rp), _p(ci), 1 if lower else 0, pad, None, ct.byref(ln))
    order = np.zeros(ln.value, np.int32)
    assert lib.rbicg_host_levels(n, _p(rp), _p(ci), 1 if lower else 0, pad, _p(order),
                                 ct.byref(ln)) == nl
    return nl, order


@pytest.mark.parametrize("lower", [True, False])
def test_level_schedule_is_valid(lower):
    """Every row once; levels padded to whole 64-lane waves; a row's
    dependencies lie in earlier waves; the level count is the longest
    dependency chain (computed here by a plain recursion); a tridiagonal
    factor is one chain (n levels)."""
    A = next(_mats())[1]
    L, U = pc.ilut(A, 0.05)
    T = L if lower else U
    n = T.shape[0]
    nl, order = _levels(T, lower)
    assert len(order) % 64 == 0
    rows = order[order >= 0]
    assert sorted(rows.tolist()) == list(range(n))
    # the invariant the device solve relies on: a row's dependencies sit in
    # earlier 64-lane waves of the order
    wave = np.full(n, -1)
    pos = np.flatnonzero(order >= 0)
    wave[order[pos]] = pos // 64
    T = T.tocsr()
    depth = np.zeros(n, int)
    rng = range(n) if lower else range(n - 1, -1, -1)
    for i in rng:
        deps = [j for j in T.indices[T.indptr[i]:T.indptr[i + 1]] if (j < i if lower else j > i)]
        depth[i] = 1 + max((depth[j] for j in deps), default=-1)
        for j in deps:
            assert wave[j] < wave[i]
    assert nl == depth.max() + 1
    Tri = sp.diags([np.ones(99), np.full(100, 2.0)], [-1, 0], format="csr")
    assert _levels(Tri, True)[0] == 100


def test_jump_convdiff2d_generator():
    """The jumping-coefficient 2D operator: with contrast 1 and no
    convection it is the 5-point Laplacian (4/h^2 diagonal, -1/h^2
    neighbours); with convection the skew part is the central difference
    (A - A^T)/2 = beta_x/(2h) on the x-neighbours; with contrast the
    symmetric part stays symmetric with zero row sums away from the
    boundary (a conservative flux form)."""
    N = 15
    h = 1.0 / (N + 1)
    A = wl.jump_convdiff2d(N, contrast=1.0, beta=(0.0, 0.0))
    M = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n)).toarray()
    L = wl.convdiff(N, 2, [0.0, 0.0])
    Lm = sp.csr_matrix((L.vals, L.colind, L.rowptr), shape=(L.n, L.n)).toarray()
    assert np.allclose(M, Lm, rtol=1e-14, atol=0)
    A = wl.jump_convdiff2d(N, contrast=1.0, beta=(8.0, 0.0))
    M = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n)).toarray()
    K = (M - M.T) / 2
    assert np.isclose(K[5, 6], 8.0 / (2 * h)) and np.isclose(K[5, 4], -8.0 / (2 * h))
    A = wl.jump_convdiff2d(N, contrast=1e3, beta=(0.0, 0.0))
    M = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n)).toarray()
    assert np.allclose(M, M.T, rtol=1e-14)
    inner = [i + N * j for j in range(1, N - 1) for i in range(1, N - 1)]
    assert np.abs(M[inner].sum(axis=1)).max() <= 1e-9 * np.abs(M).max()
    assert len(set(np.round(np.diag(M) * h**2, 6))) > 2   # the coefficient jumps
