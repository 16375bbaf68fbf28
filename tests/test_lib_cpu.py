"""CPU checks of the C-ABI library: it loads, exports every symbol the public
headers declare, and its host FP64 dense linear algebra (used at cycle ends)
agrees with numpy/scipy.  No GPU call is made."""
import ctypes as ct
import glob
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

from paper_1010_0762_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names.update(re.findall(r"\b(rbicg_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 15
    for nm in sorted(names):
        assert hasattr(lib, nm), nm
        assert nm in _lib.SIGNATURES, nm


def _c(a):
    a = np.asfortranarray(a.astype(np.complex128))
    return np.ascontiguousarray(a.T.reshape(-1)).view(np.float64).copy()  # column-major interleaved


def _uc(buf, m, n):
    return buf.view(np.complex128).reshape(n, m).T


@pytest.mark.parametrize("m,cplx,gen", [(12, False, False), (30, True, False), (25, True, True),
                                        (41, False, True)])
def test_host_eig_matches_scipy(m, cplx, gen):
    lib = _lib.load()
    rng = np.random.default_rng(m)
    P = rng.standard_normal((m, m)) + (1j * rng.standard_normal((m, m)) if cplx else 0)
    Q = (np.eye(m) + 0.2 * rng.standard_normal((m, m))) if gen else None
    lam = np.zeros(2 * m); W = np.zeros(2 * m * m); Wl = np.zeros(2 * m * m)
    Pb = _c(P); Qb = _c(Q) if gen else None
    rc = lib.rbicg_host_eig(m, _lib.dptr(Pb), _lib.dptr(Qb) if gen else None, _lib.dptr(lam),
                            _lib.dptr(W), _lib.dptr(Wl))
    assert rc == 0
    lam = lam.view(np.complex128)
    W = _uc(W, m, m); Wl = _uc(Wl, m, m)
    ref = sla.eigvals(P, Q)
    for l in ref:
        assert np.min(np.abs(lam - l)) <= 1e-9 * max(1, abs(l))
    Qm = Q if gen else np.eye(m)
    scale = np.linalg.norm(P, 2) + np.abs(lam).max() * np.linalg.norm(Qm, 2)
    for j in range(m):
        assert np.linalg.norm(P @ W[:, j] - lam[j] * Qm @ W[:, j]) <= 1e-10 * scale
        y = Wl[:, j]
        assert np.linalg.norm(y.conj() @ P - lam[j] * (y.conj() @ Qm)) <= 1e-10 * scale
        assert abs(np.linalg.norm(W[:, j]) - 1) < 1e-12


def test_host_svd_and_heig():
    lib = _lib.load()
    rng = np.random.default_rng(5)
    for m, n in [(9, 9), (20, 13)]:
        A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
        U = np.zeros(2 * m * n); s = np.zeros(n); V = np.zeros(2 * n * n)
        assert lib.rbicg_host_svd(m, n, _lib.dptr(_c(A)), _lib.dptr(U), _lib.dptr(s), _lib.dptr(V)) == 0
        U = _uc(U, m, n); V = _uc(V, n, n)
        assert np.allclose(s, np.linalg.svd(A, compute_uv=False), rtol=1e-12)
        assert np.allclose(U @ np.diag(s) @ V.conj().T, A, atol=1e-12)
    H = rng.standard_normal((15, 15)) + 1j * rng.standard_normal((15, 15))
    H = H + H.conj().T
    w = np.zeros(15); V = np.zeros(2 * 225)
    assert lib.rbicg_host_heig(15, _lib.dptr(_c(H)), _lib.dptr(w), _lib.dptr(V)) == 0
    V = _uc(V, 15, 15)
    assert np.allclose(w, np.linalg.eigvalsh(H), atol=1e-12)
    assert np.allclose(V @ np.diag(w) @ V.conj().T, H, atol=1e-11)


def test_host_select_real_pairs_and_order():
    lib = _lib.load()
    # real matrix with known spectrum: 1, 2, 3+-1i, 10, 20
    rng = np.random.default_rng(7)
    Lam = np.zeros((6, 6))
    Lam[0, 0], Lam[1, 1] = 1.0, 2.0
    Lam[2:4, 2:4] = [[3.0, 1.0], [-1.0, 3.0]]
    Lam[4, 4], Lam[5, 5] = 10.0, 20.0
    S = np.eye(6) + 0.3 * rng.standard_normal((6, 6))
    M = S @ Lam @ np.linalg.inv(S)
    m = 6
    lam = np.zeros(2 * m); W = np.zeros(2 * m * m); Wl = np.zeros(2 * m * m)
    lib.rbicg_host_eig(m, _lib.dptr(_c(M)), None, _lib.dptr(lam), _lib.dptr(W), _lib.dptr(Wl))
    for k, expect in [(4, 4), (3, 2), (5, 5)]:
        Ws = np.zeros(2 * m * m); Wls = np.zeros(2 * m * m)
        got = lib.rbicg_host_select(m, _lib.dptr(lam), _lib.dptr(W), _lib.dptr(Wl), k, 1,
                                    _lib.dptr(Ws), _lib.dptr(Wls))
        assert got == expect
        Wsel = _uc(Ws, m, m)[:, :got]
        assert np.abs(Wsel.imag).max() == 0.0
        # the selected real columns span the invariant subspace of the smallest eigenvalues
        ref = S[:, :got]
        ang = sla.subspace_angles(Wsel.real, ref)
        assert ang.max() < 1e-8


def test_host_biorth_gives_identity():
    lib = _lib.load()
    rng = np.random.default_rng(9)
    n, k = 200, 7
    C = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    Ct = C + 0.3 * (rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    Gcc, Gtt, Gtc = C.conj().T @ C, Ct.conj().T @ Ct, Ct.conj().T @ C
    TU = np.zeros(2 * k * k); TUt = np.zeros(2 * k * k)
    p = lib.rbicg_host_biorth(k, _lib.dptr(_c(Gcc)), _lib.dptr(_c(Gtt)), _lib.dptr(_c(Gtc)), 1e-2,
                              _lib.dptr(TU), _lib.dptr(TUt))
    assert p == k
    TU = _uc(TU, k, k)[:, :p]; TUt = _uc(TUt, k, k)[:, :p]
    G = (Ct @ TUt).conj().T @ (C @ TU)
    assert np.abs(G - np.eye(p)).max() < 1e-12
    # cosines of principal angles decide the truncation
    cos = np.cos(sla.subspace_angles(C, Ct))
    Ct2 = Ct.copy(); Ct2[:, 0] = rng.standard_normal(n)  # nearly orthogonal direction
    q1, _ = np.linalg.qr(C); q2, _ = np.linalg.qr(Ct2)
    sv = np.linalg.svd(q2.conj().T @ q1, compute_uv=False)
    p2 = lib.rbicg_host_biorth(k, _lib.dptr(_c(Gcc)), _lib.dptr(_c(Ct2.conj().T @ Ct2)),
                               _lib.dptr(_c(Ct2.conj().T @ C)), 0.5, _lib.dptr(TU.copy()),
                               _lib.dptr(TUt.copy()))
    assert p2 == int(np.sum(sv >= 0.5))


def test_host_eig_ill_conditioned_pencil_matches_qz():
    """cond(Q) ~ 1e9 (as in the harmonic Ritz pencils): the pencil is solved
    without forming Q^{-1} P, so the small eigenvalues agree with LAPACK's QZ."""
    lib = _lib.load()
    rng = np.random.default_rng(11)
    m = 40
    U1, _ = np.linalg.qr(rng.standard_normal((m, m)))
    U2, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Q = U1 @ np.diag(np.logspace(0, -9, m)) @ U2
    P = rng.standard_normal((m, m))
    lam = np.zeros(2 * m); W = np.zeros(2 * m * m); Wl = np.zeros(2 * m * m)
    assert lib.rbicg_host_eig(m, _lib.dptr(_c(P)), _lib.dptr(_c(Q)), _lib.dptr(lam), _lib.dptr(W),
                              _lib.dptr(Wl)) == 0
    lam = lam.view(np.complex128)
    ref = sla.eigvals(P, Q)
    small = ref[np.argsort(np.abs(ref))[:8]]
    for l in small:
        assert np.min(np.abs(lam - l)) <= 1e-7 * abs(l), l
    W = _uc(W, m, m)
    for j in np.argsort(np.abs(lam))[:8]:
        res = np.linalg.norm(P @ W[:, j] - lam[j] * (Q @ W[:, j]))
        assert res <= 1e-12 * (np.linalg.norm(P, 2) + abs(lam[j]) * np.linalg.norm(Q, 2))


@pytest.mark.parametrize("seed", range(6))
def test_host_eig_real_pencils_backward_error(seed):
    """Real pencils take the real double-shift QZ: every right and left
    eigenpair has a backward error at rounding level, conjugate pairs stay
    paired, and the eigenvalues match scipy's, also with an ill-conditioned Q
    (condition 1e9, as the harmonic Ritz pencils reach)."""
    lib = _lib.load()
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(5, 61))
    P = rng.standard_normal((m, m))
    Q = rng.standard_normal((m, m))
    if seed % 2:
        U, _, Vt = np.linalg.svd(Q)
        Q = U @ np.diag(np.logspace(0, -9, m)) @ Vt
    lam = np.zeros(2 * m); W = np.zeros(2 * m * m); Wl = np.zeros(2 * m * m)
    Pb, Qb = _c(P), _c(Q)
    assert lib.rbicg_host_eig(m, _lib.dptr(Pb), _lib.dptr(Qb), _lib.dptr(lam), _lib.dptr(W),
                              _lib.dptr(Wl)) == 0
    lam = lam.view(np.complex128)
    W = _uc(W, m, m); Wl = _uc(Wl, m, m)
    nP, nQ = np.linalg.norm(P, 2), np.linalg.norm(Q, 2)
    for i in range(m):
        if not np.isfinite(lam[i]) or abs(lam[i]) > 1e8:
            continue
        sc = nP + abs(lam[i]) * nQ
        assert np.linalg.norm(P @ W[:, i] - lam[i] * (Q @ W[:, i])) <= 1e-12 * sc
        assert np.linalg.norm(Wl[:, i].conj() @ P - lam[i] * (Wl[:, i].conj() @ Q)) <= 1e-12 * sc
        if abs(lam[i].imag) > 1e-8 * abs(lam[i]):
            assert np.min(np.abs(lam - np.conj(lam[i]))) <= 1e-8 * abs(lam[i])
    ref = sla.eigvals(P, Q)
    ref = ref[np.isfinite(ref) & (np.abs(ref) < 1e6)]
    for z in ref:
        assert np.min(np.abs(lam - z)) <= 1e-6 * max(1.0, abs(z))


def test_matrix_info_rejects_null_arguments():
    """rbicg_matrix_info is host-only: null arguments are RBICG_EINVAL with a
    message, and no device call is made."""
    lib = _lib.load()
    info = (ct.c_int64 * 5)()
    assert lib.rbicg_matrix_info(None, info) == _lib.RBICG_EINVAL
    assert b"null" in lib.rbicg_last_error()
    assert lib.rbicg_matrix_info(None, None) == _lib.RBICG_EINVAL


def test_entry_points_reject_bad_arguments_before_any_device_call():
    """The sequence, split-preconditioning and batch entry points check their
    arguments on the host: null handles, out-of-range settings and a matrix
    whose ILUT meets a zero pivot are RBICG_EINVAL with a message, and
    destroying a null object is a no-op."""
    lib = _lib.load()
    E = _lib.RBICG_EINVAL
    P = ct.c_void_p
    # a whole sequence needs a handle and (for nsys > 0) its arrays
    assert lib.rbicg_solve_sequence(None, 1, None, None, None, None, None, 1, 1e-8, None) == E
    assert b"null" in lib.rbicg_last_error()
    # split preconditioning: null objects
    info = (ct.c_int64 * 8)()
    assert lib.rbicg_ilu_info(None, info) == E
    assert lib.rbicg_ilu_set_waves(None, 512) == E
    assert lib.rbicg_ilu_attach(None, None) == E
    assert lib.rbicg_ilu_rhs(None, None, None, None, None, 0, None) == E
    assert lib.rbicg_ilu_solution(None, None, None, None, None, 0, None) == E
    assert lib.rbicg_ilu_destroy(None) == _lib.RBICG_OK
    # ILUT: bad thresholds, an invalid descriptor, a zero pivot without pivoting
    rowptr = np.array([0, 1, 2], dtype=np.int32)
    colind = np.array([1, 0], dtype=np.int32)
    vals = np.array([1.0, 1.0])
    A = _lib.rbicg_csr()
    A.n, A.nnz = 2, 2
    A.rowptr, A.colind, A.values = rowptr.ctypes.data, colind.ctypes.data, vals.ctypes.data
    A.values_complex, A.on_device = 0, 0
    out = P()
    assert lib.rbicg_ilut_create(ct.byref(A), -1.0, -1, 0.0, ct.byref(out)) == E
    assert b"droptol" in lib.rbicg_last_error()
    assert lib.rbicg_ilut_create(ct.byref(A), 0.0, -1, -0.5, ct.byref(out)) == E
    assert b"permtol" in lib.rbicg_last_error()
    assert lib.rbicg_ilut_create(ct.byref(A), 0.0, -1, 0.0, None) == E
    bad = _lib.rbicg_csr()
    bad.n, bad.nnz = 0, 0
    assert lib.rbicg_ilut_create(ct.byref(bad), 0.0, -1, 0.0, ct.byref(out)) == E
    assert b"CSR" in lib.rbicg_last_error()
    assert lib.rbicg_ilut_create(ct.byref(A), 0.0, -1, 0.0, ct.byref(out)) == E
    assert b"zero pivot in row 0" in lib.rbicg_last_error()
    assert not out.value
    # batches: slot count and window are range-checked before any stream exists
    assert lib.rbicg_batch_create(0, 50.0, ct.byref(out)) == E
    assert lib.rbicg_batch_create(17, 50.0, ct.byref(out)) == E
    assert lib.rbicg_batch_create(4, -1.0, ct.byref(out)) == E
    assert lib.rbicg_batch_create(4, 50.0, None) == E
    assert lib.rbicg_batch_use_graphs(None, 1) == E
    assert lib.rbicg_batch_stats(None, None) == E
    assert lib.rbicg_batch_destroy(None) == _lib.RBICG_OK


def test_empty_and_mismatched_inputs_are_rejected_on_the_host():
    """Degenerate inputs end in RBICG_EINVAL before any device call: an empty
    (n = 0) matrix, an A^H of another size, and options out of range (k above
    the maximum, a cycle shorter than two iterations)."""
    lib = _lib.load()
    E = _lib.RBICG_EINVAL
    out = ct.c_void_p()
    empty = _lib.rbicg_csr()
    empty.n, empty.nnz = 0, 0
    assert lib.rbicg_matrix_create(ct.byref(empty), None, ct.byref(out)) == E
    assert b"CSR" in lib.rbicg_last_error()
    opts = _lib.rbicg_opts()
    lib.rbicg_default_opts(ct.byref(opts))
    assert lib.rbicg_create(ct.byref(empty), None, ct.byref(opts), ct.byref(out)) == E
    assert b"positive" in lib.rbicg_last_error()

    def csr(n):
        rowptr = np.arange(n + 1, dtype=np.int32)
        colind = np.arange(n, dtype=np.int32)
        vals = np.ones(n)
        s = _lib.rbicg_csr()
        s.n, s.nnz = n, n
        s.rowptr, s.colind, s.values = rowptr.ctypes.data, colind.ctypes.data, vals.ctypes.data
        s.values_complex, s.on_device = 0, 0
        return s, (rowptr, colind, vals)

    A2, keep2 = csr(2)
    A3, keep3 = csr(3)
    assert lib.rbicg_matrix_create(ct.byref(A2), ct.byref(A3), ct.byref(out)) == E
    assert b"size mismatch" in lib.rbicg_last_error()
    bad = _lib.rbicg_opts()
    lib.rbicg_default_opts(ct.byref(bad))
    bad.k = 65
    assert lib.rbicg_create(ct.byref(A2), None, ct.byref(bad), ct.byref(out)) == E
    assert b"k must be" in lib.rbicg_last_error()
    lib.rbicg_default_opts(ct.byref(bad))
    bad.s = 1
    assert lib.rbicg_create(ct.byref(A2), None, ct.byref(bad), ct.byref(out)) == E
    assert not out.value
