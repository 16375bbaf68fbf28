"""Pins of the CPU oracle against facts that do not come from the oracle itself:
published generator outputs, dense direct solves, textbook special cases (CG,
SciPy's BiCG), exact eigenvector deflation, the biorthogonality invariants of
Sec. 3.1, the T-from-scalars identity of Sec. 4.1, and harmonic Ritz exactness
on invariant subspaces (eq. harmonic1)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import recycle as rc
from oracle.krylov import as_csr
from paper_1010_0762_amd import workloads as wl

from cases import eig_case, stall_case


def _rand_nonsym(n, seed, cplx=False, shift=6.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    if cplx:
        A = A + 1j * rng.standard_normal((n, n)) / np.sqrt(n)
    return A + shift * np.eye(n)


def _eig_system(n, seed, lam):
    """A = S diag(lam) S^{-1} with a well conditioned random S."""
    rng = np.random.default_rng(seed)
    S = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    Y = np.linalg.inv(S).conj().T          # left eigenvectors: Y^H A = diag(lam) Y^H
    return A, S, Y


# --------------------------------------------------------------------------
def test_splitmix64_published_outputs():
    # First three outputs of SplitMix64 seeded with 0 (Steele et al. 2014;
    # the reference C code by Vigna prints these).
    g = oracle.rng.GAMMA
    assert oracle.splitmix64(1 * g) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(2 * g) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64(3 * g) == 0x06C45D188009454F
    v = oracle.reseed_vector(7, 1000, False)
    assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.1


@pytest.mark.parametrize("cplx", [False, True])
def test_bicg_matches_dense_solve(cplx):
    n = 120
    A = _rand_nonsym(n, 1, cplx)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    bt = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    res = oracle.bicg(A, b, bt, tol=1e-10, maxit=500)
    assert res.status == "ok"
    kappa = np.linalg.cond(A)
    xs = np.linalg.solve(A, b)
    xts = np.linalg.solve(A.conj().T, bt)
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) <= 10 * kappa * 1e-10
    assert np.linalg.norm(res.xt - xts) / np.linalg.norm(xts) <= 10 * kappa * 1e-10


def test_bicg_convdiff_dense_solve():
    A = wl.convdiff(10, 2, [10.0, 5.0])
    D = A.to_dense()
    rng = np.random.default_rng(3)
    b, bt = rng.uniform(size=100), rng.uniform(size=100)
    res = oracle.bicg(A, b, bt, tol=1e-10, maxit=1000)
    xs = np.linalg.solve(D, b)
    xts = np.linalg.solve(D.T, bt)
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) <= 10 * kappa * 1e-10
    assert np.linalg.norm(res.xt - xts) / np.linalg.norm(xts) <= 10 * kappa * 1e-10


def test_bicg_equals_cg_for_spd():
    """SPD A, b~ = b, x~_0 = x_0: BiCG's iterates are CG's (textbook case)."""
    A = sp.csr_matrix(wl.convdiff(12, 2, [0.0, 0.0]).to_dense())
    rng = np.random.default_rng(4)
    b = rng.standard_normal(A.shape[0])
    res = oracle.bicg(A, b, b.copy(), tol=1e-12, maxit=40, keep_history=True)
    cg_iter = []
    spla.cg(A, b, rtol=1e-30, atol=0.0, maxiter=40, callback=lambda xk: cg_iter.append(xk.copy()))
    m = min(25, len(res.history), len(cg_iter))
    assert m >= 20
    for i in range(m):
        err = np.linalg.norm(res.history[i] - cg_iter[i]) / np.linalg.norm(cg_iter[i])
        assert err < 1e-9, (i, err)


def test_bicg_equals_scipy_bicg_iterates():
    """Real nonsymmetric A with b~ = b: the primal iterates equal SciPy's BiCG
    (its shadow residual is r_0)."""
    A = sp.csr_matrix(wl.convdiff(10, 2, [10.0, 5.0]).to_dense())
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A.shape[0])
    res = oracle.bicg(A, b, b.copy(), tol=1e-12, maxit=30, keep_history=True)
    it = []
    spla.bicg(A, b, rtol=1e-30, atol=0.0, maxiter=30, callback=lambda xk: it.append(xk.copy()))
    m = min(len(it), len(res.history), 25)
    assert m >= 20
    for i in range(m):
        err = np.linalg.norm(res.history[i] - it[i]) / np.linalg.norm(it[i])
        assert err < 1e-9, (i, err)


@pytest.mark.parametrize("cplx", [False, True])
def test_rbicg_without_recycling_is_bicg_bitwise(cplx):
    A = wl.convdiff(12, 2, [8.0, 3.0]) if not cplx else wl.random_sparse(150, 5, 9, 5.0, True)
    n = A.n
    rng = np.random.default_rng(6)
    b = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    bt = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    r0 = oracle.bicg(A, b, bt, tol=1e-9, maxit=400)
    r1 = oracle.rbicg(A, b, bt, tol=1e-9, maxit=400, update=False, max_restarts=0)
    assert r0.iters == r1.iters
    assert np.array_equal(r0.x, r1.x) and np.array_equal(r0.xt, r1.xt)


def _exact_recycle(A, S, Y, idx):
    U = S[:, idx].astype(np.complex128)
    Ut = Y[:, idx].astype(np.complex128)
    Asp = as_csr(A)
    return rc.biorthogonalize(Asp, Asp.conj().T.tocsr(), U, Ut, 1e-8)


def test_exact_eigenvector_deflation():
    """Recycling exact right/left eigenvectors deflates them (Sec. 1): a right
    side in range(U) is solved at step 0, and one with m non-recycled
    eigencomponents terminates in at most m steps."""
    n, k, m = 60, 6, 5
    lam = np.linspace(1.0, 12.0, n)
    A, S, Y = _eig_system(n, 11, lam)
    U, Ut, C, Ct = _exact_recycle(A, S, Y, np.arange(k))
    assert U.shape[1] == k
    rng = np.random.default_rng(12)
    b = S[:, :k] @ rng.standard_normal(k)
    bt = Y[:, :k] @ rng.standard_normal(k)
    res = oracle.rbicg(A, b, bt, None, None, U, Ut, C, Ct, tol=1e-10, maxit=50, update=False)
    assert res.iters == 0 and res.relres < 1e-10 and res.relres_dual < 1e-10
    # m non-recycled components plus recycled ones
    cb = np.zeros(n); cb[:k] = rng.standard_normal(k); cb[k + 10:k + 10 + m] = rng.standard_normal(m)
    cbt = np.zeros(n); cbt[:k] = rng.standard_normal(k); cbt[k + 10:k + 10 + m] = rng.standard_normal(m)
    res = oracle.rbicg(A, S @ cb, Y @ cbt, None, None, U, Ut, C, Ct, tol=1e-9, maxit=50,
                       update=False)
    assert res.status == "ok" and res.iters <= m
    res0 = oracle.rbicg(A, S @ cb, Y @ cbt, tol=1e-9, maxit=50, update=False)
    assert res0.iters > m   # without recycling the recycled components cost steps


def test_biorthogonality_after_every_update():
    seq = wl.cfg1_sequence(3)
    res, (U, Ut) = oracle.rbicg_sequence(seq.mats, seq.b, seq.bt, seq.k, seq.s, seq.tol)
    assert all(r.status == "ok" for r in res)
    for A in seq.mats:
        Asp = as_csr(A)
        U2, Ut2, C, Ct = rc.biorthogonalize(Asp, Asp.T.tocsr(), U, Ut)
        G = Ct.conj().T @ C
        assert np.abs(G - np.eye(G.shape[0])).max() <= 1e-12


def test_t_from_scalars_and_lanczos_biorthogonality():
    """T_i built from alpha, beta, ||r|| equals the projected operator
    V~^H (I - C C^^H) A V (Sec. 4.1), T~ = T^H, and [C V] is biorthogonal to
    [C~ V~] (eq. biorth), on a complex problem with a recycle space."""
    n = 80
    lam = np.linspace(0.5, 8.0, n) + 0.3j * np.sin(np.arange(n))
    A, S, Y = _eig_system(n, 21, lam)
    U, Ut, C, Ct = _exact_recycle(A, S, Y, np.arange(4))
    rng = np.random.default_rng(22)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    bt = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    res = oracle.rbicg(A, b, bt, None, None, U, Ut, C, Ct, tol=1e-12, maxit=14,
                       update=False, keep_lanczos=True, max_restarts=0)
    m = 12
    V = np.stack(res.lanczos["V"][:m], 1)
    Vt = np.stack(res.lanczos["Vt"][:m], 1)
    alpha = res.log["alpha"][:m]
    beta = res.log["beta"][:m]          # beta_{i-1} for i = 1..m (beta_0 = 0)
    # ||r_{i-1}||, i = 1..m: ||r_0|| of the projected initial residual (eq. minusXR
    # with x_{-1} = 0), then the logged norms
    rnorm = np.concatenate([[np.linalg.norm(b - C @ (Ct.conj().T @ b))],
                            res.log["rnorm"][:m - 1]])
    T = rc.t_from_scalars(alpha, beta, rnorm)
    Pi = np.eye(n) - C @ Ct.conj().T
    Tex = Vt.conj().T @ Pi @ A @ V
    assert np.abs(T - Tex).max() <= 1e-9 * np.abs(Tex).max()
    Pit = np.eye(n) - Ct @ C.conj().T
    Ttex = V.conj().T @ Pit @ A.conj().T @ Vt
    assert np.abs(Ttex - T.conj().T).max() <= 1e-9 * np.abs(Tex).max()
    assert np.abs(Vt.conj().T @ V - np.eye(m)).max() <= 1e-9
    assert np.abs(Ct.conj().T @ V).max() <= 1e-10 and np.abs(C.conj().T @ Vt).max() <= 1e-10


def test_harmonic_ritz_exact_on_invariant_subspace():
    n = 40
    lam = np.linspace(1.0, 9.0, n)
    A, S, Y = _eig_system(n, 31, lam)
    rng = np.random.default_rng(32)
    Phi = np.concatenate([S[:, :3], rng.standard_normal((n, 4))], 1)
    Phit = np.concatenate([Y[:, :3], rng.standard_normal((n, 4))], 1)
    Asp = as_csr(A)
    P, Q, Pt, Qt = rc.harmonic_pencils(Asp, Asp.conj().T.tocsr(), Phi, Phit)
    mu = sla.eig(P, Q, right=False)
    for l in lam[:3]:
        assert np.min(np.abs(mu - l)) <= 1e-10 * abs(l)
    # the dual pencil is the conjugate transpose pencil
    assert np.allclose(Pt, P.conj().T) and np.allclose(Qt, Q.conj().T)
    W, Wt, ls = rc.pencil_eigvecs(P, Q, 3, True)
    assert np.allclose(np.sort(ls.real), lam[:3], rtol=1e-10)
    ang = sla.subspace_angles(Phi @ W, S[:, :3])
    angt = sla.subspace_angles(Phit @ Wt, Y[:, :3])
    assert ang.max() < 1e-8 and angt.max() < 1e-8


def test_rbicg_with_recycling_solves_and_keeps_invariants():
    seq = wl.cfg1_sequence(2)
    res, _ = oracle.rbicg_sequence(seq.mats, seq.b, seq.bt, seq.k, seq.s, seq.tol)
    for A, r in zip(seq.mats, res):
        D = A.to_dense()
        xs = np.linalg.solve(D, seq.b[0])
        kappa = np.linalg.cond(D)
        assert r.status == "ok" and r.relres <= 1e-8 and r.relres_dual <= 1e-8
        assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 10 * kappa * 1e-8
    # final true residual equals the recurrence residual (Alg 2 step 7)
    r1 = res[1]
    assert abs(r1.relres * np.linalg.norm(seq.b[1]) - r1.log["rnorm"][-1]) <= \
        1e-6 * r1.log["rnorm"][-1]


def test_recycling_reduces_iterations_and_subspace_improves():
    """Qualitative claims of Sec. 6.1 (values parity unpinned): recycling lowers
    the iteration count, and re-solving the same pair moves the recycle space
    towards the invariant subspace of the smallest eigenvalues (Table 1)."""
    seq = wl.cfg1_sequence(5)
    res, _ = oracle.rbicg_sequence(seq.mats, seq.b, seq.bt, seq.k, seq.s, seq.tol)
    res0, _ = oracle.rbicg_sequence(seq.mats, seq.b, seq.bt, 0, seq.s, seq.tol)
    assert sum(r.iters for r in res[1:]) < 0.8 * sum(r.iters for r in res0[1:])
    A = seq.mats[0]
    D = A.to_dense()
    w, V = np.linalg.eig(D)
    Vs = V[:, np.argsort(np.abs(w))[:4]]
    cos = []
    U = None; Ut = None
    for run in range(3):
        rr, (U, Ut) = oracle.rbicg_sequence([A], [seq.b[0]], [seq.bt[0]], seq.k, seq.s,
                                            seq.tol, U0=U, Ut0=Ut)
        cos.append(np.cos(sla.subspace_angles(U, Vs)).min())
    assert cos[-1] > cos[0] + 0.05, cos


def test_bilinear_form_quadratic_error():
    n = 100
    A = _rand_nonsym(n, 41, True, 5.0)
    rng = np.random.default_rng(42)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    exact = np.vdot(u, np.linalg.solve(A, w))
    ainv = np.linalg.norm(np.linalg.inv(A), 2)
    errs = []
    for tol in (1e-3, 1e-6):
        val, rr, res = oracle.bilinear(A, u, w, tol=tol)
        err = abs(val - exact)
        assert err <= rr * ainv * 1.0001 + 1e-13
        errs.append(err / abs(exact))
    assert errs[1] < errs[0] * 1e-4      # quadratic: the error falls much faster than tol


def test_reseed_when_dual_residual_orthogonal():
    A = wl.convdiff(8, 2, [4.0, 2.0])
    n = A.n
    rng = np.random.default_rng(51)
    b = rng.standard_normal(n)
    # b~ orthogonal to r_0 = b (x_0 = 0)
    bt = rng.standard_normal(n)
    bt -= b * (b @ bt) / (b @ b)
    res = oracle.rbicg(A, b, bt, tol=1e-9, maxit=300, update=False)
    assert res.reseeds == 1 and res.status == "ok"
    assert res.relres <= 1e-9 and res.relres_dual <= 1e-9


def test_mixed_precision_refinement_reaches_fp64_tolerance():
    seq = wl.cfg4_sequence(nsys=2, N=12)
    A = as_csr(seq.mats[0])
    U = Ut = None
    for j in range(2):
        x, xt, info, (U, Ut) = oracle.mixed_refine(A, seq.b[j], seq.bt[j], U, Ut, k=seq.k,
                                                    s=seq.s, tol=1e-10, inner_tol=1e-5)
        rel = np.linalg.norm(seq.b[j] - A @ x) / np.linalg.norm(seq.b[j])
        relt = np.linalg.norm(seq.bt[j] - A.T @ xt) / np.linalg.norm(seq.bt[j])
        assert rel <= 1e-10 and relt <= 1e-10, info
        assert info["outer"] >= 2          # FP32 inner cannot reach 1e-10 alone


def test_shifted_pairs_shared_recycle():
    A, b, c, sweeps = wl.cfg3_shifts(nsweeps=2, N=8)
    Asp = as_csr(A)
    n = Asp.shape[0]
    U = Ut = None
    xs = None
    for sig in sweeps:
        res, (U, Ut) = oracle.shifted_pairs(Asp, b, c, sig, U, Ut, k=20, s=40, tol=1e-8,
                                            x0s=xs, xt0s=None)
        xs = [r.x for r in res]
        for sg, r in zip(sig, res):
            M = sg * np.eye(n) - Asp.toarray()
            assert np.linalg.norm(b - M @ r.x) <= 1.01e-8 * np.linalg.norm(b)
            assert np.linalg.norm(c - M.conj().T @ r.xt) <= 1.01e-8 * np.linalg.norm(c)
        # conjugate shifts of a real problem have conjugate solutions
        for i in range(0, 8, 2):
            M = sig[i] * np.eye(n) - Asp.toarray()
            kappa = np.linalg.cond(M)
            d = np.linalg.norm(res[i + 1].x - np.conj(res[i].x)) / np.linalg.norm(res[i].x)
            assert d <= 4 * kappa * 1e-8
    assert U is not None and U.shape[1] > 0


# ---------------------------------------------------------- added pins
@pytest.mark.parametrize("cplx", [False, True])
def test_first_cycle_dual_space_is_left_eigenvectors(cplx):
    """First cycle of the first system (Sec. 4.2): U_1 = V_1 W_1 from the
    right and U~_1 = V~_1 W~_1 from the left eigenvectors of T_1.  With b in
    the span of m right eigenvectors of A = S Lambda S^{-1} and b~ in the span
    of the matching left eigenvectors (columns of S^{-H}), a cycle of s = m
    iterations spans exactly those invariant subspaces, so U_1 and U~_1 are
    the right and left eigenvectors of the k eigenvalues of smallest modulus.
    A swap of left and right vectors, or a wrong conjugation, moves U~_1 by
    an O(1) angle."""
    m, k = 6, 3
    A, b, bt, S, Y = eig_case(cplx, m=m)
    res = oracle.rbicg(A, b, bt, tol=1e-10, maxit=50, s=m, k=k, update=True)
    assert res.status == "ok" and res.iters == m and res.cycles == 1
    assert res.U_next.shape[1] == k and res.Ut_next.shape[1] == k
    assert sla.subspace_angles(res.U_next, S[:, :k]).max() <= 1e-8
    assert sla.subspace_angles(res.Ut_next, Y[:, :k]).max() <= 1e-8
    # the dual space is not the right eigenvector space (the pin can fail)
    assert sla.subspace_angles(res.Ut_next, S[:, :k]).max() >= 0.1


def test_plain_rbicg_has_no_stall_stop():
    """Without stall_window the oracle is plain Algorithm 2: on the stall case
    it runs to maxit (no restart, no stop of its own)."""
    A, b, bt, U, Ut, C, Ct = stall_case()
    assert U.shape[1] == 4
    res = oracle.rbicg(A, b, bt, None, None, U, Ut, C, Ct, tol=1e-10, maxit=600, s=20, k=6)
    assert res.status == "maxit" and res.iters == 600 and res.restarts == 0
    assert res.relres > 1e-6


def test_restart_on_stall_driver():
    """The restart driver (not in the paper): its first run is plain
    Algorithm 2 up to the stall (same iterates as the run without the stop);
    the stall is at a cycle end where the smallest cycle-end residual has
    not halved over four cycles; the second run is bitwise the plain run
    from the initial guesses without recycling; the result solves the
    systems (dense solve)."""
    A, b, bt, U, Ut, C, Ct = stall_case()
    s, tol = 20, 1e-10
    res = oracle.drivers.rbicg_restart_on_stall(A, b, bt, None, None, U, Ut, C, Ct, tol=tol,
                                                maxit=1500, s=s, k=6, stall_window=4)
    at = res.stalled_at
    assert at % s == 0 and at >= 4 * s and res.restarts == 1 and res.status == "ok"
    plain = oracle.rbicg(A, b, bt, None, None, U, Ut, C, Ct, tol=tol, maxit=at, s=s, k=6)
    np.testing.assert_array_equal(res.log["rnorm"][:at], plain.log["rnorm"])
    bn, btn = np.linalg.norm(b), np.linalg.norm(bt)
    h = np.maximum(plain.log["rnorm"] / bn, plain.log["rtnorm"] / btn)
    # cycle-end values, with the projected initial residuals r_0 = b - C C~^H b,
    # r~_0 = b~ - C~ C^H b~ (eq. minusXR with x = x~ = 0) in front
    h0 = max(np.linalg.norm(b - C @ (Ct.T @ b)) / bn, np.linalg.norm(bt - Ct @ (C.T @ bt)) / btn)
    ends = [h0] + [h[c * s - 1] for c in range(1, at // s + 1)]
    best = np.minimum.accumulate(ends)
    cs = at // s
    assert best[cs] >= 0.5 * best[cs - 4]
    assert all(best[c] < 0.5 * best[c - 4] for c in range(4, cs))
    fresh = oracle.rbicg(A, b, bt, None, None, tol=tol, maxit=1500 - at, s=s, k=6)
    assert res.iters == at + fresh.iters
    np.testing.assert_array_equal(res.x, fresh.x)
    D = A.toarray()
    xs = np.linalg.solve(D, b)
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) <= 10 * kappa * tol
    assert res.relres <= tol and res.relres_dual <= tol


def test_fp32_simulation_is_bicg_on_rounded_data():
    """FP32 storage (k = 0, no guard firing): the simulated iterates equal
    FP64 BiCG on the float-rounded matrix and right-hand sides up to float
    rounding.  After one iteration the difference is one rounding of
    x_1 = alpha p (at most 2 eps32, and not zero: the simulation does round);
    after a few iterations it stays at float-rounding level; the converged
    corrections solve the rounded systems to the inner tolerance in BiCG's
    iteration count (+-1)."""
    from oracle.drivers import rbicg_fp32_inner, EPS32
    A = as_csr(wl.convdiff(12, 2, [10.0, 5.0]))
    AH = A.T.tocsr()
    A32, AH32 = A.astype(np.float32), AH.astype(np.float32)
    Ar = A32.astype(np.float64)
    rng = np.random.default_rng(3)
    b, bt = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    b32 = b.astype(np.float32).astype(np.float64)
    bt32 = bt.astype(np.float32).astype(np.float64)
    for j, bound in ((1, 2 * EPS32), (2, 1e-5), (5, 1e-5)):
        d, dt, it, _, div = rbicg_fp32_inner(A32, AH32, b, bt, None, None, None, None, 1e-30, j,
                                             40, 0, False, A64=A, AH64=AH)
        ref = oracle.bicg(Ar, b32, bt32, tol=1e-30, maxit=j)
        assert it == j and not div
        for got, want in ((d, ref.x), (dt, ref.xt)):
            e = np.linalg.norm(got - want) / np.linalg.norm(want)
            assert 1e-10 <= e <= bound
    d, dt, it, _, div = rbicg_fp32_inner(A32, AH32, b, bt, None, None, None, None, 1e-5, 1000, 40,
                                         0, False, A64=A, AH64=AH)
    ref = oracle.bicg(Ar, b32, bt32, tol=1e-5, maxit=1000)
    assert not div and abs(it - ref.iters) <= 1
    assert np.linalg.norm(b32 - Ar @ d) / np.linalg.norm(b32) <= 2e-5
    assert np.linalg.norm(bt32 - Ar.T @ dt) / np.linalg.norm(bt32) <= 2e-5
    assert np.linalg.norm(d - ref.x) / np.linalg.norm(ref.x) <= 1e-3
