"""GPU parity of the HIP path against the CPU oracle, element by element on the
same seeded inputs, through the C ABI (python binding -> librbicg.so).

Bars (from the method's use): true relative residual <= tol on both sides,
iteration counts within 5% of the oracle's, solutions within 1e-6 relative of
the oracle's, and early per-iteration scalars (alpha, beta, ||r||) to 1e-9
relative where both sides start from the same recycle space."""
import numpy as np
import pytest

import oracle
from oracle import recycle as rc
from oracle.krylov import as_csr
from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(*a, **kw):
    from paper_1010_0762_amd.solver import Solver
    return Solver(*a, **kw)


def _t(v, dtype=None):
    dt = dtype or (torch.complex128 if np.iscomplexobj(v) else torch.float64)
    return torch.as_tensor(np.ascontiguousarray(v)).to(device="cuda", dtype=dt)


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _iters_close(a, b, frac=0.05):
    return abs(a - b) <= max(1, int(np.ceil(frac * b)))


def test_bicg_k0_matches_oracle_iterates():
    seq = wl.cfg1_sequence(1)
    A, b, bt = seq.mats[0], seq.b[0], seq.bt[0]
    ref = oracle.bicg(A, b, bt, tol=1e-8, maxit=2000)
    S = _solver(A, k=0, s=40, update=False)
    x, xt, st = S.solve(_t(b), _t(bt), tol=1e-8)
    assert st["status"] == 0
    assert _iters_close(st["iters"], ref.iters, 0.0)
    lg = S.log()
    m = min(30, len(lg))
    alpha = ref.log["alpha"][:m]
    assert np.allclose(lg[:m, 0], alpha, rtol=1e-9, atol=0)
    assert np.allclose(lg[:m, 6], ref.log["rnorm"][1:m + 1], rtol=1e-9, atol=0)
    assert st["relres"] <= 1e-8 and st["relres_dual"] <= 1e-8
    assert _rel(_np(x), ref.x) <= 1e-6 and _rel(_np(xt), ref.xt) <= 1e-6


def test_injected_recycle_space_matches_oracle():
    """The oracle's recycle space from system 0, installed on the GPU
    (Algorithm 2 step 1), then system 1 solved without updating: the oblique
    projector is basis independent, so the iterations agree to rounding."""
    seq = wl.cfg1_sequence(2)
    A0, A1 = as_csr(seq.mats[0]), as_csr(seq.mats[1])
    r0 = oracle.rbicg(A0, seq.b[0], seq.bt[0], tol=1e-8, maxit=2000, s=40, k=10)
    U, Ut, C, Ct = rc.biorthogonalize(A1, A1.T.tocsr(), r0.U_next, r0.Ut_next)
    ref = oracle.rbicg(A1, seq.b[1], seq.bt[1], None, None, U, Ut, C, Ct, tol=1e-8, maxit=2000,
                       update=False)
    S = _solver(seq.mats[1], k=10, s=40, update=False)
    S.set_recycle(_t(r0.U_next), _t(r0.Ut_next))
    Ug, Utg, Cg, Ctg = (_np(t) for t in S.get_recycle())
    assert Ug.shape[1] == U.shape[1]
    assert np.abs(Ctg.T @ Cg - np.eye(Ug.shape[1])).max() <= 1e-12
    x, xt, st = S.solve(_t(seq.b[1]), _t(seq.bt[1]), tol=1e-8)
    assert st["status"] == 0 and st["k_used"] == U.shape[1]
    assert _iters_close(st["iters"], ref.iters)
    lg = S.log()
    m = 15
    assert np.allclose(lg[:m, 0], ref.log["alpha"][:m], rtol=1e-9, atol=0)
    assert np.allclose(lg[:m, 6], ref.log["rnorm"][:m], rtol=1e-9, atol=0)
    assert st["relres"] <= 1e-8 and st["relres_dual"] <= 1e-8
    assert _rel(_np(x), ref.x) <= 1e-6 and _rel(_np(xt), ref.xt) <= 1e-6


@pytest.mark.parametrize("nsys", [5])
def test_sequence_cfg1_matches_oracle(nsys):
    """2D convection-diffusion 32x32 sequence (k=10, s=40, tol 1e-8) with the
    GPU's own cycle-wise recycle updates."""
    seq = wl.cfg1_sequence(nsys)
    ref, _ = oracle.rbicg_sequence(seq.mats, seq.b, seq.bt, seq.k, seq.s, seq.tol)
    S = _solver(seq.mats[0], k=seq.k, s=seq.s)
    its = []
    for j in range(nsys):
        if j:
            S.update_recycle(seq.mats[j])
        x, xt, st = S.solve(_t(seq.b[j]), _t(seq.bt[j]), tol=seq.tol)
        its.append(st["iters"])
        assert st["status"] == 0, (j, st)
        assert st["relres"] <= seq.tol and st["relres_dual"] <= seq.tol, (j, st)
        assert _iters_close(st["iters"], ref[j].iters), (j, st["iters"], ref[j].iters)
        assert _rel(_np(x), ref[j].x) <= 1e-6 and _rel(_np(xt), ref[j].xt) <= 1e-6
        assert st["cycles"] == ref[j].cycles
    assert sum(its[1:]) < sum(r.iters for r in ref[:1]) * (nsys - 1)


def test_ragged_size_and_determinism():
    """n = 37^2 = 1369 (not a multiple of the 64-row slice or 256-row block)."""
    A = wl.convdiff(37, 2, [6.0, 3.0])
    rng = np.random.default_rng(77)
    b, bt = rng.standard_normal(A.n), rng.standard_normal(A.n)
    ref, _ = oracle.rbicg_sequence([A, A], [b, b], [bt, bt], 10, 40, 1e-9)
    S = _solver(A, k=10, s=40)
    x0, xt0, st0 = S.solve(_t(b), _t(bt), tol=1e-9)
    assert _iters_close(st0["iters"], ref[0].iters)
    S.update_recycle()
    x1, xt1, st1 = S.solve(_t(b), _t(bt), tol=1e-9)
    assert _iters_close(st1["iters"], ref[1].iters)
    assert st1["relres"] <= 1e-9 and _rel(_np(x1), ref[1].x) <= 1e-6
    # bitwise determinism: the same handle state gives the same result
    S2 = _solver(A, k=10, s=40)
    y0, yt0, _ = S2.solve(_t(b), _t(bt), tol=1e-9)
    assert torch.equal(x0, y0) and torch.equal(xt0, yt0)


def test_complex_sequence_matches_oracle():
    A = wl.random_sparse(700, 6, 31, 6.0, complex_vals=True)
    rng = np.random.default_rng(32)
    b = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    bt = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    A2 = wl.CSR(A.n, A.rowptr, A.colind, A.vals * (1 + 0.01j))
    ref, _ = oracle.rbicg_sequence([A, A2], [b, b], [bt, bt], 8, 20, 1e-9)
    S = _solver(A, k=8, s=20, prec="c128")
    for j, M in enumerate([A, A2]):
        if j:
            S.update_recycle(M)
        x, xt, st = S.solve(_t(b), _t(bt), tol=1e-9)
        assert st["status"] == 0
        assert _iters_close(st["iters"], ref[j].iters), (st["iters"], ref[j].iters)
        assert st["relres"] <= 1e-9 and st["relres_dual"] <= 1e-9
        assert _rel(_np(x), ref[j].x) <= 1e-6 and _rel(_np(xt), ref[j].xt) <= 1e-6


def test_layout_sharing_and_unshared_real_sequence():
    """A^H keeps A's index arrays when it has A's pattern in the same row
    order (a stencil) and its own when not (a random nonsymmetric pattern);
    the real iteration kernels on the unshared layout match the oracle too."""
    from paper_1010_0762_amd.solver import DeviceMatrix
    Ac = wl.convdiff(8, 2, [4.0, 2.0])
    mc = DeviceMatrix(Ac)
    ic = mc.info()
    assert ic["shared_pattern"] and not ic["complex"]
    assert ic["n"] == Ac.n and ic["nnz"] == len(Ac.colind) and ic["nnz_padded"] >= ic["nnz"]
    mc.close()
    # a pencil sigma E - A inherits the sharing; so does a red-black black block
    from paper_1010_0762_amd.solver import RBILU
    A5, E5 = DeviceMatrix(wl.aniso_diffusion(5)), DeviceMatrix(wl.mass_like(5))
    P5 = DeviceMatrix.pencil(A5, E5, 2.0 + 1.0j)
    ip = P5.info()
    assert ip["shared_pattern"] and ip["complex"] and ip["nnz_padded"] == A5.info()["nnz_padded"]
    for m in (P5, A5, E5):
        m.close()
    rb = RBILU(wl.convdiff(8, 3, [4.0, 2.0, 1.0]))
    assert rb.black.info()["shared_pattern"]
    rb.close()
    A = wl.random_sparse(700, 6, 33, 6.0)
    m = DeviceMatrix(A)
    assert not m.info()["shared_pattern"]
    m.close()
    rng = np.random.default_rng(34)
    b = rng.standard_normal(A.n)
    bt = rng.standard_normal(A.n)
    A2 = wl.CSR(A.n, A.rowptr, A.colind, A.vals * (1 + 0.05 * rng.standard_normal(len(A.vals))))
    ref, _ = oracle.rbicg_sequence([A, A2], [b, b], [bt, bt], 8, 20, 1e-9)
    S = _solver(A, k=8, s=20)
    for j, M in enumerate([A, A2]):
        if j:
            S.update_recycle(M)
        x, xt, st = S.solve(_t(b), _t(bt), tol=1e-9)
        assert st["status"] == 0
        assert _iters_close(st["iters"], ref[j].iters), (st["iters"], ref[j].iters)
        assert st["relres"] <= 1e-9 and st["relres_dual"] <= 1e-9
        assert _rel(_np(x), ref[j].x) <= 1e-6 and _rel(_np(xt), ref[j].xt) <= 1e-6


def test_reseed_matches_oracle():
    A = wl.convdiff(8, 2, [4.0, 2.0])
    rng = np.random.default_rng(51)
    b = rng.standard_normal(A.n)
    bt = rng.standard_normal(A.n)
    bt -= b * (b @ bt) / (b @ b)
    ref = oracle.rbicg(A, b, bt, tol=1e-9, maxit=300, update=False)
    S = _solver(A, k=0, s=40, update=False)
    x, xt, st = S.solve(_t(b), _t(bt), tol=1e-9)
    assert st["reseeds"] == ref.reseeds == 1
    assert st["iters"] == ref.iters
    assert _rel(_np(xt), ref.xt) <= 1e-8


@pytest.mark.parametrize("xt0", ["random", "zero"])
def test_zero_dual_rhs_matches_oracle(xt0):
    """b~ = 0: the unprojected initial dual residual replaces ||b~|| as the
    dual scale; with x~_0 = 0 that residual vanishes, (r~_0, r_0) = 0 forces a
    re-seed, and the scale is taken after it (as in the oracle)."""
    A = wl.convdiff(10, 2, [3.0, 1.0])
    rng = np.random.default_rng(77)
    b = rng.standard_normal(A.n)
    bt = np.zeros(A.n)
    xt = rng.standard_normal(A.n) if xt0 == "random" else np.zeros(A.n)
    ref = oracle.rbicg(A, b, bt, xt=xt.copy(), tol=1e-9, maxit=400, update=False)
    S = _solver(A, k=0, s=40, update=False)
    x0 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    x, xtg, st = S.solve(_t(b), _t(bt), x0, _t(xt), tol=1e-9)
    assert st["status"] == 0, st
    assert st["reseeds"] == ref.reseeds == (1 if xt0 == "zero" else 0)
    assert abs(st["iters"] - ref.iters) <= 1, (st["iters"], ref.iters)
    assert st["relres"] <= 1e-9 and st["relres_dual"] <= 1e-9
    assert abs(st["relres_dual"] - ref.relres_dual) <= 1e-10
    assert _rel(_np(x), ref.x) <= 1e-8


def test_bilinear_form():
    A = wl.convdiff(20, 2, [5.0, 2.0])
    D = A.to_dense()
    rng = np.random.default_rng(61)
    u, w = rng.standard_normal(A.n), rng.standard_normal(A.n)
    exact = u @ np.linalg.solve(D, w)
    S = _solver(A, k=0, s=40, update=False)
    val, err, st = S.bilinear(_t(u), _t(w), tol=1e-6)
    ainv = np.linalg.norm(np.linalg.inv(D), 2)
    assert abs(val - exact) <= err * ainv * 1.001 + 1e-12 * abs(exact)
    ov, orr, _ = oracle.bilinear(A, u, w, tol=1e-6)
    assert abs(val - ov) <= 1e-6 * abs(exact)


def test_maxit_and_bad_args():
    from paper_1010_0762_amd import _lib
    A = wl.convdiff(16, 2, [4.0, 2.0])
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.n)
    S = _solver(A, k=0, s=40, update=False, maxit=5)
    x, xt, st = S.solve(_t(b), _t(b), tol=1e-12)
    assert st["status"] == _lib.RBICG_NOT_CONVERGED and st["iters"] == 5
    with pytest.raises(TypeError):
        S.solve(_t(b[:10]), _t(b), tol=1e-8)
    with pytest.raises(_lib.RBiCGError):
        _solver(A, k=65)


@pytest.mark.parametrize("cplx", [False, True])
def test_first_cycle_spaces_are_eigenvectors(cplx):
    """First cycle of the first system on the GPU (Sec. 4.2, eigenvectors of
    T_1 from the iteration scalars): with b, b~ in invariant subspaces of
    dimension m = s, the space built for the next system is the right and
    the left eigenvectors of the k eigenvalues of smallest modulus, as the
    oracle's is."""
    from scipy.linalg import subspace_angles
    from cases import eig_case
    m, k = 6, 3
    A, b, bt, S_, Y = eig_case(cplx, m=m)
    ref = oracle.rbicg(A, b, bt, tol=1e-10, maxit=50, s=m, k=k, update=True)
    S = _solver(sp_csr(A), k=k, s=m, prec="c128" if cplx else "f64")
    x, xt, st = S.solve(_t(b), _t(bt), tol=1e-10)
    assert st["status"] == 0 and st["iters"] == ref.iters == m
    U, Ut, _, _ = S.get_recycle(next=True, kcap=k)
    U, Ut = _np(U), _np(Ut)
    assert U.shape[1] == Ut.shape[1] == k
    assert subspace_angles(U, S_[:, :k]).max() <= 1e-7
    assert subspace_angles(Ut, Y[:, :k]).max() <= 1e-7
    assert subspace_angles(U, ref.U_next).max() <= 1e-7
    assert subspace_angles(Ut, ref.Ut_next).max() <= 1e-7
    S.close()


def sp_csr(A):
    import scipy.sparse as sp
    return sp.csr_matrix(A)


def test_stall_guard_matches_oracle_driver():
    """Stall guard (opts.stall_window, not in the paper) against the oracle's
    restart driver on a case where plain Algorithm 2 does not converge: the
    GPU stalls at a cycle end (iteration a multiple of s, at least four
    cycles in), restarts without the recycle space and converges; the
    restarted run's count is within 5% of the oracle's fresh run, and the
    solution matches the oracle's.  Without the guard the GPU, like plain
    Algorithm 2, runs to maxit."""
    from cases import stall_case
    A, b, bt, U, Ut, C, Ct = stall_case()
    s, tol = 20, 1e-10
    ref = oracle.drivers.rbicg_restart_on_stall(A, b, bt, None, None, U, Ut, C, Ct, tol=tol,
                                                maxit=1500, s=s, k=6, stall_window=4)
    assert ref.status == "ok" and ref.restarts == 1
    fresh_ref = ref.iters - ref.stalled_at
    S = _solver(A, k=6, s=s, svd_tol=1e-7, maxit=1500, stall_window=4)
    S.set_recycle(_t(U), _t(Ut))
    x, xt, st = S.solve(_t(b), _t(bt), tol=tol)
    assert st["status"] == 0 and st["restarts"] >= 1
    assert st["relres"] <= tol and st["relres_dual"] <= tol
    lg = S.log()
    at = int(np.argmax(lg[:, 9] >= 1))      # first iteration of the restarted run
    assert at % s == 0 and at >= 4 * s
    assert _iters_close(st["iters"] - at, fresh_ref)
    assert _rel(_np(x), ref.x) <= 1e-6 and _rel(_np(xt), ref.xt) <= 1e-6
    S.close()
    from paper_1010_0762_amd import _lib
    P = _solver(A, k=6, s=s, svd_tol=1e-7, maxit=600, update=True)
    P.set_recycle(_t(U), _t(Ut))
    try:
        x, xt, st = P.solve(_t(b), _t(bt), tol=tol)
        assert st["status"] == 1 and st["iters"] == 600 and st["restarts"] == 0
    except _lib.RBiCGError as e:   # a drifting iteration may also break down
        assert e.code == _lib.RBICG_BREAKDOWN
    P.close()


def test_solve_sequence_equals_one_by_one():
    """rbicg_solve_sequence (the whole sequence in one library call) gives
    bitwise the iterates and counts of the same calls made one by one
    (rbicg_update_recycle_on, zeroed guesses, rbicg_solve_dual), over two
    passes of a recycled 2D sequence with an unchanged matrix in between."""
    from paper_1010_0762_amd.solver import DeviceMatrix, Solver
    seq = wl.cfg1_sequence(nsys=4)
    mats = [DeviceMatrix(A) for A in seq.mats]
    mats.insert(2, mats[1])            # the same matrix twice in a row
    bs = [torch.as_tensor(seq.b[0], device="cuda")] * len(mats)
    bts = [torch.as_tensor(seq.bt[0], device="cuda")] * len(mats)
    S1 = Solver(mats[0], k=seq.k, s=seq.s)
    S2 = Solver(mats[0], k=seq.k, s=seq.s)
    for rep in range(2):
        S1.set_recycle(None, None)
        one = []
        for j, M in enumerate(mats):
            if j > 0 or M is not S1.matrix:
                S1.update_recycle(M)
            x, xt, st = S1.solve(bs[j], bts[j], tol=seq.tol)
            one.append((x, xt, st))
        S2.set_recycle(None, None)
        xs, xts, sts = S2.solve_sequence(mats, bs, bts, tol=seq.tol)
        print("rep", rep, [o[2]["iters"] for o in one], [s["iters"] for s in sts], flush=True)
        for (x, xt, st), xs_, xts_, st2 in zip(one, xs, xts, sts):
            assert st["iters"] == st2["iters"] and st["k_used"] == st2["k_used"]
            assert st2["status"] == 0
            assert torch.equal(x, xs_) and torch.equal(xt, xts_)
    S1.close()
    S2.close()


@pytest.mark.parametrize("cplx", [False, True])
def test_wide_recycle_spaces_match_oracle(cplx):
    """k = 40: the cycle-end tall-skinny products write three 16-column output
    tiles, and from a system's second cycle on Phi = [U, V] has up to 80
    columns (W staged in LDS in two batches of rows).  Real: the 2D
    convection-diffusion sequence (126, 65, 65 iterations in the oracle, with
    30-37 vectors kept); complex: a random sparse pair and its matrix scaled
    by 1 + 0.01i (two cycles per system).  Iterations within 5%, solutions to
    1e-6, and the space carried out of the last system against the oracle's
    (dimension within one, C~^H C = I, principal angles within ten times the
    oracle's own spread: at k = 40 the largest angle between the oracle's
    spaces for b and for b perturbed by 1e-13 relative reaches 1e-2 on the
    real sequence, with the same iteration counts, so the spread is the
    largest over four perturbed runs)."""
    from scipy.linalg import subspace_angles
    if cplx:
        A = wl.random_sparse(1500, 6, 41, 4.5, complex_vals=True)
        rng = np.random.default_rng(42)
        b = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
        bt = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
        mats = [A, wl.CSR(A.n, A.rowptr, A.colind, A.vals * (1 + 0.01j))]
        bs, bts, tol = [b, b], [bt, bt], 1e-9
    else:
        seq = wl.cfg1_sequence(3)
        mats, bs, bts, tol = seq.mats, seq.b, seq.bt, seq.tol
    k, s = 40, 40
    ref, (Ur, Utr) = oracle.rbicg_sequence(mats, bs, bts, k, s, tol)
    rng = np.random.default_rng(9)
    spread = 0.0
    for _ in range(4):
        bp = [v * (1 + 1e-13 * rng.standard_normal(v.shape)) for v in bs]
        _, (Ur2, Utr2) = oracle.rbicg_sequence(mats, bp, bts, k, s, tol)
        spread = max(spread, subspace_angles(Ur, Ur2).max(), subspace_angles(Utr, Utr2).max())
    S = _solver(mats[0], k=k, s=s, prec="c128" if cplx else "f64")
    for j, M in enumerate(mats):
        if j:
            S.update_recycle(M)
        x, xt, st = S.solve(_t(bs[j]), _t(bts[j]), tol=tol)
        assert st["status"] == 0, (j, st)
        assert st["relres"] <= tol and st["relres_dual"] <= tol, (j, st)
        assert _iters_close(st["iters"], ref[j].iters), (j, st["iters"], ref[j].iters)
        assert st["cycles"] == ref[j].cycles, (j, st["cycles"], ref[j].cycles)
        assert _rel(_np(x), ref[j].x) <= 1e-6 and _rel(_np(xt), ref[j].xt) <= 1e-6
    Ug, Utg, Cg, Ctg = (_np(v) for v in S.get_recycle(next=True, kcap=k))
    assert Ug.shape[1] > 32 and abs(Ug.shape[1] - Ur.shape[1]) <= 1, (Ug.shape, Ur.shape)
    ang = max(subspace_angles(Ug, Ur).max(), subspace_angles(Utg, Utr).max())
    print(f"k=40 {'complex' if cplx else 'real'}: p gpu={Ug.shape[1]} oracle={Ur.shape[1]} "
          f"angle {ang:.2e} oracle spread {spread:.2e}", flush=True)
    assert np.linalg.norm(Ctg.conj().T @ Cg - np.eye(Ug.shape[1])) <= 1e-12
    assert ang <= max(1e-6, 10.0 * spread), (ang, spread)


@pytest.mark.parametrize("k,s,cplx", [(64, 40, False), (20, 107, False), (64, 40, True)])
def test_largest_recycle_space_and_cycle_match_oracle(k, s, cplx):
    """The documented limits: k = 64 (the largest recycle dimension; the
    cycle-end products write four 16-column tiles from up to 80 input
    columns, the pencil Gram has 105 x 209 entries) and s + k + 1 = 128 (the
    longest cycle: a 107-vector first cycle, a 128-column Gram, a 127 x 127
    pencil on the host).  The 2D convection-diffusion sequence, and at k = 64
    also the complex random sparse pair of the k = 40 test (the products'
    largest LDS use: complex W rows of four tiles), against the oracle: iterations within 5%, cycles, solutions to 1e-6, the carried
    space's dimension (within two), C~^H C = I, and its principal angles
    within ten times the oracle's own spread over four 1e-13-perturbed runs
    where that spread is small (at k = 64 it reaches 0.15 rad, so the angles
    carry no information there)."""
    from scipy.linalg import subspace_angles
    if cplx:
        A = wl.random_sparse(1500, 6, 41, 4.5, complex_vals=True)
        rng = np.random.default_rng(42)
        b = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
        bt = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
        mats = [A, wl.CSR(A.n, A.rowptr, A.colind, A.vals * (1 + 0.01j))]
        bs, bts, tol = [b, b], [bt, bt], 1e-9
    else:
        seq = wl.cfg1_sequence(3)
        mats, bs, bts, tol = seq.mats, seq.b, seq.bt, seq.tol
    ref, (Ur, Utr) = oracle.rbicg_sequence(mats, bs, bts, k, s, tol)
    rng = np.random.default_rng(9)
    spread = 0.0
    for _ in range(4):
        bp = [v * (1 + 1e-13 * rng.standard_normal(v.shape)) for v in bs]
        _, (Ur2, Utr2) = oracle.rbicg_sequence(mats, bp, bts, k, s, tol)
        spread = max(spread, subspace_angles(Ur, Ur2).max(), subspace_angles(Utr, Utr2).max())
    S = _solver(mats[0], k=k, s=s, prec="c128" if cplx else "f64")
    for j, M in enumerate(mats):
        if j:
            S.update_recycle(M)
        x, xt, st = S.solve(_t(bs[j]), _t(bts[j]), tol=tol)
        assert st["status"] == 0, (j, st)
        assert st["relres"] <= tol and st["relres_dual"] <= tol, (j, st)
        assert _iters_close(st["iters"], ref[j].iters), (j, st["iters"], ref[j].iters)
        assert st["cycles"] == ref[j].cycles, (j, st["cycles"], ref[j].cycles)
        assert _rel(_np(x), ref[j].x) <= 1e-6 and _rel(_np(xt), ref[j].xt) <= 1e-6
    Ug, Utg, Cg, Ctg = (_np(v) for v in S.get_recycle(next=True, kcap=k))
    assert Ug.shape[1] > 0 and abs(Ug.shape[1] - Ur.shape[1]) <= 2, (Ug.shape, Ur.shape)
    ang = max(subspace_angles(Ug, Ur).max(), subspace_angles(Utg, Utr).max())
    print(f"k={k} s={s} {'complex' if cplx else 'real'}: p gpu={Ug.shape[1]} oracle={Ur.shape[1]} angle {ang:.2e} "
          f"oracle spread {spread:.2e}", flush=True)
    assert np.linalg.norm(Ctg.conj().T @ Cg - np.eye(Ug.shape[1])) <= 1e-11
    if spread < 1e-3:
        assert ang <= max(1e-6, 10.0 * spread), (ang, spread)
