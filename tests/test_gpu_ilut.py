"""Split ILUT preconditioning on the GPU (rbicg_ilut_create, rbicg_ilu_*,
solver.ILUT, solver.solve_ilut_sequence) against the oracle
(oracle/precond.py: ILUT, the explicitly formed operator L^{-1} A U^{-1},
RBiCG on it): the right-hand-side and solution transforms element by
element (device level-scheduled triangular solves), preconditioned
sequences with recycling on a 2D convection-diffusion operator (iteration
counts, retained recycle dimensions, solutions), a matrix whose pattern is
not two-colourable, a complex pair, repeated solves of one system, and the
refusals."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle.precond as pc
from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(v):
    return torch.as_tensor(np.ascontiguousarray(v), device="cuda")


def _csr(A):
    return sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n))


def _mats_2d(N, m):
    return wl.ilut2d_sequence(nsys=m, N=N).mats


@pytest.mark.parametrize("kind", ["convdiff", "random_real", "random_complex"])
def test_transforms_match_oracle(kind):
    """L^{-1} b, U^{-H} b~, U^{-1} y, L^{-H} y~ from the device solves equal
    the oracle's sparse triangular solves (n = 1600, 1500: several blocks
    with a ragged tail; a pattern that is not two-colourable)."""
    from paper_1010_0762_amd.solver import ILUT
    rng = np.random.default_rng(3)
    if kind == "convdiff":
        A = _csr(_mats_2d(40, 1)[0])
    else:
        R = wl.random_sparse(1500, 6, 21, diag_shift=10.0, complex_vals=(kind == "random_complex"))
        A = _csr(R)
    n = A.shape[0]
    cplx = np.iscomplexobj(A.data)
    print("case", kind, n, flush=True)
    ss = pc.IlutSystem(A, 0.05)
    P = ILUT(A, 0.05)
    info = P.info()
    assert info["n"] == n and info["nnz_L"] == sp.tril(ss.L, -1).nnz and info["nnz_U"] == ss.U.nnz
    vecs = []
    for _ in range(4):
        v = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
        vecs.append(v)
    b, bt, y, yt = vecs
    bh, ch = P.rhs(_t(b), _t(bt))
    bhr, chr_ = ss.rhs(b, bt)
    x, xt = P.solution(_t(y), _t(yt))
    xr, xtr = ss.solution(y, yt)
    for got, ref in ((bh, bhr), (ch, chr_), (x, xr), (xt, xtr)):
        g = got.cpu().numpy()
        ref = ref if cplx else ref.real
        assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()
    if not cplx:  # complex vectors with real factors
        bc, cc = P.rhs(_t(b.astype(np.complex128)), _t(bt.astype(np.complex128)))
        assert np.abs(bc.cpu().numpy() - bhr).max() <= 1e-12 * np.abs(bhr).max()
    assert P.info()["wait_error"] == 0
    P.close()


GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ilut_convdiff2d_40.json")


def _perturbed(v, j):
    rng = np.random.default_rng(wl.BASE_SEED + 9000 + j)
    return v * (1.0 + 1e-13 * rng.standard_normal(v.shape))


def _run_sequence(seq, tau, prec, real, ranges):
    """GPU sequence against the oracle's unperturbed run (solutions) and the
    ranges of its counts and carried dimensions (ranges[i] = (iters list,
    k list) over the oracle's runs for system i)."""
    from paper_1010_0762_amd.solver import solve_ilut_sequence
    ref_sols, ref = pc.rbicg_ilut_sequence(seq.mats, seq.b, seq.bt, seq.k, seq.s, seq.tol, tau,
                                           real=real)
    out = solve_ilut_sequence(seq.mats, [_t(b) for b in seq.b], [_t(b) for b in seq.bt],
                              droptol=tau, k=seq.k, s=seq.s, tol=seq.tol, prec=prec)
    print("iters gpu", [o[2]["iters"] for o in out], "oracle", [r.iters for r in ref],
          "k gpu", [o[2]["k_used"] for o in out], "oracle", [r.k_used for r in ref], flush=True)
    for i, (A, (x, xt, st), (xr, xtr), b, bt) in enumerate(zip(seq.mats, out, ref_sols, seq.b, seq.bt)):
        As = _csr(A) if hasattr(A, "rowptr") else A
        its, ks = ranges[i]
        lo, hi = min(its), max(its)
        slack = max(2, int(np.ceil(0.05 * hi)))
        assert st["status"] == 0
        assert st["relres"] <= seq.tol and st["relres_dual"] <= seq.tol
        assert lo - slack <= st["iters"] <= hi + slack, (i, st["iters"], lo, hi)
        assert min(ks) <= st["k_used"] <= max(ks), (i, st["k_used"], ks)
        xv, xtv = x.cpu().numpy(), xt.cpu().numpy()
        assert np.linalg.norm(xv - xr) <= 1e-6 * np.linalg.norm(xr)
        assert np.linalg.norm(xtv - xtr) <= 1e-6 * np.linalg.norm(xtr)
        assert np.linalg.norm(b - As @ xv) <= 1e-5 * np.linalg.norm(b)
        assert np.linalg.norm(bt - As.conj().T @ xtv) <= 1e-5 * np.linalg.norm(bt)
    return out


def _gold_ranges(name):
    with open(GOLD) as f:
        g = json.load(f)[name]
    nsys = len(g["iters"])
    return [([run[i] for run in g["iters_runs"]], [run[i] for run in g["k_runs"]]) for i in range(nsys)]


def test_ilut_sequence_matches_oracle():
    """Four 2D convection-diffusion systems (n = 1600) with a drifting
    convection field, ILUT(0.2) each (a weaker factorization than the 0.05
    of Sec. 6.1, so that these small systems take several cycles), k = 5,
    s = 10, tol 1e-8: solutions within 1e-6 of the oracle's, counts and
    carried dimensions inside the oracle's own spread under 1e-13
    perturbations of b, b~ (stored by tests/golden/make_golden.py)."""
    seq = wl.ilut2d_sequence()
    print("case", seq.name, flush=True)
    _run_sequence(seq, seq.extra["droptol"], "f64", True, _gold_ranges(seq.name))


def test_ilut_same_system_repeated():
    """The same preconditioned pair solved four times (the set-up of the 2D
    experiment of Sec. 6.1, with x0 = 0, ILUT(0.2), k = 10, s = 20): the
    recycled solves need fewer iterations than the first, on the GPU as in
    the oracle, and match it."""
    seq = wl.ilut2d_sequence(repeat=True)
    print("case", seq.name, flush=True)
    out = _run_sequence(seq, seq.extra["droptol"], "f64", True, _gold_ranges(seq.name))
    assert all(o[2]["iters"] < out[0][2]["iters"] for o in out[1:])


def test_ilut_unstructured_and_complex():
    """A random sparse matrix with odd cycles in its graph (the red-black
    set-up refuses it) and a complex pair of such matrices, ILUT(0.1), k = 4,
    s = 8; ranges from the oracle's unperturbed run and three perturbed ones."""
    for cplx in (False, True):
        A0 = _csr(wl.random_sparse(1200, 5, 30, diag_shift=4.0, complex_vals=cplx))
        A1 = A0.copy()
        A1.data = A1.data * (1 + 0.01 * np.cos(np.arange(A1.nnz)))
        mats = [A0, A1.tocsr()]
        rng = np.random.default_rng(40 + cplx)
        n = A0.shape[0]
        bs = [rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0) for _ in mats]
        bts = [rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0) for _ in mats]
        seq = wl.DualSequence("random", mats, bs, bts, 4, 8, 1e-9)
        runs = []
        for j in range(4):
            bp = bs if j == 0 else [_perturbed(v, 800 + 10 * j + i) for i, v in enumerate(bs)]
            _, res = pc.rbicg_ilut_sequence(mats, bp, bts, 4, 8, 1e-9, 0.1, real=not cplx)
            runs.append(res)
        ranges = [([r[i].iters for r in runs], [r[i].k_used for r in runs]) for i in range(2)]
        print("case ilut unstructured complex", cplx, ranges, flush=True)
        _run_sequence(seq, 0.1, "c128" if cplx else "f64", not cplx, ranges)


def test_ilut_refusals():
    """Host-side refusals: a zero pivot; a preconditioner of another order;
    a mixed-precision handle; batching a preconditioned handle."""
    from paper_1010_0762_amd.solver import ILUT, Batch, Solver
    from paper_1010_0762_amd._lib import RBiCGError
    with pytest.raises(RBiCGError, match="pivot"):
        ILUT(sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]])), 0.0)
    A = _mats_2d(20, 1)[0]
    P = ILUT(A, 0.05)
    S = Solver(_mats_2d(21, 1)[0], k=0, s=20)
    with pytest.raises(RBiCGError):
        S.attach_ilu(P)
    S.close()
    S = Solver(A, k=0, s=20, prec="mixed")
    with pytest.raises(RBiCGError):
        S.attach_ilu(P)
    S.close()
    B = Batch(max_slots=2)
    S = Solver(A, k=0, s=20, batch=B)
    with pytest.raises(RBiCGError):
        S.attach_ilu(P)
    S.close()
    B.close()
    P.close()


def _rowperm(A, seed):
    As = _csr(A) if hasattr(A, "rowptr") else sp.csr_matrix(A)
    rows = np.random.default_rng(seed).permutation(As.shape[0])
    return sp.csr_matrix(As[rows])


@pytest.mark.parametrize("kind", ["convdiff_rowperm", "random_complex_rowperm"])
def test_ilutp_transforms_match_oracle(kind):
    """ILUTP (column pivoting, permtol 1) on row-permuted operators whose
    diagonal is mostly zero: L^{-1} b, U^{-H} Q^T b~, Q U^{-1} y, L^{-H} y~
    element by element against the oracle's (n = 1600, 1500)."""
    from paper_1010_0762_amd.solver import ILUT
    if kind == "convdiff_rowperm":
        A = _rowperm(_mats_2d(40, 1)[0], 1)
    else:
        A = _rowperm(wl.random_sparse(1500, 6, 21, diag_shift=10.0, complex_vals=True), 2)
    n = A.shape[0]
    cplx = np.iscomplexobj(A.data)
    print("case ilutp", kind, n, flush=True)
    ss = pc.IlutpSystem(A, 0.05, permtol=1.0)
    P = ILUT(A, 0.05, permtol=1.0)
    info = P.info()
    assert info["moved"] == int((ss.perm != np.arange(n)).sum()) > n // 2
    rng = np.random.default_rng(4)
    b, bt, y, yt = (rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
                    for _ in range(4))
    bh, ch = P.rhs(_t(b), _t(bt))
    x, xt = P.solution(_t(y), _t(yt))
    refs = ss.rhs(b, bt) + ss.solution(y, yt)
    for got, ref in zip((bh, ch, x, xt), refs):
        ref = ref if cplx else ref.real
        assert np.abs(got.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert P.info()["wait_error"] == 0
    P.close()


def test_ilutp_sequence_matches_oracle():
    """Two row-permuted 2D convection-diffusion systems (n = 1600; ILUT
    without pivoting meets zero pivots on them) with ILUTP(0.2, permtol 1),
    k = 5, s = 10: solutions within 1e-6 of the oracle's, counts and carried
    dimensions inside the oracle's spread over its unperturbed run and three
    runs with b, b~ perturbed by 1e-13."""
    base = wl.ilut2d_sequence(nsys=2)
    mats = [_rowperm(A, 10 + j) for j, A in enumerate(base.mats)]
    with pytest.raises(ZeroDivisionError):
        pc.ilut(mats[0], 0.2)
    seq = wl.DualSequence("rowperm", mats, base.b, base.bt, 5, 10, 1e-8)
    runs = []
    for j in range(4):
        bp = seq.b if j == 0 else [_perturbed(v, 900 + 10 * j + i) for i, v in enumerate(seq.b)]
        _, res = pc.rbicg_ilut_sequence(mats, bp, seq.bt, 5, 10, 1e-8, 0.2, permtol=1.0)
        runs.append(res)
    ranges = [([r[i].iters for r in runs], [r[i].k_used for r in runs]) for i in range(2)]
    print("case ilutp sequence", ranges, flush=True)
    _run_sequence_p(seq, 0.2, 1.0, ranges)


def _run_sequence_p(seq, tau, permtol, ranges):
    from paper_1010_0762_amd.solver import solve_ilut_sequence
    ref_sols, ref = pc.rbicg_ilut_sequence(seq.mats, seq.b, seq.bt, seq.k, seq.s, seq.tol, tau,
                                           permtol=permtol)
    out = solve_ilut_sequence(seq.mats, [_t(b) for b in seq.b], [_t(b) for b in seq.bt],
                              droptol=tau, permtol=permtol, k=seq.k, s=seq.s, tol=seq.tol)
    print("iters gpu", [o[2]["iters"] for o in out], "oracle", [r.iters for r in ref], flush=True)
    for i, (A, (x, xt, st), (xr, xtr), b, bt) in enumerate(zip(seq.mats, out, ref_sols, seq.b, seq.bt)):
        its, ks = ranges[i]
        slack = max(2, int(np.ceil(0.05 * max(its))))
        assert st["status"] == 0 and st["relres"] <= seq.tol and st["relres_dual"] <= seq.tol
        assert min(its) - slack <= st["iters"] <= max(its) + slack, (i, st["iters"], its)
        assert min(ks) <= st["k_used"] <= max(ks), (i, st["k_used"], ks)
        xv, xtv = x.cpu().numpy(), xt.cpu().numpy()
        assert np.linalg.norm(xv - xr.real) <= 1e-6 * np.linalg.norm(xr)
        assert np.linalg.norm(xtv - xtr.real) <= 1e-6 * np.linalg.norm(xtr)
        assert np.linalg.norm(b - A @ xv) <= 1e-5 * np.linalg.norm(b)
        assert np.linalg.norm(bt - A.T @ xtv) <= 1e-5 * np.linalg.norm(bt)
