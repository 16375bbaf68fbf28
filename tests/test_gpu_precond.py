"""Split ILU(0) preconditioning in red-black ordering on the GPU
(rbicg_rbilu_*, solver.RBILU, solver.solve_split_sequence) against the
oracle (oracle/precond.py): the black block of the split-preconditioned
operator (products against dense), the right-hand-side and solution
transforms (element by element), a split-preconditioned sequence with
recycling (iteration counts and true residuals), the complex path, and the
refusal of patterns that are not two-colourable."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.precond import SplitSystem, rbicg_split_sequence
from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(v):
    return torch.as_tensor(np.ascontiguousarray(v), device="cuda")


def _csr(A):
    return sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n))


def test_rbilu_black_block_and_transforms_match_oracle():
    from paper_1010_0762_amd.solver import RBILU, Solver
    A = wl.convdiff(7, 3, [20.0, 10.0, 5.0])
    ss = SplitSystem(A)
    MB = ss.black_block().toarray().real
    P = RBILU(A)
    assert P.nb == A.n - ss.nr
    rng = np.random.default_rng(2)
    m = 3
    X, Xt = rng.standard_normal((m, P.nb)), rng.standard_normal((m, P.nb))
    S = Solver(P.black, k=0, s=40, prec="c128")   # rbicg_project takes complex bases
    G, _ = S.project(_t(X.astype(np.complex128)), _t(Xt.astype(np.complex128)))
    assert np.allclose(G, Xt @ MB @ X.T, rtol=1e-12, atol=1e-10 * np.abs(MB).max())
    b, bt = rng.standard_normal(A.n), rng.standard_normal(A.n)
    bB, cB = P.rhs(_t(b), _t(bt))
    bh, ch = ss.rhs(b, bt)
    assert np.allclose(bB.cpu().numpy(), bh[ss.nr:].real, rtol=1e-13, atol=1e-13)
    assert np.allclose(cB.cpu().numpy(), ch[ss.nr:].real, rtol=1e-13, atol=1e-13)
    yB, ytB = rng.standard_normal(P.nb), rng.standard_normal(P.nb)
    x, xt = P.solution(_t(b), _t(bt), _t(yB), _t(ytB))
    xr, xtr = ss.solution(np.concatenate([bh[:ss.nr], yB]), np.concatenate([ch[:ss.nr], ytB]))
    assert np.allclose(x.cpu().numpy(), xr.real, rtol=1e-12, atol=1e-12)
    assert np.allclose(xt.cpu().numpy(), xtr.real, rtol=1e-12, atol=1e-12)
    S.close()
    P.close()


def test_split_sequence_matches_oracle():
    from paper_1010_0762_amd.solver import solve_split_sequence
    N = 12
    mats = [wl.convdiff(N, 3, [20.0 * (1 + 0.02 * j), 10.0 * (1 + 0.02 * j), 5.0 * (1 + 0.02 * j)])
            for j in range(4)]
    rng = np.random.default_rng(9)
    b, bt = rng.standard_normal(N ** 3), rng.standard_normal(N ** 3)
    ref_sols, ref = rbicg_split_sequence(mats, [b] * 4, [bt] * 4, k=8, s=20, tol=1e-9)
    out = solve_split_sequence(mats, [_t(b)] * 4, [_t(bt)] * 4, k=8, s=20, tol=1e-9)
    print("iters gpu", [o[2]["iters"] for o in out], "oracle", [r.iters for r in ref], flush=True)
    for A, (x, xt, st), r in zip(mats, out, ref):
        As = _csr(A)
        assert st["status"] == 0
        assert abs(st["iters"] - r.iters) <= max(2, r.iters // 20)
        xv, xtv = x.cpu().numpy(), xt.cpu().numpy()
        assert np.linalg.norm(b - As @ xv) <= 1e-6 * np.linalg.norm(b)
        assert np.linalg.norm(bt - As.T @ xtv) <= 1e-6 * np.linalg.norm(bt)


def test_complex_rbilu_pair():
    from paper_1010_0762_amd.solver import RBILU, Solver
    rng = np.random.default_rng(6)
    A = wl.convdiff(6, 3, [20.0, 10.0, 5.0])
    As = _csr(A).astype(np.complex128)
    As = (As + 1j * sp.diags(rng.uniform(1.0, 5.0, A.n)) +
          1j * 0.3 * sp.csr_matrix((rng.uniform(-1, 1, A.nnz), A.colind, A.rowptr),
                                   shape=(A.n, A.n))).tocsr()
    b = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    bt = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    P = RBILU(As)
    S = Solver(P.black, k=0, s=40, prec="c128")
    bB, cB = P.rhs(_t(b), _t(bt))
    yB, ytB, st = S.solve(bB, cB, tol=1e-11)
    x, xt = P.solution(_t(b), _t(bt), yB, ytB)
    assert st["status"] == 0
    xv, xtv = x.cpu().numpy(), xt.cpu().numpy()
    assert np.linalg.norm(b - As @ xv) <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm(bt - As.conj().T @ xtv) <= 1e-8 * np.linalg.norm(bt)
    S.close()
    P.close()


def test_rbilu_refuses_odd_cycles():
    from paper_1010_0762_amd.solver import RBILU
    from paper_1010_0762_amd._lib import RBiCGError
    T = sp.csr_matrix(np.array([[4.0, 1, 1], [1, 4, 1], [1, 1, 4]]))
    with pytest.raises(RBiCGError):
        RBILU(T)


def test_refresh_matches_fresh_setup():
    """New values on the same pattern, recomputed on the device, against a
    fresh host set-up of the new matrix; another pattern is refused."""
    from paper_1010_0762_amd.solver import RBILU, Solver
    from paper_1010_0762_amd._lib import RBiCGError
    A0 = wl.convdiff(7, 3, [20.0, 10.0, 5.0])
    A1 = wl.convdiff(7, 3, [23.0, 9.0, 6.5])
    P = RBILU(A0)
    P.refresh(A1)
    Q = RBILU(A1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    m = 3
    X = (rng.standard_normal((m, P.nb)) + 0j).astype(np.complex128)
    Xt = (rng.standard_normal((m, P.nb)) + 0j).astype(np.complex128)
    SP = Solver(P.black, k=0, s=40, prec="c128")
    SQ = Solver(Q.black, k=0, s=40, prec="c128")
    GP, _ = SP.project(_t(X), _t(Xt))
    GQ, _ = SQ.project(_t(X), _t(Xt))
    assert np.allclose(GP, GQ, rtol=1e-13, atol=1e-12 * np.abs(GQ).max())
    b, bt = rng.standard_normal(A1.n), rng.standard_normal(A1.n)
    (u, v), (uq, vq) = P.rhs(_t(b), _t(bt)), Q.rhs(_t(b), _t(bt))
    assert np.allclose(u.cpu().numpy(), uq.cpu().numpy(), rtol=1e-13, atol=1e-13)
    assert np.allclose(v.cpu().numpy(), vq.cpu().numpy(), rtol=1e-13, atol=1e-13)
    yB, ytB = _t(rng.standard_normal(P.nb)), _t(rng.standard_normal(P.nb))
    xp, xtp = P.solution(_t(b), _t(bt), yB, ytB)
    xq, xtq = Q.solution(_t(b), _t(bt), yB, ytB)
    assert np.allclose(xp.cpu().numpy(), xq.cpu().numpy(), rtol=1e-13, atol=1e-13)
    assert np.allclose(xtp.cpu().numpy(), xtq.cpu().numpy(), rtol=1e-13, atol=1e-13)
    with pytest.raises(RBiCGError):
        P.refresh(wl.aniso_diffusion(6))
    # the values-only form gives the same block
    P2 = RBILU(A0)
    P2.refresh_values(_t(A1.vals))
    torch.cuda.synchronize()
    S2 = Solver(P2.black, k=0, s=40, prec="c128")
    G2, _ = S2.project(_t(X), _t(Xt))
    assert np.array_equal(G2, GP)
    for h in (SP, SQ, S2):
        h.close()
    for h in (P, Q, P2):
        h.close()
