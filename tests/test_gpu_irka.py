"""GPU IRKA (paper_1010_0762_amd/irka.py over rbicg_solve_shifted and
rbicg_project) against the oracle's IRKA with direct solves
(oracle/irka.py), Algorithm 3 with E = I on the anisotropic operator.

Bars: rbicg_project equals the dense products to rounding; IRKA converges in
the oracle's number of steps (+-1), to the oracle's shifts within 2e-6
relative (twice the IRKA tolerance: the stopping test of Algorithm 3 bounds
the last step's relative shift change by the tolerance, and two runs whose
shifted solves round differently may stop one step apart, each within about
the tolerance of the fixed point), and the GPU's reduced model Hermite-interpolates
the full model (evaluated by direct solves on the CPU) at its final shifts to
1e-7 (the shifted solves run to 1e-10)."""
import numpy as np
import pytest

import oracle
from oracle.irka import transfer, transfer_deriv, transfer_reduced, transfer_reduced_deriv
from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    return abs(a - b) / abs(b)


def test_project_matches_dense():
    from paper_1010_0762_amd.solver import Solver
    A = wl.aniso_diffusion(7)
    n = A.n
    rng = np.random.default_rng(11)
    m = 5
    X = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Xt = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    S = Solver(A, k=4, s=40, prec="c128")
    t = lambda v: torch.as_tensor(np.ascontiguousarray(v), device="cuda")
    Ar, Er, br, cr = S.project(t(X), t(Xt), t(b), t(c))
    D = A.to_dense()
    V, W = X.T, Xt.T
    assert np.allclose(Ar, W.conj().T @ D @ V, rtol=1e-12, atol=1e-9)
    assert np.allclose(Er, W.conj().T @ V, rtol=1e-12, atol=1e-12)
    assert np.allclose(br, W.conj().T @ b, rtol=1e-12, atol=1e-12)
    assert np.allclose(cr, V.conj().T @ c, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,r,k,per_shift", [(10, 6, 10, False), (12, 8, 20, False),
                                             (10, 6, 10, True)])
def test_irka_matches_oracle(N, r, k, per_shift):
    from paper_1010_0762_amd.solver import DeviceMatrix, Solver
    from paper_1010_0762_amd.irka import irka
    A, b, c, s0 = wl.irka_problem(N=N, r=r)
    ref = oracle.irka.irka(A, b, c, s0, tol=1e-6, maxit=40)
    if per_shift:
        M = DeviceMatrix(A)
        S = [Solver(M, k=k, s=40, prec="c128", stream=torch.cuda.Stream()) for _ in range(r)]
    else:
        S = Solver(A, k=k, s=40, prec="c128")
    t = lambda v: torch.as_tensor(np.ascontiguousarray(v.astype(np.complex128)), device="cuda")
    run = irka(S, t(b), t(c), s0, tol=1e-6, maxit=40, solve_tol=1e-10)
    print("steps gpu", run.steps, "oracle", ref.steps, "iters", run.iters, flush=True)
    assert ref.converged and run.converged and run.all_solved
    assert abs(run.steps - ref.steps) <= 1
    sg, so = run.shifts[-1], ref.shifts[-1]
    assert np.max(np.abs(sg - so) / np.abs(so)) <= 2e-6
    for s in sg:
        assert _rel(transfer_reduced(run.Ar, run.Er, run.br, run.cr, s), transfer(A, b, c, s)) <= 1e-7
        assert _rel(transfer_reduced_deriv(run.Ar, run.Er, run.br, run.cr, s),
                    transfer_deriv(A, b, c, s)) <= 1e-6


# ---------------------------------------------------------------- E != I

def test_pencil_matches_dense():
    """rbicg_matrix_pencil: alpha E + beta A and its conjugate transpose,
    created and then rewritten in place, against dense products and direct
    solves; a pattern mismatch is refused."""
    import scipy.sparse as sp
    from paper_1010_0762_amd.solver import DeviceMatrix, Solver
    from paper_1010_0762_amd._lib import RBiCGError
    A, E = wl.aniso_diffusion(5), wl.mass_like(5)
    n = A.n
    Ad, Ed = A.to_dense(), E.to_dense()
    MA, ME = DeviceMatrix(A), DeviceMatrix(E)
    rng = np.random.default_rng(21)
    m = 4
    X = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Xt = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    t = lambda v: torch.as_tensor(np.ascontiguousarray(v), device="cuda")
    P = None
    for alpha, beta in [(30.0 + 5.0j, -1.0), (2.0 - 7.0j, 0.5 + 0.25j)]:
        P = DeviceMatrix.pencil(MA, ME, alpha, beta, out=P)
        torch.cuda.synchronize()
        Pd = alpha * Ed + beta * Ad
        S = Solver(P, k=0, s=40, prec="c128")
        Pr, _ = S.project(t(X), t(Xt))
        assert np.allclose(Pr, Xt.conj() @ Pd @ X.T, rtol=1e-12, atol=1e-9)
        x, xt, st = S.solve(t(b), t(c), tol=1e-11)
        assert st["status"] == 0
        xr = np.linalg.solve(Pd, b)
        xtr = np.linalg.solve(Pd.conj().T, c)
        assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-8 * np.linalg.norm(xr)
        assert np.linalg.norm(xt.cpu().numpy() - xtr) <= 1e-8 * np.linalg.norm(xtr)
        S.close()
    D = wl.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    MD = DeviceMatrix(D)
    with pytest.raises(RBiCGError):
        DeviceMatrix.pencil(MA, MD, 1.0)
    for mm in (P, MD, ME, MA):
        mm.close()


@pytest.mark.parametrize("recycle", ["per_shift", "pool", "none"])
def test_irka_pencil_matches_oracle(recycle):
    from paper_1010_0762_amd.solver import DeviceMatrix
    from paper_1010_0762_amd.irka import irka_pencil
    A, E, b, c, s0 = wl.irka_problem_e(N=8, r=4)
    ref = oracle.irka.irka(A, b, c, s0, tol=1e-6, maxit=60, E=E)
    MA, ME = DeviceMatrix(A), DeviceMatrix(E)
    t = lambda v: torch.as_tensor(np.ascontiguousarray(v.astype(np.complex128)), device="cuda")
    run = irka_pencil(MA, ME, t(b), t(c), s0, k=10, s=40, tol=1e-6, maxit=60, solve_tol=1e-10,
                      recycle=recycle)
    print("steps gpu", run.steps, "oracle", ref.steps, "iters", run.iters[-1], flush=True)
    assert ref.converged and run.converged and run.all_solved
    assert abs(run.steps - ref.steps) <= 1
    sg, so = run.shifts[-1], ref.shifts[-1]
    assert np.max(np.abs(sg - so) / np.abs(so)) <= 2e-6
    for s in sg:
        assert _rel(transfer_reduced(run.Ar, run.Er, run.br, run.cr, s),
                    transfer(A, b, c, s, E=E)) <= 1e-7
        assert _rel(transfer_reduced_deriv(run.Ar, run.Er, run.br, run.cr, s),
                    transfer_deriv(A, b, c, s, E=E)) <= 1e-6
    MA.close()
    ME.close()
