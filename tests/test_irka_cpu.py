"""Pins of the oracle's IRKA (Algorithm 3; oracle/irka.py) against what
the interpolation theory of Sec. 5 fixes, independently of the algorithm's own
arithmetic:
  - Petrov-Galerkin projection with V = (sigma I - A)^{-1} b columns and
    W = (sigma I - A)^{-H} c columns makes G_r a Hermite interpolant of G at
    every shift used (G = G_r and G' = G_r' there);
  - at convergence the shifts are a fixed point: the mirror images of the
    reduced poles;
  - with r = n the reduced model is the full one (G_r = G everywhere)."""
import numpy as np
import pytest

import oracle
from oracle.irka import irka, order_shifts, transfer, transfer_deriv, transfer_reduced, transfer_reduced_deriv
from paper_1010_0762_amd import workloads as wl


def _rel(a, b):
    return abs(a - b) / abs(b)


@pytest.fixture(scope="module")
def run6():
    A, b, c, s0 = wl.irka_problem(N=6, r=4)
    return A, b, c, irka(A, b, c, s0, tol=1e-8, maxit=60)


def test_hermite_interpolation_at_shifts(run6):
    A, b, c, res = run6
    for s in res.shifts[-1]:
        g, gr = transfer(A, b, c, s), transfer_reduced(res.Ar, res.Er, res.br, res.cr, s)
        d, dr = transfer_deriv(A, b, c, s), transfer_reduced_deriv(res.Ar, res.Er, res.br, res.cr, s)
        assert _rel(gr, g) <= 1e-10
        assert _rel(dr, d) <= 1e-9
    # away from the shifts the reduced model is only an approximation
    s = 3.0 + 0.0j
    assert _rel(transfer_reduced(res.Ar, res.Er, res.br, res.cr, s), transfer(A, b, c, s)) > 1e-8


def test_fixed_point_at_convergence(run6):
    A, b, c, res = run6
    assert res.converged and res.changes[-1] < 1e-8
    import scipy.linalg as sla
    mirror = order_shifts(-sla.eigvals(res.Ar, res.Er))
    assert np.max(np.abs(mirror - res.shifts[-1]) / np.abs(res.shifts[-1])) <= 1e-7
    # symmetric negative definite A, nearly collocated b, c: positive real shifts
    assert np.all(res.shifts[-1].real > 0) and np.max(np.abs(res.shifts[-1].imag)) < 1e-6


def test_full_order_is_exact():
    A, b, c, _ = wl.irka_problem(N=2, r=8)   # n = 8 = r
    rng = np.random.default_rng(3)
    s0 = np.array([1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0], dtype=np.complex128)
    res = irka(A, b, c, s0, tol=1e-6, maxit=1)
    for s in rng.uniform(0.5, 300.0, 5) + 1j * rng.uniform(-10.0, 10.0, 5):
        assert _rel(transfer_reduced(res.Ar, res.Er, res.br, res.cr, s), transfer(A, b, c, s)) <= 1e-9


def test_order_keeps_conjugate_pairs_adjacent():
    s = order_shifts([2 - 1j, 5, 2 + 1j + 1e-14, 1])
    assert s[0] == 1 and s[3] == 5
    assert abs(s[1] - np.conj(s[2])) < 1e-12


def test_hermite_interpolation_at_complex_shifts():
    """One step from complex conjugate shifts (a missing conjugation in W^H or
    in the solves breaks the interpolation there)."""
    A, b, c, _ = wl.irka_problem(N=5, r=4)
    s0 = np.array([3 + 4j, 3 - 4j, 40 + 10j, 40 - 10j])
    res = irka(A, b, c, s0, tol=1e-6, maxit=1)
    for s in res.shifts[0]:
        assert _rel(transfer_reduced(res.Ar, res.Er, res.br, res.cr, s), transfer(A, b, c, s)) <= 1e-10
        assert _rel(transfer_reduced_deriv(res.Ar, res.Er, res.br, res.cr, s),
                    transfer_deriv(A, b, c, s)) <= 1e-9


# ---------------------------------------------------------------- E != I
# The model G(s) = c^H (s E - A)^{-1} b of Sec. 5 with an SPD E on A's
# pattern.  Derivatives are checked by central differences of G itself, so
# that the pins do not reuse the derivative formula.

def _fd(f, s, h):
    return (f(s + h) - f(s - h)) / (2 * h)


@pytest.fixture(scope="module")
def run6e():
    A, E, b, c, s0 = wl.irka_problem_e(N=6, r=4)
    return A, E, b, c, irka(A, b, c, s0, tol=1e-8, maxit=80, E=E)


def test_hermite_interpolation_with_e(run6e):
    A, E, b, c, res = run6e
    assert res.converged
    Ed = E.to_dense()
    for s in res.shifts[-1]:
        # G from a dense solve of (s E - A), G' by central differences
        g = np.vdot(c, np.linalg.solve(s * Ed - A.to_dense(), b))
        h = 1e-4 * abs(s)
        d = _fd(lambda z: transfer(A, b, c, z, E=E), s, h)
        assert _rel(transfer_reduced(res.Ar, res.Er, res.br, res.cr, s), g) <= 1e-10
        assert _rel(transfer_reduced_deriv(res.Ar, res.Er, res.br, res.cr, s), d) <= 1e-6
    # the E = I model is a different one: its interpolant misses G here
    s = res.shifts[-1][0]
    res_i = irka(A, b, c, res.shifts[-1], tol=1e-6, maxit=1)
    assert _rel(transfer_reduced(res_i.Ar, res_i.Er, res_i.br, res_i.cr, s),
                transfer(A, b, c, s, E=E)) > 1e-3


def test_diagonal_e_equals_rescaled_identity_model():
    """With E = D diagonal, (s D - A)^{-1} = D^{-1/2} (s I - A^)^{-1} D^{-1/2}
    for A^ = D^{-1/2} A D^{-1/2}: IRKA on (D, A, b, c) and on (I, A^,
    D^{-1/2} b, D^{-1/2} c) build the same reduced pencils and shifts."""
    import scipy.sparse as sp
    A, b, c, s0 = wl.irka_problem(N=5, r=4)
    rng = np.random.default_rng(5)
    d = rng.uniform(0.5, 2.0, A.n)
    As = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n))
    Dm = sp.diags(d).tocsr()
    Dh = sp.diags(1.0 / np.sqrt(d))
    r1 = irka(As, b, c, s0, tol=1e-9, maxit=60, E=Dm)
    r2 = irka((Dh @ As @ Dh).tocsr(), b / np.sqrt(d), c / np.sqrt(d), s0, tol=1e-9, maxit=60)
    assert r1.converged and r2.converged and r1.steps == r2.steps
    assert np.max(np.abs(r1.shifts[-1] - r2.shifts[-1]) / np.abs(r2.shifts[-1])) <= 1e-8
    for s in (2.0 + 1j, 30.0):
        assert _rel(transfer_reduced(r1.Ar, r1.Er, r1.br, r1.cr, s),
                    transfer_reduced(r2.Ar, r2.Er, r2.br, r2.cr, s)) <= 1e-9


def test_full_order_is_exact_with_e():
    A = wl.aniso_diffusion(2)
    E = wl.mass_like(2)
    rng = np.random.default_rng(7)
    b, c = rng.standard_normal(8), rng.standard_normal(8)
    s0 = np.array([1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0], dtype=np.complex128)
    res = irka(A, b, c, s0, tol=1e-6, maxit=1, E=E)
    Ad, Ed = A.to_dense(), E.to_dense()
    for s in rng.uniform(0.5, 300.0, 5) + 1j * rng.uniform(-10.0, 10.0, 5):
        g = np.vdot(c, np.linalg.solve(s * Ed - Ad, b))
        assert _rel(transfer_reduced(res.Ar, res.Er, res.br, res.cr, s), g) <= 1e-9


def test_transfer_deriv_with_e_matches_differences():
    A, E, b, c, _ = wl.irka_problem_e(N=4, r=2)
    for s in (3.0 + 2.0j, 150.0 + 0.0j):
        h = 1e-4 * abs(s)
        assert _rel(transfer_deriv(A, b, c, s, E=E),
                    _fd(lambda z: transfer(A, b, c, z, E=E), s, h)) <= 1e-6
