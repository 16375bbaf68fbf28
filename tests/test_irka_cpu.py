"""Pins of the oracle's IRKA (Algorithm 3, E = I; oracle/irka.py) against what
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
