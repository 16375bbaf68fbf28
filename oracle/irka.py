"""IRKA (Algorithm 3) with direct sparse solves -- TEST INFRASTRUCTURE.

Only tests/, the package smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

The model is G(s) = c^H (s E - A)^{-1} b (eq. orginalModel, Sec. 5; E = I
when not given).  Algorithm 3: starting from shifts sigma_1..sigma_r, repeat
    V = [(sigma_i E - A)^{-1} b],  W = [(sigma_i E - A)^{-H} c],
    A_r = W^H A V,  E_r = W^H E V,
    sigma_i <- -lambda_i(A_r, E_r)
until the relative change of the shifts is below tol; the reduced model is
(E_r, A_r, b_r = W^H b, c_r = V^H c) with transfer function
G_r(s) = c_r^H (s E_r - A_r)^{-1} b_r.  Reading: step 4 of the printed
algorithm writes E_r = W_r^* A V_r; the pencil's second matrix is the
Petrov-Galerkin projection of E, W^H E V, which is what is used.

At a fixed point G_r Hermite-interpolates G at the shifts (the first-order
H2-optimality conditions quoted in Sec. 5), which the pins check.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import as_csr


def order_shifts(sig: np.ndarray) -> np.ndarray:
    """Canonical order: by real part, then imaginary part (rounded so that
    conjugate pairs computed with rounding stay adjacent)."""
    sig = np.asarray(sig, dtype=np.complex128)
    key = np.lexsort((np.round(sig.imag, 12), np.round(sig.real, 12)))
    return sig[key]


def _pencil(A, E, s):
    """s E - A as a complex CSC matrix (E = I when None)."""
    A = as_csr(A)
    n = A.shape[0]
    En = sp.identity(n, dtype=np.complex128, format="csr") if E is None else as_csr(E)
    return (s * En.astype(np.complex128) - A.astype(np.complex128)).tocsc()


def transfer(A, b, c, s, E=None) -> complex:
    """G(s) = c^H (s E - A)^{-1} b by a direct solve."""
    return complex(np.vdot(c, spla.spsolve(_pencil(A, E, s), b.astype(np.complex128))))


def transfer_reduced(Ar, Er, br, cr, s) -> complex:
    return complex(np.vdot(cr, np.linalg.solve(s * Er - Ar, br)))


def transfer_reduced_deriv(Ar, Er, br, cr, s) -> complex:
    """d/ds of c_r^H (s E_r - A_r)^{-1} b_r = -c_r^H M^{-1} E_r M^{-1} b_r."""
    M = s * Er - Ar
    return complex(-np.vdot(cr, np.linalg.solve(M, Er @ np.linalg.solve(M, br))))


def transfer_deriv(A, b, c, s, E=None) -> complex:
    """G'(s) = -c^H (s E - A)^{-1} E (s E - A)^{-1} b."""
    lu = spla.splu(_pencil(A, E, s))
    y = lu.solve(b.astype(np.complex128))
    if E is not None:
        y = as_csr(E) @ y
    return complex(-np.vdot(c, lu.solve(y)))


@dataclass
class IrkaResult:
    shifts: List[np.ndarray] = field(default_factory=list)   # shifts used at each step
    changes: List[float] = field(default_factory=list)
    steps: int = 0
    converged: bool = False
    Ar: np.ndarray = None
    Er: np.ndarray = None
    br: np.ndarray = None
    cr: np.ndarray = None


def irka(A, b, c, sigma0, tol=1e-6, maxit=50, E=None) -> IrkaResult:
    """Algorithm 3 (E = I when not given); every shifted pair by a direct
    sparse LU of sigma_i E - A."""
    A = as_csr(A).astype(np.complex128)
    n = A.shape[0]
    En = sp.identity(n, dtype=np.complex128, format="csr") if E is None else \
        as_csr(E).astype(np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128)
    sig = order_shifts(sigma0)
    res = IrkaResult()
    for step in range(maxit):
        V = np.empty((n, len(sig)), np.complex128)
        W = np.empty((n, len(sig)), np.complex128)
        for i, s in enumerate(sig):
            lu = spla.splu((s * En - A).tocsc())
            V[:, i] = lu.solve(b)
            W[:, i] = lu.solve(c, trans="H")
        Ar = W.conj().T @ (A @ V)
        Er = W.conj().T @ (En @ V)
        res.shifts.append(sig.copy())
        res.Ar, res.Er = Ar, Er
        res.br, res.cr = W.conj().T @ b, V.conj().T @ c
        res.steps = step + 1
        new = order_shifts(-sla.eigvals(Ar, Er))
        change = float(np.max(np.abs(new - sig) / np.abs(sig)))
        res.changes.append(change)
        sig = new
        if change < tol:
            res.converged = True
            break
    return res
