"""Recycle-space computation of RBiCG (Sec. 4), oracle side, plain definitions.

Conventions (shared by every oracle module):
  * (a, b) = a^H b, conjugate in the first argument.
  * The paper's * is written ^H here.
  * C~^H C = I after biorthogonalization, so C^ = C~ and C-check = C.

Functions
  t_from_scalars      -- tridiagonal T_i from alpha, beta, ||r|| (Sec. 4.1).
  first_cycle_eigvecs -- right and left eigenvectors of T for the first cycle of
                         the first system (Sec. 4.2).
  harmonic_pencils    -- primal pencil of eq. finalGenEigValue, formed from the
                         explicit products A Phi and A^H Phi~ (eq. harmonic1),
                         and its dual mirror (reading: the dual derivation is
                         deferred by the paper to another work).
  select_eigvecs      -- the k eigenvalues closest to the origin; real problems
                         keep real bases by splitting conjugate pairs into
                         real and imaginary parts.
  biorthogonalize     -- C = A U, C~ = A^H U~, SVD of C~^H C, truncation, and
                         scaling to C~^H C = I (Sec. 4.3).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def t_from_scalars(alpha, beta, rnorm) -> np.ndarray:
    """Tridiagonal T_m of Sec. 4.1 from the iteration scalars.

    alpha[i-1] = alpha_i (i = 1..m), beta[i] = beta_i (i = 0..m-1, beta_0 = 0),
    rnorm[i] = ||r_i|| (i = 0..m-1).  Entries (1-based):
      T(i,i)   = 1/alpha_i + beta_{i-1}/alpha_{i-1}
      T(i+1,i) = -(||r_i|| / ||r_{i-1}||) / alpha_i
      T(i-1,i) = -(||r_{i-2}|| / ||r_{i-1}||) * beta_{i-1} / alpha_{i-1}
    """
    alpha = np.asarray(alpha)
    m = len(alpha)
    dt = np.result_type(alpha.dtype, np.asarray(beta).dtype, np.float64)
    T = np.zeros((m, m), dtype=dt)
    for i in range(1, m + 1):
        a_i = alpha[i - 1]
        T[i - 1, i - 1] = 1.0 / a_i
        if i >= 2:
            T[i - 1, i - 1] += beta[i - 1] / alpha[i - 2]
            T[i - 2, i - 1] = -(rnorm[i - 2] / rnorm[i - 1]) * beta[i - 1] / alpha[i - 2]
        if i <= m - 1:
            T[i, i - 1] = -(rnorm[i] / rnorm[i - 1]) / a_i
    return T


def _order(lam: np.ndarray) -> np.ndarray:
    """Indices of finite eigenvalues sorted by (|lambda|, Re, Im)."""
    finite = np.nonzero(np.isfinite(lam))[0]
    keys = [(abs(lam[i]), lam[i].real, lam[i].imag, i) for i in finite]
    keys.sort()
    return np.array([k[3] for k in keys], dtype=np.int64)


def select_eigvecs(lam: np.ndarray, W: np.ndarray, k: int, real_problem: bool,
                   Wl: np.ndarray | None = None):
    """Pick eigenvectors for the k eigenvalues closest to the origin.

    For a real problem a complex pair (lambda, conj lambda) contributes the two
    real vectors [Re w, Im w] (same span as [w, conj w]); if the k-th slot would
    split a pair, only k-1 vectors are taken.  Infinite or NaN eigenvalues are
    discarded.  ``Wl`` (optional) holds matching left eigenvectors that are
    selected and split the same way.  Returns (W_sel, Wl_sel, lam_sel).
    """
    order = _order(lam)
    cols, lcols, lams = [], [], []
    if not real_problem:
        for i in order[:k]:
            cols.append(W[:, i]); lams.append(lam[i])
            if Wl is not None:
                lcols.append(Wl[:, i])
    else:
        scale = max(1.0, float(np.max(np.abs(lam[np.isfinite(lam)]), initial=1.0)))
        used = np.zeros(len(lam), dtype=bool)
        for i in order:
            if len(cols) >= k:
                break
            if used[i]:
                continue
            if abs(lam[i].imag) <= 1e-12 * max(abs(lam[i]), 1e-300) or lam[i].imag == 0.0:
                used[i] = True
                cols.append(np.real(W[:, i])); lams.append(lam[i].real)
                if Wl is not None:
                    lcols.append(np.real(Wl[:, i]))
                continue
            # complex: find its conjugate partner
            cand = [j for j in order if not used[j] and j != i]
            if not cand:
                break
            j = min(cand, key=lambda t: abs(lam[t] - np.conj(lam[i])))
            if abs(lam[j] - np.conj(lam[i])) > 1e-8 * scale:
                # unpaired complex value of a real pencil: treat alone
                used[i] = True
                cols.append(np.real(W[:, i])); lams.append(lam[i])
                if Wl is not None:
                    lcols.append(np.real(Wl[:, i]))
                continue
            if len(cols) + 2 > k:
                break
            used[i] = used[j] = True
            ip = i if lam[i].imag > 0 else j
            cols.append(np.real(W[:, ip])); cols.append(np.imag(W[:, ip]))
            lams.extend([lam[ip], np.conj(lam[ip])])
            if Wl is not None:
                lcols.append(np.real(Wl[:, ip])); lcols.append(np.imag(Wl[:, ip]))
    if not cols:
        m = W.shape[0]
        dt = np.float64 if real_problem else W.dtype
        return np.zeros((m, 0), dt), (np.zeros((m, 0), dt) if Wl is not None else None), np.zeros(0)
    Ws = np.stack(cols, axis=1)
    Wls = np.stack(lcols, axis=1) if Wl is not None else None
    return Ws, Wls, np.asarray(lams)


def first_cycle_eigvecs(T: np.ndarray, k: int, real_problem: bool):
    """Right eigenvectors W and left eigenvectors W~ of T (T~ = T^H, so the
    left eigenvectors of T are the eigenvectors of T~) for the k eigenvalues
    of T closest to the origin (Sec. 4.2, first cycle of the first system)."""
    lam, vl, vr = sla.eig(T, left=True, right=True)
    W, Wt, lam_sel = select_eigvecs(lam, vr, k, real_problem, Wl=vl)
    return W, Wt, lam_sel


def harmonic_pencils(A, AH, Phi: np.ndarray, Phit: np.ndarray):
    """Matrices of the two harmonic Ritz problems.

    Primal (eq. harmonic1 / finalGenEigValue): (A u - lambda u) orthogonal to
    range(A^H Phi~), u = Phi w:
        (A^H Phi~)^H (A Phi) w = lambda (A^H Phi~)^H Phi w.
    Dual (reading, mirror image): (A^H u~ - mu u~) orthogonal to range(A Phi),
    u~ = Phi~ w~:
        (A Phi)^H (A^H Phi~) w~ = mu (A Phi)^H Phi~ w~.
    A Phi and A^H Phi~ are formed by explicit sparse products.
    Returns (P, Q, Pt, Qt)."""
    APhi = A @ Phi
    AHPhit = AH @ Phit
    P = AHPhit.conj().T @ APhi
    Q = AHPhit.conj().T @ Phi
    Pt = APhi.conj().T @ AHPhit
    Qt = APhi.conj().T @ Phit
    return P, Q, Pt, Qt


def pencil_eigvecs(P: np.ndarray, Q: np.ndarray, k: int, real_problem: bool):
    """Right and left generalized eigenvectors of P w = lambda Q w for the k
    finite eigenvalues closest to the origin (QZ via scipy.linalg.eig).

    The dual harmonic problem (A Phi)^H (A^H Phi~) w~ = mu (A Phi)^H Phi~ w~ is
    the pencil (P^H, Q^H), whose eigenvectors are the left eigenvectors of
    (P, Q) with mu = conj(lambda).  Taking them from the same decomposition
    pairs each right vector with the left vector of the same eigenvalue, as in
    the first cycle, instead of ranking the two spectra separately.
    Returns (W, W~, lambda_selected)."""
    lam, vl, vr = sla.eig(P, Q, left=True, right=True)
    Ws, Wls, lam_sel = select_eigvecs(lam, vr, k, real_problem, Wl=vl)
    return Ws, Wls, lam_sel


def biorthogonalize(A, AH, U: np.ndarray, Ut: np.ndarray, svd_tol: float = 1e-2):
    """Bi-orthogonal C, C~ (Sec. 4.3, eqs. equationSVD and equationForUC).

    The paper takes the SVD of C~^H C and keeps the singular values above a
    tolerance, leaving the scaling of the bases open.  Reading: the SVD is taken
    with orthonormal bases of range(C) and range(C~), so the singular values are
    the cosines of the principal angles between the two spaces and the
    tolerance is scale free:
        C = A U = Q R,  C~ = A^H U~ = Q~ R~       (thin Householder QR)
        Q~^H Q = M Sigma N^H,  p = #{sigma_i >= svd_tol}
        U  <- U R^{-1} N_p Sigma_p^{-1/2},   U~ <- U~ R~^{-1} M_p Sigma_p^{-1/2}
        C = A U,  C~ = A^H U~                 so that C~^H C = I_p.
    (The paper keeps Sigma_p on the diagonal of C~^H C instead; the spans are
    the same.)  Returns (U, Ut, C, Ct); C, Ct are None when p = 0."""
    if U is None or U.shape[1] == 0:
        return U, Ut, None, None
    TU, TUt = biorth_transforms(A, AH, U, Ut, svd_tol)
    if TU.shape[1] == 0:
        return U[:, :0], Ut[:, :0], None, None
    U = U @ TU
    Ut = Ut @ TUt
    C = A @ U
    Ct = AH @ Ut
    return U, Ut, C, Ct


def biorth_transforms(A, AH, U: np.ndarray, Ut: np.ndarray, svd_tol: float = 1e-2):
    """The transforms of ``biorthogonalize``: (TU, TU~) with
    U <- U TU, U~ <- U~ TU~ (m x p each; p = 0 when nothing is kept)."""
    C = A @ U
    Ct = AH @ Ut
    Q, R = np.linalg.qr(C)
    Qt, Rt = np.linalg.qr(Ct)
    M, sig, NH = np.linalg.svd(Qt.conj().T @ Q)
    p = int(np.sum(sig >= svd_tol))
    m = U.shape[1]
    if p == 0 or not np.all(np.isfinite(sig)):
        return np.zeros((m, 0), U.dtype), np.zeros((m, 0), Ut.dtype)
    s_inv_half = 1.0 / np.sqrt(sig[:p])
    TU = sla.solve_triangular(R, NH.conj().T[:, :p]) * s_inv_half
    TUt = sla.solve_triangular(Rt, M[:, :p]) * s_inv_half
    return TU, TUt
