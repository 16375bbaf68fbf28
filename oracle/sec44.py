"""Set-up of the harmonic Ritz pencil by the recurrences of Sec. 4.4, oracle side.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The pencil of eq. finalGenEigValue is
    (H~_j^H Psi~_j^H Psi_j H_j) w = lambda (H~_j^H Psi~_j^H Phi_j) w,
with (Sec. 4.1, eq. firstKW)
    Phi_j = [U_{j-1}, V_j],  Psi_j = [C, C_{j-1}, Upsilon_j],
    H_j = [[0, B_j], [I, 0], [0, Gamma_j]],  B_j = C^^H A V_j,
and the dual analogues (~).  ``recycle.harmonic_pencils`` forms it from the
explicit products A Phi and A^H Phi~ (the plain definition).  Sec. 4.4 instead
assembles Psi~_j^H Psi_j and Psi~_j^H Phi_j from blocks carried over from the
previous cycle, using the biorthogonality of the Lanczos vectors, C~^H r = 0,
C^H r~ = 0 and the construction of C_{j-1}; the only O(n) product left is
Upsilon~_j^H U_{j-1}.  B_j comes from the restrictions zeta_i = C~^H z_i of the
iteration: A r_{i-1} = z_i - beta_{i-1} z_{i-1}.

Conventions: C~^H C = I after biorthogonalization (so C^ = C~, C-check = C,
D_c = I, Sigma_{j-1} = I); U_{j-1} = Phi_{j-1} (W N)_{j-1} and
U~_{j-1} = Phi~_{j-1} (W~ M)_{j-1}, where (W N) and (W~ M) are the products of
the eigenvector selection and of the biorthogonalizing transform.

Cases (Sec. 4.2):
  * first cycle of the first system: eigenvectors of T_1 (not handled here);
  * first cycle of a later system: Phi_1 = [U, V_1], Psi_1 = [C, V_1 underbar]
    with V_1 underbar = [V_1, v_{s+1}], H_1 = [[I, B_1], [0, T_1 underbar]];
    Psi~_1^H Psi_1 = blockdiag(D_c, I) and Psi~_1^H Phi_1 needs C~^H U and
    V~_1 underbar^H U;
  * every later cycle of the same Lanczos process (the general form; without
    a system recycle space the C rows and columns are absent).

Readings (the passage is terse or garbled here):
  * Gamma_j's extra top row holds the coefficient of v_{(j-1)s} in
    A v_{(j-1)s+1} (zero in the first cycle of a Lanczos run); Gamma~_j is
    built from T~ = T^H (Sec. 4.1 scaling), entry (l, i) = conj(T(i, l)).
  * V~_{j-1}^H A V_{j-1} in the block C~_{j-1}^H U_{j-1} is T_{j-1} (the middle
    rows of Gamma_{j-1}); the printed T~_{j-1} is read as this product.
  * Upsilon~_{j-1}^H Upsilon_j has ones at (s, 0) and (s+1, 1) (the shared
    vectors v_{(j-1)s}, v_{(j-1)s+1}); its transpose gives Upsilon~_j^H
    Upsilon_{j-1}.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def t_entries(alpha, beta_prev, rnorm, rn_end, beta_end, alpha_before=None,
              rnorm_before=None):
    """Entries of the Lanczos tridiagonal for one cycle of s iterations
    i = i0 .. i0+s-1 (Sec. 4.1):
      alpha[c] = alpha_i, beta_prev[c] = beta_{i-1}, rnorm[c] = ||r_{i-1}||,
      rn_end = ||r_{i0+s-1}||, beta_end = beta_{i0+s-1},
      alpha_before = alpha_{i0-1}, rnorm_before = ||r_{i0-2}|| (previous
      cycle of the same run; None in the first cycle of a run).
    Returns (diag, sub, sup) of length s with
      diag[c] = T(i, i), sub[c] = T(i+1, i), sup[c] = T(i-1, i),
    and (sub_before, sup_end) = (T(i0, i0-1), T(i0+s-1, i0+s))."""
    alpha = np.asarray(alpha)
    s = len(alpha)
    dt = np.result_type(alpha.dtype, np.asarray(beta_prev).dtype, np.float64)
    diag = np.zeros(s, dt)
    sub = np.zeros(s, dt)
    sup = np.zeros(s, dt)

    def alpha_m1(c):
        return alpha[c - 1] if c >= 1 else alpha_before

    def rn_m2(c):
        return rnorm[c - 1] if c >= 1 else rnorm_before

    for c in range(s):
        diag[c] = 1.0 / alpha[c]
        if beta_prev[c] != 0:
            diag[c] += beta_prev[c] / alpha_m1(c)
            sup[c] = -(rn_m2(c) / rnorm[c]) * beta_prev[c] / alpha_m1(c)
        rn_next = rnorm[c + 1] if c + 1 < s else rn_end
        sub[c] = -(rn_next / rnorm[c]) / alpha[c]
    sub_before = 0.0
    if alpha_before is not None:
        sub_before = -(rnorm[0] / rnorm_before) / alpha_before
    sup_end = -(rnorm[s - 1] / rn_end) * beta_end / alpha[s - 1]
    return diag, sub, sup, sub_before, sup_end


def gamma_blocks(alpha, beta_prev, rnorm, rn_end, beta_end, alpha_before=None,
                 rnorm_before=None):
    """Gamma_j and Gamma~_j ((s+2) x s, eq. augBiLanExtend): rows are the
    coefficients of v_{(j-1)s}, V_j, v_{js+1} (and of the dual vectors)."""
    diag, sub, sup, sub_before, sup_end = t_entries(alpha, beta_prev, rnorm, rn_end, beta_end,
                                                    alpha_before, rnorm_before)
    s = len(diag)
    G = np.zeros((s + 2, s), dtype=np.result_type(diag.dtype, np.complex128)
                 if np.iscomplexobj(diag) else diag.dtype)
    Gt = np.zeros_like(G)
    for c in range(s):
        G[c, c] = sup[c]
        G[c + 1, c] = diag[c]
        G[c + 2, c] = sub[c]
        # dual column c: conj(T(i, i-1)), conj(T(i, i)), conj(T(i, i+1))
        t_i_im1 = sub[c - 1] if c >= 1 else sub_before
        t_i_ip1 = sup[c + 1] if c + 1 < s else sup_end
        Gt[c, c] = np.conj(t_i_im1)
        Gt[c + 1, c] = np.conj(diag[c])
        Gt[c + 2, c] = np.conj(t_i_ip1)
    return G, Gt


def b_blocks(zeta, zetat, zeta_before, zetat_before, beta_prev, vscale, vtscale):
    """B_j = C^^H A V_j and B~_j = C-check^H A^H V~_j (k x s) from the
    iteration's restrictions: zeta[c] = C~^H z_i, zetat[c] = C^H z~_i,
    zeta_before = zeta_{i0-1} (ignored when beta_prev[0] = 0); v_i = vscale[c]
    r_{i-1}, v~_i = vtscale[c] r~_{i-1}; A r_{i-1} = z_i - beta_{i-1} z_{i-1},
    A^H r~_{i-1} = z~_i - conj(beta_{i-1}) z~_{i-1}."""
    zeta = np.asarray(zeta)
    zetat = np.asarray(zetat)
    s = len(beta_prev)
    k = zeta.shape[1] if zeta.ndim == 2 else 0
    B = np.zeros((k, s), np.result_type(zeta.dtype, np.asarray(beta_prev).dtype))
    Bt = np.zeros((k, s), B.dtype)
    for c in range(s):
        prev = zeta[c - 1] if c >= 1 else zeta_before
        prevt = zetat[c - 1] if c >= 1 else zetat_before
        d = zeta[c] - (beta_prev[c] * prev if beta_prev[c] != 0 else 0)
        dt_ = zetat[c] - (np.conj(beta_prev[c]) * prevt if beta_prev[c] != 0 else 0)
        B[:, c] = d * vscale[c]
        Bt[:, c] = dt_ * vtscale[c]
    return B, Bt


def _e(s):
    """Upsilon~_{j-1}^H Upsilon_j ((s+2) x (s+2))."""
    E = np.zeros((s + 2, s + 2))
    E[s, 0] = 1.0
    E[s + 1, 1] = 1.0
    return E


@dataclass
class Blocks:
    """Blocks of Psi~_j^H Psi_j and Psi~_j^H Phi_j that do not need the cycle j
    data, carried from the end of cycle j-1 (kC = dim C, kp = dim U_{j-1}):
      XCC  = C~^H C_{j-1}          (kC x kp)
      XCtC = C~_{j-1}^H C          (kp x kC)
      XCtY = C~_{j-1}^H Upsilon_j  (kp x (s+2))
      XYtC = Upsilon~_j^H C_{j-1}  ((s+2) x kp)
      XCU  = C~^H U_{j-1}          (kC x kp)
      XCtU = C~_{j-1}^H U_{j-1}    (kp x kp)
    """
    XCC: np.ndarray
    XCtC: np.ndarray
    XCtY: np.ndarray
    XYtC: np.ndarray
    XCU: np.ndarray
    XCtU: np.ndarray


def system_start_blocks(CtU: np.ndarray, s: int) -> Blocks:
    """The carried blocks at the start of a later system, reading U_0 = U,
    C_0 = C (used only by the recurrences after the first cycle, whose own
    pencil has the reduced form of Sec. 4.2): C~^H C = D_c = I,
    C~^H Upsilon_1 = 0 (r_0 is projected), C~^H U."""
    k = CtU.shape[0]
    dt = CtU.dtype
    return Blocks(np.eye(k, dtype=dt), np.eye(k, dtype=dt), np.zeros((k, s + 2), dt),
                  np.zeros((s + 2, k), dt), CtU, CtU)


def empty_blocks(s: int, dt) -> Blocks:
    """No recycle space before the cycle (first cycle of the first system)."""
    z = lambda a, b: np.zeros((a, b), dt)
    return Blocks(z(0, 0), z(0, 0), z(0, s + 2), z(s + 2, 0), z(0, 0), z(0, 0))


def pencil_general(X: Blocks, YtU, B, Bt, G, Gt):
    """(P, Q) of eq. finalGenEigValue for Phi_j = [U_{j-1}, V_j],
    Psi_j = [C, C_{j-1}, Upsilon_j] from the carried blocks X, the explicit
    YtU = Upsilon~_j^H U_{j-1}, B_j, B~_j, Gamma_j, Gamma~_j."""
    kC, kp = X.XCU.shape
    s = G.shape[1]
    dt = np.result_type(X.XCtU.dtype, YtU.dtype, B.dtype, G.dtype, Gt.dtype)
    m1 = kC + kp + s + 2
    G1 = np.zeros((m1, m1), dt)
    G1[:kC, :kC] = np.eye(kC)
    G1[:kC, kC:kC + kp] = X.XCC
    G1[kC:kC + kp, :kC] = X.XCtC
    G1[kC:kC + kp, kC:kC + kp] = np.eye(kp)
    G1[kC:kC + kp, kC + kp:] = X.XCtY
    G1[kC + kp:, kC:kC + kp] = X.XYtC
    G1[kC + kp:, kC + kp:] = np.eye(s + 2)
    G2 = np.zeros((m1, kp + s), dt)
    G2[:kC, :kp] = X.XCU
    G2[kC:kC + kp, :kp] = X.XCtU
    G2[kC:kC + kp, kp:] = X.XCtY[:, 1:s + 1]
    G2[kC + kp:, :kp] = YtU
    G2[kC + kp + 1:kC + kp + 1 + s, kp:] = np.eye(s)
    H = np.zeros((m1, kp + s), dt)
    Ht = np.zeros((m1, kp + s), dt)
    H[:kC, kp:] = B
    Ht[:kC, kp:] = Bt
    H[kC:kC + kp, :kp] = np.eye(kp)
    Ht[kC:kC + kp, :kp] = np.eye(kp)
    H[kC + kp:, kp:] = G
    Ht[kC + kp:, kp:] = Gt
    P = Ht.conj().T @ G1 @ H
    Q = Ht.conj().T @ G2
    return P, Q


def pencil_first_cycle(CtU, VtU, B, Bt, G, Gt):
    """(P, Q) for the first cycle of a later system (Sec. 4.2): Phi_1 =
    [U, V_1], Psi_1 = [C, V_1 underbar], H_1 = [[I, B_1], [0, T_1 underbar]];
    CtU = C~^H U, VtU = V~_1 underbar^H U ((s+1) x k)."""
    k = CtU.shape[0]
    s = G.shape[1]
    dt = np.result_type(CtU.dtype, VtU.dtype, B.dtype, G.dtype, Gt.dtype)
    m1 = k + s + 1
    G2 = np.zeros((m1, k + s), dt)
    G2[:k, :k] = CtU
    G2[k:, :k] = VtU
    G2[k:k + s, k:] = np.eye(s)
    H = np.zeros((m1, k + s), dt)
    Ht = np.zeros((m1, k + s), dt)
    H[:k, :k] = np.eye(k)
    Ht[:k, :k] = np.eye(k)
    H[:k, k:] = B
    Ht[:k, k:] = Bt
    H[k:, k:] = G[1:, :]
    Ht[k:, k:] = Gt[1:, :]
    # Psi~_1^H Psi_1 = blockdiag(D_c, I) = I
    P = Ht.conj().T @ H
    Q = Ht.conj().T @ G2
    return P, Q


def next_blocks(X: Blocks, WN, WtM, B, Bt, G, Gt) -> Blocks:
    """Carried blocks for cycle j+1 from those of cycle j (X), the cycle's
    Gamma_j, Gamma~_j, B_j, B~_j and U_j = Phi_j WN, U~_j = Phi~_j WtM
    (the recurrences of Sec. 4.4 with j-1 -> j)."""
    kC, kp = X.XCU.shape
    s = G.shape[1]
    E = _e(s)
    T = G[1:s + 1, :]
    WtMh = WtM.conj().T
    XCC = np.hstack([X.XCC, B]) @ WN
    XCtC = WtMh @ np.vstack([X.XCtC, Bt.conj().T])
    XCtY = WtMh @ np.vstack([np.zeros((kp, s + 2)), Gt.conj().T @ E])
    XYtC = np.hstack([np.zeros((s + 2, kp)), E.T @ G]) @ WN
    XCU = np.hstack([X.XCU, np.zeros((kC, s))]) @ WN
    M = np.block([[X.XCtU, X.XCtY[:, 1:s + 1]], [X.XYtC[1:s + 1, :], T]])
    XCtU = WtMh @ M @ WN
    return Blocks(XCC, XCtC, XCtY, XYtC, XCU, XCtU)
