// Host set-up of the harmonic Ritz pencil by the recurrences of Sec. 4.4
// (efficient set-up of the generalized eigenvalue problem).  Small dense
// complex matrices only; the one O(n) input, Upsilon~_j^H U_{j-1} (or, in the
// first cycle of a later system, V~_1 underbar^H U and C~^H U), comes from a
// device Gram.
//
// Notation (Sec. 4.1): Phi_j = [U_{j-1}, V_j], Psi_j = [C, C_{j-1}, Upsilon_j],
// H_j = [[0, B_j], [I, 0], [0, Gamma_j]], and the dual analogues; the pencil
// is P = H~^H (Psi~^H Psi) H, Q = H~^H (Psi~^H Phi) (eq. finalGenEigValue).
// C~^H C = I after every biorthogonalization, so D_c = I and Sigma_{j-1} = I.
#pragma once
#include <complex>
#include <vector>

namespace sec44 {

using cplx = std::complex<double>;

// Column-major dense matrix.
struct Mat {
  int r = 0, c = 0;
  std::vector<cplx> a;
  Mat() = default;
  Mat(int rr, int cc) : r(rr), c(cc), a((size_t)rr * cc, cplx(0.0)) {}
  cplx &operator()(int i, int j) { return a[(size_t)i + (size_t)j * r]; }
  cplx operator()(int i, int j) const { return a[(size_t)i + (size_t)j * r]; }
};

Mat mul(const Mat &A, const Mat &B);    // A B
Mat mul_h(const Mat &A, const Mat &B);  // A^H B
Mat eye(int n);

// Scalars of one cycle of s iterations i = i0 .. i0+s-1 (Sec. 4.1):
//   alpha[c] = alpha_i, beta[c] = beta_{i-1}, rn[c] = ||r_{i-1}||,
//   rn_end = ||r_{i0+s-1}||, beta_end = beta_{i0+s-1};
//   first = 1 in the first cycle of a Lanczos run (no v_{i0-1}), else
//   alpha_before = alpha_{i0-1}, rn_before = ||r_{i0-2}||.
struct CycleScalars {
  int s = 0;
  std::vector<cplx> alpha, beta;
  std::vector<double> rn;
  double rn_end = 0.0;
  cplx beta_end = 0.0;
  bool first = true;
  cplx alpha_before = 0.0;
  double rn_before = 0.0;
};

// Gamma_j and Gamma~_j ((s+2) x s): coefficients of v_{i0-1}, V_j, v_{i0+s}
// in (I - C C~^H) A V_j, and of the dual vectors in (I - C~ C^H) A^H V~_j,
// with T~ = T^H (entry (l, i) of Gamma~ is conj(T(i, l))).
void gamma_blocks(const CycleScalars &cs, Mat &G, Mat &Gt);

// Blocks of Psi~_j^H Psi_j and Psi~_j^H Phi_j carried from the end of cycle
// j-1 (kC = dim C, kp = dim U_{j-1}).
struct Blocks {
  Mat XCC;   // C~^H C_{j-1}          kC x kp
  Mat XCtC;  // C~_{j-1}^H C          kp x kC
  Mat XCtY;  // C~_{j-1}^H Upsilon_j  kp x (s+2)
  Mat XYtC;  // Upsilon~_j^H C_{j-1}  (s+2) x kp
  Mat XCU;   // C~^H U_{j-1}          kC x kp
  Mat XCtU;  // C~_{j-1}^H U_{j-1}    kp x kp
};

// Before the first cycle of the first system (nothing recycled yet).
Blocks empty_blocks(int s);
// At the start of a later system, reading U_0 = U, C_0 = C (only the
// recurrences after the first cycle use them): D_c, C~^H Upsilon_1 = 0, C~^H U.
Blocks system_start_blocks(const Mat &CtU, int s);

// Pencil of a later cycle of the same Lanczos run: X carried, YtU the
// explicit Upsilon~_j^H U_{j-1} ((s+2) x kp), B, Bt (kC x s).
void pencil_general(const Blocks &X, const Mat &YtU, const Mat &B, const Mat &Bt, const Mat &G,
                    const Mat &Gt, Mat &P, Mat &Q);
// Pencil of the first cycle of a later system (Sec. 4.2): Phi_1 = [U, V_1],
// Psi_1 = [C, V_1 underbar], H_1 = [[I, B_1], [0, T_1 underbar]]; CtU = C~^H U,
// VtU = V~_1 underbar^H U ((s+1) x k).
void pencil_first(const Mat &CtU, const Mat &VtU, const Mat &B, const Mat &Bt, const Mat &G,
                  const Mat &Gt, Mat &P, Mat &Q);
// Blocks for cycle j+1 from those of cycle j and U_j = Phi_j WN,
// U~_j = Phi~_j WtM (Phi in terms of the normalized Lanczos vectors).
Blocks next_blocks(const Blocks &X, const Mat &WN, const Mat &WtM, const Mat &B, const Mat &Bt,
                   const Mat &G, const Mat &Gt);

}  // namespace sec44
