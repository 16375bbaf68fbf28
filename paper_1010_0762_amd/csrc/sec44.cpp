// Sec. 4.4 recurrences for the harmonic Ritz pencil (see sec44.h).
#include "sec44.h"

namespace sec44 {

Mat mul(const Mat &A, const Mat &B) {
  Mat R(A.r, B.c);
  for (int j = 0; j < B.c; ++j)
    for (int l = 0; l < A.c; ++l) {
      const cplx b = B(l, j);
      if (b == cplx(0.0)) continue;
      for (int i = 0; i < A.r; ++i) R(i, j) += A(i, l) * b;
    }
  return R;
}

Mat mul_h(const Mat &A, const Mat &B) {
  Mat R(A.c, B.c);
  for (int j = 0; j < B.c; ++j)
    for (int i = 0; i < A.c; ++i) {
      cplx acc = 0.0;
      for (int l = 0; l < A.r; ++l) acc += std::conj(A(l, i)) * B(l, j);
      R(i, j) = acc;
    }
  return R;
}

Mat eye(int n) {
  Mat I(n, n);
  for (int i = 0; i < n; ++i) I(i, i) = 1.0;
  return I;
}

namespace {

// Copy src into dst at (r0, c0).
void put(Mat &dst, int r0, int c0, const Mat &src) {
  for (int j = 0; j < src.c; ++j)
    for (int i = 0; i < src.r; ++i) dst(r0 + i, c0 + j) = src(i, j);
}

Mat rows(const Mat &A, int r0, int nr) {
  Mat R(nr, A.c);
  for (int j = 0; j < A.c; ++j)
    for (int i = 0; i < nr; ++i) R(i, j) = A(r0 + i, j);
  return R;
}

Mat cols(const Mat &A, int c0, int nc) {
  Mat R(A.r, nc);
  for (int j = 0; j < nc; ++j)
    for (int i = 0; i < A.r; ++i) R(i, j) = A(i, c0 + j);
  return R;
}

}  // namespace

void gamma_blocks(const CycleScalars &cs, Mat &G, Mat &Gt) {
  const int s = cs.s;
  // T(i, i), T(i+1, i), T(i-1, i) for the cycle's columns
  std::vector<cplx> diag(s), sub(s), sup(s, cplx(0.0));
  auto alpha_m1 = [&](int c) { return c >= 1 ? cs.alpha[c - 1] : cs.alpha_before; };
  auto rn_m2 = [&](int c) { return c >= 1 ? cs.rn[c - 1] : cs.rn_before; };
  for (int c = 0; c < s; ++c) {
    diag[c] = 1.0 / cs.alpha[c];
    if (cs.beta[c] != cplx(0.0)) {
      diag[c] += cs.beta[c] / alpha_m1(c);
      sup[c] = -(rn_m2(c) / cs.rn[c]) * cs.beta[c] / alpha_m1(c);
    }
    const double rn_next = c + 1 < s ? cs.rn[c + 1] : cs.rn_end;
    sub[c] = -(rn_next / cs.rn[c]) / cs.alpha[c];
  }
  // T(i0, i0-1) and T(i0+s-1, i0+s) for the dual boundary entries
  const cplx sub_before = cs.first ? cplx(0.0) : -(cs.rn[0] / cs.rn_before) / cs.alpha_before;
  const cplx sup_end = -(cs.rn[s - 1] / cs.rn_end) * cs.beta_end / cs.alpha[s - 1];
  G = Mat(s + 2, s);
  Gt = Mat(s + 2, s);
  for (int c = 0; c < s; ++c) {
    G(c, c) = sup[c];
    G(c + 1, c) = diag[c];
    G(c + 2, c) = sub[c];
    Gt(c, c) = std::conj(c >= 1 ? sub[c - 1] : sub_before);
    Gt(c + 1, c) = std::conj(diag[c]);
    Gt(c + 2, c) = std::conj(c + 1 < s ? sup[c + 1] : sup_end);
  }
}

Blocks empty_blocks(int s) {
  Blocks X;
  X.XCC = Mat(0, 0);
  X.XCtC = Mat(0, 0);
  X.XCtY = Mat(0, s + 2);
  X.XYtC = Mat(s + 2, 0);
  X.XCU = Mat(0, 0);
  X.XCtU = Mat(0, 0);
  return X;
}

Blocks system_start_blocks(const Mat &CtU, int s) {
  const int k = CtU.r;
  Blocks X;
  X.XCC = eye(k);
  X.XCtC = eye(k);
  X.XCtY = Mat(k, s + 2);
  X.XYtC = Mat(s + 2, k);
  X.XCU = CtU;
  X.XCtU = CtU;
  return X;
}

void pencil_general(const Blocks &X, const Mat &YtU, const Mat &B, const Mat &Bt, const Mat &G,
                    const Mat &Gt, Mat &P, Mat &Q) {
  const int kC = X.XCU.r, kp = X.XCU.c, s = G.c;
  const int m1 = kC + kp + s + 2, mm = kp + s;
  // Psi~^H Psi
  Mat G1(m1, m1);
  put(G1, 0, 0, eye(kC));
  put(G1, 0, kC, X.XCC);
  put(G1, kC, 0, X.XCtC);
  put(G1, kC, kC, eye(kp));
  put(G1, kC, kC + kp, X.XCtY);
  put(G1, kC + kp, kC, X.XYtC);
  put(G1, kC + kp, kC + kp, eye(s + 2));
  // Psi~^H Phi
  Mat G2(m1, mm);
  put(G2, 0, 0, X.XCU);
  put(G2, kC, 0, X.XCtU);
  put(G2, kC, kp, cols(X.XCtY, 1, s));
  put(G2, kC + kp, 0, YtU);
  for (int c = 0; c < s; ++c) G2(kC + kp + 1 + c, kp + c) = 1.0;
  // H, H~
  Mat H(m1, mm), Ht(m1, mm);
  put(H, 0, kp, B);
  put(Ht, 0, kp, Bt);
  put(H, kC, 0, eye(kp));
  put(Ht, kC, 0, eye(kp));
  put(H, kC + kp, kp, G);
  put(Ht, kC + kp, kp, Gt);
  P = mul_h(Ht, mul(G1, H));
  Q = mul_h(Ht, G2);
}

void pencil_first(const Mat &CtU, const Mat &VtU, const Mat &B, const Mat &Bt, const Mat &G,
                  const Mat &Gt, Mat &P, Mat &Q) {
  const int k = CtU.r, s = G.c;
  const int m1 = k + s + 1, mm = k + s;
  Mat G2(m1, mm);
  put(G2, 0, 0, CtU);
  put(G2, k, 0, VtU);
  for (int c = 0; c < s; ++c) G2(k + c, k + c) = 1.0;
  Mat H(m1, mm), Ht(m1, mm);
  put(H, 0, 0, eye(k));
  put(Ht, 0, 0, eye(k));
  put(H, 0, k, B);
  put(Ht, 0, k, Bt);
  put(H, k, k, rows(G, 1, s + 1));
  put(Ht, k, k, rows(Gt, 1, s + 1));
  // Psi~_1^H Psi_1 = blockdiag(D_c, I) = I
  P = mul_h(Ht, H);
  Q = mul_h(Ht, G2);
}

Blocks next_blocks(const Blocks &X, const Mat &WN, const Mat &WtM, const Mat &B, const Mat &Bt,
                   const Mat &G, const Mat &Gt) {
  const int kC = X.XCU.r, kp = X.XCU.c, s = G.c;
  // E = Upsilon~_j^H Upsilon_{j+1}: ones at (s, 0) and (s+1, 1)
  auto times_E = [&](const Mat &M) {  // M E  (columns s, s+1 of M move to 0, 1)
    Mat R(M.r, s + 2);
    for (int i = 0; i < M.r; ++i) {
      R(i, 0) = M(i, s);
      R(i, 1) = M(i, s + 1);
    }
    return R;
  };
  auto Et_times = [&](const Mat &M) {  // E^T M  (rows s, s+1 of M move to 0, 1)
    Mat R(s + 2, M.c);
    for (int j = 0; j < M.c; ++j) {
      R(0, j) = M(s, j);
      R(1, j) = M(s + 1, j);
    }
    return R;
  };
  Blocks Y;
  {  // C~^H C_j = [C~^H C_{j-1}, D_c B_j] WN
    Mat L(kC, kp + s);
    put(L, 0, 0, X.XCC);
    put(L, 0, kp, B);
    Y.XCC = mul(L, WN);
  }
  {  // C~_j^H C = (W~M)^H [C~_{j-1}^H C; B~_j^H D_c]
    Mat R(kp + s, kC);
    put(R, 0, 0, X.XCtC);
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < kC; ++j) R(kp + i, j) = std::conj(Bt(j, i));
    Y.XCtC = mul_h(WtM, R);
  }
  {  // C~_j^H Upsilon_{j+1} = (W~M)^H [0; Gamma~_j^H E]
    Mat GtE = times_E(mul_h(Gt, eye(s + 2)));
    Mat R(kp + s, s + 2);
    put(R, kp, 0, GtE);
    Y.XCtY = mul_h(WtM, R);
  }
  {  // Upsilon~_{j+1}^H C_j = [0, E^T Gamma_j] WN
    Mat L(s + 2, kp + s);
    put(L, 0, kp, Et_times(G));
    Y.XYtC = mul(L, WN);
  }
  {  // C~^H U_j = [C~^H U_{j-1}, 0] WN
    Mat L(kC, kp + s);
    put(L, 0, 0, X.XCU);
    Y.XCU = mul(L, WN);
  }
  {  // C~_j^H U_j = (W~M)^H [[C~_{j-1}^H U_{j-1}, C~_{j-1}^H V_j], [V~_j^H C_{j-1}, T_j]] WN
    Mat M(kp + s, kp + s);
    put(M, 0, 0, X.XCtU);
    put(M, 0, kp, cols(X.XCtY, 1, s));
    put(M, kp, 0, rows(X.XYtC, 1, s));
    put(M, kp, kp, rows(G, 1, s));
    Y.XCtU = mul_h(WtM, mul(M, WN));
  }
  return Y;
}

}  // namespace sec44
