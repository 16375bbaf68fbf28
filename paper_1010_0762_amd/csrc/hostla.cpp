// Host FP64 dense linear algebra for the cycle-end computations of recycling
// BiCG: the small eigenproblems of Sec. 4.1/4.2 and the biorthogonalization of
// Sec. 4.3.  Sizes are at most a few hundred, so plain O(m^3) algorithms are
// used: Householder Hessenberg reduction + shifted complex QR (Schur form),
// triangular back-substitution for eigenvectors, LU with partial pivoting,
// cyclic Jacobi for Hermitian matrices and one-sided Jacobi for the SVD.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <vector>

#include "rbicg_hostla.h"
#include "errors.h"

namespace {

using cplx = std::complex<double>;
const double kEps = 2.220446049250313e-16;

struct CMat {
  int m = 0, n = 0;
  std::vector<cplx> a;
  CMat() {}
  CMat(int m_, int n_) : m(m_), n(n_), a((size_t)m_ * n_) {}
  cplx &operator()(int i, int j) { return a[(size_t)i + (size_t)j * m]; }
  const cplx &operator()(int i, int j) const { return a[(size_t)i + (size_t)j * m]; }
};

CMat load(int m, int n, const double *p) {
  CMat A(m, n);
  for (size_t t = 0; t < (size_t)m * n; ++t) A.a[t] = cplx(p[2 * t], p[2 * t + 1]);
  return A;
}
void store(const CMat &A, double *p) {
  for (size_t t = 0; t < A.a.size(); ++t) {
    p[2 * t] = A.a[t].real();
    p[2 * t + 1] = A.a[t].imag();
  }
}
double abs1(cplx z) { return std::fabs(z.real()) + std::fabs(z.imag()); }
// modulus without hypot's overflow guard (entries here are far from the limits)
inline double cabs(cplx z) { return std::sqrt(z.real() * z.real() + z.imag() * z.imag()); }

// LU with partial pivoting; solves A X = B in place (B overwritten by X).
bool lu_solve(CMat A, CMat &B) {
  const int m = A.m;
  std::vector<int> piv(m);
  double anorm = 0;
  for (auto &z : A.a) anorm = std::max(anorm, std::abs(z));
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = std::abs(A(k, k));
    for (int i = k + 1; i < m; ++i)
      if (std::abs(A(i, k)) > best) { best = std::abs(A(i, k)); p = i; }
    if (best <= anorm * 1e-300 || best == 0.0) return false;
    piv[k] = p;
    if (p != k) {
      for (int j = 0; j < m; ++j) std::swap(A(k, j), A(p, j));
      for (int j = 0; j < B.n; ++j) std::swap(B(k, j), B(p, j));
    }
    for (int i = k + 1; i < m; ++i) {
      cplx f = A(i, k) / A(k, k);
      A(i, k) = f;
      for (int j = k + 1; j < m; ++j) A(i, j) -= f * A(k, j);
      for (int j = 0; j < B.n; ++j) B(i, j) -= f * B(k, j);
    }
  }
  for (int j = 0; j < B.n; ++j)
    for (int i = m - 1; i >= 0; --i) {
      cplx s = B(i, j);
      for (int l = i + 1; l < m; ++l) s -= A(i, l) * B(l, j);
      B(i, j) = s / A(i, i);
    }
  return true;
}

bool inverse(const CMat &A, CMat &Ainv) {
  Ainv = CMat(A.m, A.m);
  for (int i = 0; i < A.m; ++i) Ainv(i, i) = 1.0;
  return lu_solve(A, Ainv);
}

// Householder reduction to upper Hessenberg form: A = Z H Z^H.
void hessenberg(CMat &H, CMat &Z) {
  const int m = H.m;
  Z = CMat(m, m);
  for (int i = 0; i < m; ++i) Z(i, i) = 1.0;
  std::vector<cplx> v(m);
  for (int k = 0; k + 2 < m; ++k) {
    double xnorm = 0;
    for (int i = k + 1; i < m; ++i) xnorm += std::norm(H(i, k));
    xnorm = std::sqrt(xnorm);
    if (xnorm == 0.0) continue;
    cplx x0 = H(k + 1, k);
    cplx ph = (std::abs(x0) == 0.0) ? cplx(1.0, 0.0) : x0 / std::abs(x0);
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int i = k + 1; i < m; ++i) v[i] = H(i, k);
    v[k + 1] += ph * xnorm;
    double vn = 0;
    for (int i = k + 1; i < m; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    // H <- (I - 2 v v^H / vn) H (I - 2 v v^H / vn)
    for (int j = 0; j < m; ++j) {
      cplx s = 0;
      for (int i = k + 1; i < m; ++i) s += std::conj(v[i]) * H(i, j);
      s *= 2.0 / vn;
      for (int i = k + 1; i < m; ++i) H(i, j) -= v[i] * s;
    }
    for (int i = 0; i < m; ++i) {
      cplx s = 0;
      for (int j = k + 1; j < m; ++j) s += H(i, j) * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < m; ++j) H(i, j) -= s * std::conj(v[j]);
    }
    for (int i = 0; i < m; ++i) {
      cplx s = 0;
      for (int j = k + 1; j < m; ++j) s += Z(i, j) * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < m; ++j) Z(i, j) -= s * std::conj(v[j]);
    }
    for (int i = k + 2; i < m; ++i) H(i, k) = 0.0;
  }
}

// Shifted complex QR iteration (explicit Givens form, Wilkinson shifts with
// occasional exceptional shifts) on a Hessenberg matrix; on return H is upper
// triangular (complex Schur form) and Z accumulates the unitary similarity.
bool schur_qr(CMat &H, CMat &Z) {
  const int m = H.m;
  double hnorm = 0;
  for (auto &z : H.a) hnorm = std::max(hnorm, abs1(z));
  if (hnorm == 0.0) return true;
  int hi = m - 1, iter = 0, total = 0;
  std::vector<cplx> cs(m), sn(m);
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      double s = abs1(H(l - 1, l - 1)) + abs1(H(l, l));
      if (s == 0.0) s = hnorm;
      if (abs1(H(l, l - 1)) <= kEps * s) {
        H(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    ++iter;
    if (++total > 60 * m) return false;
    cplx mu;
    if (iter % 10 == 0) {
      mu = H(hi, hi) + cplx(0.75 * std::abs(H(hi, hi - 1)), 0.0);
    } else {
      cplx a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
      cplx half = 0.5 * (a - d);
      cplx disc = std::sqrt(half * half + b * c);
      cplx l1 = 0.5 * (a + d) + disc, l2 = 0.5 * (a + d) - disc;
      mu = (std::abs(l1 - d) < std::abs(l2 - d)) ? l1 : l2;
    }
    for (int k = l; k <= hi; ++k) H(k, k) -= mu;
    for (int k = l; k < hi; ++k) {
      cplx x = H(k, k), y = H(k + 1, k);
      double r = std::sqrt(std::norm(x) + std::norm(y));
      cplx c = 1.0, s = 0.0;
      if (r != 0.0) { c = x / r; s = y / r; }
      cs[k] = c; sn[k] = s;
      // rows k, k+1 <- [[conj c, conj s], [-s, c]] [row k; row k+1]
      for (int j = k; j < m; ++j) {
        cplx a = H(k, j), b = H(k + 1, j);
        H(k, j) = std::conj(c) * a + std::conj(s) * b;
        H(k + 1, j) = -s * a + c * b;
      }
    }
    for (int k = l; k < hi; ++k) {
      cplx c = cs[k], s = sn[k];
      // columns k, k+1 <- [col k, col k+1] [[c, -conj s], [s, conj c]]
      int rmax = std::min(k + 1, hi);
      for (int i = 0; i <= rmax; ++i) {
        cplx a = H(i, k), b = H(i, k + 1);
        H(i, k) = a * c + b * s;
        H(i, k + 1) = -a * std::conj(s) + b * std::conj(c);
      }
      for (int i = 0; i < m; ++i) {
        cplx a = Z(i, k), b = Z(i, k + 1);
        Z(i, k) = a * c + b * s;
        Z(i, k + 1) = -a * std::conj(s) + b * std::conj(c);
      }
    }
    for (int k = l; k <= hi; ++k) H(k, k) += mu;
  }
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) H(i, j) = 0.0;
  return true;
}

void normalize_cols(CMat &X) {
  for (int j = 0; j < X.n; ++j) {
    double s = 0;
    for (int i = 0; i < X.m; ++i) s += std::norm(X(i, j));
    s = std::sqrt(s);
    if (s > 0)
      for (int i = 0; i < X.m; ++i) X(i, j) /= s;
  }
}

// Eigenvalues and right eigenvectors of a general complex matrix.
bool eig_general(const CMat &M, std::vector<cplx> &lam, CMat &X) {
  const int m = M.m;
  CMat H = M, Z;
  hessenberg(H, Z);
  if (!schur_qr(H, Z)) return false;
  lam.resize(m);
  for (int i = 0; i < m; ++i) lam[i] = H(i, i);
  double tnorm = 0;
  for (auto &z : H.a) tnorm = std::max(tnorm, std::abs(z));
  double small = std::max(tnorm * kEps, 1e-300);
  CMat Y(m, m);
  for (int j = 0; j < m; ++j) {
    Y(j, j) = 1.0;
    for (int i = j - 1; i >= 0; --i) {
      cplx s = 0;
      for (int l = i + 1; l <= j; ++l) s += H(i, l) * Y(l, j);
      cplx d = H(i, i) - lam[j];
      if (std::abs(d) < small) d = small;
      Y(i, j) = -s / d;
    }
  }
  X = CMat(m, m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      cplx s = 0;
      for (int l = 0; l <= j; ++l) s += Z(i, l) * Y(l, j);
      X(i, j) = s;
    }
  normalize_cols(X);
  return true;
}

// Cyclic Jacobi for a Hermitian matrix: A = V diag(w) V^H.
void herm_jacobi(CMat A, std::vector<double> &w, CMat &V) {
  const int m = A.m;
  V = CMat(m, m);
  for (int i = 0; i < m; ++i) V(i, i) = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        tot += std::norm(A(i, j));
        if (i != j) off += std::norm(A(i, j));
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        cplx apq = A(p, q);
        double b = std::abs(apq);
        if (b == 0.0) continue;
        double app = A(p, p).real(), aqq = A(q, q).real();
        cplx e = apq / b;  // e^{i phi}
        double tau = (aqq - app) / (2.0 * b);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        cplx em = std::conj(e);
        // A <- A J, J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
        for (int k = 0; k < m; ++k) {
          cplx akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * em * akq;
          A(k, q) = s * akp + c * em * akq;
        }
        // A <- J^H A
        for (int k = 0; k < m; ++k) {
          cplx apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * e * aqk;
          A(q, k) = s * apk + c * e * aqk;
        }
        for (int k = 0; k < m; ++k) {
          cplx vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * em * vkq;
          V(k, q) = s * vkp + c * em * vkq;
        }
      }
  }
  w.resize(m);
  for (int i = 0; i < m; ++i) w[i] = A(i, i).real();
  std::vector<int> idx(m);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] < w[b]; });
  CMat V2(m, m);
  std::vector<double> w2(m);
  for (int j = 0; j < m; ++j) {
    w2[j] = w[idx[j]];
    for (int i = 0; i < m; ++i) V2(i, j) = V(i, idx[j]);
  }
  w = w2;
  V = V2;
}

// One-sided Jacobi SVD, m >= n: A = U diag(s) V^H, s descending.
void svd_jacobi(const CMat &A, CMat &U, std::vector<double> &s, CMat &V) {
  const int m = A.m, n = A.n;
  U = A;
  V = CMat(n, n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double alpha = 0, beta = 0;
        cplx gamma = 0;
        for (int i = 0; i < m; ++i) {
          alpha += std::norm(U(i, p));
          beta += std::norm(U(i, q));
          gamma += std::conj(U(i, p)) * U(i, q);
        }
        double g = std::abs(gamma);
        if (g == 0.0 || g <= 1e-15 * std::sqrt(alpha * beta)) continue;
        rotated = true;
        cplx e = gamma / g, em = std::conj(e);
        double tau = (beta - alpha) / (2.0 * g);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        for (int i = 0; i < m; ++i) {
          cplx up = U(i, p), uq = U(i, q);
          U(i, p) = c * up - sn * em * uq;
          U(i, q) = sn * up + c * em * uq;
        }
        for (int i = 0; i < n; ++i) {
          cplx vp = V(i, p), vq = V(i, q);
          V(i, p) = c * vp - sn * em * vq;
          V(i, q) = sn * vp + c * em * vq;
        }
      }
    if (!rotated) break;
  }
  s.resize(n);
  for (int j = 0; j < n; ++j) {
    double t = 0;
    for (int i = 0; i < m; ++i) t += std::norm(U(i, j));
    s[j] = std::sqrt(t);
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return s[a] > s[b]; });
  CMat U2(m, n), V2(n, n);
  std::vector<double> s2(n);
  for (int j = 0; j < n; ++j) {
    int o = idx[j];
    s2[j] = s[o];
    for (int i = 0; i < m; ++i) U2(i, j) = (s[o] > 0) ? U(i, o) / s[o] : (i == j ? 1.0 : 0.0);
    for (int i = 0; i < n; ++i) V2(i, j) = V(i, o);
  }
  U = U2;
  V = V2;
  s = s2;
}


// Complex Givens rotation G = [[c, s], [-conj(s), c]] (c real) with
// G [x; y] = [r; 0].
struct Giv {
  double c;
  cplx s;
};
Giv givens(cplx x, cplx y) {
  const double ax = cabs(x), ay = cabs(y);
  if (ay == 0.0) return {1.0, 0.0};
  if (ax == 0.0) return {0.0, std::conj(y) / ay};
  const double r = std::sqrt(ax * ax + ay * ay);
  const cplx ph = x / ax;
  return {ax / r, ph * std::conj(y) / r};
}
// rows (i, j) of M <- G [row i; row j], columns c0..c1-1
void rot_rows(CMat &M, int i, int j, const Giv &g, int c0, int c1) {
  for (int c = c0; c < c1; ++c) {
    const cplx a = M(i, c), b = M(j, c);
    M(i, c) = g.c * a + g.s * b;
    M(j, c) = -std::conj(g.s) * a + g.c * b;
  }
}
// columns (i, j) of M <- [col i, col j] G^H, rows r0..r1-1
void rot_cols(CMat &M, int i, int j, const Giv &g, int r0, int r1) {
  for (int r = r0; r < r1; ++r) {
    const cplx a = M(r, i), b = M(r, j);
    M(r, i) = g.c * a + std::conj(g.s) * b;
    M(r, j) = -g.s * a + g.c * b;
  }
}
// column rotation that zeroes M(r, i) against M(r, j): [M(r,i), M(r,j)] G^H = [0, *]
Giv givens_col_zero_left(cplx mi, cplx mj) {
  // want a c + b conj(s) = 0 with a = mi, b = mj: take G from (conj(mj), -conj(mi)) style
  const double ai = cabs(mi), aj = cabs(mj);
  if (ai == 0.0) return {1.0, 0.0};
  if (aj == 0.0) return {0.0, 1.0};
  const double r = std::sqrt(ai * ai + aj * aj);
  // c = |mj| / r, s such that mi c + mj conj(s) = 0  ->  conj(s) = -mi c / mj
  const double c = aj / r;
  const cplx sc = -mi * c / mj;
  return {c, std::conj(sc)};
}

// Generalized complex Schur form of the pencil (A, B): Q^H A Z = S, Q^H B Z = T
// with S, T upper triangular (QZ algorithm of Moler and Stewart: Hessenberg-
// triangular reduction, then implicit single-shift QZ sweeps).
bool qz(CMat &A, CMat &B, CMat &Q, CMat &Z) {
  const int m = A.m;
  Q = CMat(m, m);
  Z = CMat(m, m);
  for (int i = 0; i < m; ++i) { Q(i, i) = 1.0; Z(i, i) = 1.0; }
  // B = QR by Givens, applied to A as well
  for (int j = 0; j < m; ++j)
    for (int i = m - 1; i > j; --i) {
      const Giv g = givens(B(i - 1, j), B(i, j));
      rot_rows(B, i - 1, i, g, 0, m);
      rot_rows(A, i - 1, i, g, 0, m);
      // Q <- Q G^H
      rot_cols(Q, i - 1, i, g, 0, m);
      B(i, j) = 0.0;
    }
  // A to Hessenberg keeping B triangular
  for (int j = 0; j + 2 < m; ++j)
    for (int i = m - 1; i > j + 1; --i) {
      const Giv g = givens(A(i - 1, j), A(i, j));
      rot_rows(A, i - 1, i, g, 0, m);
      rot_rows(B, i - 1, i, g, 0, m);
      rot_cols(Q, i - 1, i, g, 0, m);
      A(i, j) = 0.0;
      // fill-in B(i, i-1): zero it with a column rotation on (i-1, i)
      const Giv h = givens_col_zero_left(B(i, i - 1), B(i, i));
      rot_cols(B, i - 1, i, h, 0, m);
      rot_cols(A, i - 1, i, h, 0, m);
      rot_cols(Z, i - 1, i, h, 0, m);
      B(i, i - 1) = 0.0;
    }
  double anorm = 0, bnorm = 0;
  for (auto &z : A.a) anorm = std::max(anorm, abs1(z));
  for (auto &z : B.a) bnorm = std::max(bnorm, abs1(z));
  if (anorm == 0.0) anorm = 1.0;
  if (bnorm == 0.0) bnorm = 1.0;
  int hi = m - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      if (abs1(A(l, l - 1)) <= kEps * (abs1(A(l - 1, l - 1)) + abs1(A(l, l)) + 1e-300 * anorm) ||
          abs1(A(l, l - 1)) <= kEps * anorm * 1e-3) {
        A(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    ++iter;
    if (++total > 80 * m) return false;
    // tiny diagonal entries of B: set to a floor (infinite eigenvalues become huge)
    for (int i = l; i <= hi; ++i)
      if (cabs(B(i, i)) < kEps * bnorm) B(i, i) = kEps * bnorm;
    // shift: eigenvalue of the trailing 2x2 of A B^{-1} closest to A(hi,hi)/B(hi,hi)
    cplx mu;
    {
      const cplx b11 = B(hi - 1, hi - 1), b12 = B(hi - 1, hi), b22 = B(hi, hi);
      const cplx a11 = A(hi - 1, hi - 1), a12 = A(hi - 1, hi), a21 = A(hi, hi - 1), a22 = A(hi, hi);
      // M = [a] [b]^{-1}, b upper triangular 2x2
      const cplx i11 = 1.0 / b11, i22 = 1.0 / b22, i12 = -b12 / (b11 * b22);
      const cplx m11 = a11 * i11, m12 = a11 * i12 + a12 * i22;
      const cplx m21 = a21 * i11, m22 = a21 * i12 + a22 * i22;
      const cplx half = 0.5 * (m11 - m22);
      const cplx disc = std::sqrt(half * half + m12 * m21);
      const cplx e1 = 0.5 * (m11 + m22) + disc, e2 = 0.5 * (m11 + m22) - disc;
      const cplx tgt = a22 / b22;
      mu = (cabs(e1 - tgt) < cabs(e2 - tgt)) ? e1 : e2;
      if (iter % 10 == 0) mu = tgt + cplx(0.75 * cabs(a21 / b11), 0.0);
    }
    // first rotation from the first column of A - mu B
    Giv g = givens(A(l, l) - mu * B(l, l), A(l + 1, l));
    for (int k = l; k < hi; ++k) {
      if (k > l) g = givens(A(k, k - 1), A(k + 1, k - 1));
      rot_rows(A, k, k + 1, g, std::max(l, k - 1), m);
      rot_rows(B, k, k + 1, g, k, m);
      rot_cols(Q, k, k + 1, g, 0, m);
      if (k > l) A(k + 1, k - 1) = 0.0;
      // B(k+1, k) fill-in: column rotation on (k, k+1)
      const Giv h = givens_col_zero_left(B(k + 1, k), B(k + 1, k + 1));
      rot_cols(B, k, k + 1, h, 0, k + 2);
      rot_cols(A, k, k + 1, h, 0, std::min(k + 3, hi + 1));
      rot_cols(Z, k, k + 1, h, 0, m);
      B(k + 1, k) = 0.0;
    }
  }
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) {
      A(i, j) = 0.0;
      B(i, j) = 0.0;
    }
  return true;
}

// Eigenvalues of a complex pencil via QZ, and right eigenvectors W
// (A w = lambda B w) and left eigenvectors Y (y^H A = lambda y^H B) for the
// eigenvalue indices in `want` (all when empty); W and Y hold one column per
// wanted index, in the order given.
struct PencilSchur {
  CMat S, T, Q, Z;
  std::vector<cplx> lam;
};
bool pencil_schur(CMat A, CMat B, PencilSchur &ps) {
  const int m = A.m;
  if (!qz(A, B, ps.Q, ps.Z)) return false;
  ps.S = A;
  ps.T = B;
  ps.lam.resize(m);
  for (int i = 0; i < m; ++i) ps.lam[i] = A(i, i) / B(i, i);
  return true;
}
void pencil_vectors(const PencilSchur &ps, const std::vector<int> &want, CMat &W, CMat &Y) {
  const CMat &A = ps.S, &B = ps.T;
  const int m = A.m, nw = (int)want.size();
  double snorm = 0;
  for (auto &z : A.a) snorm = std::max(snorm, cabs(z));
  for (auto &z : B.a) snorm = std::max(snorm, cabs(z));
  const double small = std::max(snorm * kEps, 1e-300);
  W = CMat(m, nw);
  Y = CMat(m, nw);
  std::vector<cplx> yr(m), yl(m);
  for (int c = 0; c < nw; ++c) {
    const int j = want[c];
    const cplx lj = ps.lam[j];
    std::fill(yr.begin(), yr.end(), cplx(0.0));
    std::fill(yl.begin(), yl.end(), cplx(0.0));
    // right: (S - lam T) y = 0 with y supported on rows 0..j
    yr[j] = 1.0;
    for (int i = j - 1; i >= 0; --i) {
      cplx sacc = 0;
      for (int l = i + 1; l <= j; ++l) sacc += (A(i, l) - lj * B(i, l)) * yr[l];
      cplx d = A(i, i) - lj * B(i, i);
      if (cabs(d) < small) d = small;
      yr[i] = -sacc / d;
    }
    // left: u^H (S - lam T) = 0 with u supported on rows j..m-1
    yl[j] = 1.0;
    for (int i = j + 1; i < m; ++i) {
      cplx sacc = 0;
      for (int l = j; l < i; ++l) sacc += std::conj(yl[l]) * (A(l, i) - lj * B(l, i));
      cplx d = A(i, i) - lj * B(i, i);
      if (cabs(d) < small) d = small;
      yl[i] = std::conj(-sacc / d);
    }
    for (int i = 0; i < m; ++i) {
      cplx a = 0, b = 0;
      for (int l = 0; l <= j; ++l) a += ps.Z(i, l) * yr[l];
      for (int l = j; l < m; ++l) b += ps.Q(i, l) * yl[l];
      W(i, c) = a;
      Y(i, c) = b;
    }
  }
  normalize_cols(W);
  normalize_cols(Y);
}

bool finite(cplx z) { return std::isfinite(z.real()) && std::isfinite(z.imag()); }

}  // namespace

extern "C" int rbicg_host_eig(int32_t m, const double *P, const double *Q, double *lam,
                              double *W, double *Wl) {
  if (m <= 0 || !P) return rbicg_fail(-1, "host_eig: bad arguments");
  CMat Pm = load(m, m, P);
  CMat Qm(m, m);
  if (Q) {
    Qm = load(m, m, Q);
  } else {
    for (int i = 0; i < m; ++i) Qm(i, i) = 1.0;
  }
  PencilSchur ps;
  if (!pencil_schur(Pm, Qm, ps)) return rbicg_fail(-1, "host_eig: QZ iteration did not converge");
  std::vector<cplx> &ev = ps.lam;
  CMat X, Y;
  std::vector<int> all(m);
  std::iota(all.begin(), all.end(), 0);
  if (W || Wl) pencil_vectors(ps, all, X, Y);
  if (lam)
    for (int i = 0; i < m; ++i) { lam[2 * i] = ev[i].real(); lam[2 * i + 1] = ev[i].imag(); }
  if (W) store(X, W);
  if (Wl) store(Y, Wl);
  return 0;
}

namespace {
// One selected eigenvalue and how its vector enters the recycle space:
// 0 as is (complex problem), 1 real eigenvalue of a real problem (phase
// removed, real part), 2 conjugate pair of a real problem ([Re w, Im w]),
// 3 complex value without a partner in a real problem (real part only).
struct SelItem {
  int idx, kind;
};

std::vector<SelItem> select_indices(const std::vector<cplx> &lam, int k, bool real_problem,
                                    int &ncols) {
  const int m = (int)lam.size();
  std::vector<int> order;
  for (int i = 0; i < m; ++i)
    if (finite(lam[i])) order.push_back(i);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const double ma = cabs(lam[a]), mb = cabs(lam[b]);
    if (ma != mb) return ma < mb;
    if (lam[a].real() != lam[b].real()) return lam[a].real() < lam[b].real();
    if (lam[a].imag() != lam[b].imag()) return lam[a].imag() < lam[b].imag();
    return a < b;
  });
  std::vector<SelItem> out;
  ncols = 0;
  if (!real_problem) {
    for (size_t t = 0; t < order.size() && ncols < k; ++t) {
      out.push_back({order[t], 0});
      ++ncols;
    }
    return out;
  }
  double scale = 1.0;
  for (int i : order) scale = std::max(scale, cabs(lam[i]));
  std::vector<char> used(m, 0);
  for (size_t t = 0; t < order.size() && ncols < k; ++t) {
    const int i = order[t];
    if (used[i]) continue;
    if (std::fabs(lam[i].imag()) <= 1e-9 * std::max(cabs(lam[i]), 1e-300)) {
      used[i] = 1;
      out.push_back({i, 1});
      ++ncols;
      continue;
    }
    int jbest = -1;
    double dbest = 0;
    for (int j : order) {
      if (used[j] || j == i) continue;
      const double d = cabs(lam[j] - std::conj(lam[i]));
      if (jbest < 0 || d < dbest) { jbest = j; dbest = d; }
    }
    if (jbest < 0) break;
    if (dbest > 1e-8 * scale) {
      used[i] = 1;
      out.push_back({i, 3});
      ++ncols;
      continue;
    }
    if (ncols + 2 > k) break;
    used[i] = used[jbest] = 1;
    out.push_back({lam[i].imag() > 0 ? i : jbest, 2});
    ncols += 2;
  }
  return out;
}

std::vector<cplx> dephase(std::vector<cplx> c) {
  int im = 0;
  for (size_t i = 1; i < c.size(); ++i)
    if (cabs(c[i]) > cabs(c[im])) im = (int)i;
  const cplx ph = (cabs(c[im]) > 0) ? std::conj(c[im]) / cabs(c[im]) : cplx(1.0);
  for (auto &z : c) z = cplx((z * ph).real(), 0.0);
  return c;
}

// Expand the selection into output columns (m x ncols, column-major,
// interleaved); col(c) gives the vector of selection entry c.
template <class F>
void emit(const std::vector<SelItem> &sel, int m, F col, double *out) {
  int c = 0;
  auto put = [&](const std::vector<cplx> &v) {
    for (int i = 0; i < m; ++i) {
      out[2 * ((size_t)i + (size_t)c * m)] = v[i].real();
      out[2 * ((size_t)i + (size_t)c * m) + 1] = v[i].imag();
    }
    ++c;
  };
  for (size_t t = 0; t < sel.size(); ++t) {
    std::vector<cplx> v = col((int)t);
    switch (sel[t].kind) {
      case 0: put(v); break;
      case 1: put(dephase(v)); break;
      case 2: {
        std::vector<cplx> re(m), im(m);
        for (int i = 0; i < m; ++i) { re[i] = v[i].real(); im[i] = v[i].imag(); }
        put(re);
        put(im);
        break;
      }
      default: {
        std::vector<cplx> re(m);
        for (int i = 0; i < m; ++i) re[i] = v[i].real();
        put(re);
      }
    }
  }
}
}  // namespace

extern "C" int rbicg_host_select(int32_t m, const double *lamp, const double *Wp,
                                 const double *Wlp, int32_t k, int32_t real_problem,
                                 double *Wsel, double *Wlsel) {
  if (m <= 0 || k < 0 || !lamp || !Wp || !Wsel) return rbicg_fail(-1, "host_select: bad arguments");
  std::vector<cplx> lam(m);
  for (int i = 0; i < m; ++i) lam[i] = cplx(lamp[2 * i], lamp[2 * i + 1]);
  const CMat W = load(m, m, Wp);
  CMat Wl;
  if (Wlp) Wl = load(m, m, Wlp);
  int ncols = 0;
  const std::vector<SelItem> sel = select_indices(lam, k, real_problem != 0, ncols);
  auto colW = [&](int t) {
    std::vector<cplx> v(m);
    for (int i = 0; i < m; ++i) v[i] = W(i, sel[t].idx);
    return v;
  };
  emit(sel, m, colW, Wsel);
  if (Wlp && Wlsel) {
    auto colL = [&](int t) {
      std::vector<cplx> v(m);
      for (int i = 0; i < m; ++i) v[i] = Wl(i, sel[t].idx);
      return v;
    };
    emit(sel, m, colL, Wlsel);
  }
  return ncols;
}

extern "C" int rbicg_host_eig_select(int32_t m, const double *P, const double *Q, int32_t k,
                                     int32_t real_problem, double *Wsel, double *Wlsel) {
  if (m <= 0 || k < 0 || !P || !Wsel || !Wlsel) return rbicg_fail(-1, "host_eig_select: bad arguments");
  CMat Pm = load(m, m, P);
  CMat Qm(m, m);
  if (Q) {
    Qm = load(m, m, Q);
  } else {
    for (int i = 0; i < m; ++i) Qm(i, i) = 1.0;
  }
  PencilSchur ps;
  if (!pencil_schur(Pm, Qm, ps)) return rbicg_fail(-1, "host_eig_select: QZ iteration did not converge");
  int ncols = 0;
  const std::vector<SelItem> sel = select_indices(ps.lam, k, real_problem != 0, ncols);
  std::vector<int> want;
  for (const auto &it : sel) want.push_back(it.idx);
  CMat W, Y;
  pencil_vectors(ps, want, W, Y);
  auto colW = [&](int t) {
    std::vector<cplx> v(m);
    for (int i = 0; i < m; ++i) v[i] = W(i, t);
    return v;
  };
  auto colY = [&](int t) {
    std::vector<cplx> v(m);
    for (int i = 0; i < m; ++i) v[i] = Y(i, t);
    return v;
  };
  emit(sel, m, colW, Wsel);
  emit(sel, m, colY, Wlsel);
  return ncols;
}

extern "C" int rbicg_host_svd(int32_t m, int32_t n, const double *A, double *U, double *s,
                              double *V) {
  if (m <= 0 || n <= 0 || m < n || !A) return rbicg_fail(-1, "host_svd: bad arguments");
  CMat Am = load(m, n, A), Um, Vm;
  std::vector<double> sv;
  svd_jacobi(Am, Um, sv, Vm);
  if (U) store(Um, U);
  if (V) store(Vm, V);
  if (s) std::copy(sv.begin(), sv.end(), s);
  return 0;
}

extern "C" int rbicg_host_heig(int32_t m, const double *A, double *w, double *V) {
  if (m <= 0 || !A) return rbicg_fail(-1, "host_heig: bad arguments");
  CMat Am = load(m, m, A), Vm;
  std::vector<double> wv;
  herm_jacobi(Am, wv, Vm);
  if (w) std::copy(wv.begin(), wv.end(), w);
  if (V) store(Vm, V);
  return 0;
}

namespace {
// Columns spanning range(C) with orthonormal images: L = V_r diag(w_r^{-1/2}).
CMat whitening(const CMat &G) {
  std::vector<double> w;
  CMat V;
  herm_jacobi(G, w, V);
  const int k = G.m;
  double wmax = 0;
  for (double x : w) wmax = std::max(wmax, x);
  std::vector<int> keep;
  for (int i = k - 1; i >= 0; --i)
    if (w[i] > 1e-13 * wmax && w[i] > 0) keep.push_back(i);
  CMat L(k, (int)keep.size());
  for (size_t j = 0; j < keep.size(); ++j) {
    double f = 1.0 / std::sqrt(w[keep[j]]);
    for (int i = 0; i < k; ++i) L(i, (int)j) = V(i, keep[j]) * f;
  }
  return L;
}
CMat mul(const CMat &A, const CMat &B, bool conjA = false) {
  int m = conjA ? A.n : A.m, kk = conjA ? A.m : A.n;
  CMat C(m, B.n);
  for (int j = 0; j < B.n; ++j)
    for (int i = 0; i < m; ++i) {
      cplx s = 0;
      for (int l = 0; l < kk; ++l) s += (conjA ? std::conj(A(l, i)) : A(i, l)) * B(l, j);
      C(i, j) = s;
    }
  return C;
}
}  // namespace

extern "C" int rbicg_host_biorth(int32_t k, const double *Gcc, const double *Gtt,
                                 const double *Gtc, double tol, double *TU, double *TUt) {
  if (k <= 0 || !Gcc || !Gtt || !Gtc || !TU || !TUt) return rbicg_fail(-1, "host_biorth: bad arguments");
  CMat L = whitening(load(k, k, Gcc));
  CMat Lt = whitening(load(k, k, Gtt));
  if (L.n == 0 || Lt.n == 0) return 0;
  CMat K = mul(Lt, mul(load(k, k, Gtc), L), true);  // Q~^H Q  (rt x r)
  CMat M, N;
  std::vector<double> sv;
  if (K.m >= K.n) {
    svd_jacobi(K, M, sv, N);  // K = M S N^H
  } else {
    CMat KH(K.n, K.m);
    for (int i = 0; i < K.m; ++i)
      for (int j = 0; j < K.n; ++j) KH(j, i) = std::conj(K(i, j));
    svd_jacobi(KH, N, sv, M);  // K^H = N S M^H
  }
  int p = 0;
  for (double x : sv)
    if (std::isfinite(x) && x >= tol) ++p;
  for (int j = 0; j < p; ++j) {
    double f = 1.0 / std::sqrt(sv[j]);
    for (int i = 0; i < k; ++i) {
      cplx a = 0, b = 0;
      for (int l = 0; l < L.n; ++l) a += L(i, l) * N(l, j);
      for (int l = 0; l < Lt.n; ++l) b += Lt(i, l) * M(l, j);
      a *= f;
      b *= f;
      TU[2 * (i + j * k)] = a.real();
      TU[2 * (i + j * k) + 1] = a.imag();
      TUt[2 * (i + j * k)] = b.real();
      TUt[2 * (i + j * k) + 1] = b.imag();
    }
  }
  return p;
}
