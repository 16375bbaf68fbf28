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

// ------------------------------------------------------------- real QZ
// Real pencils (the harmonic Ritz pencils of real problems) take the real
// double-shift QZ algorithm of Moler and Stewart: Householder QR of B,
// Givens reduction of A to Hessenberg form with B kept triangular, then
// implicit double-shift sweeps (3 x 3 Householder reflections chasing the
// bulge) until A is quasi-triangular (1 x 1 and 2 x 2 diagonal blocks).
// Complex eigenvalues of the 2 x 2 blocks come in conjugate pairs.
struct RMat {
  int m = 0, n = 0;
  std::vector<double> a;
  RMat() {}
  RMat(int m_, int n_) : m(m_), n(n_), a((size_t)m_ * n_, 0.0) {}
  double &operator()(int i, int j) { return a[(size_t)i + (size_t)j * m]; }
  double operator()(int i, int j) const { return a[(size_t)i + (size_t)j * m]; }
};

// Householder vector of x (len entries): (I - beta v v^T) x = -+||x|| e_0,
// v[0] = 1 (Golub and Van Loan, Algorithm 5.1.1).
void house(const double *x, int len, double *v, double &beta) {
  double sigma = 0.0;
  for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
  v[0] = 1.0;
  for (int i = 1; i < len; ++i) v[i] = x[i];
  if (sigma == 0.0) {
    beta = 0.0;
    return;
  }
  const double mu = std::sqrt(x[0] * x[0] + sigma);
  const double v0 = x[0] <= 0.0 ? x[0] - mu : -sigma / (x[0] + mu);
  beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
  for (int i = 1; i < len; ++i) v[i] /= v0;
}
// rows r0..r0+len-1 of M <- (I - beta v v^T) M, columns c0..c1-1
void house_left(RMat &M, int r0, int len, const double *v, double beta, int c0, int c1) {
  if (beta == 0.0) return;
  for (int j = c0; j < c1; ++j) {
    double t = 0.0;
    for (int i = 0; i < len; ++i) t += v[i] * M(r0 + i, j);
    t *= beta;
    for (int i = 0; i < len; ++i) M(r0 + i, j) -= t * v[i];
  }
}
// columns c0..c0+len-1 of M <- M (I - beta v v^T), rows r0..r1-1
void house_right(RMat &M, int c0, int len, const double *v, double beta, int r0, int r1) {
  if (beta == 0.0) return;
  for (int i = r0; i < r1; ++i) {
    double t = 0.0;
    for (int j = 0; j < len; ++j) t += M(i, c0 + j) * v[j];
    t *= beta;
    for (int j = 0; j < len; ++j) M(i, c0 + j) -= t * v[j];
  }
}
// rows (i, i+1) <- G [row i; row i+1] with G = [c s; -s c], columns c0..c1-1
void grot_rows(RMat &M, int i, double c, double s, int c0, int c1) {
  for (int j = c0; j < c1; ++j) {
    const double a = M(i, j), b = M(i + 1, j);
    M(i, j) = c * a + s * b;
    M(i + 1, j) = -s * a + c * b;
  }
}
// columns (j, j+1) <- [col j, col j+1] [c -s; s c], rows r0..r1-1
// (with (c, s) from (M(r, j+1), M(r, j)) this zeroes M(r, j))
void grot_cols(RMat &M, int j, double c, double s, int r0, int r1) {
  for (int i = r0; i < r1; ++i) {
    const double a = M(i, j), b = M(i, j + 1);
    M(i, j) = c * a - s * b;
    M(i, j + 1) = s * a + c * b;
  }
}
void givens_r(double a, double b, double &c, double &s) {
  const double r = std::hypot(a, b);
  if (r == 0.0) {
    c = 1.0;
    s = 0.0;
  } else {
    c = a / r;
    s = b / r;
  }
}
// zero B(r, j) against B(r, j+1) by a rotation of columns (j, j+1)
void zero_col_entry(RMat &B, RMat &A, RMat &Z, int r, int j, int arows, int brows) {
  double c, s;
  givens_r(B(r, j + 1), B(r, j), c, s);
  grot_cols(B, j, c, s, 0, brows);
  grot_cols(A, j, c, s, 0, arows);
  grot_cols(Z, j, c, s, 0, Z.m);
  B(r, j) = 0.0;
}

bool qz_real(RMat &A, RMat &B, RMat &Q, RMat &Z) {
  const int m = A.m;
  Q = RMat(m, m);
  Z = RMat(m, m);
  for (int i = 0; i < m; ++i) {
    Q(i, i) = 1.0;
    Z(i, i) = 1.0;
  }
  std::vector<double> x(m), v(m);
  // B = Q R
  for (int j = 0; j + 1 < m; ++j) {
    const int len = m - j;
    for (int i = 0; i < len; ++i) x[i] = B(j + i, j);
    double beta;
    house(x.data(), len, v.data(), beta);
    house_left(B, j, len, v.data(), beta, j, m);
    house_left(A, j, len, v.data(), beta, 0, m);
    house_right(Q, j, len, v.data(), beta, 0, m);
    for (int i = j + 1; i < m; ++i) B(i, j) = 0.0;
  }
  // A to Hessenberg form, B kept upper triangular
  for (int j = 0; j + 2 < m; ++j)
    for (int i = m - 1; i > j + 1; --i) {
      double c, s;
      givens_r(A(i - 1, j), A(i, j), c, s);
      grot_rows(A, i - 1, c, s, j, m);
      grot_rows(B, i - 1, c, s, i - 1, m);
      // Q <- Q G^T on columns (i-1, i)
      for (int r = 0; r < m; ++r) {
        const double a = Q(r, i - 1), b = Q(r, i);
        Q(r, i - 1) = c * a + s * b;
        Q(r, i) = -s * a + c * b;
      }
      A(i, j) = 0.0;
      zero_col_entry(B, A, Z, i, i - 1, m, i + 1);
    }
  double anorm = 0.0, bnorm = 0.0;
  for (double z : A.a) anorm = std::max(anorm, std::fabs(z));
  for (double z : B.a) bnorm = std::max(bnorm, std::fabs(z));
  if (anorm == 0.0) anorm = 1.0;
  if (bnorm == 0.0) bnorm = 1.0;
  int hi = m - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      const double sub = std::fabs(A(l, l - 1));
      if (sub <= kEps * (std::fabs(A(l - 1, l - 1)) + std::fabs(A(l, l))) || sub <= kEps * anorm * 1e-3) {
        A(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {  // 1 x 1 block
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {  // 2 x 2 block: kept (its eigenvalues come from the quadratic)
      hi -= 2;
      iter = 0;
      continue;
    }
    ++iter;
    if (++total > 60 * m) return false;
    // tiny diagonal entries of B: floored (infinite eigenvalues become huge)
    for (int i = l; i <= hi; ++i)
      if (std::fabs(B(i, i)) < kEps * bnorm) B(i, i) = B(i, i) < 0.0 ? -kEps * bnorm : kEps * bnorm;
    // shifts: eigenvalues of the trailing 2 x 2 block of M = A B^{-1}
    double sh, tt;
    {
      const double b11 = B(hi - 2, hi - 2), b12 = B(hi - 2, hi - 1), b13 = B(hi - 2, hi);
      const double b22 = B(hi - 1, hi - 1), b23 = B(hi - 1, hi), b33 = B(hi, hi);
      const double i12 = -b12 / (b11 * b22), i22 = 1.0 / b22;
      const double i13 = (b12 * b23 - b13 * b22) / (b11 * b22 * b33), i23 = -b23 / (b22 * b33), i33 = 1.0 / b33;
      const double m11 = A(hi - 1, hi - 2) * i12 + A(hi - 1, hi - 1) * i22;
      const double m12 = A(hi - 1, hi - 2) * i13 + A(hi - 1, hi - 1) * i23 + A(hi - 1, hi) * i33;
      const double m21 = A(hi, hi - 1) * i22;
      const double m22 = A(hi, hi - 1) * i23 + A(hi, hi) * i33;
      sh = m11 + m22;
      tt = m11 * m22 - m12 * m21;
      if (iter % 10 == 0) {  // exceptional shift
        const double w = std::fabs(A(hi, hi - 1) / B(hi - 1, hi - 1)) +
                         std::fabs(A(hi - 1, hi - 2) / B(hi - 2, hi - 2));
        sh = 1.5 * w;
        tt = w * w;
      }
    }
    // first column of (M - a1 I)(M - a2 I) restricted to rows l..l+2
    double v0, v1, v2;
    {
      const double bll = B(l, l), bl1 = B(l, l + 1), b22 = B(l + 1, l + 1);
      const double y1 = A(l, l) / bll, y2 = A(l + 1, l) / bll;
      const double u2 = y2 / b22, u1 = (y1 - bl1 * u2) / bll;
      const double w0 = A(l, l) * u1 + A(l, l + 1) * u2;
      const double w1 = A(l + 1, l) * u1 + A(l + 1, l + 1) * u2;
      const double w2 = A(l + 2, l + 1) * u2;
      v0 = w0 - sh * y1 + tt;
      v1 = w1 - sh * y2;
      v2 = w2;
      const double sc = std::max(std::fabs(v0), std::max(std::fabs(v1), std::fabs(v2)));
      if (sc > 0.0) {
        v0 /= sc;
        v1 /= sc;
        v2 /= sc;
      }
    }
    for (int k = l; k <= hi - 2; ++k) {
      if (k > l) {
        v0 = A(k, k - 1);
        v1 = A(k + 1, k - 1);
        v2 = A(k + 2, k - 1);
      }
      double xv[3] = {v0, v1, v2}, hv[3], beta;
      house(xv, 3, hv, beta);
      const int c0 = k > l ? k - 1 : l;
      house_left(A, k, 3, hv, beta, c0, m);
      house_left(B, k, 3, hv, beta, k, m);
      house_right(Q, k, 3, hv, beta, 0, m);
      if (k > l) {
        A(k + 1, k - 1) = 0.0;
        A(k + 2, k - 1) = 0.0;
      }
      // restore B: zero B(k+2, k), B(k+2, k+1) by a reflection of columns
      // k..k+2 built from the reversed row, then B(k+1, k) by a rotation
      {
        double xr[3] = {B(k + 2, k + 2), B(k + 2, k + 1), B(k + 2, k)}, vr[3], br;
        house(xr, 3, vr, br);
        double vv[3] = {vr[2], vr[1], vr[0]};
        const int ar = std::min(k + 4, hi + 1);
        house_right(B, k, 3, vv, br, 0, k + 3);
        house_right(A, k, 3, vv, br, 0, ar);
        house_right(Z, k, 3, vv, br, 0, m);
        B(k + 2, k) = 0.0;
        B(k + 2, k + 1) = 0.0;
        zero_col_entry(B, A, Z, k + 1, k, ar, k + 2);
      }
    }
    // last step: rows (hi-1, hi), then B(hi, hi-1)
    {
      double c, s;
      givens_r(A(hi - 1, hi - 2), A(hi, hi - 2), c, s);
      grot_rows(A, hi - 1, c, s, hi - 2, m);
      grot_rows(B, hi - 1, c, s, hi - 1, m);
      for (int r = 0; r < m; ++r) {
        const double a = Q(r, hi - 1), b = Q(r, hi);
        Q(r, hi - 1) = c * a + s * b;
        Q(r, hi) = -s * a + c * b;
      }
      A(hi, hi - 2) = 0.0;
      zero_col_entry(B, A, Z, hi, hi - 1, hi + 1, hi + 1);
    }
  }
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) {
      B(i, j) = 0.0;
      if (i > j + 1) A(i, j) = 0.0;
    }
  return true;
}

// Generalized real Schur form and eigenvalues (blk[i] = 1 when i starts a
// 2 x 2 block, 2 for its second row, 0 for a 1 x 1 block).
struct RPencil {
  RMat S, T, Q, Z;
  std::vector<cplx> lam;
  std::vector<int> blk;
};
bool rpencil_schur(const CMat &P, const CMat &Qc, RPencil &ps) {
  const int m = P.m;
  RMat A(m, m), B(m, m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      A(i, j) = P(i, j).real();
      B(i, j) = Qc(i, j).real();
    }
  if (!qz_real(A, B, ps.Q, ps.Z)) return false;
  ps.S = A;
  ps.T = B;
  ps.lam.assign(m, cplx(0.0));
  ps.blk.assign(m, 0);
  for (int i = 0; i < m;) {
    if (i + 1 < m && A(i + 1, i) != 0.0) {
      ps.blk[i] = 1;
      ps.blk[i + 1] = 2;
      // det(S_b - lambda T_b) = 0, T_b upper triangular
      const double s11 = A(i, i), s12 = A(i, i + 1), s21 = A(i + 1, i), s22 = A(i + 1, i + 1);
      const double t11 = B(i, i), t12 = B(i, i + 1), t22 = B(i + 1, i + 1);
      const double qa = t11 * t22, qb = -(s11 * t22 + s22 * t11 - s21 * t12), qc = s11 * s22 - s12 * s21;
      const cplx disc = std::sqrt(cplx(qb * qb - 4.0 * qa * qc, 0.0));
      if (qa == 0.0) {
        ps.lam[i] = ps.lam[i + 1] = cplx(INFINITY, 0.0);
      } else {
        // the root of larger modulus from the stable form, the other from the product
        const cplx q = -0.5 * (cplx(qb, 0.0) + (qb >= 0.0 ? disc : -disc));
        cplx r1 = q / qa, r2 = q != cplx(0.0) ? cplx(qc, 0.0) / q : cplx(0.0);
        if (r1.imag() < r2.imag() || (r1.imag() == r2.imag() && r1.real() < r2.real())) std::swap(r1, r2);
        ps.lam[i] = r1;
        ps.lam[i + 1] = r2;
      }
      i += 2;
    } else {
      ps.lam[i] = B(i, i) != 0.0 ? cplx(A(i, i) / B(i, i), 0.0) : cplx(INFINITY, 0.0);
      ++i;
    }
  }
  return true;
}

// Right (w: P w = lambda Q w) and left (y: y^H P = lambda y^H Q) eigenvectors
// of the eigenvalue indices in `want`, by complex back- and forward
// substitution on the quasi-triangular form.
void rpencil_vectors(const RPencil &ps, const std::vector<int> &want, CMat &W, CMat &Y) {
  const RMat &S = ps.S, &T = ps.T;
  const int m = S.m, nw = (int)want.size();
  double snorm = 0;
  for (double z : S.a) snorm = std::max(snorm, std::fabs(z));
  for (double z : T.a) snorm = std::max(snorm, std::fabs(z));
  const double small = std::max(snorm * kEps, 1e-300);
  W = CMat(m, nw);
  Y = CMat(m, nw);
  std::vector<cplx> yr(m), yl(m);
  auto D = [&](int i, int j, cplx lj) { return cplx(S(i, j), 0.0) - lj * T(i, j); };
  auto solve2 = [&](cplx a, cplx b, cplx c, cplx d, cplx r0, cplx r1, cplx &x0, cplx &x1) {
    cplx det = a * d - b * c;
    if (cabs(det) < small * small) det = small * small;
    x0 = (r0 * d - b * r1) / det;
    x1 = (a * r1 - c * r0) / det;
  };
  for (int cidx = 0; cidx < nw; ++cidx) {
    const int j = want[cidx];
    const cplx lj = ps.lam[j];
    const int js = ps.blk[j] == 2 ? j - 1 : j;             // first row of j's block
    const int je = ps.blk[j] == 1 || ps.blk[j] == 2 ? js + 1 : j;  // last row
    std::fill(yr.begin(), yr.end(), cplx(0.0));
    std::fill(yl.begin(), yl.end(), cplx(0.0));
    // right vector: null vector of the block, then rows js-1 .. 0
    if (js == je) {
      yr[js] = 1.0;
    } else {
      const cplx a = D(js, js, lj), b = D(js, je, lj), c = D(je, js, lj), d = D(je, je, lj);
      if (cabs(a) + cabs(b) >= cabs(c) + cabs(d)) {
        yr[js] = -b;
        yr[je] = a;
      } else {
        yr[js] = d;
        yr[je] = -c;
      }
    }
    for (int i = js - 1; i >= 0;) {
      if (ps.blk[i] == 2) {  // rows (i-1, i) form a block
        cplx r0 = 0, r1 = 0;
        for (int q = i + 1; q <= je; ++q) {
          r0 -= D(i - 1, q, lj) * yr[q];
          r1 -= D(i, q, lj) * yr[q];
        }
        solve2(D(i - 1, i - 1, lj), D(i - 1, i, lj), D(i, i - 1, lj), D(i, i, lj), r0, r1, yr[i - 1], yr[i]);
        i -= 2;
      } else {
        cplx acc = 0;
        for (int q = i + 1; q <= je; ++q) acc += D(i, q, lj) * yr[q];
        cplx d = D(i, i, lj);
        if (cabs(d) < small) d = small;
        yr[i] = -acc / d;
        --i;
      }
    }
    // left vector: u^H (S - lam T) = 0, i.e. (S - lam T)^H u = 0, supported on js..m-1
    if (js == je) {
      yl[js] = 1.0;
    } else {
      // rows of (S - lam T)^H on the block: conj of the block's columns
      const cplx a = std::conj(D(js, js, lj)), b = std::conj(D(je, js, lj));
      const cplx c = std::conj(D(js, je, lj)), d = std::conj(D(je, je, lj));
      if (cabs(a) + cabs(b) >= cabs(c) + cabs(d)) {
        yl[js] = -b;
        yl[je] = a;
      } else {
        yl[js] = d;
        yl[je] = -c;
      }
    }
    for (int i = je + 1; i < m;) {
      if (ps.blk[i] == 1) {  // rows (i, i+1) form a block
        cplx r0 = 0, r1 = 0;
        for (int q = js; q < i; ++q) {
          r0 -= std::conj(D(q, i, lj)) * yl[q];
          r1 -= std::conj(D(q, i + 1, lj)) * yl[q];
        }
        solve2(std::conj(D(i, i, lj)), std::conj(D(i + 1, i, lj)), std::conj(D(i, i + 1, lj)),
               std::conj(D(i + 1, i + 1, lj)), r0, r1, yl[i], yl[i + 1]);
        i += 2;
      } else {
        cplx acc = 0;
        for (int q = js; q < i; ++q) acc += std::conj(D(q, i, lj)) * yl[q];
        cplx d = std::conj(D(i, i, lj));
        if (cabs(d) < small) d = small;
        yl[i] = -acc / d;
        ++i;
      }
    }
    for (int i = 0; i < m; ++i) {
      cplx a = 0, b = 0;
      for (int l = 0; l <= je; ++l) a += ps.Z(i, l) * yr[l];
      for (int l = js; l < m; ++l) b += ps.Q(i, l) * yl[l];
      W(i, cidx) = a;
      Y(i, cidx) = b;
    }
  }
  normalize_cols(W);
  normalize_cols(Y);
}

bool is_real(const CMat &M) {
  for (const cplx &z : M.a)
    if (z.imag() != 0.0) return false;
  return true;
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
  std::vector<cplx> ev;
  CMat X, Y;
  std::vector<int> all(m);
  std::iota(all.begin(), all.end(), 0);
  if (is_real(Pm) && is_real(Qm)) {
    RPencil rp;
    if (!rpencil_schur(Pm, Qm, rp)) return rbicg_fail(-1, "host_eig: QZ iteration did not converge");
    ev = rp.lam;
    if (W || Wl) rpencil_vectors(rp, all, X, Y);
  } else {
    PencilSchur ps;
    if (!pencil_schur(Pm, Qm, ps)) return rbicg_fail(-1, "host_eig: QZ iteration did not converge");
    ev = ps.lam;
    if (W || Wl) pencil_vectors(ps, all, X, Y);
  }
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
  int ncols = 0;
  std::vector<SelItem> sel;
  CMat W, Y;
  if (is_real(Pm) && is_real(Qm)) {
    RPencil rp;
    if (!rpencil_schur(Pm, Qm, rp)) return rbicg_fail(-1, "host_eig_select: QZ iteration did not converge");
    sel = select_indices(rp.lam, k, real_problem != 0, ncols);
    std::vector<int> want;
    for (const auto &it : sel) want.push_back(it.idx);
    rpencil_vectors(rp, want, W, Y);
  } else {
    PencilSchur ps;
    if (!pencil_schur(Pm, Qm, ps)) return rbicg_fail(-1, "host_eig_select: QZ iteration did not converge");
    sel = select_indices(ps.lam, k, real_problem != 0, ncols);
    std::vector<int> want;
    for (const auto &it : sel) want.push_back(it.idx);
    pencil_vectors(ps, want, W, Y);
  }
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

// Real counterparts of herm_jacobi, svd_jacobi and whitening for real Gram
// matrices (real problems): the same rotations, with the phase e = a_pq / |a_pq|
// reduced to a sign, in real arithmetic (a quarter of the complex work).
void sym_jacobi(RMat A, std::vector<double> &w, RMat &V) {
  const int m = A.m;
  V = RMat(m, m);
  for (int i = 0; i < m; ++i) V(i, i) = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        tot += A(i, j) * A(i, j);
        if (i != j) off += A(i, j) * A(i, j);
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A(p, q), b = std::fabs(apq);
        if (b == 0.0) continue;
        const double app = A(p, p), aqq = A(q, q), e = apq / b;
        const double tau = (aqq - app) / (2.0 * b);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        const double se = sn * e, ce = c * e;
        for (int r = 0; r < m; ++r) {
          const double akp = A(r, p), akq = A(r, q);
          A(r, p) = c * akp - se * akq;
          A(r, q) = sn * akp + ce * akq;
        }
        for (int r = 0; r < m; ++r) {
          const double apk = A(p, r), aqk = A(q, r);
          A(p, r) = c * apk - se * aqk;
          A(q, r) = sn * apk + ce * aqk;
        }
        for (int r = 0; r < m; ++r) {
          const double vkp = V(r, p), vkq = V(r, q);
          V(r, p) = c * vkp - se * vkq;
          V(r, q) = sn * vkp + ce * vkq;
        }
      }
  }
  w.resize(m);
  for (int i = 0; i < m; ++i) w[i] = A(i, i);
  std::vector<int> idx(m);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] < w[b]; });
  RMat V2(m, m);
  std::vector<double> w2(m);
  for (int j = 0; j < m; ++j) {
    w2[j] = w[idx[j]];
    for (int i = 0; i < m; ++i) V2(i, j) = V(i, idx[j]);
  }
  w = w2;
  V = V2;
}

void svd_jacobi_real(const RMat &A, RMat &U, std::vector<double> &s, RMat &V) {
  const int m = A.m, n = A.n;
  U = A;
  V = RMat(n, n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double alpha = 0, beta = 0, gamma = 0;
        for (int i = 0; i < m; ++i) {
          alpha += U(i, p) * U(i, p);
          beta += U(i, q) * U(i, q);
          gamma += U(i, p) * U(i, q);
        }
        const double g = std::fabs(gamma);
        if (g == 0.0 || g <= 1e-15 * std::sqrt(alpha * beta)) continue;
        rotated = true;
        const double e = gamma / g;
        const double tau = (beta - alpha) / (2.0 * g);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        const double se = sn * e, ce = c * e;
        for (int i = 0; i < m; ++i) {
          const double up = U(i, p), uq = U(i, q);
          U(i, p) = c * up - se * uq;
          U(i, q) = sn * up + ce * uq;
        }
        for (int i = 0; i < n; ++i) {
          const double vp = V(i, p), vq = V(i, q);
          V(i, p) = c * vp - se * vq;
          V(i, q) = sn * vp + ce * vq;
        }
      }
    if (!rotated) break;
  }
  s.resize(n);
  for (int j = 0; j < n; ++j) {
    double t = 0;
    for (int i = 0; i < m; ++i) t += U(i, j) * U(i, j);
    s[j] = std::sqrt(t);
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return s[a] > s[b]; });
  RMat U2(m, n), V2(n, n);
  std::vector<double> s2(n);
  for (int j = 0; j < n; ++j) {
    const int o = idx[j];
    s2[j] = s[o];
    for (int i = 0; i < m; ++i) U2(i, j) = (s[o] > 0) ? U(i, o) / s[o] : (i == j ? 1.0 : 0.0);
    for (int i = 0; i < n; ++i) V2(i, j) = V(i, o);
  }
  U = U2;
  V = V2;
  s = s2;
}

RMat load_real(int m, int n, const double *p) {
  RMat A(m, n);
  for (size_t t = 0; t < (size_t)m * n; ++t) A.a[t] = p[2 * t];
  return A;
}
RMat whitening_real(const RMat &G) {
  std::vector<double> w;
  RMat V;
  sym_jacobi(G, w, V);
  const int k = G.m;
  double wmax = 0;
  for (double x : w) wmax = std::max(wmax, x);
  std::vector<int> keep;
  for (int i = k - 1; i >= 0; --i)
    if (w[i] > 1e-13 * wmax && w[i] > 0) keep.push_back(i);
  RMat L(k, (int)keep.size());
  for (size_t j = 0; j < keep.size(); ++j) {
    const double f = 1.0 / std::sqrt(w[keep[j]]);
    for (int i = 0; i < k; ++i) L(i, (int)j) = V(i, keep[j]) * f;
  }
  return L;
}
RMat mul_real(const RMat &A, const RMat &B, bool transA = false) {
  const int m = transA ? A.n : A.m, kk = transA ? A.m : A.n;
  RMat C(m, B.n);
  for (int j = 0; j < B.n; ++j)
    for (int i = 0; i < m; ++i) {
      double s = 0;
      for (int l = 0; l < kk; ++l) s += (transA ? A(l, i) : A(i, l)) * B(l, j);
      C(i, j) = s;
    }
  return C;
}
bool all_real(int k, const double *G) {
  for (size_t t = 0; t < (size_t)k * k; ++t)
    if (G[2 * t + 1] != 0.0) return false;
  return true;
}

// rbicg_host_biorth for real Grams (same steps, real arithmetic)
int biorth_real(int k, const double *Gcc, const double *Gtt, const double *Gtc, double tol,
                double *TU, double *TUt) {
  RMat L = whitening_real(load_real(k, k, Gcc));
  RMat Lt = whitening_real(load_real(k, k, Gtt));
  if (L.n == 0 || Lt.n == 0) return 0;
  RMat K = mul_real(Lt, mul_real(load_real(k, k, Gtc), L), true);  // Q~^T Q
  RMat M, N;
  std::vector<double> sv;
  if (K.m >= K.n) {
    svd_jacobi_real(K, M, sv, N);
  } else {
    RMat KT(K.n, K.m);
    for (int i = 0; i < K.m; ++i)
      for (int j = 0; j < K.n; ++j) KT(j, i) = K(i, j);
    svd_jacobi_real(KT, N, sv, M);
  }
  int p = 0;
  for (double x : sv)
    if (std::isfinite(x) && x >= tol) ++p;
  for (int j = 0; j < p; ++j) {
    const double f = 1.0 / std::sqrt(sv[j]);
    for (int i = 0; i < k; ++i) {
      double a = 0, b = 0;
      for (int l = 0; l < L.n; ++l) a += L(i, l) * N(l, j);
      for (int l = 0; l < Lt.n; ++l) b += Lt(i, l) * M(l, j);
      TU[2 * (i + j * k)] = a * f;
      TU[2 * (i + j * k) + 1] = 0.0;
      TUt[2 * (i + j * k)] = b * f;
      TUt[2 * (i + j * k) + 1] = 0.0;
    }
  }
  return p;
}
}  // namespace

extern "C" int rbicg_host_biorth(int32_t k, const double *Gcc, const double *Gtt,
                                 const double *Gtc, double tol, double *TU, double *TUt) {
  if (k <= 0 || !Gcc || !Gtt || !Gtc || !TU || !TUt) return rbicg_fail(-1, "host_biorth: bad arguments");
  if (all_real(k, Gcc) && all_real(k, Gtt) && all_real(k, Gtc))
    return biorth_real(k, Gcc, Gtt, Gtc, tol, TU, TUt);
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
