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

bool finite(cplx z) { return std::isfinite(z.real()) && std::isfinite(z.imag()); }

}  // namespace

extern "C" int rbicg_host_eig(int32_t m, const double *P, const double *Q, double *lam,
                              double *W, double *Wl) {
  if (m <= 0 || !P) return rbicg_fail(-1, "host_eig: bad arguments");
  CMat Pm = load(m, m, P);
  CMat M = Pm;
  CMat Qm;
  if (Q) {
    Qm = load(m, m, Q);
    if (!lu_solve(Qm, M)) return rbicg_fail(-1, "host_eig: Q is singular");
  }
  std::vector<cplx> ev;
  CMat X;
  if (!eig_general(M, ev, X)) return rbicg_fail(-1, "host_eig: QR iteration did not converge");
  if (lam)
    for (int i = 0; i < m; ++i) { lam[2 * i] = ev[i].real(); lam[2 * i + 1] = ev[i].imag(); }
  if (W) store(X, W);
  if (Wl) {
    // y^H P = lambda y^H Q  <=>  y = Q^{-H} g with g the columns of X^{-H}.
    CMat Xi;
    if (!inverse(X, Xi)) return rbicg_fail(-1, "host_eig: eigenvector matrix is singular");
    CMat G(m, m);  // X^{-H}
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) G(i, j) = std::conj(Xi(j, i));
    if (Q) {
      CMat QH(m, m);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) QH(i, j) = std::conj(Qm(j, i));
      if (!lu_solve(QH, G)) return rbicg_fail(-1, "host_eig: Q is singular");
    }
    normalize_cols(G);
    store(G, Wl);
  }
  return 0;
}

extern "C" int rbicg_host_select(int32_t m, const double *lamp, const double *Wp,
                                 const double *Wlp, int32_t k, int32_t real_problem,
                                 double *Wsel, double *Wlsel) {
  if (m <= 0 || k < 0 || !lamp || !Wp || !Wsel) return rbicg_fail(-1, "host_select: bad arguments");
  std::vector<cplx> lam(m);
  for (int i = 0; i < m; ++i) lam[i] = cplx(lamp[2 * i], lamp[2 * i + 1]);
  CMat W = load(m, m, Wp);
  CMat Wl;
  if (Wlp) Wl = load(m, m, Wlp);
  std::vector<int> order;
  for (int i = 0; i < m; ++i)
    if (finite(lam[i])) order.push_back(i);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    double ma = std::abs(lam[a]), mb = std::abs(lam[b]);
    if (ma != mb) return ma < mb;
    if (lam[a].real() != lam[b].real()) return lam[a].real() < lam[b].real();
    if (lam[a].imag() != lam[b].imag()) return lam[a].imag() < lam[b].imag();
    return a < b;
  });
  std::vector<std::vector<cplx>> cols, lcols;
  auto column = [&](const CMat &A, int j) {
    std::vector<cplx> c(m);
    for (int i = 0; i < m; ++i) c[i] = A(i, j);
    return c;
  };
  // phase that makes the largest entry real positive
  auto dephase = [&](std::vector<cplx> c) {
    int im = 0;
    for (int i = 1; i < m; ++i)
      if (std::abs(c[i]) > std::abs(c[im])) im = i;
    cplx ph = (std::abs(c[im]) > 0) ? std::conj(c[im]) / std::abs(c[im]) : cplx(1.0);
    for (auto &z : c) z = cplx((z * ph).real(), 0.0);
    return c;
  };
  auto repart = [&](const std::vector<cplx> &c, bool imagpart) {
    std::vector<cplx> o(m);
    for (int i = 0; i < m; ++i) o[i] = imagpart ? cplx(c[i].imag(), 0.0) : cplx(c[i].real(), 0.0);
    return o;
  };
  if (!real_problem) {
    for (size_t t = 0; t < order.size() && (int)cols.size() < k; ++t) {
      cols.push_back(column(W, order[t]));
      if (Wlp) lcols.push_back(column(Wl, order[t]));
    }
  } else {
    double scale = 1.0;
    for (int i : order) scale = std::max(scale, std::abs(lam[i]));
    std::vector<char> used(m, 0);
    for (size_t t = 0; t < order.size() && (int)cols.size() < k; ++t) {
      int i = order[t];
      if (used[i]) continue;
      if (std::fabs(lam[i].imag()) <= 1e-9 * std::max(std::abs(lam[i]), 1e-300)) {
        used[i] = 1;
        cols.push_back(dephase(column(W, i)));
        if (Wlp) lcols.push_back(dephase(column(Wl, i)));
        continue;
      }
      int jbest = -1;
      double dbest = 0;
      for (int j : order) {
        if (used[j] || j == i) continue;
        double d = std::abs(lam[j] - std::conj(lam[i]));
        if (jbest < 0 || d < dbest) { jbest = j; dbest = d; }
      }
      if (jbest < 0) break;
      if (dbest > 1e-8 * scale) {
        used[i] = 1;
        cols.push_back(repart(column(W, i), false));
        if (Wlp) lcols.push_back(repart(column(Wl, i), false));
        continue;
      }
      if ((int)cols.size() + 2 > k) break;
      used[i] = used[jbest] = 1;
      int ip = lam[i].imag() > 0 ? i : jbest;
      auto w = column(W, ip);
      cols.push_back(repart(w, false));
      cols.push_back(repart(w, true));
      if (Wlp) {
        auto wl = column(Wl, ip);
        lcols.push_back(repart(wl, false));
        lcols.push_back(repart(wl, true));
      }
    }
  }
  for (size_t j = 0; j < cols.size(); ++j)
    for (int i = 0; i < m; ++i) {
      Wsel[2 * (i + j * m)] = cols[j][i].real();
      Wsel[2 * (i + j * m) + 1] = cols[j][i].imag();
      if (Wlp && Wlsel) {
        Wlsel[2 * (i + j * m)] = lcols[j][i].real();
        Wlsel[2 * (i + j * m) + 1] = lcols[j][i].imag();
      }
    }
  return (int)cols.size();
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
