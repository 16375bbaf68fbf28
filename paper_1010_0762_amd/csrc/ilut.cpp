// Host ILUT factorization and level schedules (see ilut.h).
#include "ilut.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <queue>
#include <string>

#include "errors.h"
#include "rbicg_hostla.h"

namespace ilut {

int factor(const Csr &A, double tau, int p, Csr &L, Csr &U, std::string &msg) {
  const int n = A.n;
  // column 2-norms of A
  std::vector<double> cn(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) cn[A.ci[e]] += std::norm(A.v[e]);
  for (auto &c : cn) c = std::sqrt(c);
  L = Csr();
  U = Csr();
  L.n = U.n = n;
  L.rp.assign(1, 0);
  U.rp.assign(1, 0);
  std::vector<int> udiag(n, -1);   // position of u_kk in U
  std::vector<cplx> w(n, 0.0);     // working row
  std::vector<int> mark(n, -1);    // mark[j] == i: column j is in the working row
  std::vector<int> upper;          // columns >= i of the working row
  std::priority_queue<int, std::vector<int>, std::greater<int>> heap;  // columns < i, ascending
  std::vector<std::pair<int, cplx>> lrow, urow;
  for (int i = 0; i < n; ++i) {
    upper.clear();
    lrow.clear();
    urow.clear();
    for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int j = A.ci[e];
      if (mark[j] != i) {
        mark[j] = i;
        w[j] = 0.0;
        if (j < i) heap.push(j);
        else upper.push_back(j);
      }
      w[j] += A.v[e];
    }
    while (!heap.empty()) {
      const int k = heap.top();
      heap.pop();
      cplx wk = w[k];
      w[k] = 0.0;
      if (std::abs(wk) < tau * cn[k]) continue;  // dropped: no update
      wk /= U.v[udiag[k]];
      lrow.emplace_back(k, wk);
      for (int e = udiag[k] + 1; e < U.rp[k + 1]; ++e) {
        const int j = U.ci[e];
        if (mark[j] != i) {
          mark[j] = i;
          w[j] = 0.0;
          if (j < i) heap.push(j);
          else upper.push_back(j);
        }
        w[j] -= wk * U.v[e];
      }
    }
    cplx d = 0.0;
    for (int j : upper) {
      if (j == i) d = w[j];
      else if (std::abs(w[j]) >= tau * cn[j]) urow.emplace_back(j, w[j]);
    }
    if (d == cplx(0.0)) {
      msg = "ILUT: zero pivot in row " + std::to_string(i);
      return -1;
    }
    auto limit = [p](std::vector<std::pair<int, cplx>> &row) {
      if (p >= 0 && (int)row.size() > p) {
        std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) {
          const double ma = std::abs(a.second), mb = std::abs(b.second);
          return ma != mb ? ma > mb : a.first < b.first;
        });
        row.resize(p);
      }
      std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    };
    limit(lrow);
    limit(urow);
    for (auto &t : lrow) {
      L.ci.push_back(t.first);
      L.v.push_back(t.second);
    }
    L.rp.push_back((int)L.ci.size());
    udiag[i] = (int)U.ci.size();
    U.ci.push_back(i);
    U.v.push_back(d);
    for (auto &t : urow) {
      U.ci.push_back(t.first);
      U.v.push_back(t.second);
    }
    U.rp.push_back((int)U.ci.size());
  }
  return 0;
}

int factor_pivoted(const Csr &A, double tau, int p, double permtol, Csr &L, Csr &U,
                   std::vector<int> &perm, std::string &msg) {
  const int n = A.n;
  std::vector<double> cn(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) cn[A.ci[e]] += std::norm(A.v[e]);
  for (auto &c : cn) c = std::sqrt(c);
  perm.resize(n);
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) perm[i] = pos[i] = i;
  // U rows in columns of A: off-pivot entries and the pivot apart
  std::vector<std::vector<std::pair<int, cplx>>> urows(n);
  std::vector<cplx> piv(n);
  L = Csr();
  L.n = n;
  L.rp.assign(1, 0);
  std::vector<cplx> w(n, 0.0);
  std::vector<int> mark(n, -1);
  std::vector<int> upper;
  std::priority_queue<int, std::vector<int>, std::greater<int>> heap;  // positions < i
  std::vector<std::pair<int, cplx>> lrow, urow;
  for (int i = 0; i < n; ++i) {
    upper.clear();
    lrow.clear();
    urow.clear();
    auto touch = [&](int c) {
      if (mark[c] != i) {
        mark[c] = i;
        w[c] = 0.0;
        if (pos[c] < i) heap.push(pos[c]);
        else upper.push_back(c);
      }
    };
    for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      touch(A.ci[e]);
      w[A.ci[e]] += A.v[e];
    }
    while (!heap.empty()) {
      const int k = heap.top();
      heap.pop();
      const int c = perm[k];
      cplx wk = w[c];
      w[c] = 0.0;
      if (std::abs(wk) < tau * cn[c]) continue;  // dropped: no update
      wk /= piv[k];
      lrow.emplace_back(k, wk);
      for (const auto &t : urows[k]) {
        touch(t.first);
        w[t.first] -= wk * t.second;
      }
    }
    int dcol = perm[i];
    const cplx wd = mark[dcol] == i ? w[dcol] : cplx(0.0);
    // kept remaining entries (the unpivoted diagonal always)
    std::vector<int> kept;
    for (int c : upper)
      if (c == dcol || std::abs(w[c]) >= tau * cn[c]) kept.push_back(c);
    int best = dcol;
    double bmod = std::abs(wd);
    for (int c : kept) {
      const double m = std::abs(w[c]);
      if (m > bmod || (m == bmod && pos[c] < pos[best])) {
        best = c;
        bmod = m;
      }
    }
    if (best != dcol && bmod * permtol > std::abs(wd)) {
      const int j = pos[best];
      perm[i] = best;
      perm[j] = dcol;
      pos[best] = i;
      pos[dcol] = j;
      dcol = best;
    }
    const cplx d = mark[dcol] == i ? w[dcol] : cplx(0.0);
    if (d == cplx(0.0)) {
      msg = "ILUTP: zero pivot in row " + std::to_string(i);
      return -1;
    }
    for (int c : kept)
      if (c != dcol) urow.emplace_back(c, w[c]);
    if (p >= 0 && (int)lrow.size() > p) {
      std::sort(lrow.begin(), lrow.end(), [](const auto &a, const auto &b) {
        const double ma = std::abs(a.second), mb = std::abs(b.second);
        return ma != mb ? ma > mb : a.first < b.first;
      });
      lrow.resize(p);
    }
    std::sort(lrow.begin(), lrow.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    if (p >= 0 && (int)urow.size() > p) {
      std::sort(urow.begin(), urow.end(), [&](const auto &a, const auto &b) {
        const double ma = std::abs(a.second), mb = std::abs(b.second);
        return ma != mb ? ma > mb : pos[a.first] < pos[b.first];
      });
      urow.resize(p);
    }
    for (auto &t : lrow) {
      L.ci.push_back(t.first);
      L.v.push_back(t.second);
    }
    L.rp.push_back((int)L.ci.size());
    urows[i] = urow;
    piv[i] = d;
  }
  // U in positions, columns ascending, pivot first
  U = Csr();
  U.n = n;
  U.rp.assign(1, 0);
  std::vector<std::pair<int, cplx>> row;
  for (int i = 0; i < n; ++i) {
    row.clear();
    row.emplace_back(i, piv[i]);
    for (const auto &t : urows[i]) row.emplace_back(pos[t.first], t.second);
    std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (auto &t : row) {
      U.ci.push_back(t.first);
      U.v.push_back(t.second);
    }
    U.rp.push_back((int)U.ci.size());
  }
  return 0;
}

Csr conj_transpose(const Csr &T) {
  Csr R;
  R.n = T.n;
  R.rp.assign(T.n + 1, 0);
  for (int c : T.ci) ++R.rp[c + 1];
  for (int i = 0; i < T.n; ++i) R.rp[i + 1] += R.rp[i];
  R.ci.resize(T.ci.size());
  R.v.resize(T.v.size());
  std::vector<int> pos(R.rp.begin(), R.rp.end() - 1);
  for (int i = 0; i < T.n; ++i)
    for (int e = T.rp[i]; e < T.rp[i + 1]; ++e) {
      const int q = pos[T.ci[e]]++;
      R.ci[q] = i;
      R.v[q] = std::conj(T.v[e]);
    }
  return R;
}

int levels(const Csr &T, bool lower, int pad, std::vector<int> &order) {
  const int n = T.n;
  std::vector<int> lev(n, 0);
  int nl = 0;
  auto visit = [&](int i) {
    int l = 0;
    for (int e = T.rp[i]; e < T.rp[i + 1]; ++e) {
      const int j = T.ci[e];
      if (lower ? j < i : j > i) l = std::max(l, lev[j] + 1);
    }
    lev[i] = l;
    nl = std::max(nl, l + 1);
  };
  if (lower)
    for (int i = 0; i < n; ++i) visit(i);
  else
    for (int i = n - 1; i >= 0; --i) visit(i);
  std::vector<std::vector<int>> by(nl);
  for (int i = 0; i < n; ++i) by[lev[i]].push_back(i);
  order.clear();
  for (auto &rows : by) {
    order.insert(order.end(), rows.begin(), rows.end());
    while (order.size() % pad) order.push_back(-1);
  }
  return nl;
}

}  // namespace ilut

// ------------------------------------------------------------- C exports

namespace {
int load_host(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, ilut::Csr &A) {
  if (n <= 0 || !rp || !ci || !v || rp[0] != 0) return -1;
  A.n = n;
  A.rp.assign(rp, rp + n + 1);
  for (int i = 0; i < n; ++i)
    if (A.rp[i + 1] < A.rp[i]) return -1;
  const int nnz = A.rp[n];
  A.ci.assign(ci, ci + nnz);
  for (int c : A.ci)
    if (c < 0 || c >= n) return -1;
  A.v.resize(nnz);
  for (int e = 0; e < nnz; ++e) A.v[e] = ilut::cplx(v[2 * e], v[2 * e + 1]);
  return 0;
}

void store(const ilut::Csr &T, int32_t *rp, int32_t *ci, double *v) {
  for (size_t i = 0; i < T.rp.size(); ++i) rp[i] = T.rp[i];
  for (size_t e = 0; e < T.ci.size(); ++e) {
    ci[e] = T.ci[e];
    v[2 * e] = T.v[e].real();
    v[2 * e + 1] = T.v[e].imag();
  }
}
}  // namespace

extern "C" int rbicg_host_ilut(int32_t n, const int32_t *rowptr, const int32_t *colind,
                               const double *values, double tau, int32_t p, double permtol,
                               int64_t *nnz, int32_t *Lrp, int32_t *Lci, double *Lv, int32_t *Urp,
                               int32_t *Uci, double *Uv, int32_t *perm) {
  ilut::Csr A, L, U;
  if (!nnz || load_host(n, rowptr, colind, values, A) < 0 || !(tau >= 0.0) || !(permtol >= 0.0))
    return rbicg_fail(-1, "host_ilut: bad arguments");
  std::string msg;
  std::vector<int> pv;
  const int rc = permtol > 0.0 ? ilut::factor_pivoted(A, tau, p, permtol, L, U, pv, msg)
                               : ilut::factor(A, tau, p, L, U, msg);
  if (rc < 0) return rbicg_fail(-1, "%s", msg.c_str());
  nnz[0] = (int64_t)L.ci.size();
  nnz[1] = (int64_t)U.ci.size();
  if (Lrp && Lci && Lv) store(L, Lrp, Lci, Lv);
  if (Urp && Uci && Uv) store(U, Urp, Uci, Uv);
  if (perm)
    for (int i = 0; i < n; ++i) perm[i] = pv.empty() ? i : pv[i];
  return 0;
}

extern "C" int rbicg_host_levels(int32_t n, const int32_t *rowptr, const int32_t *colind,
                                 int32_t lower, int32_t pad, int32_t *order, int64_t *len) {
  if (n <= 0 || !rowptr || !colind || !len || pad <= 0) return rbicg_fail(-1, "host_levels: bad arguments");
  ilut::Csr T;
  T.n = n;
  T.rp.assign(rowptr, rowptr + n + 1);
  T.ci.assign(colind, colind + T.rp[n]);
  for (int c : T.ci)
    if (c < 0 || c >= n) return rbicg_fail(-1, "host_levels: column index out of range");
  std::vector<int> ord;
  const int nl = ilut::levels(T, lower != 0, pad, ord);
  *len = (int64_t)ord.size();
  if (order) std::copy(ord.begin(), ord.end(), order);
  return nl;
}
