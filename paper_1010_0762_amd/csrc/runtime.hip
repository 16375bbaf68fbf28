// Host runtime of librbicg: handle, matrix repacking, the RBiCG solve driver
// (Algorithm 2) and the cycle-wise recycle-space update (Sec. 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rbicg.h"
#include "rbicg_hostla.h"
#include "device.h"
#include "errors.h"
#include "kernels.h"

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

int rbicg_fail(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

extern "C" const char *rbicg_last_error(void) { return g_last_error.c_str(); }

#define HIPCHECK(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return rbicg_fail(RBICG_EHIP, "%s failed at %s:%d: %s", #call, __FILE__, __LINE__, \
                        hipGetErrorString(e_));                                          \
  } while (0)

#define TRY(call)                 \
  do {                            \
    int rc_ = (call);             \
    if (rc_ < 0) return rc_;      \
  } while (0)

using cplx = std::complex<double>;

namespace {

// ------------------------------------------------------------ device matrix
struct DevSell {
  int n = 0, nslices = 0;
  int *sliceptr = nullptr;
  int *col = nullptr;
  void *val = nullptr;
  size_t nnzpad = 0;
  int64_t nnz = 0;
  int vbytes = 0;
  template <class M> Sell<M> view() const {
    Sell<M> s;
    s.n = n;
    s.nslices = nslices;
    s.sliceptr = sliceptr;
    s.col = col;
    s.val = (const M *)val;
    return s;
  }
  void release() {
    if (sliceptr) (void)hipFree(sliceptr);
    if (col) (void)hipFree(col);
    if (val) (void)hipFree(val);
    sliceptr = nullptr;
    col = nullptr;
    val = nullptr;
  }
};

// Host CSR with complex values (real matrices have zero imaginary parts).
struct HostCsr {
  int n = 0;
  std::vector<int> rowptr, col;
  std::vector<cplx> val;
  bool complex_vals = false;
};

int read_csr(const rbicg_csr *A, HostCsr &out) {
  if (!A || A->n <= 0 || A->nnz < 0 || !A->rowptr || (A->nnz > 0 && (!A->colind || !A->values)))
    return rbicg_fail(RBICG_EINVAL, "invalid CSR descriptor");
  if (A->nnz >= (int64_t)1 << 31) return rbicg_fail(RBICG_EINVAL, "nnz exceeds int32 range");
  const int n = A->n;
  const size_t nnz = (size_t)A->nnz;
  out.n = n;
  out.complex_vals = A->values_complex != 0;
  out.rowptr.resize(n + 1);
  out.col.resize(nnz);
  std::vector<double> raw(nnz * (out.complex_vals ? 2 : 1));
  if (A->on_device) {
    HIPCHECK(hipMemcpy(out.rowptr.data(), A->rowptr, (n + 1) * sizeof(int), hipMemcpyDeviceToHost));
    if (nnz) {
      HIPCHECK(hipMemcpy(out.col.data(), A->colind, nnz * sizeof(int), hipMemcpyDeviceToHost));
      HIPCHECK(hipMemcpy(raw.data(), A->values, raw.size() * sizeof(double), hipMemcpyDeviceToHost));
    }
  } else {
    std::memcpy(out.rowptr.data(), A->rowptr, (n + 1) * sizeof(int));
    if (nnz) {
      std::memcpy(out.col.data(), A->colind, nnz * sizeof(int));
      std::memcpy(raw.data(), A->values, raw.size() * sizeof(double));
    }
  }
  if (out.rowptr[0] != 0 || (size_t)out.rowptr[n] != nnz)
    return rbicg_fail(RBICG_EINVAL, "CSR row pointers do not span nnz");
  for (int i = 0; i < n; ++i)
    if (out.rowptr[i + 1] < out.rowptr[i]) return rbicg_fail(RBICG_EINVAL, "CSR row pointers decrease");
  for (size_t e = 0; e < nnz; ++e)
    if (out.col[e] < 0 || out.col[e] >= n) return rbicg_fail(RBICG_EINVAL, "CSR column index out of range");
  out.val.resize(nnz);
  for (size_t e = 0; e < nnz; ++e)
    out.val[e] = out.complex_vals ? cplx(raw[2 * e], raw[2 * e + 1]) : cplx(raw[e], 0.0);
  return 0;
}

// Conjugate transpose by a counting sort over columns (O(nnz)).
HostCsr conj_transpose(const HostCsr &A) {
  HostCsr T;
  T.n = A.n;
  T.complex_vals = A.complex_vals;
  T.rowptr.assign(A.n + 1, 0);
  for (int c : A.col) T.rowptr[c + 1]++;
  for (int i = 0; i < A.n; ++i) T.rowptr[i + 1] += T.rowptr[i];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int> fill(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int i = 0; i < A.n; ++i)
    for (int e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
      const int c = A.col[e];
      const int d = fill[c]++;
      T.col[d] = i;
      T.val[d] = std::conj(A.val[e]);
    }
  return T;
}

// Repack CSR into the wave-sliced ELL layout and upload.  vkind: 0 double,
// 1 complex double, 2 float.
int upload_sell(const HostCsr &A, int vkind, DevSell &D) {
  const int n = A.n;
  const int ns = (n + RBICG_WAVE - 1) / RBICG_WAVE;
  std::vector<int> sp(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    int w = 0;
    for (int r = s * RBICG_WAVE; r < std::min(n, (s + 1) * RBICG_WAVE); ++r)
      w = std::max(w, A.rowptr[r + 1] - A.rowptr[r]);
    if ((int64_t)sp[s] + (int64_t)w * RBICG_WAVE >= ((int64_t)1 << 31))
      return rbicg_fail(RBICG_EINVAL, "padded matrix exceeds int32 range");
    sp[s + 1] = sp[s] + w * RBICG_WAVE;
  }
  const size_t total = (size_t)sp[ns];
  std::vector<int> col(total);
  const int vb = vkind == 1 ? 16 : (vkind == 0 ? 8 : 4);
  std::vector<unsigned char> val(total * vb, 0);
  for (int s = 0; s < ns; ++s) {
    const int w = (sp[s + 1] - sp[s]) / RBICG_WAVE;
    for (int lane = 0; lane < RBICG_WAVE; ++lane) {
      const int r = s * RBICG_WAVE + lane;
      const int rr = std::min(r, n - 1);
      const int len = r < n ? A.rowptr[r + 1] - A.rowptr[r] : 0;
      for (int j = 0; j < w; ++j) {
        const size_t e = (size_t)sp[s] + (size_t)j * RBICG_WAVE + lane;
        if (j < len) {
          const int src = A.rowptr[r] + j;
          col[e] = A.col[src];
          const cplx v = A.val[src];
          if (vkind == 0) {
            double d = v.real();
            std::memcpy(&val[e * 8], &d, 8);
          } else if (vkind == 1) {
            double d[2] = {v.real(), v.imag()};
            std::memcpy(&val[e * 16], d, 16);
          } else {
            float f = (float)v.real();
            std::memcpy(&val[e * 4], &f, 4);
          }
        } else {
          col[e] = rr;
        }
      }
    }
  }
  D.release();
  D.n = n;
  D.nslices = ns;
  D.nnzpad = total;
  D.nnz = (int64_t)A.col.size();
  D.vbytes = vb;
  HIPCHECK(hipMalloc(&D.sliceptr, (ns + 1) * sizeof(int)));
  HIPCHECK(hipMalloc(&D.col, std::max<size_t>(total, 1) * sizeof(int)));
  HIPCHECK(hipMalloc(&D.val, std::max<size_t>(total, 1) * vb));
  HIPCHECK(hipMemcpy(D.sliceptr, sp.data(), (ns + 1) * sizeof(int), hipMemcpyHostToDevice));
  if (total) {
    HIPCHECK(hipMemcpy(D.col, col.data(), total * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(D.val, val.data(), total * vb, hipMemcpyHostToDevice));
  }
  return 0;
}

}  // namespace

// ====================================================================== handle
struct rbicg_s {
  rbicg_opts opt{};
  int n = 0;
  int ld = 0;
  hipStream_t st = nullptr;
  int vkind = 0;  // 0 double, 1 complex
  bool mat_complex = false;
  size_t vb = 8;
  int kcap = 0, scap = 0;
  DevSell A, AH;
  // iteration vectors (x, x~ are the caller's)
  void *r = nullptr, *rt = nullptr, *p[2] = {nullptr, nullptr}, *pt[2] = {nullptr, nullptr};
  void *z = nullptr, *zt = nullptr, *q = nullptr, *qt = nullptr, *t1 = nullptr, *t2 = nullptr;
  // recycle space of the current system
  void *U = nullptr, *Ut = nullptr, *C = nullptr, *Ct = nullptr;
  int ksys = 0;
  // recycle space built by the cycles (double-buffered)
  void *Uc[2] = {}, *Utc[2] = {}, *Cc[2] = {}, *Ctc[2] = {};
  int kcyc = 0, cur = 0;
  bool have_cyc = false;
  // scratch for U_j before biorthogonalization
  void *Ua = nullptr, *Uta = nullptr, *Ca = nullptr, *Cta = nullptr;
  // cycle rings: raw residuals r_{i-1} (s slots) and z_i (s+1 slots)
  void *R = nullptr, *Rt = nullptr, *Z = nullptr, *Zt = nullptr;
  Scalars *S = nullptr;
  double *log = nullptr;
  int logcap = 0;
  double *partial = nullptr;
  double *gpart = nullptr;
  size_t gpart_bytes = 0;
  double *Gd = nullptr;
  cd *Wd = nullptr;
  // pinned host staging
  Scalars *hS = nullptr;
  double *hG = nullptr;
  cd *hW = nullptr;
  double *hlog = nullptr;
  // last solve's log (host copy) for rbicg_get_log
  std::vector<double> last_log;
  int last_count = 0;
  std::vector<void *> allocs;
};

namespace {

int dalloc(rbicg_s *h, void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) return rbicg_fail(RBICG_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  h->allocs.push_back(*p);
  return 0;
}

inline char *col_ptr(void *base, int j, const rbicg_s *h) {
  return (char *)base + (size_t)j * h->ld * h->vb;
}

int sync(rbicg_s *h) {
  HIPCHECK(hipStreamSynchronize(h->st));
  return 0;
}

int pull_scalars(rbicg_s *h) {
  HIPCHECK(hipMemcpyAsync(h->hS, h->S, sizeof(Scalars), hipMemcpyDeviceToHost, h->st));
  return sync(h);
}
int push_scalars(rbicg_s *h) {
  HIPCHECK(hipMemcpyAsync(h->S, h->hS, sizeof(Scalars), hipMemcpyHostToDevice, h->st));
  return 0;
}

// bytes per algorithmic iteration (matrix streams + 29 vector streams + C, C~ twice)
double alg_bytes_iter(const rbicg_s *h, int k) {
  const double ba = (double)h->A.vbytes;
  const double nnz = (double)h->A.nnz;
  const double n = h->n;
  return 2.0 * (nnz * (ba + 4.0) + 4.0 * (n + 1.0)) + (29.0 + 4.0 * k) * n * (double)h->vb;
}

// ---------------------------------------------------------- typed helpers
template <class V> struct VK;
template <> struct VK<double> { static constexpr int kind = 0; };
template <> struct VK<cd> { static constexpr int kind = 1; };

// Gram G = X^H Y (mx x my, complex, row-major by (i, j)) into h->hG.
template <class V>
int gram(rbicg_s *h, const std::vector<const void *> &X, const std::vector<const void *> &Y) {
  const int mx = (int)X.size(), my = (int)Y.size();
  if (mx > RBICG_MAXCOLS || my > RBICG_MAXCOLS) return rbicg_fail(RBICG_EINVAL, "gram too wide");
  ColList xl{}, yl{};
  for (int i = 0; i < mx; ++i) xl.p[i] = X[i];
  for (int i = 0; i < my; ++i) yl.p[i] = Y[i];
  int nchunks = std::max(1, std::min(64, (h->n + 4095) / 4096));
  const size_t need = (size_t)nchunks * mx * my * 2 * sizeof(double);
  if (need > h->gpart_bytes) return rbicg_fail(RBICG_EINVAL, "gram workspace too small");
  launch_gram<V>(h->st, h->n, xl, mx, yl, my, h->gpart, h->Gd, nchunks);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(h->hG, h->Gd, (size_t)mx * my * 2 * sizeof(double), hipMemcpyDeviceToHost, h->st));
  return sync(h);
}
inline cplx G_at(const rbicg_s *h, int my, int i, int j) {
  const double *g = h->hG + ((size_t)i * my + j) * 2;
  return cplx(g[0], g[1]);
}

// Y (ld columns) = X W with W given on the host (m x p, column-major, complex).
template <class V>
int tsgemm(rbicg_s *h, const std::vector<const void *> &X, const std::vector<cplx> &W, int p,
           void *Y) {
  const int m = (int)X.size();
  if (m > RBICG_MAXCOLS) return rbicg_fail(RBICG_EINVAL, "tsgemm too wide");
  if (p == 0 || m == 0) return 0;
  // the staging buffer may still be read by a previous GEMM on the stream
  TRY(sync(h));
  for (int t = 0; t < m * p; ++t) h->hW[t] = cd{W[t].real(), W[t].imag()};
  HIPCHECK(hipMemcpyAsync(h->Wd, h->hW, (size_t)m * p * sizeof(cd), hipMemcpyHostToDevice, h->st));
  ColList xl{};
  for (int i = 0; i < m; ++i) xl.p[i] = X[i];
  launch_tsgemm<V>(h->st, h->n, xl, m, h->Wd, p, (V *)Y, h->ld);
  HIPCHECK(hipGetLastError());
  return 0;
}

template <class V, class M> struct MatOf;

// Apply the biorthogonalization of Sec. 4.3 to U_j = Ua, U~_j = Uta (m columns):
// C = A U, C~ = A^H U~, Grams, host SVD, and write the biorthogonal pair
// (p columns) to (Uo, Uto, Co, Cto).  Returns p (>= 0) or an error.
template <class V, class M>
int biorth(rbicg_s *h, int m, void *Uo, void *Uto, void *Co, void *Cto) {
  if (m == 0) return 0;
  Sell<M> A = h->A.view<M>(), AH = h->AH.view<M>();
  launch_spmm<V, M>(h->st, A, (const V *)h->Ua, (V *)h->Ca, h->ld, m);
  launch_spmm<V, M>(h->st, AH, (const V *)h->Uta, (V *)h->Cta, h->ld, m);
  HIPCHECK(hipGetLastError());
  std::vector<const void *> X;
  for (int j = 0; j < m; ++j) X.push_back(col_ptr(h->Ca, j, h));
  for (int j = 0; j < m; ++j) X.push_back(col_ptr(h->Cta, j, h));
  TRY(gram<V>(h, X, X));
  const int w = 2 * m;
  std::vector<double> Gcc(2 * m * m), Gtt(2 * m * m), Gtc(2 * m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      // column-major (i, j) for the host routines
      cplx a = G_at(h, w, i, j), b = G_at(h, w, m + i, m + j), c = G_at(h, w, m + i, j);
      Gcc[2 * (i + j * m)] = a.real(); Gcc[2 * (i + j * m) + 1] = a.imag();
      Gtt[2 * (i + j * m)] = b.real(); Gtt[2 * (i + j * m) + 1] = b.imag();
      Gtc[2 * (i + j * m)] = c.real(); Gtc[2 * (i + j * m) + 1] = c.imag();
    }
  std::vector<double> TU(2 * m * m), TUt(2 * m * m);
  const int p = rbicg_host_biorth(m, Gcc.data(), Gtt.data(), Gtc.data(), h->opt.svd_tol,
                                  TU.data(), TUt.data());
  if (p < 0) return rbicg_fail(RBICG_EINVAL, "biorthogonalization failed: %s", rbicg_last_error());
  if (p == 0) return 0;
  std::vector<cplx> W(m * p), Wt(m * p);
  for (int t = 0; t < m * p; ++t) {
    W[t] = cplx(TU[2 * t], TU[2 * t + 1]);
    Wt[t] = cplx(TUt[2 * t], TUt[2 * t + 1]);
  }
  std::vector<const void *> XU, XC, XUt, XCt;
  for (int j = 0; j < m; ++j) {
    XU.push_back(col_ptr(h->Ua, j, h));
    XC.push_back(col_ptr(h->Ca, j, h));
    XUt.push_back(col_ptr(h->Uta, j, h));
    XCt.push_back(col_ptr(h->Cta, j, h));
  }
  TRY(tsgemm<V>(h, XU, W, p, Uo));
  TRY(tsgemm<V>(h, XC, W, p, Co));
  TRY(tsgemm<V>(h, XUt, Wt, p, Uto));
  TRY(tsgemm<V>(h, XCt, Wt, p, Cto));
  TRY(sync(h));
  return p;
}

// One log entry of iteration i (1-based, global index within the solve).
struct LogEntry {
  cplx alpha, beta_prev, rho;
  double rn, rtn;
};

// End of a cycle (Sec. 4): build U_j, U~_j from the ring and the logged
// scalars, then biorthogonalize into the cycle buffers.
template <class V, class M>
int cycle_update(rbicg_s *h, int e, int run_start, double rn0, cplx rho0) {
  const int s = h->opt.s;
  const bool real_problem = (VK<V>::kind == 0);
  // pull log entries e-s .. e (entry run_start is the run's initial state)
  const int lo = e - s;
  HIPCHECK(hipMemcpyAsync(h->hlog, h->log + (size_t)lo * LOG_STRIDE,
                          (size_t)(s + 1) * LOG_STRIDE * sizeof(double), hipMemcpyDeviceToHost, h->st));
  TRY(sync(h));
  std::vector<LogEntry> L(s + 1);
  for (int t = 0; t <= s; ++t) {
    const double *q = h->hlog + (size_t)t * LOG_STRIDE;
    L[t].alpha = cplx(q[0], q[1]);
    L[t].beta_prev = cplx(q[2], q[3]);
    L[t].rho = cplx(q[4], q[5]);
    L[t].rn = q[6];
    L[t].rtn = q[7];
  }
  if (lo == run_start) {
    L[0].rn = rn0;
    L[0].rho = rho0;
  }
  // cycle iteration c (0..s-1) is i = lo + 1 + c; ||r_{i-1}|| = L[c].rn, rho_{i-1} = L[c].rho
  std::vector<double> a(s);
  std::vector<cplx> at(s), alpha(s), beta(s);
  for (int c = 0; c < s; ++c) {
    a[c] = 1.0 / L[c].rn;
    at[c] = L[c].rn / std::conj(L[c].rho);
    alpha[c] = L[c + 1].alpha;
    beta[c] = L[c + 1].beta_prev;
  }
  const int k = h->opt.k;
  int m = 0;
  std::vector<cplx> Wc, Wtc;
  std::vector<const void *> XU, XUt;
  if (!h->have_cyc && h->ksys == 0) {
    // first cycle of the first system: eigenvectors of T_s (Sec. 4.2)
    std::vector<double> T(2 * s * s, 0.0);
    auto setT = [&](int i, int j, cplx v) {
      T[2 * (i + j * s)] = v.real();
      T[2 * (i + j * s) + 1] = v.imag();
    };
    for (int i = 1; i <= s; ++i) {
      cplx d = 1.0 / alpha[i - 1];
      if (i >= 2) {
        d += beta[i - 1] / alpha[i - 2];
        setT(i - 2, i - 1, -(L[i - 2].rn / L[i - 1].rn) * beta[i - 1] / alpha[i - 2]);
      }
      setT(i - 1, i - 1, d);
      if (i <= s - 1) setT(i, i - 1, -(L[i].rn / L[i - 1].rn) / alpha[i - 1]);
    }
    std::vector<double> lam(2 * s), W(2 * s * s), Wl(2 * s * s), Ws(2 * s * s), Wls(2 * s * s);
    if (rbicg_host_eig(s, T.data(), nullptr, lam.data(), W.data(), Wl.data()) != 0)
      return rbicg_fail(RBICG_EINVAL, "cycle eigenproblem failed: %s", rbicg_last_error());
    m = rbicg_host_select(s, lam.data(), W.data(), Wl.data(), k, real_problem ? 1 : 0, Ws.data(), Wls.data());
    if (m < 0) return m;
    Wc.resize(s * m);
    Wtc.resize(s * m);
    for (int c = 0; c < m; ++c)
      for (int l = 0; l < s; ++l) {
        Wc[l + c * s] = a[l] * cplx(Ws[2 * (l + c * s)], Ws[2 * (l + c * s) + 1]);
        Wtc[l + c * s] = at[l] * cplx(Wls[2 * (l + c * s)], Wls[2 * (l + c * s) + 1]);
      }
    for (int c = 0; c < s; ++c) {
      XU.push_back(col_ptr(h->R, c, h));
      XUt.push_back(col_ptr(h->Rt, c, h));
    }
  } else {
    // Phi = [U_prev, V_j]; harmonic Ritz pencil of eq. finalGenEigValue
    void *Up = h->have_cyc ? h->Uc[h->cur] : h->U;
    void *Utp = h->have_cyc ? h->Utc[h->cur] : h->Ut;
    void *Cp = h->have_cyc ? h->Cc[h->cur] : h->C;
    void *Ctp = h->have_cyc ? h->Ctc[h->cur] : h->Ct;
    const int kp = h->have_cyc ? h->kcyc : h->ksys;
    const int mm = kp + s;       // columns of Phi
    const int mz = kp + s + 1;   // columns of [C_prev, Z ring]
    std::vector<const void *> X1, Y1, Y2;
    for (int j = 0; j < kp; ++j) {
      X1.push_back(col_ptr(Ctp, j, h));
      Y1.push_back(col_ptr(Cp, j, h));
      Y2.push_back(col_ptr(Up, j, h));
      XU.push_back(col_ptr(Up, j, h));
      XUt.push_back(col_ptr(Utp, j, h));
    }
    for (int c = 0; c <= s; ++c) {
      X1.push_back(col_ptr(h->Zt, c, h));
      Y1.push_back(col_ptr(h->Z, c, h));
    }
    for (int c = 0; c < s; ++c) {
      Y2.push_back(col_ptr(h->R, c, h));
      XU.push_back(col_ptr(h->R, c, h));
      XUt.push_back(col_ptr(h->Rt, c, h));
    }
    // transforms: A Phi = [C_p, Z] B, A^H Phi~ = [C~_p, Z~] Bt, Phi = [U_p, R] D
    std::vector<cplx> B((size_t)mz * mm, 0.0), Bt((size_t)mz * mm, 0.0), D((size_t)mm * mm, 0.0);
    for (int j = 0; j < kp; ++j) {
      B[j + (size_t)j * mz] = 1.0;
      Bt[j + (size_t)j * mz] = 1.0;
      D[j + (size_t)j * mm] = 1.0;
    }
    for (int c = 0; c < s; ++c) {
      const int col = kp + c;
      B[(kp + c + 1) + (size_t)col * mz] = a[c];
      B[(kp + c) + (size_t)col * mz] = -beta[c] * a[c];
      Bt[(kp + c + 1) + (size_t)col * mz] = at[c];
      Bt[(kp + c) + (size_t)col * mz] = -std::conj(beta[c]) * at[c];
      D[col + (size_t)col * mm] = a[c];
    }
    TRY(gram<V>(h, X1, Y1));
    std::vector<cplx> G1((size_t)mz * mz);
    for (int i = 0; i < mz; ++i)
      for (int j = 0; j < mz; ++j) G1[i + (size_t)j * mz] = G_at(h, mz, i, j);
    TRY(gram<V>(h, X1, Y2));
    std::vector<cplx> G2((size_t)mz * mm);
    for (int i = 0; i < mz; ++i)
      for (int j = 0; j < mm; ++j) G2[i + (size_t)j * mz] = G_at(h, mm, i, j);
    // P = Bt^H G1 B, Q = Bt^H G2 D
    auto mulH = [&](const std::vector<cplx> &Lm, int lr, int lc, const std::vector<cplx> &Mm,
                    int mc) {  // Lm^H (lr x lc)^H * Mm (lr x mc) -> lc x mc
      std::vector<cplx> O((size_t)lc * mc, 0.0);
      for (int j = 0; j < mc; ++j)
        for (int i = 0; i < lc; ++i) {
          cplx sacc = 0;
          for (int l = 0; l < lr; ++l) sacc += std::conj(Lm[l + (size_t)i * lr]) * Mm[l + (size_t)j * lr];
          O[i + (size_t)j * lc] = sacc;
        }
      return O;
    };
    auto mul = [&](const std::vector<cplx> &Lm, int lr, int lc, const std::vector<cplx> &Mm,
                   int mc) {  // (lr x lc) * (lc x mc)
      std::vector<cplx> O((size_t)lr * mc, 0.0);
      for (int j = 0; j < mc; ++j)
        for (int l = 0; l < lc; ++l) {
          const cplx f = Mm[l + (size_t)j * lc];
          if (f == 0.0) continue;
          for (int i = 0; i < lr; ++i) O[i + (size_t)j * lr] += Lm[i + (size_t)l * lr] * f;
        }
      return O;
    };
    std::vector<cplx> P = mulH(Bt, mz, mm, mul(G1, mz, mz, B, mm), mm);
    std::vector<cplx> Q = mulH(Bt, mz, mm, mul(G2, mz, mm, D, mm), mm);
    std::vector<double> Pd(2 * (size_t)mm * mm), Qd(2 * (size_t)mm * mm);
    for (size_t t = 0; t < (size_t)mm * mm; ++t) {
      Pd[2 * t] = P[t].real(); Pd[2 * t + 1] = P[t].imag();
      Qd[2 * t] = Q[t].real(); Qd[2 * t + 1] = Q[t].imag();
    }
    std::vector<double> lam(2 * mm), W(2 * (size_t)mm * mm), Wl(2 * (size_t)mm * mm),
        Ws(2 * (size_t)mm * mm), Wls(2 * (size_t)mm * mm);
    if (rbicg_host_eig(mm, Pd.data(), Qd.data(), lam.data(), W.data(), Wl.data()) != 0)
      return rbicg_fail(RBICG_EINVAL, "harmonic Ritz problem failed: %s", rbicg_last_error());
    m = rbicg_host_select(mm, lam.data(), W.data(), Wl.data(), k, real_problem ? 1 : 0, Ws.data(), Wls.data());
    if (m < 0) return m;
    std::vector<cplx> Wsel((size_t)mm * m), Wlsel((size_t)mm * m);
    for (size_t t = 0; t < (size_t)mm * m; ++t) {
      Wsel[t] = cplx(Ws[2 * t], Ws[2 * t + 1]);
      Wlsel[t] = cplx(Wls[2 * t], Wls[2 * t + 1]);
    }
    // U_j = [U_p, R] (D W), U~_j = [U~_p, R~] (Dt W~), Dt = blockdiag(I, diag(at))
    Wc = mul(D, mm, mm, Wsel, m);
    std::vector<cplx> Dt((size_t)mm * mm, 0.0);
    for (int j = 0; j < kp; ++j) Dt[j + (size_t)j * mm] = 1.0;
    for (int c = 0; c < s; ++c) Dt[(kp + c) + (size_t)(kp + c) * mm] = at[c];
    Wtc = mul(Dt, mm, mm, Wlsel, m);
  }
  if (m == 0) return 0;
  TRY(tsgemm<V>(h, XU, Wc, m, h->Ua));
  TRY(tsgemm<V>(h, XUt, Wtc, m, h->Uta));
  const int nxt = h->have_cyc ? 1 - h->cur : h->cur;
  const int p = biorth<V, M>(h, m, h->Uc[nxt], h->Utc[nxt], h->Cc[nxt], h->Ctc[nxt]);
  if (p < 0) return p;
  if (p > 0) {
    h->cur = nxt;
    h->kcyc = p;
    h->have_cyc = true;
  }
  return 0;
}

// ------------------------------------------------------------------ solve
template <class V, class M>
int solve_impl(rbicg_s *h, const V *b, const V *bt, V *x, V *xt, double tol, rbicg_stats *stp) {
  rbicg_stats st{};
  const int n = h->n, ld = h->ld, s = h->opt.s;
  Sell<M> A = h->A.view<M>(), AH = h->AH.view<M>();
  hipEvent_t ev0, ev1;
  HIPCHECK(hipEventCreate(&ev0));
  HIPCHECK(hipEventCreate(&ev1));
  HIPCHECK(hipEventRecord(ev0, h->st));
  const bool update = h->opt.update && h->opt.k > 0;
  h->have_cyc = false;
  V *r = (V *)h->r, *rt = (V *)h->rt;
  const int ks = h->ksys;
  const V *U = (const V *)h->U, *Ut = (const V *)h->Ut, *C = (const V *)h->C, *Ct = (const V *)h->Ct;
  // reference norms
  launch_dots<V>(h->st, n, b, b, bt, bt, nullptr, nullptr, h->partial, h->S);
  HIPCHECK(hipGetLastError());
  TRY(pull_scalars(h));
  double bn = std::sqrt(std::fabs(h->hS->red[0])), btn = std::sqrt(std::fabs(h->hS->red[2]));
  int total = 0, restarts = 0, reseeds = 0, status = ST_MAXIT;
  double relres = NAN, relres_dual = NAN;
  bool first = true;
  std::vector<double> fulllog;
  while (true) {
    // eq. minusXR: r_{-1} = b - A x, projection with C, C~
    launch_residual<V, M>(h->st, A, b, x, r);
    launch_residual<V, M>(h->st, AH, bt, xt, rt);
    if (first && (bn == 0.0 || btn == 0.0)) {
      launch_dots<V>(h->st, n, r, r, rt, rt, nullptr, nullptr, h->partial, h->S);
      TRY(pull_scalars(h));
      if (bn == 0.0) bn = std::sqrt(std::fabs(h->hS->red[0]));
      if (btn == 0.0) btn = std::sqrt(std::fabs(h->hS->red[2]));
      if (bn == 0.0) bn = 1.0;
      if (btn == 0.0) btn = 1.0;
    }
    if (ks > 0) {
      launch_restrict<V>(h->st, n, r, Ct, rt, C, ks, ld, h->partial, h->S);
      launch_expand2<V>(h->st, n, x, U, 1.0, r, C, -1.0, xt, Ut, 1.0, rt, Ct, -1.0, ks, ld, 0, h->S);
    }
    launch_dots<V>(h->st, n, rt, r, r, r, rt, rt, h->partial, h->S);
    HIPCHECK(hipGetLastError());
    TRY(pull_scalars(h));
    cplx rho(h->hS->red[0], h->hS->red[1]);
    double rn = std::sqrt(std::fabs(h->hS->red[2])), rtn = std::sqrt(std::fabs(h->hS->red[4]));
    // Algorithm 2 step 3: re-seed x~ if (r_0, r~_0) vanishes
    while (std::abs(rho) <= 1e-14 * rn * rtn && rn > 0 && reseeds < 3) {
      launch_reseed<V>(h->st, xt, (size_t)n, (unsigned long long)(h->opt.seed + reseeds));
      launch_residual<V, M>(h->st, AH, bt, xt, rt);
      if (ks > 0) {
        launch_restrict<V>(h->st, n, r, Ct, rt, C, ks, ld, h->partial, h->S);
        launch_expand2<V>(h->st, n, nullptr, U, 0.0, nullptr, C, 0.0, xt, Ut, 1.0, rt, Ct, -1.0, ks, ld, 0, h->S);
      }
      launch_dots<V>(h->st, n, rt, r, r, r, rt, rt, h->partial, h->S);
      TRY(pull_scalars(h));
      rho = cplx(h->hS->red[0], h->hS->red[1]);
      rn = std::sqrt(std::fabs(h->hS->red[2]));
      rtn = std::sqrt(std::fabs(h->hS->red[4]));
      ++reseeds;
    }
    first = false;
    const int run_start = total;
    // scalar block for the run
    Scalars *hs = h->hS;
    std::memset(hs, 0, sizeof(Scalars));
    hs->rho = cd{rho.real(), rho.imag()};
    hs->tol = tol;
    hs->bn = bn;
    hs->btn = btn;
    hs->rn = rn;
    hs->rtn = rtn;
    hs->iter = total;
    hs->maxit = h->opt.maxit;
    hs->log_base = 0;
    bool conv0 = rn <= tol * bn && rtn <= tol * btn;
    hs->done = conv0 ? 1 : 0;
    hs->status = conv0 ? ST_CONVERGED : ST_RUNNING;
    if (total >= h->opt.maxit && !conv0) {
      hs->done = 1;
      hs->status = ST_MAXIT;
    }
    TRY(push_scalars(h));
    launch_fill_zero<V>(h->st, (V *)h->p[0], (size_t)n);
    launch_fill_zero<V>(h->st, (V *)h->pt[0], (size_t)n);
    if (update) {
      launch_fill_zero<V>(h->st, (V *)h->Z, (size_t)ld);
      launch_fill_zero<V>(h->st, (V *)h->Zt, (size_t)ld);
    }
    int pc = 0;
    int launched = total;  // iterations enqueued
    int done = hs->done, dev_status = hs->status;
    const int chunk_def = h->opt.chunk > 0 ? h->opt.chunk : 8;
    while (!done) {
      int in_run = launched - run_start;
      int chunk = chunk_def;
      if (update) chunk = std::min(chunk, s - (in_run % s));
      chunk = std::min(chunk, h->opt.maxit - launched);
      if (chunk <= 0) break;
      for (int c = 0; c < chunk; ++c) {
        const int pos = (launched - run_start) % s;
        V *capR = nullptr, *capRt = nullptr, *capZ = nullptr, *capZt = nullptr;
        if (update) {
          capR = (V *)col_ptr(h->R, pos, h);
          capRt = (V *)col_ptr(h->Rt, pos, h);
          capZ = (V *)col_ptr(h->Z, pos + 1, h);
          capZt = (V *)col_ptr(h->Zt, pos + 1, h);
        }
        V *pn = (V *)h->p[1 - pc], *ptn = (V *)h->pt[1 - pc];
        launch_iter_spmv<V, M>(h->st, A, AH, r, (const V *)h->p[pc], rt, (const V *)h->pt[pc], pn, ptn,
                               (V *)h->z, (V *)h->zt, C, Ct, ks, ld, capR, capRt, capZ, capZt,
                               h->partial, h->S);
        launch_iter_expand<V>(h->st, n, (const V *)h->z, (const V *)h->zt, C, Ct, ks, ld, ptn,
                              (V *)h->q, (V *)h->qt, h->partial, h->S);
        const V *qq = ks > 0 ? (const V *)h->q : (const V *)h->z;
        const V *qqt = ks > 0 ? (const V *)h->qt : (const V *)h->zt;
        launch_iter_update<V>(h->st, n, x, xt, r, rt, pn, ptn, qq, qqt, h->partial, h->S, h->log);
        pc = 1 - pc;
        ++launched;
      }
      HIPCHECK(hipGetLastError());
      TRY(pull_scalars(h));
      done = h->hS->done;
      dev_status = h->hS->status;
      const int it = h->hS->iter;
      // no-op launches after convergence do not advance the count or the parity
      if (it != launched) {
        if ((launched - it) % 2) pc = 1 - pc;
        launched = it;
      }
      if (update && it > run_start && (it - run_start) % s == 0 &&
          (dev_status == ST_RUNNING || dev_status == ST_CONVERGED || dev_status == ST_MAXIT)) {
        TRY((cycle_update<V, M>(h, it, run_start, rn, rho)));
        st.cycles++;
        // z_{js} becomes slot 0 of the next cycle
        HIPCHECK(hipMemcpyAsync(h->Z, col_ptr(h->Z, s, h), (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
        HIPCHECK(hipMemcpyAsync(h->Zt, col_ptr(h->Zt, s, h), (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
      }
    }
    total = h->hS->iter;
    status = h->hS->status;
    // keep this run's log
    if (total > run_start) {
      std::vector<double> tmp((size_t)(total - run_start) * LOG_STRIDE);
      HIPCHECK(hipMemcpy(tmp.data(), h->log + (size_t)(run_start + 1) * LOG_STRIDE,
                         tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (size_t t = 0; t < tmp.size(); t += LOG_STRIDE) tmp[t + 8] = restarts;
      fulllog.insert(fulllog.end(), tmp.begin(), tmp.end());
    }
    // Algorithm 2 step 7: x -= U zeta_c, x~ -= U~ zeta~_c
    if (ks > 0)
      launch_expand2<V>(h->st, n, x, U, -1.0, nullptr, C, 0.0, xt, Ut, -1.0, nullptr, Ct, 0.0, ks, ld, 1, h->S);
    // true residuals
    launch_residual<V, M>(h->st, A, b, x, (V *)h->t1);
    launch_residual<V, M>(h->st, AH, bt, xt, (V *)h->t2);
    launch_dots<V>(h->st, n, (V *)h->t1, (V *)h->t1, (V *)h->t2, (V *)h->t2, nullptr, nullptr, h->partial, h->S);
    HIPCHECK(hipGetLastError());
    TRY(pull_scalars(h));
    const double tr = std::sqrt(std::fabs(h->hS->red[0])), trt = std::sqrt(std::fabs(h->hS->red[2]));
    relres = tr / bn;
    relres_dual = trt / btn;
    const bool true_ok = tr <= tol * bn && trt <= tol * btn;
    if (status == ST_CONVERGED && !true_ok && restarts < h->opt.max_restarts && total < h->opt.maxit) {
      ++restarts;
      continue;
    }
    if (status == ST_CONVERGED && !true_ok) status = ST_MAXIT;
    break;
  }
  HIPCHECK(hipEventRecord(ev1, h->st));
  HIPCHECK(hipEventSynchronize(ev1));
  float ms = 0;
  HIPCHECK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  h->last_log = fulllog;
  h->last_count = (int)(fulllog.size() / LOG_STRIDE);
  st.status = status == ST_CONVERGED ? RBICG_OK : (status == ST_BREAKDOWN ? RBICG_BREAKDOWN : RBICG_NOT_CONVERGED);
  st.iters = total;
  st.restarts = restarts;
  st.reseeds = reseeds;
  st.k_used = ks;
  st.relres = relres;
  st.relres_dual = relres_dual;
  st.time_ms = ms;
  st.alg_bytes = alg_bytes_iter(h, ks) * total;
  if (stp) *stp = st;
  return st.status;
}

template <class V, class M>
int install_recycle(rbicg_s *h, const void *Usrc, const void *Utsrc, int k) {
  if (k == 0) {
    h->ksys = 0;
    return 0;
  }
  if (Usrc != h->Ua) HIPCHECK(hipMemcpy2DAsync(h->Ua, h->ld * h->vb, Usrc, h->ld * h->vb, h->n * h->vb, k, hipMemcpyDeviceToDevice, h->st));
  if (Utsrc != h->Uta) HIPCHECK(hipMemcpy2DAsync(h->Uta, h->ld * h->vb, Utsrc, h->ld * h->vb, h->n * h->vb, k, hipMemcpyDeviceToDevice, h->st));
  const int p = biorth<V, M>(h, k, h->U, h->Ut, h->C, h->Ct);
  if (p < 0) return p;
  h->ksys = p;
  return 0;
}

template <class F>
int dispatch(rbicg_s *h, F &&f) {
  if (h->vkind == 0) return f((double *)nullptr, (double *)nullptr);
  if (h->mat_complex) return f((cd *)nullptr, (cd *)nullptr);
  return f((cd *)nullptr, (double *)nullptr);
}

int alloc_workspace(rbicg_s *h) {
  const size_t vbytes = (size_t)h->ld * h->vb;
  void **vecs[] = {&h->r, &h->rt, &h->p[0], &h->p[1], &h->pt[0], &h->pt[1], &h->z, &h->zt,
                   &h->q, &h->qt, &h->t1, &h->t2};
  for (void **v : vecs) TRY(dalloc(h, v, vbytes));
  const size_t kb = vbytes * std::max(1, h->kcap);
  void **bases[] = {&h->U, &h->Ut, &h->C, &h->Ct, &h->Ua, &h->Uta, &h->Ca, &h->Cta,
                    &h->Uc[0], &h->Utc[0], &h->Cc[0], &h->Ctc[0],
                    &h->Uc[1], &h->Utc[1], &h->Cc[1], &h->Ctc[1]};
  for (void **v : bases) TRY(dalloc(h, v, kb));
  if (h->kcap > 0 && h->opt.update) {
    TRY(dalloc(h, &h->R, vbytes * h->scap));
    TRY(dalloc(h, &h->Rt, vbytes * h->scap));
    TRY(dalloc(h, &h->Z, vbytes * (h->scap + 1)));
    TRY(dalloc(h, &h->Zt, vbytes * (h->scap + 1)));
  }
  TRY(dalloc(h, (void **)&h->S, sizeof(Scalars)));
  HIPCHECK(hipMemset(h->S, 0, sizeof(Scalars)));
  h->logcap = h->opt.maxit + 2;
  TRY(dalloc(h, (void **)&h->log, (size_t)h->logcap * LOG_STRIDE * sizeof(double)));
  const size_t nblocks = (h->n + RBICG_BLOCK - 1) / RBICG_BLOCK;
  TRY(dalloc(h, (void **)&h->partial, nblocks * 4 * KMAXD * sizeof(double)));
  const int w = std::max(2 * h->kcap, h->kcap + h->scap + 1);
  h->gpart_bytes = (size_t)64 * w * w * 2 * sizeof(double);
  TRY(dalloc(h, (void **)&h->gpart, h->gpart_bytes));
  TRY(dalloc(h, (void **)&h->Gd, (size_t)w * w * 2 * sizeof(double)));
  TRY(dalloc(h, (void **)&h->Wd, (size_t)RBICG_MAXCOLS * KMAXD * sizeof(cd)));
  HIPCHECK(hipHostMalloc((void **)&h->hS, sizeof(Scalars), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&h->hG, (size_t)w * w * 2 * sizeof(double), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&h->hW, (size_t)RBICG_MAXCOLS * KMAXD * sizeof(cd), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&h->hlog, (size_t)(h->scap + 2) * LOG_STRIDE * sizeof(double), hipHostMallocDefault));
  return 0;
}

int set_matrix(rbicg_s *h, const rbicg_csr *A, const rbicg_csr *AH) {
  HostCsr hA, hAH;
  TRY(read_csr(A, hA));
  if (hA.n != h->n) return rbicg_fail(RBICG_EINVAL, "matrix size %d does not match handle n=%d", hA.n, h->n);
  if (AH) {
    TRY(read_csr(AH, hAH));
    if (hAH.n != h->n) return rbicg_fail(RBICG_EINVAL, "A^H size mismatch");
  } else {
    hAH = conj_transpose(hA);
  }
  const bool cm = hA.complex_vals || hAH.complex_vals;
  if (cm && h->vkind == 0) return rbicg_fail(RBICG_EINVAL, "complex matrix needs a RBICG_C128 handle");
  h->mat_complex = cm;
  const int kind = cm ? 1 : 0;
  TRY(upload_sell(hA, kind, h->A));
  TRY(upload_sell(hAH, kind, h->AH));
  return 0;
}

}  // namespace

// ====================================================================== C ABI
extern "C" void rbicg_default_opts(rbicg_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->k = 20;
  o->s = 40;
  o->maxit = 10000;
  o->max_restarts = 2;
  o->update = 1;
  o->svd_tol = 1e-2;
  o->seed = 0;
  o->prec = RBICG_F64;
  o->inner_tol = 1e-5;
  o->max_outer = 30;
  o->stream = nullptr;
  o->chunk = 0;
}

extern "C" int rbicg_create(const rbicg_csr *A, const rbicg_csr *AH, const rbicg_opts *opt,
                            rbicg_handle *out) {
  if (!A || !opt || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (opt->k < 0 || opt->k > RBICG_KMAX) return rbicg_fail(RBICG_EINVAL, "k must be in [0, %d]", RBICG_KMAX);
  if (opt->s < 2 || opt->s + opt->k + 1 > RBICG_MAXCOLS || opt->s > 120)
    return rbicg_fail(RBICG_EINVAL, "cycle length s=%d out of range", opt->s);
  if (opt->maxit < 1) return rbicg_fail(RBICG_EINVAL, "maxit must be positive");
  if (opt->prec != RBICG_F64 && opt->prec != RBICG_C128)
    return rbicg_fail(RBICG_EINVAL, "precision mode %d is not available", (int)opt->prec);
  if (A->n <= 0) return rbicg_fail(RBICG_EINVAL, "n must be positive");
  rbicg_s *h = new rbicg_s();
  h->opt = *opt;
  h->n = A->n;
  h->ld = (A->n + 255) / 256 * 256;
  h->st = (hipStream_t)opt->stream;
  h->vkind = opt->prec == RBICG_C128 ? 1 : 0;
  h->vb = h->vkind ? 16 : 8;
  h->kcap = opt->k;
  h->scap = opt->s;
  int rc = set_matrix(h, A, AH);
  if (rc >= 0) rc = alloc_workspace(h);
  if (rc < 0) {
    rbicg_destroy(h);
    return rc;
  }
  *out = h;
  return RBICG_OK;
}

extern "C" int rbicg_destroy(rbicg_handle h) {
  if (!h) return RBICG_OK;
  if (h->st) (void)hipStreamSynchronize(h->st);
  else (void)hipDeviceSynchronize();
  h->A.release();
  h->AH.release();
  for (void *p : h->allocs) (void)hipFree(p);
  if (h->hS) (void)hipHostFree(h->hS);
  if (h->hG) (void)hipHostFree(h->hG);
  if (h->hW) (void)hipHostFree(h->hW);
  if (h->hlog) (void)hipHostFree(h->hlog);
  delete h;
  return RBICG_OK;
}

extern "C" int rbicg_solve_dual(rbicg_handle h, const void *b, const void *bt, void *x, void *xt,
                                double tol, rbicg_stats *st) {
  if (!h || !b || !bt || !x || !xt) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (!(tol > 0)) return rbicg_fail(RBICG_EINVAL, "tol must be positive");
  return dispatch(h, [&](auto *vp, auto *mp) {
    using V = std::remove_pointer_t<decltype(vp)>;
    using M = std::remove_pointer_t<decltype(mp)>;
    return solve_impl<V, M>(h, (const V *)b, (const V *)bt, (V *)x, (V *)xt, tol, st);
  });
}

extern "C" int rbicg_update_recycle(rbicg_handle h, const rbicg_csr *A_next, const rbicg_csr *AH_next) {
  if (!h) return rbicg_fail(RBICG_EINVAL, "null handle");
  if (A_next) TRY(set_matrix(h, A_next, AH_next));
  const void *Us = h->have_cyc ? h->Uc[h->cur] : h->U;
  const void *Uts = h->have_cyc ? h->Utc[h->cur] : h->Ut;
  const int k = h->have_cyc ? h->kcyc : h->ksys;
  h->have_cyc = false;
  return dispatch(h, [&](auto *vp, auto *mp) {
    using V = std::remove_pointer_t<decltype(vp)>;
    using M = std::remove_pointer_t<decltype(mp)>;
    return install_recycle<V, M>(h, Us, Uts, k);
  });
}

extern "C" int rbicg_set_recycle(rbicg_handle h, const void *U, const void *Ut, int32_t k) {
  if (!h) return rbicg_fail(RBICG_EINVAL, "null handle");
  if (k < 0 || k > h->kcap) return rbicg_fail(RBICG_EINVAL, "k=%d exceeds the handle's capacity %d", k, h->kcap);
  if (k > 0 && (!U || !Ut)) return rbicg_fail(RBICG_EINVAL, "null recycle basis");
  h->have_cyc = false;
  if (k == 0) {
    h->ksys = 0;
    return 0;
  }
  // caller layout has leading dimension n; the handle uses ld
  HIPCHECK(hipMemcpy2DAsync(h->Ua, h->ld * h->vb, U, h->n * h->vb, h->n * h->vb, k, hipMemcpyDeviceToDevice, h->st));
  HIPCHECK(hipMemcpy2DAsync(h->Uta, h->ld * h->vb, Ut, h->n * h->vb, h->n * h->vb, k, hipMemcpyDeviceToDevice, h->st));
  return dispatch(h, [&](auto *vp, auto *mp) {
    using V = std::remove_pointer_t<decltype(vp)>;
    using M = std::remove_pointer_t<decltype(mp)>;
    return install_recycle<V, M>(h, h->Ua, h->Uta, k);
  });
}

extern "C" int rbicg_get_recycle(rbicg_handle h, void *U, void *Ut, void *C, void *Ct, int32_t kcap,
                                 int32_t next, int32_t *k) {
  if (!h || !k) return rbicg_fail(RBICG_EINVAL, "null argument");
  const bool use_cyc = next && h->have_cyc;
  const int kk = use_cyc ? h->kcyc : h->ksys;
  *k = kk;
  const int m = std::min(kk, (int)kcap);
  void *src[4] = {use_cyc ? h->Uc[h->cur] : h->U, use_cyc ? h->Utc[h->cur] : h->Ut,
                  use_cyc ? h->Cc[h->cur] : h->C, use_cyc ? h->Ctc[h->cur] : h->Ct};
  void *dst[4] = {U, Ut, C, Ct};
  for (int t = 0; t < 4; ++t)
    if (dst[t] && m > 0)
      HIPCHECK(hipMemcpy2DAsync(dst[t], h->n * h->vb, src[t], h->ld * h->vb, h->n * h->vb, m, hipMemcpyDeviceToDevice, h->st));
  HIPCHECK(hipStreamSynchronize(h->st));
  return RBICG_OK;
}

extern "C" int rbicg_get_log(rbicg_handle h, double *out, int32_t cap, int32_t *count) {
  if (!h || !count) return rbicg_fail(RBICG_EINVAL, "null argument");
  const int c = std::min(h->last_count, (int)cap);
  if (out && c > 0) std::memcpy(out, h->last_log.data(), (size_t)c * LOG_STRIDE * sizeof(double));
  *count = h->last_count;
  return RBICG_OK;
}

extern "C" int rbicg_bilinear(rbicg_handle h, const void *u, const void *w, double tol, void *value,
                              double *err_est, rbicg_stats *st) {
  if (!h || !u || !w || !value) return rbicg_fail(RBICG_EINVAL, "null argument");
  void *x = nullptr, *xt = nullptr;
  const size_t bytes = (size_t)h->ld * h->vb;
  HIPCHECK(hipMalloc(&x, bytes));
  HIPCHECK(hipMalloc(&xt, bytes));
  int rc = dispatch(h, [&](auto *vp, auto *mp) {
    using V = std::remove_pointer_t<decltype(vp)>;
    using M = std::remove_pointer_t<decltype(mp)>;
    launch_fill_zero<V>(h->st, (V *)x, (size_t)h->n);
    launch_fill_zero<V>(h->st, (V *)xt, (size_t)h->n);
    // A x = w (primal), A^H x~ = u (dual)
    int r1 = solve_impl<V, M>(h, (const V *)w, (const V *)u, (V *)x, (V *)xt, tol, st);
    if (r1 < 0 && r1 != RBICG_BREAKDOWN) return r1;
    // value = u^H x + x~^H r with r = w - A x;  ||r||, ||r~||
    launch_residual<V, M>(h->st, h->A.view<M>(), (const V *)w, (const V *)x, (V *)h->t1);
    launch_residual<V, M>(h->st, h->AH.view<M>(), (const V *)u, (const V *)xt, (V *)h->t2);
    launch_dots<V>(h->st, h->n, (const V *)u, (const V *)x, (const V *)xt, (const V *)h->t1,
                   (const V *)h->t1, (const V *)h->t1, h->partial, h->S);
    TRY(pull_scalars(h));
    const double *red = h->hS->red;
    const double vr = red[0] + red[2], vi = red[1] + red[3];
    const double rnorm = std::sqrt(std::fabs(red[4]));
    launch_dots<V>(h->st, h->n, (const V *)h->t2, (const V *)h->t2, nullptr, nullptr, nullptr,
                   nullptr, h->partial, h->S);
    TRY(pull_scalars(h));
    const double rtnorm = std::sqrt(std::fabs(h->hS->red[0]));
    double *out = (double *)value;
    out[0] = vr;
    if (h->vkind == 1) out[1] = vi;
    if (err_est) *err_est = rnorm * rtnorm;
    return r1;
  });
  (void)hipFree(x);
  (void)hipFree(xt);
  return rc;
}

extern "C" int rbicg_solve_shifted(rbicg_handle h, int32_t S, const double *sigma, const void *b,
                                   const void *c, void *X, void *Xt, double tol, int32_t update_from,
                                   rbicg_stats *st) {
  (void)h; (void)S; (void)sigma; (void)b; (void)c; (void)X; (void)Xt; (void)tol; (void)update_from; (void)st;
  return rbicg_fail(RBICG_EINVAL, "rbicg_solve_shifted: not built yet");
}
