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
#include <deque>
#include <future>
#include <memory>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "rbicg.h"
#include "rbicg_hostla.h"
#include "device.h"
#include "errors.h"
#include "kernels.h"
#include "matviews.h"
#include "sec44.h"
#include "batch.h"
#include "ilut.h"

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
  float *val32 = nullptr;  // float copy of real values (FP32-inner mode), made on demand
  size_t nnzpad = 0;
  int64_t nnz = 0;
  int vbytes = 0;
  // sliceptr and col belong to another DevSell of the same matrix object (a
  // conjugate transpose with the matrix's own pattern) and are not freed here
  bool borrowed = false;
  template <class M> Sell<M> view() const {
    Sell<M> s;
    s.n = n;
    s.nslices = nslices;
    s.sliceptr = sliceptr;
    s.col = col;
    if constexpr (std::is_same<M, float>::value) s.val = val32;
    else s.val = (const M *)val;
    s.shifted = 0;
    s.shr = 0.0;
    s.shi = 0.0;
    return s;
  }
  void release() {
    if (sliceptr && !borrowed) (void)hipFree(sliceptr);
    if (col && !borrowed) (void)hipFree(col);
    borrowed = false;
    if (val) (void)hipFree(val);
    if (val32) (void)hipFree(val32);
    sliceptr = nullptr;
    col = nullptr;
    val = nullptr;
    val32 = nullptr;
  }
  // float copy of the (real, FP64) values
  int make_f32(hipStream_t st) {
    if (val32) return 0;
    if (vbytes != 8) return rbicg_fail(RBICG_EINVAL, "FP32-inner mode needs a real FP64 matrix");
    HIPCHECK(hipMalloc(&val32, std::max<size_t>(nnzpad, 1) * sizeof(float)));
    launch_d2f(st, (const double *)val, val32, nnzpad);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
    return 0;
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
// Conjugate transpose by a counting sort over columns (O(nnz)); with map,
// map[e] is the entry of the result that entry e of A became.
HostCsr conj_transpose_map(const HostCsr &A, std::vector<int> *map);
HostCsr conj_transpose(const HostCsr &A) { return conj_transpose_map(A, nullptr); }
HostCsr conj_transpose_map(const HostCsr &A, std::vector<int> *map) {
  if (map) map->assign(A.col.size(), 0);
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
      if (map) (*map)[e] = d;
    }
  return T;
}

// Position in the wave-sliced ELL layout of upload_sell of every CSR entry
// of A (entry j of row r at slice(r) + j 64 + r mod 64).
std::vector<int> sell_index(const HostCsr &A) {
  const int n = A.n;
  const int ns = (n + RBICG_WAVE - 1) / RBICG_WAVE;
  std::vector<int> idx(A.col.size());
  int base = 0;
  for (int s = 0; s < ns; ++s) {
    int w = 0;
    for (int r = s * RBICG_WAVE; r < std::min(n, (s + 1) * RBICG_WAVE); ++r)
      w = std::max(w, A.rowptr[r + 1] - A.rowptr[r]);
    for (int r = s * RBICG_WAVE; r < std::min(n, (s + 1) * RBICG_WAVE); ++r)
      for (int e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e)
        idx[e] = base + (e - A.rowptr[r]) * RBICG_WAVE + (r - s * RBICG_WAVE);
    base += w * RBICG_WAVE;
  }
  return idx;
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

// When the conjugate transpose has the matrix's own pattern (rows with the
// same column indices in the same order, e.g. any structurally symmetric
// stencil with sorted rows), its sliced-ELL slice pointers and column indices
// equal the matrix's (upload_sell depends on rowptr and col only): keep one
// copy, so that a pass over both reads the indices once.
int share_pattern(const HostCsr &hA, const HostCsr &hAH, DevSell &A, DevSell &AH) {
  if (hA.rowptr != hAH.rowptr || hA.col != hAH.col) return 0;
  if (AH.nnzpad != A.nnzpad || AH.nslices != A.nslices) return 0;
  HIPCHECK(hipFree(AH.sliceptr));
  HIPCHECK(hipFree(AH.col));
  AH.sliceptr = A.sliceptr;
  AH.col = A.col;
  AH.borrowed = true;
  return 0;
}

}  // namespace

// A device-resident matrix: A and its explicit conjugate transpose, repacked.
struct rbicg_mat_s {
  int n = 0;
  bool complex_vals = false;
  DevSell A, AH;
  // set for a pencil alpha E + beta A made by rbicg_matrix_pencil
  const rbicg_mat_s *pencil_a = nullptr, *pencil_e = nullptr;
};

// Workspace of rbicg_solve_shifted, allocated on the first call (n x S batch
// vectors, the shared basis [U, A U], [U~, A^H U~], Gram buffers, scalars).
struct ShiftWs {
  int Scap = 0, kcap = 0;
  std::vector<void *> allocs;
  cd *R = nullptr, *Rt = nullptr, *P[2] = {}, *Pt[2] = {}, *Z = nullptr, *Zt = nullptr;
  cd *X = nullptr, *Xt = nullptr;
  cd *BU = nullptr, *BUt = nullptr;
  cd *Y = nullptr, *Yt = nullptr, *Yx = nullptr, *Yxt = nullptr;
  double *gpart = nullptr, *G = nullptr, *P3 = nullptr, *rec = nullptr;
  size_t gpart_bytes = 0, G_bytes = 0;
  int reccap = 0;
  ShScalars *Sh = nullptr, *hSh = nullptr;
  ShScalars *hShd = nullptr;  // device view of hSh (chunk-end done flags)
  ShCoef *Co = nullptr, *hCo = nullptr;
  double *hG = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~ShiftWs() {
    for (void *p : allocs) (void)hipFree(p);
    if (hSh) (void)hipHostFree(hSh);
    if (hCo) (void)hipHostFree(hCo);
    if (hG) (void)hipHostFree(hG);
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// ==================================================== split preconditioner
// ILUT factors of one matrix on the device: L (unit lower), U (upper), and
// their conjugate transposes for the dual operator, each as its strictly
// triangular part, its diagonal (U, U^H) and a level-scheduled row order;
// three workspaces (iteration stream, cycle-end stream, rhs/solution calls),
// each with four n-vectors and the chunk counter of the triangular solves.
struct rbicg_ilu_s {
  int n = 0;
  bool complex_vals = false;
  int waves = 512;  // waves that work through the chunks of a triangular solve
  // ILUTP's column permutation (NULL without pivoting): perm[j] = the column
  // of A at position j, pos = its inverse; moved = columns out of place
  int *perm = nullptr, *pos = nullptr;
  int64_t moved = 0;
  struct Tri {
    int len = 0, levels = 0;
    int64_t nnz = 0;
    int *order = nullptr, *rp = nullptr, *ci = nullptr;
    void *v = nullptr, *diag = nullptr;
  } L, U, LH, UH;
  struct Ws {
    void *q[4] = {};
    int *counter = nullptr;
  } ws[3];
  int *err = nullptr;
  std::vector<void *> allocs;
  ~rbicg_ilu_s() {
    for (void *p : allocs) (void)hipFree(p);
  }
  template <class M> TriDev<M> view(const Tri &t) const {
    TriDev<M> d;
    d.n = n;
    d.len = t.len;
    d.order = t.order;
    d.rp = t.rp;
    d.ci = t.ci;
    d.v = (const M *)t.v;
    d.diag = (const M *)t.diag;
    return d;
  }
};

// ====================================================================== handle
struct rbicg_s {
  rbicg_opts opt{};
  int n = 0;
  int ld = 0;
  hipStream_t st = nullptr;
  // cycle-end work (recycle-space update for the next system) runs on its own
  // stream, concurrently with the iterations it does not feed
  hipStream_t jst = nullptr;
  hipEvent_t jev = nullptr;
  int vkind = 0;  // 0 double, 1 complex, 2 float (FP32-inner / FP64-outer mode)
  bool mat_complex = false;
  size_t vb = 8;
  int kcap = 0, scap = 0;
  rbicg_mat_s *mat = nullptr;
  bool own_mat = false;
  // optional per-kernel timing of the iteration kernels (opts.profile)
  std::vector<hipEvent_t> pev;
  hipEvent_t sev[2] = {nullptr, nullptr};
  double prof_ms[2] = {0, 0};
  long prof_n[2] = {0, 0};
  double prof_bytes[2] = {0, 0};  // algorithmic bytes of the timed launches
  // cycle-end telemetry (always on): jobs finished, host ms of the two host
  // parts, ms from a job's first enqueue to its last, ms the iteration
  // launches waited for a job (ring reuse)
  double prof_cyc[5] = {0, 0, 0, 0, 0};
  long prof_chunks = 0;              // chunks launched since the handle was made
  // iteration vectors (x, x~ are the caller's)
  void *r = nullptr, *rt = nullptr, *p[2] = {nullptr, nullptr}, *pt[2] = {nullptr, nullptr};
  void *xs0 = nullptr, *xts0 = nullptr;  // initial guesses of the current solve
  void *z = nullptr, *zt = nullptr, *t1 = nullptr, *t2 = nullptr;
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
  double *partial = nullptr;  // host-requested reductions
  double *P1 = nullptr, *P3 = nullptr;  // iteration partials
  int nb = 1;                 // blocks of the iteration kernels
  double *gpart = nullptr;
  size_t gpart_bytes = 0;
  size_t gram_cap = 0;  // complex entries of Gd / hG (mx * my of one Gram)
  double *Gd = nullptr;
  cd *Wd = nullptr;
  // pinned host staging
  Scalars *hS = nullptr;
  Scalars *hSd = nullptr;  // device view of hS (k_itfin writes the stopping outcome there)
  double *hG = nullptr;
  cd *hW = nullptr;
  double *hlog = nullptr;
  // last solve's log (host copy) for rbicg_get_log
  std::vector<double> last_log;
  int last_count = 0;
  // FP32-inner mode: FP64 outer residuals, float right-hand sides and corrections
  double *r64 = nullptr, *rt64 = nullptr, *d64 = nullptr, *dt64 = nullptr;
  float *b32 = nullptr, *bt32 = nullptr, *d32 = nullptr, *dt32 = nullptr;
  rbicg_s *h64 = nullptr;  // FP64 inner solves after a diverged FP32 one (made on demand)
  int last_dev_status = 0;  // device status code of the last solve_impl run
  // implicit shift: while set, the handle's matrix stands for sigma I - A
  // (used for the shifted pairs of IRKA; A^H becomes conj(sigma) I - A^H)
  bool shifted = false;
  cplx shift = 0.0;
  ShiftWs *sw = nullptr;  // workspace of the batched shifted solves
  rbicg_batch batch = nullptr;  // iteration chunks launched through this batch (rbicg_batch_attach)
  rbicg_ilu ilu = nullptr;      // split preconditioner: the operator is L^{-1} A U^{-1} (rbicg_ilu_attach)
  // Sec. 4.4 set-up (opts.pencil_setup = 1): per-iteration restrictions
  // zeta_i, zeta~_i (zstride doubles per iteration, indexed like log), their
  // pinned staging for one cycle, and the blocks carried to the next cycle
  double *zlog = nullptr, *hzlog = nullptr;
  int zstride = 0;
  struct RecState {
    bool valid = false;
    int run_start = -1, cycle = -1;  // the cycle whose job produced the blocks
    sec44::Blocks X;
    double rn_last2 = 0.0;   // ||r_{e-1}|| of that cycle (e its last iteration)
    cplx at_last = 0.0;      // scale of its last dual Lanczos vector
  } rec;
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

// No-progress window of FP32 inner solves, in cycles: BiCG's residual norms
// are not monotone and can plateau for a few cycles on convection-dominated
// operators before they drop again, so a shorter window would discard float
// solves that converge.
constexpr int FP32_NOPROGRESS_CYCLES = 6;

// Cosine cut of the biorthogonalization.  FP32-inner mode raises it so that
// the attainable inner residual, about eps32 ||I - C C~^H|| <= eps32 (1 + 1/tau),
// stays ten times below the inner tolerance: tau >= 10 eps32 / inner_tol.
double svd_tol_eff(const rbicg_s *h) {
  if (h->vkind != 2) return h->opt.svd_tol;
  return std::max(h->opt.svd_tol, 10.0 * std::ldexp(1.0, -24) / h->opt.inner_tol);
}

// Algorithmic bytes of one launch of each iteration kernel (matrix values of
// the type the kernels read, int32 column indices, one slice pointer per
// row-slice rounded to one per row): k_it1 reads r, r~, p, p~ and C, C~ rows
// and writes p, p~, z, z~ (plus r_{i-1}, r~_{i-1} into the cycle rings when
// updating; z, z~ then live in their ring slots); k_it2 reads x, x~, r, r~,
// p, p~, z, z~ and C, C~ rows and writes x, x~, r, r~.
void kernel_bytes(const rbicg_s *h, int k, double out[2]) {
  const double ba = h->vkind == 2 ? 4.0 : (double)h->mat->A.vbytes;
  const double nnz = (double)h->mat->A.nnz, n = h->n, vb = (double)h->vb;
  const bool cap = h->opt.update && h->opt.k > 0;
  // the index arrays once when A^H shares A's pattern
  const double ix = h->mat->AH.borrowed ? 1.0 : 2.0;
  out[0] = 2.0 * nnz * ba + ix * (4.0 * nnz + 4.0 * (n + 1.0)) +
           (8.0 + 2.0 * k + (cap ? 2.0 : 0.0)) * n * vb;
  out[1] = (12.0 + 2.0 * k) * n * vb;
}

// bytes per algorithmic iteration: the two kernels' total
double alg_bytes_iter(const rbicg_s *h, int k) {
  double kb[2];
  kernel_bytes(h, k, kb);
  double b = kb[0] + kb[1];
  if (h->ilu) {
    // per triangular solve: the factor (values, columns, row pointers, level
    // order, diagonal), b read, x and the flags written; the SpMVs' vectors
    // (x read, y written, both directions) and the split kernels' re-reads
    // of p, p~ (the direction update) and p~ (the restriction)
    const rbicg_ilu_s *P = h->ilu;
    const double bm = (double)h->mat->A.vbytes, n = h->n, vb = (double)h->vb;
    for (const rbicg_ilu_s::Tri *T : {&P->L, &P->U, &P->LH, &P->UH})
      b += (double)T->nnz * (bm + 4.0) + 4.0 * (n + 1.0) + 4.0 * T->len +
           (T->diag ? n * bm : 0.0) + 2.0 * n * vb + 4.0 * n;
    b += 4.0 * n * vb + 3.0 * n * vb;
  }
  return b;
}

// views of the handle's matrix and of its conjugate transpose, with the
// handle's implicit shift attached
template <class M> Sell<M> view_A(const rbicg_s *h) {
  Sell<M> v = h->mat->A.view<M>();
  if (h->shifted) {
    v.shifted = 1;
    v.shr = h->shift.real();
    v.shi = h->shift.imag();
  }
  return v;
}
template <class M> Sell<M> view_AH(const rbicg_s *h) {
  Sell<M> v = h->mat->AH.view<M>();
  if (h->shifted) {
    v.shifted = 1;
    v.shr = h->shift.real();
    v.shi = -h->shift.imag();
  }
  return v;
}

// ------------------------------------------------ operator of the handle
// The handle iterates with A, or with a split preconditioner attached with
// A^ = L^{-1} A U^{-1} (dual A^^H = U^{-H} A^H L^{-H}), applied as two
// triangular solves around one SpMV.  The cycle-end stream (jst) and the
// iteration stream use separate workspaces, so that both may apply A^ at once.
rbicg_ilu_s::Ws &ilu_ws(rbicg_s *h) { return h->ilu->ws[h->st == h->jst ? 1 : 0]; }

// x0 = T_f0^{-1} b0 and, when f1 >= 0, x1 = T_f1^{-1} b1 in one pair of
// launches; factors 0 L, 1 U, 2 L^H, 3 U^H.
template <class V, class M>
void ilu_trsv(hipStream_t st, rbicg_ilu_s *P, rbicg_ilu_s::Ws &w, int f0, const V *b0, V *x0,
              int f1, const V *b1, V *x1, const Scalars *S) {
  auto tri = [&](int f) -> const rbicg_ilu_s::Tri & {
    return f == 0 ? P->L : f == 1 ? P->U : f == 2 ? P->LH : P->UH;
  };
  const TriDev<M> T0 = P->view<M>(tri(f0));
  if (f1 >= 0) {
    const TriDev<M> T1 = P->view<M>(tri(f1));
    launch_sptrsv<V, M>(st, T0, b0, x0, &T1, b1, x1, w.counter, P->waves, S, P->err);
  } else {
    launch_sptrsv<V, M>(st, T0, b0, x0, nullptr, (const V *)nullptr, (V *)nullptr, w.counter,
                        P->waves, S, P->err);
  }
}

// y0 = A^ x0 and y1 = A^^H x1, A^ = L^{-1} A Q U^{-1} (Q = I without
// pivoting; either pair may be absent; y0, y1 must not be
// workspace vectors or alias the x's): the two directions' triangular solves
// share launches.  S: the kernels do nothing once the stopping test has
// fired (NULL: always run).  FP64 and complex vectors only (FP32 handles
// never carry a preconditioner).
template <class V, class M>
void ilu_apply(rbicg_s *h, const V *x0, V *y0, const V *x1, V *y1, const Scalars *S) {
  if constexpr (sizeof(V) >= 8) {
    rbicg_ilu_s *P = h->ilu;
    rbicg_ilu_s::Ws &w = ilu_ws(h);
    V *a1 = (V *)w.q[0], *a2 = (V *)w.q[1], *d1 = (V *)w.q[2], *d2 = (V *)w.q[3];
    // A (Q a1) and Q^T (A^H d1); plain SpMVs without pivoting
    auto spmv_primal = [&]() {
      if (P->perm) launch_spmv_perm<V, M>(h->st, view_A<M>(h), a1, a2, P->pos, nullptr, S);
      else launch_spmv<V, M>(h->st, view_A<M>(h), a1, a2, S);
    };
    auto spmv_dual = [&]() {
      if (P->perm) launch_spmv_perm<V, M>(h->st, view_AH<M>(h), d1, d2, nullptr, P->perm, S);
      else launch_spmv<V, M>(h->st, view_AH<M>(h), d1, d2, S);
    };
    if (x0 && x1) {
      ilu_trsv<V, M>(h->st, P, w, 1, x0, a1, 2, x1, d1, S);  // U^{-1} x0, L^{-H} x1
      spmv_primal();
      spmv_dual();
      ilu_trsv<V, M>(h->st, P, w, 0, a2, y0, 3, d2, y1, S);  // L^{-1} ., U^{-H} .
    } else if (x0) {
      ilu_trsv<V, M>(h->st, P, w, 1, x0, a1, -1, (const V *)nullptr, (V *)nullptr, S);
      spmv_primal();
      ilu_trsv<V, M>(h->st, P, w, 0, a2, y0, -1, (const V *)nullptr, (V *)nullptr, S);
    } else if (x1) {
      ilu_trsv<V, M>(h->st, P, w, 2, x1, d1, -1, (const V *)nullptr, (V *)nullptr, S);
      spmv_dual();
      ilu_trsv<V, M>(h->st, P, w, 3, d2, y1, -1, (const V *)nullptr, (V *)nullptr, S);
    }
  }
}

// out = b - Op x (x NULL: out = b), Op = A or A^ (dual: A^H or A^^H)
template <class V, class M>
void op_residual(rbicg_s *h, bool dual, const V *b, const V *x, V *out) {
  if (!h->ilu || !x) {
    launch_residual<V, M>(h->st, dual ? view_AH<M>(h) : view_A<M>(h), b, x, out);
    return;
  }
  // A^ x into out, then out = b - out
  if (dual) ilu_apply<V, M>(h, nullptr, nullptr, x, out, nullptr);
  else ilu_apply<V, M>(h, x, out, nullptr, nullptr, nullptr);
  launch_rsub<V>(h->st, h->n, b, out, out);
}

// Y = Op X for m columns of leading dimension ld
template <class V, class M>
void op_spmm(rbicg_s *h, bool dual, const V *X, V *Y, int ld, int m) {
  if (!h->ilu) {
    launch_spmm<V, M>(h->st, dual ? view_AH<M>(h) : view_A<M>(h), X, Y, ld, m);
    return;
  }
  for (int j = 0; j < m; ++j) {
    const V *x = X + (size_t)j * ld;
    V *y = Y + (size_t)j * ld;
    if (dual) ilu_apply<V, M>(h, nullptr, nullptr, x, y, nullptr);
    else ilu_apply<V, M>(h, x, y, nullptr, nullptr, nullptr);
  }
}

// The attached preconditioner fits the handle's current matrix and mode
int ilu_check(const rbicg_s *h) {
  if (!h->ilu) return 0;
  if (h->ilu->n != h->n || h->ilu->complex_vals != h->mat->complex_vals)
    return rbicg_fail(RBICG_EINVAL, "the attached preconditioner does not match the handle's matrix");
  if (h->vkind == 2) return rbicg_fail(RBICG_EINVAL, "split preconditioning needs an FP64 or complex handle");
  return 0;
}

// ---------------------------------------------------------- typed helpers
template <class V, class M> constexpr int batch_kind() {
  return sizeof(V) == 4 ? BK_F32 : (sizeof(V) == 8 ? BK_F64 : (sizeof(M) == 16 ? BK_C128 : BK_C128_REAL_A));
}
template <class V> struct VK;
template <> struct VK<double> { static constexpr int kind = 0; };
template <> struct VK<cd> { static constexpr int kind = 1; };
template <> struct VK<float> { static constexpr int kind = 0; };

// Gram G = X^H Y (mx x my, complex): enqueue the kernels and the download
// into h->hG (no synchronization).  Y is processed in column groups so that
// every launch fits the kernel's tile and LDS budget (mx <= 128); the download
// keeps the group layout, gram_parse restores row-major (i, j) order.
template <class V>
int gram_enqueue(rbicg_s *h, const std::vector<const void *> &X, const std::vector<const void *> &Y) {
  const int mx = (int)X.size(), my = (int)Y.size();
  if (mx > 128 || mx < 1 || my < 1) return rbicg_fail(RBICG_EINVAL, "gram shape %d x %d unsupported", mx, my);
  if ((size_t)mx * my > h->gram_cap)
    return rbicg_fail(RBICG_EINVAL, "gram %d x %d exceeds the handle's Gram buffers (k, s too small)", mx, my);
  const int gy = gram_group(mx, sizeof(V) == 16 ? 1 : 0);
  const int nchunks = gram_chunks(h->n);
  ColList xl{};
  for (int i = 0; i < mx; ++i) xl.p[i] = X[i];
  for (int j0 = 0; j0 < my; j0 += gy) {
    const int g = std::min(gy, my - j0);
    const size_t need = (size_t)nchunks * mx * g * 2 * sizeof(double);
    if (need > h->gpart_bytes) return rbicg_fail(RBICG_EINVAL, "gram workspace too small");
    ColList yl{};
    for (int j = 0; j < g; ++j) yl.p[j] = Y[j0 + j];
    launch_gram<V>(h->st, h->n, xl, mx, yl, g, h->gpart, h->Gd + (size_t)2 * mx * j0, nchunks);
    HIPCHECK(hipGetLastError());
  }
  HIPCHECK(hipMemcpyAsync(h->hG, h->Gd, (size_t)mx * my * 2 * sizeof(double), hipMemcpyDeviceToHost, h->st));
  return 0;
}

// Row-major (i, j) complex Gram from the downloaded group layout (host only).
std::vector<cplx> gram_parse(const double *hG, int mx, int my, int gy) {
  std::vector<cplx> G((size_t)mx * my);
  for (int j0 = 0; j0 < my; j0 += gy) {
    const int g = std::min(gy, my - j0);
    const double *blk = hG + (size_t)2 * mx * j0;
    for (int i = 0; i < mx; ++i)
      for (int j = 0; j < g; ++j)
        G[(size_t)i * my + j0 + j] = cplx(blk[2 * ((size_t)i * g + j)], blk[2 * ((size_t)i * g + j) + 1]);
  }
  return G;
}


// Stage W (m x p, column-major, complex) into coefficient slot `slot` and
// enqueue Y = X W.  A slot is reused only after the stream has been
// synchronized at least once since its last use (every cycle update and every
// biorthogonalization synchronize to read a Gram).
#define RBICG_WSLOT ((size_t)RBICG_MAXCOLS * KMAXD)
template <class V>
int tsgemm(rbicg_s *h, const std::vector<const void *> &X, const std::vector<cplx> &W, int p,
           void *Y, int slot) {
  const int m = (int)X.size();
  if (m > RBICG_MAXCOLS || p > KMAXD) return rbicg_fail(RBICG_EINVAL, "tsgemm too wide");
  if (p == 0 || m == 0) return 0;
  cd *hw = h->hW + (size_t)slot * RBICG_WSLOT;
  cd *dw = h->Wd + (size_t)slot * RBICG_WSLOT;
  for (int t = 0; t < m * p; ++t) hw[t] = cd{W[t].real(), W[t].imag()};
  HIPCHECK(hipMemcpyAsync(dw, hw, (size_t)m * p * sizeof(cd), hipMemcpyHostToDevice, h->st));
  ColList xl{};
  for (int i = 0; i < m; ++i) xl.p[i] = X[i];
  launch_tsgemm<V>(h->st, h->n, xl, m, dw, p, (V *)Y, h->ld);
  HIPCHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------- recycle-space updates
// The update at the end of a cycle (Sec. 4) runs as a job in stages, so that
// its host work (the small eigenproblem and SVD) overlaps the iterations of
// the next cycle on the GPU:
//   begin   enqueue the download of the cycle's scalars and the Gram
//           X1^H [Y1 | Y2] of the harmonic Ritz pencil, record an event;
//   host1   (worker thread) build T or the pencil (P, Q) and pick the
//           eigenvectors of the k eigenvalues closest to the origin;
//   stage2  enqueue U_j = Phi W, U~_j = Phi~ W~ (MFMA tall-skinny products),
//           C = A U_j, C~ = A^H U~_j, their Grams, record an event;
//   host3   (worker thread) biorthogonalization (Sec. 4.3) from the Grams;
//   stage4  enqueue the rotations into the cycle buffers and install them.
// Jobs run one after another.  The cycle's captured vectors live in one of two
// ring sets; the iterations of cycle c+2 (which overwrite that set) are
// enqueued only after the job of cycle c has enqueued its last ring read.
// Points h->st at the handle's job stream for the enclosed enqueues.
struct JobStream {
  rbicg_s *h;
  hipStream_t saved;
  explicit JobStream(rbicg_s *hh) : h(hh), saved(hh->st) { h->st = h->jst; }
  ~JobStream() { h->st = saved; }
};

struct CycleJob {
  int cycle = 0, e = 0, set = 0, run_start = 0;
  int stage = 0;          // 0 pending, 1 begun, 2 host1, 3 stage2 done, 4 host3, 5 finished
  bool tpath = false;     // first cycle of the first system: eigenvectors of T
  double rn0 = 0;
  cplx rho0;
  int kp = 0, mm = 0, mz = 0, gy = 0;
  std::vector<const void *> XU, XUt;
  hipEvent_t ev = nullptr;     // the job's last enqueued stage (job stream)
  hipEvent_t ready = nullptr;  // the cycle's last iteration (iteration stream)
  std::future<int> fut;
  double host_ms[2] = {0, 0};
  std::chrono::steady_clock::time_point t_begin;
  int m = 0, p = 0;
  std::vector<cplx> Wc, Wtc, TU, TUt;
  int g2y = 0;
  std::string err;
  // Sec. 4.4 set-up: 0 explicit Grams, 1 later cycle of the same Lanczos run,
  // 2 first cycle of a later system, 3 eigenvectors of T (first cycle of the
  // first system) with the recurrence state started
  int setup = 0;
  sec44::Mat Wn, Wtn;            // eigenvectors in terms of Phi_j (normalized v)
  sec44::Mat B, Bt, G, Gt;       // B_j, B~_j, Gamma_j, Gamma~_j
  sec44::Blocks X, Xnext;        // carried blocks used, and those for the next cycle
  double rn_last2 = 0.0;
  cplx at_last = 0.0;
  // A job dropped on an error path may still have its host part running on a
  // worker thread, writing into the members above: wait for it before they
  // are destroyed (a deferred part that never ran is not started).
  ~CycleJob() {
    if (fut.valid() && fut.wait_for(std::chrono::seconds(0)) != std::future_status::deferred) fut.wait();
    if (ev) (void)hipEventDestroy(ev);
    if (ready) (void)hipEventDestroy(ready);
  }
};

struct LogEntry {
  cplx alpha, beta_prev, rho;
  double rn, rtn;
};

inline char *ring_col(void *base, int set, int slots, int c, const rbicg_s *h) {
  return (char *)base + ((size_t)set * slots + c) * h->ld * h->vb;
}
// Dual residual ring: slots 0..s-1 hold r~_{i-1} of the cycle's iterations,
// slot s the residual r~ after the cycle's last iteration, slot s+1 the
// previous cycle's last r~_{i-1} (copied at the start of the cycle); the two
// extra slots give the set-up of Sec. 4.4 the whole Upsilon~_j of the cycle.
inline char *rt_col(const rbicg_s *h, int set, int c) { return ring_col(h->Rt, set, h->opt.s + 2, c, h); }

// Stages 1, 2 and 4 enqueue on h->st, which the caller points at the job
// stream (JobStream).
template <class V>
int job_begin(rbicg_s *h, CycleJob &J) {
  const int s = h->opt.s;
  const int lo = J.e - s;
  HIPCHECK(hipStreamWaitEvent(h->st, J.ready, 0));
  HIPCHECK(hipMemcpyAsync(h->hlog, h->log + (size_t)lo * LOG_STRIDE,
                          (size_t)(s + 1) * LOG_STRIDE * sizeof(double), hipMemcpyDeviceToHost, h->st));
  J.XU.clear();
  J.XUt.clear();
  J.tpath = !h->have_cyc && h->ksys == 0;
  const bool rec_mode = h->zlog != nullptr;
  J.setup = 0;
  if (rec_mode) {
    if (J.tpath) J.setup = 3;
    else if (!h->have_cyc && h->ksys > 0 && J.cycle == 0) J.setup = 2;
    else if (h->have_cyc && h->rec.valid && h->rec.run_start == J.run_start && h->rec.cycle == J.cycle - 1)
      J.setup = 1;
  }
  if (J.setup == 0) h->rec.valid = false;
  if (h->zlog && h->ksys > 0 && (J.setup == 1 || J.setup == 2))
    HIPCHECK(hipMemcpyAsync(h->hzlog, h->zlog + (size_t)lo * h->zstride,
                            (size_t)(s + 1) * h->zstride * sizeof(double), hipMemcpyDeviceToHost, h->st));
  if (J.setup == 1 || J.setup == 2) {
    // Phi_j = [U_{j-1}, V_j] for the products U_j = Phi_j W (as below); the one
    // O(n) product of the set-up: Upsilon~_j^H U_{j-1}, or in the first cycle
    // of a later system [V~_1 underbar, C~]^H U
    const bool first = J.setup == 2;
    void *Up = first ? h->U : h->Uc[h->cur];
    void *Utp = first ? h->Ut : h->Utc[h->cur];
    const int kp = first ? h->ksys : h->kcyc;
    J.kp = kp;
    J.mm = kp + s;
    std::vector<const void *> X, Y;
    for (int j = 0; j < kp; ++j) {
      J.XU.push_back(col_ptr(Up, j, h));
      J.XUt.push_back(col_ptr(Utp, j, h));
      Y.push_back(col_ptr(Up, j, h));
    }
    for (int c = 0; c < s; ++c) {
      J.XU.push_back(ring_col(h->R, J.set, s, c, h));
      J.XUt.push_back(rt_col(h, J.set, c));
    }
    if (!first) X.push_back(rt_col(h, J.set, s + 1));
    for (int c = 0; c <= s; ++c) X.push_back(rt_col(h, J.set, c));
    if (first)
      for (int j = 0; j < kp; ++j) X.push_back(col_ptr(h->Ct, j, h));
    J.mz = (int)X.size();
    J.gy = gram_group(J.mz, sizeof(V) == 16 ? 1 : 0);
    TRY(gram_enqueue<V>(h, X, Y));
  } else if (J.tpath) {
    for (int c = 0; c < s; ++c) {
      J.XU.push_back(ring_col(h->R, J.set, s, c, h));
      J.XUt.push_back(rt_col(h, J.set, c));
    }
  } else {
    void *Up = h->have_cyc ? h->Uc[h->cur] : h->U;
    void *Utp = h->have_cyc ? h->Utc[h->cur] : h->Ut;
    void *Cp = h->have_cyc ? h->Cc[h->cur] : h->C;
    void *Ctp = h->have_cyc ? h->Ctc[h->cur] : h->Ct;
    const int kp = h->have_cyc ? h->kcyc : h->ksys;
    J.kp = kp;
    J.mm = kp + s;
    J.mz = kp + s + 1;
    std::vector<const void *> X1, Yall;
    for (int j = 0; j < kp; ++j) {
      X1.push_back(col_ptr(Ctp, j, h));
      Yall.push_back(col_ptr(Cp, j, h));
      J.XU.push_back(col_ptr(Up, j, h));
      J.XUt.push_back(col_ptr(Utp, j, h));
    }
    for (int c = 0; c <= s; ++c) {
      X1.push_back(ring_col(h->Zt, J.set, s + 1, c, h));
      Yall.push_back(ring_col(h->Z, J.set, s + 1, c, h));
    }
    for (int j = 0; j < kp; ++j) Yall.push_back(col_ptr(Up, j, h));
    for (int c = 0; c < s; ++c) {
      Yall.push_back(ring_col(h->R, J.set, s, c, h));
      J.XU.push_back(ring_col(h->R, J.set, s, c, h));
      J.XUt.push_back(rt_col(h, J.set, c));
    }
    J.gy = gram_group((int)X1.size(), sizeof(V) == 16 ? 1 : 0);
    TRY(gram_enqueue<V>(h, X1, Yall));
  }
  HIPCHECK(hipEventRecord(J.ev, h->st));
  J.stage = 1;
  return 0;
}

// Gamma_j, Gamma~_j and B_j, B~_j of the cycle (Sec. 4.1, Sec. 4.4) from the
// logged scalars and restrictions.  L[t] is the log row of iteration
// e - s + t; a[c], at[c] scale r_{i-1}, r~_{i-1} to v_i, v~_i.
int job_rec_cycle_blocks(const rbicg_s *h, CycleJob &J, const std::vector<LogEntry> &L,
                         const std::vector<double> &a, const std::vector<cplx> &at,
                         const std::vector<cplx> &alpha, const std::vector<cplx> &beta) {
  const int s = h->opt.s;
  sec44::CycleScalars cs;
  cs.s = s;
  cs.alpha = alpha;
  cs.beta = beta;
  cs.rn.resize(s);
  for (int c = 0; c < s; ++c) cs.rn[c] = L[c].rn;
  cs.rn_end = L[s].rn;
  cs.beta_end = L[s].rho / L[s - 1].rho;
  cs.first = J.cycle == 0;
  if (!cs.first) {
    cs.alpha_before = L[0].alpha;
    cs.rn_before = h->rec.rn_last2;
  }
  sec44::gamma_blocks(cs, J.G, J.Gt);
  const int kC = J.setup == 3 ? 0 : h->ksys;
  J.B = sec44::Mat(kC, s);
  J.Bt = sec44::Mat(kC, s);
  if (kC > 0) {
    const int nd = h->vkind == 1 ? 2 : 1;
    auto zeta = [&](int row, int j) -> cplx {  // restriction j (< 2 kC) of log row e - s + row
      const double *z = h->hzlog + (size_t)row * h->zstride + (size_t)j * nd;
      return nd == 2 ? cplx(z[0], z[1]) : cplx(z[0], 0.0);
    };
    for (int c = 0; c < s; ++c)
      for (int j = 0; j < kC; ++j) {
        cplx d = zeta(c + 1, j), dt = zeta(c + 1, kC + j);
        if (beta[c] != cplx(0.0)) {
          d -= beta[c] * zeta(c, j);
          dt -= std::conj(beta[c]) * zeta(c, kC + j);
        }
        J.B(j, c) = d * a[c];
        J.Bt(j, c) = dt * at[c];
      }
  }
  J.rn_last2 = L[s - 1].rn;
  J.at_last = at[s - 1];
  return 0;
}

// Host part 1 with the Sec. 4.4 set-up (J.setup 1 or 2): the pencil from the
// carried blocks and the cycle's small Gram, its eigenvectors, and the
// coefficient matrices of U_j = Phi_j W, U~_j = Phi~_j W~.
int job_host1_sec44(const rbicg_s *h, CycleJob &J, const std::vector<LogEntry> &L,
                    const std::vector<double> &a, const std::vector<cplx> &at,
                    const std::vector<cplx> &alpha, const std::vector<cplx> &beta, bool real_problem) {
  const int s = h->opt.s, k = h->opt.k, kp = J.kp, mm = J.mm;
  TRY(job_rec_cycle_blocks(h, J, L, a, at, alpha, beta));
  // the Gram X^H Y of job_begin: X = raw dual residuals (and C~), Y = U_{j-1}
  const std::vector<cplx> Gr = gram_parse(h->hG, J.mz, kp, J.gy);
  const cplx at_end = L[s].rn / std::conj(L[s].rho);
  sec44::Mat P, Q;
  if (J.setup == 1) {
    // rows: v~_{e-s}, V~_j, v~_{e+1}
    sec44::Mat YtU(s + 2, kp);
    for (int i = 0; i < s + 2; ++i) {
      const cplx sc = std::conj(i == 0 ? h->rec.at_last : (i <= s ? at[i - 1] : at_end));
      for (int j = 0; j < kp; ++j) YtU(i, j) = sc * Gr[(size_t)i * kp + j];
    }
    J.X = h->rec.X;
    sec44::pencil_general(J.X, YtU, J.B, J.Bt, J.G, J.Gt, P, Q);
  } else {
    // rows: V~_1, v~_{s+1}, then C~
    sec44::Mat VtU(s + 1, kp), CtU(kp, kp);
    for (int i = 0; i < s + 1; ++i) {
      const cplx sc = std::conj(i < s ? at[i] : at_end);
      for (int j = 0; j < kp; ++j) VtU(i, j) = sc * Gr[(size_t)i * kp + j];
    }
    for (int i = 0; i < kp; ++i)
      for (int j = 0; j < kp; ++j) CtU(i, j) = Gr[(size_t)(s + 1 + i) * kp + j];
    J.X = sec44::system_start_blocks(CtU, s);
    sec44::pencil_first(CtU, VtU, J.B, J.Bt, J.G, J.Gt, P, Q);
  }
  std::vector<double> Pd(2 * (size_t)mm * mm), Qd(2 * (size_t)mm * mm);
  for (int j = 0; j < mm; ++j)
    for (int i = 0; i < mm; ++i) {
      Pd[2 * (i + (size_t)j * mm)] = P(i, j).real();
      Pd[2 * (i + (size_t)j * mm) + 1] = P(i, j).imag();
      Qd[2 * (i + (size_t)j * mm)] = Q(i, j).real();
      Qd[2 * (i + (size_t)j * mm) + 1] = Q(i, j).imag();
    }
  std::vector<double> Ws(2 * (size_t)mm * mm), Wls(2 * (size_t)mm * mm);
  const int m = rbicg_host_eig_select(mm, Pd.data(), Qd.data(), k, real_problem ? 1 : 0, Ws.data(), Wls.data());
  if (m < 0) {
    J.err = std::string("harmonic Ritz problem failed: ") + rbicg_last_error();
    return -1;
  }
  J.Wn = sec44::Mat(mm, m);
  J.Wtn = sec44::Mat(mm, m);
  J.Wc.assign((size_t)mm * m, 0.0);
  J.Wtc.assign((size_t)mm * m, 0.0);
  for (int c = 0; c < m; ++c)
    for (int l = 0; l < mm; ++l) {
      const cplx w = cplx(Ws[2 * (l + (size_t)c * mm)], Ws[2 * (l + (size_t)c * mm) + 1]);
      const cplx wl = cplx(Wls[2 * (l + (size_t)c * mm)], Wls[2 * (l + (size_t)c * mm) + 1]);
      J.Wn(l, c) = w;
      J.Wtn(l, c) = wl;
      J.Wc[l + (size_t)c * mm] = (l < kp ? cplx(1.0) : cplx(a[l - kp])) * w;
      J.Wtc[l + (size_t)c * mm] = (l < kp ? cplx(1.0) : at[l - kp]) * wl;
    }
  J.m = m;
  return 0;
}

// Host part 1 (no HIP calls): coefficient matrices of U_j and U~_j.
int job_host1(const rbicg_s *h, CycleJob &J, bool real_problem) {
  const int s = h->opt.s, k = h->opt.k;
  std::vector<LogEntry> L(s + 1);
  for (int t = 0; t <= s; ++t) {
    const double *q = h->hlog + (size_t)t * LOG_STRIDE;
    L[t].alpha = cplx(q[0], q[1]);
    L[t].beta_prev = cplx(q[2], q[3]);
    L[t].rho = cplx(q[4], q[5]);
    L[t].rn = q[6];
    L[t].rtn = q[7];
  }
  if (J.e - s == J.run_start) {
    L[0].rn = J.rn0;
    L[0].rho = J.rho0;
  }
  // cycle iteration c (0..s-1) is i = e - s + 1 + c: ||r_{i-1}|| = L[c].rn,
  // rho_{i-1} = L[c].rho, alpha_i = L[c+1].alpha, beta_{i-1} = L[c+1].beta_prev;
  // v_i = r_{i-1} a_i and v~_i = r~_{i-1} at_i (Sec. 4.1 scaling)
  std::vector<double> a(s);
  std::vector<cplx> at(s), alpha(s), beta(s);
  for (int c = 0; c < s; ++c) {
    a[c] = 1.0 / L[c].rn;
    at[c] = L[c].rn / std::conj(L[c].rho);
    alpha[c] = L[c + 1].alpha;
    beta[c] = L[c + 1].beta_prev;
  }
  int m = 0;
  if (J.tpath) {
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
    std::vector<double> Ws(2 * s * s), Wls(2 * s * s);
    m = rbicg_host_eig_select(s, T.data(), nullptr, k, real_problem ? 1 : 0, Ws.data(), Wls.data());
    if (m < 0) {
      J.err = std::string("cycle eigenproblem failed: ") + rbicg_last_error();
      return -1;
    }
    J.Wc.assign((size_t)s * m, 0.0);
    J.Wtc.assign((size_t)s * m, 0.0);
    for (int c = 0; c < m; ++c)
      for (int l = 0; l < s; ++l) {
        J.Wc[l + c * s] = a[l] * cplx(Ws[2 * (l + c * s)], Ws[2 * (l + c * s) + 1]);
        J.Wtc[l + c * s] = at[l] * cplx(Wls[2 * (l + c * s)], Wls[2 * (l + c * s) + 1]);
      }
    if (J.setup == 3) {
      // start of the Sec. 4.4 recurrences: Phi_1 = V_1, nothing carried
      J.kp = 0;
      J.Wn = sec44::Mat(s, m);
      J.Wtn = sec44::Mat(s, m);
      for (int c = 0; c < m; ++c)
        for (int l = 0; l < s; ++l) {
          J.Wn(l, c) = cplx(Ws[2 * (l + c * s)], Ws[2 * (l + c * s) + 1]);
          J.Wtn(l, c) = cplx(Wls[2 * (l + c * s)], Wls[2 * (l + c * s) + 1]);
        }
      J.X = sec44::empty_blocks(s);
      TRY(job_rec_cycle_blocks(h, J, L, a, at, alpha, beta));
    }
  } else if (J.setup == 1 || J.setup == 2) {
    TRY(job_host1_sec44(h, J, L, a, at, alpha, beta, real_problem));
    m = J.m;
  } else {
    const int kp = J.kp, mm = J.mm, mz = J.mz;
    const std::vector<cplx> G = gram_parse(h->hG, mz, mz + mm, J.gy);
    const int wy = mz + mm;
    // A Phi = [C_p, Z] B, A^H Phi~ = [C~_p, Z~] Bt, Phi = [U_p, R] D with
    // A v_i = (z_i - beta_{i-1} z_{i-1}) a_i and A^H v~_i likewise; then
    // P = Bt^H G1 B, Q = Bt^H G2 D (eq. finalGenEigValue).  B, Bt, D are
    // identity blocks plus (bi)diagonals, applied entrywise here.
    auto G1 = [&](int i, int j) { return G[(size_t)i * wy + j]; };
    auto G2 = [&](int i, int j) { return G[(size_t)i * wy + mz + j]; };
    auto Bcol = [&](int col, int row) -> cplx {  // B(row, col)
      if (col < kp) return row == col ? cplx(1.0) : cplx(0.0);
      const int c = col - kp;
      if (row == kp + c + 1) return a[c];
      if (row == kp + c) return -beta[c] * a[c];
      return 0.0;
    };
    auto Btcol = [&](int col, int row) -> cplx {
      if (col < kp) return row == col ? cplx(1.0) : cplx(0.0);
      const int c = col - kp;
      if (row == kp + c + 1) return at[c];
      if (row == kp + c) return -std::conj(beta[c]) * at[c];
      return 0.0;
    };
    auto rows_of = [&](int col, int *r) {  // nonzero rows of column col of B / Bt
      if (col < kp) { r[0] = col; return 1; }
      r[0] = col;       // kp + c
      r[1] = col + 1;   // kp + c + 1
      return 2;
    };
    // X1 = G1 B (mz x mm), X2 = G2 D (mz x mm)
    std::vector<cplx> X1((size_t)mz * mm), X2((size_t)mz * mm);
    for (int j = 0; j < mm; ++j) {
      int rr[2];
      const int nr = rows_of(j, rr);
      const cplx dj = j < kp ? cplx(1.0) : cplx(a[j - kp]);
      for (int i = 0; i < mz; ++i) {
        cplx acc = 0;
        for (int t = 0; t < nr; ++t) acc += G1(i, rr[t]) * Bcol(j, rr[t]);
        X1[i + (size_t)j * mz] = acc;
        X2[i + (size_t)j * mz] = G2(i, j) * dj;
      }
    }
    std::vector<double> Pd(2 * (size_t)mm * mm), Qd(2 * (size_t)mm * mm);
    for (int j = 0; j < mm; ++j)
      for (int i = 0; i < mm; ++i) {
        int rr[2];
        const int nr = rows_of(i, rr);
        cplx p = 0, q = 0;
        for (int t = 0; t < nr; ++t) {
          const cplx f = std::conj(Btcol(i, rr[t]));
          p += f * X1[rr[t] + (size_t)j * mz];
          q += f * X2[rr[t] + (size_t)j * mz];
        }
        Pd[2 * (i + (size_t)j * mm)] = p.real();
        Pd[2 * (i + (size_t)j * mm) + 1] = p.imag();
        Qd[2 * (i + (size_t)j * mm)] = q.real();
        Qd[2 * (i + (size_t)j * mm) + 1] = q.imag();
      }
    std::vector<double> Ws(2 * (size_t)mm * mm), Wls(2 * (size_t)mm * mm);
    m = rbicg_host_eig_select(mm, Pd.data(), Qd.data(), k, real_problem ? 1 : 0, Ws.data(), Wls.data());
    if (m < 0) {
      J.err = std::string("harmonic Ritz problem failed: ") + rbicg_last_error();
      return -1;
    }
    // U_j = [U_p, R] (D W), U~_j = [U~_p, R~] (Dt W~), Dt = blockdiag(I, diag(at))
    J.Wc.assign((size_t)mm * m, 0.0);
    J.Wtc.assign((size_t)mm * m, 0.0);
    for (int c = 0; c < m; ++c)
      for (int l = 0; l < mm; ++l) {
        const cplx w = cplx(Ws[2 * (l + (size_t)c * mm)], Ws[2 * (l + (size_t)c * mm) + 1]);
        const cplx wl = cplx(Wls[2 * (l + (size_t)c * mm)], Wls[2 * (l + (size_t)c * mm) + 1]);
        J.Wc[l + (size_t)c * mm] = (l < kp ? cplx(1.0) : cplx(a[l - kp])) * w;
        J.Wtc[l + (size_t)c * mm] = (l < kp ? cplx(1.0) : at[l - kp]) * wl;
      }
  }
  J.m = m;
  return 0;
}

// Enqueue U_j, U~_j into (Ua, Uta), C = A U_j, C~ = A^H U~_j and the Grams of
// [C, C~] (biorthogonalization input); record the job's event.
template <class V, class M>
int job_stage2(rbicg_s *h, CycleJob &J) {
  const int m = J.m;
  if (m > 0) {
    TRY(tsgemm<V>(h, J.XU, J.Wc, m, h->Ua, 4));
    TRY(tsgemm<V>(h, J.XUt, J.Wtc, m, h->Uta, 5));
    op_spmm<V, M>(h, false, (const V *)h->Ua, (V *)h->Ca, h->ld, m);
    op_spmm<V, M>(h, true, (const V *)h->Uta, (V *)h->Cta, h->ld, m);
    HIPCHECK(hipGetLastError());
    std::vector<const void *> X;
    for (int j = 0; j < m; ++j) X.push_back(col_ptr(h->Ca, j, h));
    for (int j = 0; j < m; ++j) X.push_back(col_ptr(h->Cta, j, h));
    J.g2y = gram_group(2 * m, sizeof(V) == 16 ? 1 : 0);
    TRY(gram_enqueue<V>(h, X, X));
  }
  HIPCHECK(hipEventRecord(J.ev, h->st));
  J.stage = 3;
  return 0;
}

// Host part 2 (no HIP calls): biorthogonalizing transforms from the Grams.
int job_host3(const rbicg_s *h, CycleJob &J) {
  const int m = J.m;
  if (m == 0) {
    J.p = 0;
    return 0;
  }
  const int w = 2 * m;
  const std::vector<cplx> G = gram_parse(h->hG, w, w, J.g2y);
  std::vector<double> Gcc(2 * m * m), Gtt(2 * m * m), Gtc(2 * m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const cplx a = G[(size_t)i * w + j], b = G[(size_t)(m + i) * w + m + j], c = G[(size_t)(m + i) * w + j];
      Gcc[2 * (i + j * m)] = a.real(); Gcc[2 * (i + j * m) + 1] = a.imag();
      Gtt[2 * (i + j * m)] = b.real(); Gtt[2 * (i + j * m) + 1] = b.imag();
      Gtc[2 * (i + j * m)] = c.real(); Gtc[2 * (i + j * m) + 1] = c.imag();
    }
  std::vector<double> TU(2 * m * m), TUt(2 * m * m);
  const int p = rbicg_host_biorth(m, Gcc.data(), Gtt.data(), Gtc.data(), svd_tol_eff(h), TU.data(), TUt.data());
  if (p < 0) {
    J.err = std::string("biorthogonalization failed: ") + rbicg_last_error();
    return -1;
  }
  J.p = p;
  J.TU.resize((size_t)m * p);
  J.TUt.resize((size_t)m * p);
  for (size_t t = 0; t < (size_t)m * p; ++t) {
    J.TU[t] = cplx(TU[2 * t], TU[2 * t + 1]);
    J.TUt[t] = cplx(TUt[2 * t], TUt[2 * t + 1]);
  }
  if (J.setup != 0 && p > 0) {
    // blocks for the next cycle (Sec. 4.4): U_j = Phi_j (W TU), U~_j = Phi~_j (W~ TU~)
    sec44::Mat T1(m, p), T2(m, p);
    for (int c = 0; c < p; ++c)
      for (int i = 0; i < m; ++i) {
        T1(i, c) = J.TU[i + (size_t)c * m];
        T2(i, c) = J.TUt[i + (size_t)c * m];
      }
    J.Xnext = sec44::next_blocks(J.X, sec44::mul(J.Wn, T1), sec44::mul(J.Wtn, T2), J.B, J.Bt, J.G, J.Gt);
  }
  return 0;
}

// Enqueue the rotations of (Ua, Ca, Uta, Cta) into the given outputs.
template <class V>
int apply_biorth(rbicg_s *h, int m, int p, const std::vector<cplx> &TU, const std::vector<cplx> &TUt,
                 void *Uo, void *Uto, void *Co, void *Cto) {
  if (p == 0) return 0;
  std::vector<const void *> XU, XC, XUt, XCt;
  for (int j = 0; j < m; ++j) {
    XU.push_back(col_ptr(h->Ua, j, h));
    XC.push_back(col_ptr(h->Ca, j, h));
    XUt.push_back(col_ptr(h->Uta, j, h));
    XCt.push_back(col_ptr(h->Cta, j, h));
  }
  TRY(tsgemm<V>(h, XU, TU, p, Uo, 0));
  TRY(tsgemm<V>(h, XC, TU, p, Co, 1));
  TRY(tsgemm<V>(h, XUt, TUt, p, Uto, 2));
  TRY(tsgemm<V>(h, XCt, TUt, p, Cto, 3));
  return 0;
}

template <class V>
int job_stage4(rbicg_s *h, CycleJob &J) {
  if (J.p > 0) {
    const int nxt = h->have_cyc ? 1 - h->cur : h->cur;
    TRY(apply_biorth<V>(h, J.m, J.p, J.TU, J.TUt, h->Uc[nxt], h->Utc[nxt], h->Cc[nxt], h->Ctc[nxt]));
    h->cur = nxt;
    h->kcyc = J.p;
    h->have_cyc = true;
  }
  // the Sec. 4.4 blocks carry to the next cycle only after a cycle set up by
  // them (or by T) that kept a space
  h->rec.valid = J.setup != 0 && J.p > 0;
  if (h->rec.valid) {
    h->rec.run_start = J.run_start;
    h->rec.cycle = J.cycle;
    h->rec.X = std::move(J.Xnext);
    h->rec.rn_last2 = J.rn_last2;
    h->rec.at_last = J.at_last;
  }
  J.stage = 5;
  return 0;
}

// Synchronous biorthogonalization of (Ua, Uta) with m columns into the
// system's recycle space (rbicg_set_recycle, rbicg_update_recycle).
template <class V, class M>
int biorth_sync(rbicg_s *h, int m) {
  TRY(ilu_check(h));
  CycleJob J;
  J.m = m;
  HIPCHECK(hipEventCreateWithFlags(&J.ev, hipEventDisableTiming));
  int rc = 0;
  if (m > 0) {
    op_spmm<V, M>(h, false, (const V *)h->Ua, (V *)h->Ca, h->ld, m);
    op_spmm<V, M>(h, true, (const V *)h->Uta, (V *)h->Cta, h->ld, m);
    std::vector<const void *> X;
    for (int j = 0; j < m; ++j) X.push_back(col_ptr(h->Ca, j, h));
    for (int j = 0; j < m; ++j) X.push_back(col_ptr(h->Cta, j, h));
    J.g2y = gram_group(2 * m, sizeof(V) == 16 ? 1 : 0);
    rc = gram_enqueue<V>(h, X, X);
    if (rc >= 0) rc = sync(h);
    if (rc >= 0 && job_host3(h, J) < 0) rc = rbicg_fail(RBICG_EINVAL, "%s", J.err.c_str());
    if (rc >= 0) rc = apply_biorth<V>(h, m, J.p, J.TU, J.TUt, h->U, h->Ut, h->C, h->Ct);
    if (rc >= 0) rc = sync(h);
  }
  if (rc < 0) return rc;
  return J.p;
}

// ------------------------------------------------------------------ solve
template <class V> constexpr int ndv() { return sizeof(V) == 16 ? 2 : 1; }

// dots (a_i, b_i) -> host values (complex)
template <class V>
int host_dots(rbicg_s *h, const V *a0, const V *b0, const V *a1, const V *b1, const V *a2,
              const V *b2, cplx out[3]) {
  launch_dots<V>(h->st, h->nb, h->n, a0, b0, a1, b1, a2, b2, h->partial, h->S->red);
  HIPCHECK(hipGetLastError());
  TRY(pull_scalars(h));
  const int nd = ndv<V>();
  for (int i = 0; i < 3; ++i)
    out[i] = cplx(h->hS->red[i * nd], nd == 2 ? h->hS->red[i * nd + 1] : 0.0);
  return 0;
}

template <class V, class M>
int solve_impl(rbicg_s *h, const V *b, const V *bt, V *x, V *xt, double tol, rbicg_stats *stp,
               bool inner = false) {
  rbicg_stats st{};
  const int n = h->n, ld = h->ld, s = h->opt.s, nb = h->nb;
  TRY(ilu_check(h));
  if (h->ilu && h->batch) return rbicg_fail(RBICG_EINVAL, "a preconditioned handle cannot be batched");
  Sell<M> A = view_A<M>(h), AH = view_AH<M>(h);
  hipEvent_t ev0, ev1;
  HIPCHECK(hipEventCreate(&ev0));
  HIPCHECK(hipEventCreate(&ev1));
  HIPCHECK(hipEventRecord(ev0, h->st));
  const bool update = h->opt.update && h->opt.k > 0;
  h->have_cyc = false;
  h->rec.valid = false;
  // Sec. 4.4 set-up: the cycle jobs read the restrictions and two extra dual
  // ring slots (rt_col)
  const bool rec_mode = update && h->zlog != nullptr;
  // FP32 storage (inner solves): every iteration re-projects r_{i-1}, r~_{i-1}
  // onto the complements of range(C), range(C~) inside k_it1/k_it2 (a no-op in
  // exact arithmetic; see k_it2)
  int rp = 0;
  V *r = (V *)h->r, *rt = (V *)h->rt;
  int ks = h->ksys;  // recycle dimension of the current run (a stalled run drops it)
  const V *U = (const V *)h->U, *Ut = (const V *)h->Ut, *C = (const V *)h->C, *Ct = (const V *)h->Ct;
  cplx d[3];
  double bn = 0.0, btn = 0.0;  // from the first pass's scalar read (below)
  const int nd = ndv<V>();
  int total = 0, restarts = 0, reseeds = 0, status = ST_MAXIT;
  double relres = NAN, relres_dual = NAN;
  bool first = true;
  std::vector<double> fulllog;
  std::deque<std::unique_ptr<CycleJob>> jobs;
  const bool guard = !inner && h->opt.stall_window > 0;
  if (ks > 0 && guard) {  // initial guesses, for a restart after a stall
    HIPCHECK(hipMemcpyAsync(h->xs0, x, (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
    HIPCHECK(hipMemcpyAsync(h->xts0, xt, (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
  }
  while (true) {
    rp = (inner && VK<V>::kind == 0 && sizeof(V) == 4 && ks > 0) ? 1 : 0;
    // eq. minusXR: r_{-1} = b - A x, projection with C, C~.  On the first
    // pass ||b||, ||b~|| and the unprojected ||r||, ||r~|| (the scale when b
    // or b~ vanishes) go to red[16..] and red[24..] and come back with the
    // initial scalars: one host round trip.
    if (first)
      launch_dots<V>(h->st, nb, n, b, b, bt, bt, nullptr, nullptr, h->partial, h->S->red + 16);
    op_residual<V, M>(h, false, b, x, r);
    op_residual<V, M>(h, true, bt, xt, rt);
    if (first)
      launch_dots<V>(h->st, nb, n, r, r, rt, rt, nullptr, nullptr, h->partial, h->S->red + 24);
    if (ks > 0) {
      launch_restrict<V>(h->st, nb, n, r, Ct, rt, C, ks, ld, h->partial, h->S->gbuf);
      launch_expand2<V>(h->st, n, x, U, 1.0, r, C, -1.0, xt, Ut, 1.0, rt, Ct, -1.0, ks, ld, h->S->gbuf);
    }
    launch_init_p3<V>(h->st, nb, n, r, rt, h->P3);
    launch_fin_red(h->st, h->P3, nb, 2 + ndv<V>(), h->S->red);
    HIPCHECK(hipGetLastError());
    TRY(pull_scalars(h));
    double rn = std::sqrt(std::fabs(h->hS->red[0])), rtn = std::sqrt(std::fabs(h->hS->red[1]));
    cplx rho(h->hS->red[2], ndv<V>() == 2 ? h->hS->red[3] : 0.0);
    // Algorithm 2 step 3: re-seed x~ if (r_0, r~_0) vanishes
    while (std::abs(rho) <= 1e-14 * rn * rtn && rn > 0 && reseeds < 3) {
      launch_reseed<V>(h->st, xt, (size_t)n, (unsigned long long)(h->opt.seed + reseeds));
      op_residual<V, M>(h, true, bt, xt, rt);
      if (first)  // the unprojected dual residual of the re-seeded guess (scale when b~ = 0)
        launch_dots<V>(h->st, nb, n, rt, rt, nullptr, nullptr, nullptr, nullptr, h->partial,
                       h->S->red + 24 + nd);
      if (ks > 0) {
        launch_restrict<V>(h->st, nb, n, r, Ct, rt, C, ks, ld, h->partial, h->S->gbuf);
        launch_expand2<V>(h->st, n, nullptr, U, 0.0, nullptr, C, 0.0, xt, Ut, 1.0, rt, Ct, -1.0, ks, ld, h->S->gbuf);
      }
      launch_init_p3<V>(h->st, nb, n, r, rt, h->P3);
      launch_fin_red(h->st, h->P3, nb, 2 + ndv<V>(), h->S->red);
      TRY(pull_scalars(h));
      rn = std::sqrt(std::fabs(h->hS->red[0]));
      rtn = std::sqrt(std::fabs(h->hS->red[1]));
      rho = cplx(h->hS->red[2], ndv<V>() == 2 ? h->hS->red[3] : 0.0);
      ++reseeds;
    }
    if (first) {
      // reference norms ||b||, ||b~||; a vanishing one is replaced by the
      // unprojected initial residual (after any re-seed)
      const double *rd = h->hS->red;
      bn = std::sqrt(std::fabs(rd[16]));
      btn = std::sqrt(std::fabs(rd[16 + nd]));
      if (bn == 0.0) bn = std::sqrt(std::fabs(rd[24]));
      if (btn == 0.0) btn = std::sqrt(std::fabs(rd[24 + nd]));
      if (bn == 0.0) bn = 1.0;
      if (btn == 0.0) btn = 1.0;
    }
    first = false;
    const int run_start = total;
    // scalar block for the run
    Scalars *hs = h->hS;
    std::memset(hs, 0, sizeof(Scalars));
    hs->tol = tol;
    hs->bn = bn;
    hs->btn = btn;
    hs->iter = total;
    hs->maxit = h->opt.maxit;
    hs->stag_base = total;
    if (inner) {
      hs->stag_s = h->opt.s;
      hs->stag_w = FP32_NOPROGRESS_CYCLES;
      hs->stag_div = 1;
      hs->stag_lim = std::sqrt(tol);
    } else if (ks > 0 && guard) {
      // stall guard (opts.stall_window; not in the paper)
      hs->stag_s = h->opt.s;
      hs->stag_w = h->opt.stall_window;
      hs->stag_div = 1;
      hs->stag_lim = 0.0;
    }
    const bool conv0 = rn <= tol * bn && rtn <= tol * btn;
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
      launch_fill_zero<V>(h->st, (V *)ring_col(h->Z, 0, s + 1, 0, h), (size_t)ld);
      launch_fill_zero<V>(h->st, (V *)ring_col(h->Zt, 0, s + 1, 0, h), (size_t)ld);
    }
    int pc = 0;
    int launched = total;          // iterations enqueued
    int known = total;             // iterations known to be complete
    int done = hs->done, dev_status = hs->status;
    int completed = total;
    const int chunk_def = h->opt.chunk > 0 ? h->opt.chunk : 8;
    struct Flight {
      int upto, slot, chunk_start, chunk;
      bool prof;
    };
    std::deque<Flight> flight;
    int slot_next = 0;
    const bool real_problem = (VK<V>::kind == 0);

    // advance the job queue; blocking: wait for what the front job needs
    // blocking: spin on the event (a sleeping wait adds wake-up latency to
    // the cycle-end chain) and run the host parts on this thread (deferred),
    // which saves the start of a worker when nothing else is left to overlap
    auto ev_ready = [&](hipEvent_t ev, bool blocking) -> hipError_t {
      hipError_t q = hipEventQuery(ev);
      while (blocking && q == hipErrorNotReady) {
        std::this_thread::yield();
        q = hipEventQuery(ev);
      }
      return q;
    };
    auto fut_ready = [](std::future<int> &f, bool blocking) {
      return blocking || f.wait_for(std::chrono::seconds(0)) != std::future_status::timeout;
    };
    auto advance = [&](bool blocking) -> int {
      bool progress = true;
      while (progress && !jobs.empty()) {
        progress = false;
        CycleJob &J = *jobs.front();
        if (J.stage == 0) {
          JobStream js(h);
          J.t_begin = std::chrono::steady_clock::now();
          TRY(job_begin<V>(h, J));
          progress = true;
        } else if (J.stage == 1) {
          const hipError_t q = ev_ready(J.ev, blocking);
          if (q == hipSuccess) {
            J.fut = std::async(blocking ? std::launch::deferred : std::launch::async, [h, &J, real_problem]() {
              const auto t0 = std::chrono::steady_clock::now();
              const int r = job_host1(h, J, real_problem);
              J.host_ms[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
              return r;
            });
            J.stage = 2;
            progress = true;
          } else if (q != hipErrorNotReady) {
            return rbicg_fail(RBICG_EHIP, "cycle event: %s", hipGetErrorString(q));
          }
        } else if (J.stage == 2) {
          if (fut_ready(J.fut, blocking)) {
            if (J.fut.get() < 0) return rbicg_fail(RBICG_EINVAL, "%s", J.err.c_str());
            JobStream js(h);
            TRY((job_stage2<V, M>(h, J)));
            progress = true;
          }
        } else if (J.stage == 3) {
          const hipError_t q = ev_ready(J.ev, blocking);
          if (q == hipSuccess) {
            J.fut = std::async(blocking ? std::launch::deferred : std::launch::async, [h, &J]() {
              const auto t0 = std::chrono::steady_clock::now();
              const int r = job_host3(h, J);
              J.host_ms[1] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
              return r;
            });
            J.stage = 4;
            progress = true;
          } else if (q != hipErrorNotReady) {
            return rbicg_fail(RBICG_EHIP, "cycle event: %s", hipGetErrorString(q));
          }
        } else if (J.stage == 4) {
          // install only once the cycle is known to have been completed
          if (J.e <= known && fut_ready(J.fut, blocking)) {
            if (J.fut.get() < 0) return rbicg_fail(RBICG_EINVAL, "%s", J.err.c_str());
            {
              JobStream js(h);
              TRY(job_stage4<V>(h, J));
            }
            h->prof_cyc[0] += 1;
            h->prof_cyc[1] += J.host_ms[0];
            h->prof_cyc[2] += J.host_ms[1];
            h->prof_cyc[3] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - J.t_begin).count();
            st.cycles++;
            jobs.pop_front();  // (its destructor frees the events)
            progress = true;
          }
        }
        if (blocking) break;
      }
      return 0;
    };

    // read the scalars of the oldest chunk in flight; while it runs, move the
    // cycle jobs along (each stage change is noticed at once instead of once
    // per chunk, so a job's stages do not wait for the iterations)
    auto read_one = [&]() -> int {
      if (flight.empty()) return 0;
      const Flight f = flight.front();
      flight.pop_front();
      while (true) {
        const hipError_t q = hipEventQuery(h->sev[f.slot]);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) return rbicg_fail(RBICG_EHIP, "chunk event: %s", hipGetErrorString(q));
        if (update && !jobs.empty()) TRY(advance(false));
        std::this_thread::yield();
      }
      const Scalars &sc = h->hS[f.slot];
      if (sc.done) {
        done = 1;
        dev_status = sc.status;
        completed = sc.iter;
      } else {
        completed = f.upto;
      }
      known = std::max(known, completed);
      if (f.prof) {
        const int eb = f.slot * 3 * f.chunk;
        double kb[2];
        kernel_bytes(h, ks, kb);
        for (int c = 0; c < completed - f.chunk_start && c < f.chunk; ++c)
          for (int kk = 0; kk < 2; ++kk) {
            float ms = 0;
            HIPCHECK(hipEventElapsedTime(&ms, h->pev[eb + 3 * c + kk], h->pev[eb + 3 * c + kk + 1]));
            h->prof_ms[kk] += ms;
            h->prof_n[kk] += 1;
            h->prof_bytes[kk] += kb[kk];
          }
      }
      return 0;
    };

    // while this run iterates, a batch it is attached to counts it among the
    // solves whose chunks it waits for
    struct BatchGuard {
      rbicg_batch b;
      explicit BatchGuard(rbicg_batch bb) : b(bb) {
        if (b) batch_enter(b);
      }
      ~BatchGuard() {
        if (b) batch_leave(b);
      }
    } batch_guard(h->batch);
    while (true) {
      // keep up to two chunks in flight
      while (!done && (int)flight.size() < 2 && launched < h->opt.maxit) {
        const int in_run = launched - run_start;
        const int cyc = in_run / s;
        // the ring set of cycle cyc was last used by cycle cyc-2: its job must
        // have enqueued all reads of that set first
        if (update) {
          auto must_wait = [&]() {
            for (const auto &j : jobs)
              if (j->cycle <= cyc - 2 && j->stage < 3) return true;
            return false;
          };
          const auto tw = std::chrono::steady_clock::now();
          while (!done && must_wait()) {
            const int before = jobs.front()->stage;
            const size_t nj = jobs.size();
            TRY(advance(true));
            if (jobs.size() == nj && jobs.front()->stage == before) TRY(read_one());
          }
          h->prof_cyc[4] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tw).count();
          if (done) break;
          // the job stream's reads of this ring set (job of cycle cyc-2, its
          // stages 1-2 enqueued: checked just above) precede this cycle's writes
          if (in_run % s == 0)
            for (const auto &j : jobs)
              if (j->cycle <= cyc - 2) HIPCHECK(hipStreamWaitEvent(h->st, j->ev, 0));
          // first chunk of cycle cyc >= 1: the z of cycle cyc-1's last iteration
          // seeds slot 0 of this cycle's set
          if (cyc >= 1 && in_run % s == 0) {
            HIPCHECK(hipMemcpyAsync(ring_col(h->Z, cyc % 2, s + 1, 0, h), ring_col(h->Z, (cyc - 1) % 2, s + 1, s, h),
                                    (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
            HIPCHECK(hipMemcpyAsync(ring_col(h->Zt, cyc % 2, s + 1, 0, h), ring_col(h->Zt, (cyc - 1) % 2, s + 1, s, h),
                                    (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
            if (rec_mode)  // v~_{(j-1)s} of Upsilon~_j: the previous cycle's last r~_{i-1}
              HIPCHECK(hipMemcpyAsync(rt_col(h, cyc % 2, s + 1), rt_col(h, (cyc - 1) % 2, s - 1),
                                      (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
          }
        }
        int chunk = chunk_def;
        if (update) chunk = std::min(chunk, s - (in_run % s));
        chunk = std::min(chunk, h->opt.maxit - launched);
        const int chunk_start = launched;
        // profiling: time every opts.profile-th chunk (events between launches)
        const bool prof = !h->batch && !h->ilu && h->opt.profile > 0 && (int)h->pev.size() >= 8 * chunk &&
                          (h->prof_chunks++ % h->opt.profile) == 0;
        const int eb = (slot_next % 2) * 3 * chunk;
        // attached to a batch: the chunk's kernel arguments are handed to it
        BatchChunk bc;
        for (int c = 0; c < chunk; ++c) {
          const int it = launched + 1;
          const int pos = (it - 1 - run_start) % s;
          const int set = ((it - 1 - run_start) / s) % 2;
          V *capR = nullptr, *capRt = nullptr, *capZ = nullptr, *capZt = nullptr;
          if (update) {
            capR = (V *)ring_col(h->R, set, s, pos, h);
            capRt = (V *)rt_col(h, set, pos);
            capZ = (V *)ring_col(h->Z, set, s + 1, pos + 1, h);
            capZt = (V *)ring_col(h->Zt, set, s + 1, pos + 1, h);
          }
          V *pn = (V *)h->p[1 - pc], *ptn = (V *)h->pt[1 - pc];
          // when updating, z and z~ live in their cycle ring slots (written once)
          V *zw = capZ ? capZ : (V *)h->z, *ztw = capZt ? capZt : (V *)h->zt;
          double *zl = rec_mode && ks > 0 ? h->zlog : nullptr;
          if (h->batch) {
            const It1Args<V, M> a1{A, AH, r, (const V *)h->p[pc], rt, (const V *)h->pt[pc], pn, ptn,
                                   zw, ztw, C, Ct, ks, ld, capR, capRt, capZ, capZt,
                                   h->P3, h->P1, h->S, h->log, it, it == run_start + 1 ? 1 : 0, rp,
                                   0, 0};
            const It2Args<V> a2{n, x, xt, r, rt, pn, ptn, zw, ztw, C, Ct,
                                ks, ld, h->P1, h->P3, h->S, h->log, it, rp, zl, h->zstride, 0, 0};
            bc.it1.insert(bc.it1.end(), (const char *)&a1, (const char *)&a1 + sizeof(a1));
            bc.it2.insert(bc.it2.end(), (const char *)&a2, (const char *)&a2 + sizeof(a2));
            pc = 1 - pc;
            ++launched;
            continue;
          }
          if (prof) HIPCHECK(hipEventRecord(h->pev[eb + 3 * c], h->st));
          if (h->ilu) {
            // k_it1's work split around the preconditioned operator
            launch_op_dir<V>(h->st, nb, n, r, (const V *)h->p[pc], rt, (const V *)h->pt[pc], pn, ptn,
                             capR, capRt, h->P3, h->S, h->log, it, it == run_start + 1 ? 1 : 0);
            ilu_apply<V, M>(h, pn, zw, ptn, ztw, h->S);
            launch_op_restr<V>(h->st, nb, n, zw, ztw, ptn, C, Ct, ks, ld, nullptr, nullptr, h->P1, h->S);
          } else {
            launch_it1<V, M>(h->st, nb, A, AH, r, (const V *)h->p[pc], rt, (const V *)h->pt[pc], pn,
                             ptn, zw, ztw, C, Ct, ks, ld, capR, capRt, capZ, capZt, h->P3,
                             h->P1, h->S, h->log, it, it == run_start + 1 ? 1 : 0, rp);
          }
          if (prof) HIPCHECK(hipEventRecord(h->pev[eb + 3 * c + 1], h->st));
          launch_it2<V>(h->st, nb, n, x, xt, r, rt, pn, ptn, zw, ztw, C,
                        Ct, ks, ld, h->P1, h->P3, h->S, h->log, it, rp, zl, h->zstride);
          if (prof) HIPCHECK(hipEventRecord(h->pev[eb + 3 * c + 2], h->st));
          pc = 1 - pc;
          ++launched;
        }
        // stopping test of the chunk's last iteration, then its scalars to the host
        const int slot = slot_next % 2;
        // (k_itfin writes done, status and iter into host slot `slot` itself; the
        // event's completion makes them visible to the host)
        if (h->batch) {
          bc.kind = batch_kind<V, M>();
          bc.one_row = iter_one_row(n, nb);
          bc.nb = nb;
          bc.lds = it1_lds_bytes<V>(ks, rp);
          bc.len = chunk;
          bc.fin = ItfinArgs{h->P3, nb, h->S, h->log, launched + 1, launched == run_start ? 1 : 0,
                             h->hSd + slot};
          bc.st = h->st;
          TRY(batch_submit(h->batch, bc));
        } else {
          launch_itfin<V>(h->st, nb, h->P3, h->S, h->log, launched + 1, launched == run_start ? 1 : 0,
                          h->hSd + slot);
        }
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipEventRecord(h->sev[slot], h->st));
        flight.push_back({launched, slot, chunk_start, chunk, prof});
        ++slot_next;
        if (update && (launched - run_start) % s == 0) {
          const int c = (launched - run_start) / s - 1;  // cycle c just ended
          if (rec_mode)  // v~_{js+1} of Upsilon~_j: the dual residual after the cycle
            HIPCHECK(hipMemcpyAsync(rt_col(h, c % 2, s), rt, (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
          auto J = std::make_unique<CycleJob>();
          J->cycle = c;
          J->e = launched;
          J->set = c % 2;
          J->run_start = run_start;
          J->rn0 = rn;
          J->rho0 = rho;
          HIPCHECK(hipEventCreateWithFlags(&J->ev, hipEventDisableTiming));
          HIPCHECK(hipEventCreateWithFlags(&J->ready, hipEventDisableTiming));
          HIPCHECK(hipEventRecord(J->ready, h->st));
          jobs.push_back(std::move(J));
        }
      }
      if (update) TRY(advance(false));
      if (flight.empty()) break;
      TRY(read_one());
      if (done) break;  // a chunk may still be in flight: drained below
    }
    if (!done) {
      // maxit reached without the stopping test firing
      completed = launched;
      dev_status = ST_MAXIT;
      known = completed;
    }
    total = completed;
    status = dev_status;
    const bool stalled = status == ST_DIVERGED && guard;
    // Algorithm 2 step 7 and the true residuals need nothing from the chunk
    // still in flight (its launches do nothing once the stopping test has
    // fired) or from the cycle updates: they are enqueued first, behind that
    // chunk on the iteration stream, and their reductions are read after the
    // drains below
    if (!stalled) {
      // x -= U zeta_c, x~ -= U~ zeta~_c
      if (ks > 0)
        launch_expand2<V>(h->st, n, x, U, -1.0, nullptr, C, 0.0, xt, Ut, -1.0, nullptr, Ct, 0.0, ks, ld, h->S->zc);
      if (!inner) {
        op_residual<V, M>(h, false, b, x, (V *)h->t1);
        op_residual<V, M>(h, true, bt, xt, (V *)h->t2);
        launch_dots<V>(h->st, nb, n, (V *)h->t1, (V *)h->t1, (V *)h->t2, (V *)h->t2, nullptr, nullptr,
                       h->partial, h->S->red);
        HIPCHECK(hipGetLastError());
      }
    }
    // the chunk still in flight (its launches returned at once)
    while (!flight.empty()) {
      HIPCHECK(hipEventSynchronize(h->sev[flight.front().slot]));
      flight.pop_front();
    }
    // cycles that ended after the last completed iteration never happened
    while (!jobs.empty() && jobs.back()->e > completed) {
      CycleJob &J = *jobs.back();
      if (J.stage == 2 || J.stage == 4) J.fut.wait();
      if (J.stage >= 1) (void)hipEventSynchronize(J.ev);
      jobs.pop_back();
    }
    // finish the remaining updates of this run; later work on the iteration
    // stream (next run, next system's recycle space) is ordered after them
    while (!jobs.empty()) TRY(advance(true));
    if (update) {
      HIPCHECK(hipEventRecord(h->jev, h->jst));
      HIPCHECK(hipStreamWaitEvent(h->st, h->jev, 0));
    }
    // keep this run's log
    if (total > run_start) {
      std::vector<double> tmp((size_t)(total - run_start) * LOG_STRIDE);
      HIPCHECK(hipMemcpy(tmp.data(), h->log + (size_t)(run_start + 1) * LOG_STRIDE,
                         tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (size_t t = 0; t < tmp.size(); t += LOG_STRIDE) tmp[t + 9] = restarts;
      fulllog.insert(fulllog.end(), tmp.begin(), tmp.end());
    }
    if (stalled) {
      // stall guard: start again from the initial guesses without the
      // recycle space (the cycle spaces of the stalled run are dropped too)
      HIPCHECK(hipMemcpyAsync(x, h->xs0, (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
      HIPCHECK(hipMemcpyAsync(xt, h->xts0, (size_t)n * h->vb, hipMemcpyDeviceToDevice, h->st));
      ks = 0;
      h->ksys = 0;
      h->have_cyc = false;
      if (restarts < h->opt.max_restarts && total < h->opt.maxit) {
        ++restarts;
        continue;
      }
      status = ST_MAXIT;
      break;
    }
    if (inner) break;  // the FP64 outer loop checks the true residual
    // true residuals (reductions enqueued before the drain)
    TRY(pull_scalars(h));
    const double tr = std::sqrt(std::fabs(h->hS->red[0])), trt = std::sqrt(std::fabs(h->hS->red[nd]));
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
  h->last_dev_status = status;
  if (h->ilu) {  // a triangular solve's dependency wait gave up: results invalid
    int e = 0;
    HIPCHECK(hipMemcpy(&e, h->ilu->err, sizeof(int), hipMemcpyDeviceToHost));
    if (e) return rbicg_fail(RBICG_EHIP, "triangular solve: dependency wait exceeded its bound");
  }
  st.status = (status == ST_CONVERGED || status == ST_STAGNATED)
                  ? RBICG_OK
                  : (status == ST_BREAKDOWN ? RBICG_BREAKDOWN : RBICG_NOT_CONVERGED);
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
  const int p = biorth_sync<V, M>(h, k);
  if (p < 0) return p;
  h->ksys = p;
  return 0;
}

// FP32-inner / FP64-outer iterative refinement (RBICG_F32_IN_F64_OUT).  Outer
// step: r = b - A x, r~ = b~ - A^H x~ with the FP64 matrix; stop when both
// relative true residuals are <= tol; else round r, r~ to float, solve
// A d = r, A^H d~ = r~ with the float RBiCG (FP64 reductions, float matrix
// values and vectors) to inner_tol relative, and add d, d~ to x, x~ in FP64.
// The latest cycle's recycle space carries over to the next outer step,
// re-biorthogonalized (cut svd_tol_eff).  Inner solves also stop at a cycle
// end without progress (stagnated near the tolerance: the iterate is used;
// diverged: the correction is discarded, the recycle space dropped and the
// next inner solve taken in FP64 by plain BiCG); a correction that raises
// max(||r||/||b||, ||r~||/||b~||) is taken back and the recycle space dropped.
int solve_mixed(rbicg_s *h, const double *b, const double *bt, double *x, double *xt, double tol,
                rbicg_stats *stp) {
  rbicg_stats st{};
  const int n = h->n;
  const Sell<double> A = h->mat->A.view<double>(), AH = h->mat->AH.view<double>();
  hipEvent_t ev0, ev1;
  HIPCHECK(hipEventCreate(&ev0));
  HIPCHECK(hipEventCreate(&ev1));
  HIPCHECK(hipEventRecord(ev0, h->st));
  cplx d[3];
  TRY(host_dots<double>(h, b, b, bt, bt, nullptr, nullptr, d));
  double bn = std::sqrt(std::fabs(d[0].real())), btn = std::sqrt(std::fabs(d[1].real()));
  if (bn == 0.0) bn = 1.0;
  if (btn == 0.0) btn = 1.0;
  const int k_first = h->ksys;
  int outer = 0, inner_total = 0, cycles = 0, status = RBICG_NOT_CONVERGED;
  double rel = NAN, relt = NAN;
  double prev = 0.0;     // residual measure before the last applied correction
  bool applied = false;  // d32, dt32 (or d64, dt64) hold the last applied correction
  bool applied64 = false, escalate = false;
  int fp64_inner = 0;
  auto residuals = [&]() -> int {
    launch_residual<double, double>(h->st, A, b, x, h->r64);
    launch_residual<double, double>(h->st, AH, bt, xt, h->rt64);
    TRY(host_dots<double>(h, h->r64, h->r64, h->rt64, h->rt64, nullptr, nullptr, d));
    rel = std::sqrt(std::fabs(d[0].real())) / bn;
    relt = std::sqrt(std::fabs(d[1].real())) / btn;
    return 0;
  };
  while (true) {
    TRY(residuals());
    if (applied && std::max(rel, relt) > prev) {
      // the correction made things worse: take it back, drop the recycle space
      if (applied64) {
        launch_add_d2d(h->st, x, h->d64, -1.0, (size_t)n);
        launch_add_d2d(h->st, xt, h->dt64, -1.0, (size_t)n);
      } else {
        launch_add_f2d(h->st, x, h->d32, -1.0, (size_t)n);
        launch_add_f2d(h->st, xt, h->dt32, -1.0, (size_t)n);
      }
      h->ksys = 0;
      h->have_cyc = false;
      TRY(residuals());
    }
    applied = false;
    if (rel <= tol && relt <= tol) {
      status = RBICG_OK;
      break;
    }
    if (outer >= h->opt.max_outer || inner_total >= h->opt.maxit) break;
    if (escalate) {
      // FP64 inner solve (plain BiCG) for this outer step, after a diverged FP32 one
      if (!h->h64) {
        rbicg_opts o = h->opt;
        o.prec = RBICG_F64;
        o.k = 0;
        o.update = 0;
        o.profile = 0;
        TRY(rbicg_create_on(h->mat, &o, &h->h64));
      }
      launch_fill_zero<double>(h->st, h->d64, (size_t)n);
      launch_fill_zero<double>(h->st, h->dt64, (size_t)n);
      rbicg_stats ist{};
      const int rc = solve_impl<double, double>(h->h64, h->r64, h->rt64, h->d64, h->dt64, h->opt.inner_tol, &ist);
      inner_total += ist.iters;
      ++outer;
      ++fp64_inner;
      escalate = false;
      if (rc < 0 && rc != RBICG_BREAKDOWN) return rc;
      if (rc == RBICG_BREAKDOWN) {
        status = RBICG_BREAKDOWN;
        break;
      }
      prev = std::max(rel, relt);
      applied = true;
      applied64 = true;
      launch_add_d2d(h->st, x, h->d64, 1.0, (size_t)n);
      launch_add_d2d(h->st, xt, h->dt64, 1.0, (size_t)n);
      HIPCHECK(hipGetLastError());
      continue;
    }
    if (h->have_cyc) {
      void *Us = h->Uc[h->cur], *Uts = h->Utc[h->cur];
      const int kc = h->kcyc;
      h->have_cyc = false;
      TRY((install_recycle<float, float>(h, Us, Uts, kc)));
    }
    launch_d2f(h->st, h->r64, h->b32, (size_t)n);
    launch_d2f(h->st, h->rt64, h->bt32, (size_t)n);
    launch_fill_zero<float>(h->st, h->d32, (size_t)n);
    launch_fill_zero<float>(h->st, h->dt32, (size_t)n);
    rbicg_stats ist{};
    const int rc = solve_impl<float, float>(h, h->b32, h->bt32, h->d32, h->dt32, h->opt.inner_tol, &ist, true);
    inner_total += ist.iters;
    cycles += ist.cycles;
    st.reseeds += ist.reseeds;
    if (rc < 0 && rc != RBICG_BREAKDOWN) return rc;
    ++outer;
    if (h->last_dev_status == ST_DIVERGED || h->last_dev_status == ST_BREAKDOWN) {
      // discard the correction; continue without a recycle space, the next
      // inner solve in FP64
      h->ksys = 0;
      h->have_cyc = false;
      escalate = true;
      continue;
    }
    prev = std::max(rel, relt);
    applied = true;
    applied64 = false;
    launch_add_f2d(h->st, x, h->d32, 1.0, (size_t)n);
    launch_add_f2d(h->st, xt, h->dt32, 1.0, (size_t)n);
    HIPCHECK(hipGetLastError());
  }
  HIPCHECK(hipEventRecord(ev1, h->st));
  HIPCHECK(hipEventSynchronize(ev1));
  float ms = 0;
  HIPCHECK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  st.status = status;
  st.iters = inner_total;
  st.outer_steps = outer;
  st.restarts = fp64_inner;
  st.cycles = cycles;
  st.k_used = k_first;
  st.relres = rel;
  st.relres_dual = relt;
  st.time_ms = ms;
  st.alg_bytes = alg_bytes_iter(h, k_first) * inner_total;
  if (stp) *stp = st;
  return status;
}

// =========================================================== shifted pairs
int shift_ws(rbicg_s *h, int S) {
  if (h->sw && h->sw->Scap >= S) return 0;
  delete h->sw;
  h->sw = new ShiftWs();
  ShiftWs &w = *h->sw;
  w.Scap = SHMAX;
  w.kcap = std::min(h->kcap, KSH);
  auto al = [&](void **p, size_t bytes) -> int {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) return rbicg_fail(RBICG_ENOMEM, "hipMalloc(%zu) failed", bytes);
    w.allocs.push_back(*p);
    return 0;
  };
  const size_t vb = (size_t)h->ld * sizeof(cd) * SHMAX;
  void **vecs[] = {(void **)&w.R, (void **)&w.Rt, (void **)&w.P[0], (void **)&w.P[1], (void **)&w.Pt[0],
                   (void **)&w.Pt[1], (void **)&w.Z, (void **)&w.Zt, (void **)&w.X, (void **)&w.Xt};
  for (void **v : vecs) TRY(al(v, vb));
  const size_t bb = (size_t)h->ld * sizeof(cd) * std::max(1, 2 * w.kcap);
  TRY(al((void **)&w.BU, bb));
  TRY(al((void **)&w.BUt, bb));
  TRY(al((void **)&w.Y, sizeof(cd) * 2 * KSH * SHMAX));
  TRY(al((void **)&w.Yt, sizeof(cd) * 2 * KSH * SHMAX));
  TRY(al((void **)&w.Yx, sizeof(cd) * KSH * SHMAX));
  TRY(al((void **)&w.Yxt, sizeof(cd) * KSH * SHMAX));
  // Gram shapes: the bases against themselves (4k x 4k at most) at the start
  // of a sweep, [bases, p~..] (4k + S columns) against [z.., z~.., p~..] (3S)
  // in every iteration
  const size_t mx = (size_t)std::max(1, 4 * w.kcap), gmax = std::max(mx * mx, (mx + SHMAX) * 3 * SHMAX);
  w.gpart_bytes = (size_t)gram_chunks(h->n) * gmax * 2 * sizeof(double);
  TRY(al((void **)&w.gpart, w.gpart_bytes));
  w.G_bytes = gmax * 2 * sizeof(double);
  TRY(al((void **)&w.G, w.G_bytes));
  TRY(al((void **)&w.P3, (size_t)sh_blocks(h->n) * SHMAX * 4 * sizeof(double)));
  w.reccap = h->opt.maxit + 2;
  TRY(al((void **)&w.rec, (size_t)w.reccap * SHMAX * SH_LOG * sizeof(double)));
  TRY(al((void **)&w.Sh, sizeof(ShScalars)));
  TRY(al((void **)&w.Co, sizeof(ShCoef)));
  HIPCHECK(hipHostMalloc((void **)&w.hSh, 2 * sizeof(ShScalars), hipHostMallocDefault));
  HIPCHECK(hipHostGetDevicePointer((void **)&w.hShd, w.hSh, 0));
  HIPCHECK(hipHostMalloc((void **)&w.hCo, sizeof(ShCoef), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&w.hG, gmax * 2 * sizeof(double), hipHostMallocDefault));
  for (auto &e : w.ev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return 0;
}

// G = X^H Y (mx <= 128 columns of X) into w.G on the device, row-major
// (i, j) complex; my must fit one column group of the Gram kernel.
int shift_gram(rbicg_s *h, const std::vector<const void *> &X, const std::vector<const void *> &Y) {
  ShiftWs &w = *h->sw;
  const int mx = (int)X.size(), my = (int)Y.size();
  if (mx < 1 || mx > RBICG_MAXCOLS || my < 1 || my > gram_group(mx, 1))
    return rbicg_fail(RBICG_EINVAL, "shifted Gram shape %d x %d unsupported", mx, my);
  const int nchunks = gram_chunks(h->n);
  if ((size_t)nchunks * mx * my * 2 * sizeof(double) > w.gpart_bytes)
    return rbicg_fail(RBICG_EINVAL, "shifted Gram workspace too small");
  ColList xl{}, yl{};
  for (int i = 0; i < mx; ++i) xl.p[i] = X[i];
  for (int j = 0; j < my; ++j) yl.p[j] = Y[j];
  launch_gram<cd>(h->st, h->n, xl, mx, yl, my, w.gpart, w.G, nchunks);
  HIPCHECK(hipGetLastError());
  return 0;
}

// Two Grams in one launch into w.G: X[0, mx0)^H Y[0, my0), then (mx1 > 0)
// X[x1, x1 + mx1)^H Y[y1, y1 + my1), each row-major.
int shift_gram2(rbicg_s *h, const std::vector<const void *> &X, const std::vector<const void *> &Y,
                int mx0, int my0, int x1, int mx1, int y1, int my1) {
  ShiftWs &w = *h->sw;
  const int nx = (int)X.size(), ny = (int)Y.size();
  const int mxm = std::max(mx0, mx1), mym = std::max(my0, my1);
  if (nx > RBICG_MAXCOLS || ny > RBICG_MAXCOLS || mx0 < 1 || my0 < 1 || mx0 > nx || my0 > ny ||
      mx1 < 0 || (mx1 > 0 && (x1 < 0 || x1 + mx1 > nx || y1 < 0 || my1 < 1 || y1 + my1 > ny)) ||
      mym > gram_group(mxm, 1))
    return rbicg_fail(RBICG_EINVAL, "shifted Gram shapes %d x %d, %d x %d unsupported", mx0, my0, mx1, my1);
  const int nchunks = gram_chunks(h->n);
  const size_t ent = (size_t)mx0 * my0 + (mx1 > 0 ? (size_t)mx1 * my1 : 0);
  if ((size_t)nchunks * ent * 2 * sizeof(double) > w.gpart_bytes || ent * 2 * sizeof(double) > w.G_bytes)
    return rbicg_fail(RBICG_EINVAL, "shifted Gram workspace too small");
  ColList xl{}, yl{};
  for (int i = 0; i < nx; ++i) xl.p[i] = X[i];
  for (int j = 0; j < ny; ++j) yl.p[j] = Y[j];
  launch_gram2<cd>(h->st, h->n, xl, mx0, yl, my0, x1, mx1, y1, mx1 > 0 ? my1 : 0, w.gpart, w.G, nchunks);
  HIPCHECK(hipGetLastError());
  return 0;
}

inline cd *bcol(cd *base, int j, const rbicg_s *h) { return base + (size_t)j * h->ld; }

// C = B S with S = [sigma I; -I] (2k x k): entries of S^H M S for a 2k x 2k
// Hermitian-form block M (host, row-major complex), as a k x k column-major
// interleaved array for rbicg_host_biorth.
static void shifted_form(const std::vector<cplx> &M, int ldm, int r0, int c0, int k, cplx a, cplx b,
                         std::vector<double> &out) {
  // out(i, j) = sum_{u, v} conj(S_a(u, i)) M(r0 + u, c0 + v) S_b(v, j),
  // S_a = [a I; -I], S_b = [b I; -I]
  out.assign(2 * (size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      const cplx m11 = M[(size_t)(r0 + i) * ldm + c0 + j], m12 = M[(size_t)(r0 + i) * ldm + c0 + k + j];
      const cplx m21 = M[(size_t)(r0 + k + i) * ldm + c0 + j], m22 = M[(size_t)(r0 + k + i) * ldm + c0 + k + j];
      const cplx v = std::conj(a) * m11 * b - std::conj(a) * m12 - m21 * b + m22;
      out[2 * (i + (size_t)j * k)] = v.real();
      out[2 * (i + (size_t)j * k) + 1] = v.imag();
    }
}

template <class M>
int solve_shifted_impl(rbicg_s *h, int S, const double *sigma, const cd *b, const cd *c, cd *Xc,
                       cd *Xtc, double tol, int update_from, rbicg_stats *stats, size_t rhs_stride = 0) {
  // rhs_stride 0: one b, c for every shift; n: column s of b, c for shift s
  const int n = h->n, ld = h->ld;
  auto bcol_of = [&](int s) { return b + (size_t)s * rhs_stride; };
  auto ccol_of = [&](int s) { return c + (size_t)s * rhs_stride; };
  std::vector<cplx> sig(S);
  for (int s = 0; s < S; ++s) sig[s] = cplx(sigma[2 * s], sigma[2 * s + 1]);
  const bool update = h->opt.update && h->opt.k > 0;
  int u0 = -1;
  if (update) {
    u0 = update_from;
    if (u0 < 0) {
      u0 = 0;
      for (int s = 1; s < S; ++s)
        if (std::abs(sig[s]) < std::abs(sig[u0])) u0 = s;
    }
    if (u0 >= S) return rbicg_fail(RBICG_EINVAL, "update_from %d out of range", u0);
  }
  // the batch kernels address 9 columns of ld complex entries with 32-bit
  // byte offsets
  if ((size_t)ld * 9 * sizeof(cd) >= ((size_t)1 << 32))
    return rbicg_fail(RBICG_EINVAL, "n = %d too large for batched shifted solves", n);
  TRY(shift_ws(h, S));
  ShiftWs &w = *h->sw;
  const cd *Usrc = (const cd *)(h->have_cyc ? h->Uc[h->cur] : h->U);
  const cd *Utsrc = (const cd *)(h->have_cyc ? h->Utc[h->cur] : h->Ut);
  int k = h->have_cyc ? h->kcyc : h->ksys;
  if (k > w.kcap) return rbicg_fail(RBICG_EINVAL, "recycle dimension %d exceeds %d for shifted solves", k, w.kcap);
  const int k2 = 2 * k;
  h->shifted = false;
  // shared basis [U, A U] and [U~, A^H U~]
  if (k > 0) {
    HIPCHECK(hipMemcpy2DAsync(w.BU, ld * sizeof(cd), Usrc, ld * sizeof(cd), n * sizeof(cd), k, hipMemcpyDeviceToDevice, h->st));
    HIPCHECK(hipMemcpy2DAsync(w.BUt, ld * sizeof(cd), Utsrc, ld * sizeof(cd), n * sizeof(cd), k, hipMemcpyDeviceToDevice, h->st));
    launch_spmm<cd, M>(h->st, view_A<M>(h), w.BU, bcol(w.BU, k, h), ld, k);
    launch_spmm<cd, M>(h->st, view_AH<M>(h), w.BUt, bcol(w.BUt, k, h), ld, k);
    HIPCHECK(hipGetLastError());
  }
  // batch = every shift except the update shift
  std::vector<int> bidx;
  for (int s = 0; s < S; ++s)
    if (s != u0) bidx.push_back(s);
  const int Sb = (int)bidx.size();
  for (int s = 0; s < S; ++s) stats[s] = rbicg_stats{};
  hipEvent_t ev0, ev1;
  HIPCHECK(hipEventCreate(&ev0));
  HIPCHECK(hipEventCreate(&ev1));
  if (Sb > 0) {
    HIPCHECK(hipEventRecord(ev0, h->st));
    ShScalars *hs = &w.hSh[0];
    std::memset(hs, 0, sizeof(ShScalars));
    hs->tol = tol;
    hs->S = Sb;
    hs->k2 = k2;
    hs->maxit = h->opt.maxit;
    // per-shift biorthogonalization from the basis Grams (Sec. 4.3 for
    // C_s = sigma_s U - A U, C~_s = conj(sigma_s) U~ - A^H U~)
    if (k > 0) {
      std::vector<const void *> Xl;
      for (int j = 0; j < k2; ++j) Xl.push_back(bcol(w.BU, j, h));
      for (int j = 0; j < k2; ++j) Xl.push_back(bcol(w.BUt, j, h));
      // in column groups that fit the Gram kernel; group j0 is row-major m4 x gg
      const int m4 = 2 * k2, grp = gram_group(m4, 1);
      for (int j0 = 0; j0 < m4; j0 += grp) {
        const int gg = std::min(grp, m4 - j0);
        std::vector<const void *> Yg(Xl.begin() + j0, Xl.begin() + j0 + gg);
        TRY(shift_gram(h, Xl, Yg));
        HIPCHECK(hipMemcpyAsync(w.hG + 2 * (size_t)m4 * j0, w.G, (size_t)m4 * gg * 2 * sizeof(double),
                                hipMemcpyDeviceToHost, h->st));
        TRY(sync(h));
      }
      std::vector<cplx> G((size_t)m4 * m4);
      for (int j0 = 0; j0 < m4; j0 += grp) {
        const int gg = std::min(grp, m4 - j0);
        const double *blk = w.hG + 2 * (size_t)m4 * j0;
        for (int i = 0; i < m4; ++i)
          for (int j = 0; j < gg; ++j)
            G[(size_t)i * m4 + j0 + j] = cplx(blk[2 * ((size_t)i * gg + j)], blk[2 * ((size_t)i * gg + j) + 1]);
      }
      std::memset(w.hCo, 0, sizeof(ShCoef));
      std::vector<double> Gcc, Gtt, Gtc, TU(2 * (size_t)k * k), TUt(2 * (size_t)k * k);
      for (int j = 0; j < Sb; ++j) {
        const cplx sg = sig[bidx[j]], sgc = std::conj(sg);
        // C^H C with C = BU [sg I; -I]; C~^H C~ with C~ = BUt [conj(sg) I; -I];
        // C~^H C (rows of BUt against columns of BU)
        shifted_form(G, m4, 0, 0, k, sg, sg, Gcc);
        shifted_form(G, m4, k2, k2, k, sgc, sgc, Gtt);
        shifted_form(G, m4, k2, 0, k, sgc, sg, Gtc);
        const int p = rbicg_host_biorth(k, Gcc.data(), Gtt.data(), Gtc.data(), svd_tol_eff(h), TU.data(), TUt.data());
        if (p < 0) return rbicg_fail(RBICG_EINVAL, "shift %d: biorthogonalization failed: %s", bidx[j], rbicg_last_error());
        hs->p[j] = p;
        auto tu = [&](int i, int l) { return cplx(TU[2 * (i + (size_t)l * k)], TU[2 * (i + (size_t)l * k) + 1]); };
        auto tut = [&](int i, int l) { return cplx(TUt[2 * (i + (size_t)l * k)], TUt[2 * (i + (size_t)l * k) + 1]); };
        auto put = [](double *m, size_t idx, cplx v) { m[2 * idx] = v.real(); m[2 * idx + 1] = v.imag(); };
        // K = TUt^H [sg I, -I]  (zeta = K [U~, A^H U~]^H z), Kt = TU^H [conj(sg) I, -I]
        // L = [sg I; -I] TU, Lt = [conj(sg) I; -I] TUt, T = TU, Tt = TUt
        for (int l = 0; l < p; ++l)
          for (int i = 0; i < k; ++i) {
            put(w.hCo->K[j], (size_t)l * k2 + i, std::conj(tut(i, l)) * sg);
            put(w.hCo->K[j], (size_t)l * k2 + k + i, -std::conj(tut(i, l)));
            put(w.hCo->Kt[j], (size_t)l * k2 + i, std::conj(tu(i, l)) * sgc);
            put(w.hCo->Kt[j], (size_t)l * k2 + k + i, -std::conj(tu(i, l)));
            put(w.hCo->L[j], (size_t)i * p + l, sg * tu(i, l));
            put(w.hCo->L[j], (size_t)(k + i) * p + l, -tu(i, l));
            put(w.hCo->Lt[j], (size_t)i * p + l, sgc * tut(i, l));
            put(w.hCo->Lt[j], (size_t)(k + i) * p + l, -tut(i, l));
            put(w.hCo->T[j], (size_t)i * p + l, tu(i, l));
            put(w.hCo->Tt[j], (size_t)i * p + l, tut(i, l));
          }
      }
      HIPCHECK(hipMemcpyAsync(w.Co, w.hCo, sizeof(ShCoef), hipMemcpyHostToDevice, h->st));
    }
    // norms of b, c (per shift when every shift has its own right-hand sides)
    cplx d[3];
    for (int j = 0; j < Sb; ++j) {
      if (j == 0 || rhs_stride) {
        TRY(host_dots<cd>(h, bcol_of(bidx[j]), bcol_of(bidx[j]), ccol_of(bidx[j]), ccol_of(bidx[j]),
                          nullptr, nullptr, d));
        double bn = std::sqrt(std::fabs(d[0].real())), cn = std::sqrt(std::fabs(d[1].real()));
        hs->bn[j] = bn == 0.0 ? 1.0 : bn;
        hs->btn[j] = cn == 0.0 ? 1.0 : cn;
      } else {
        hs->bn[j] = hs->bn[0];
        hs->btn[j] = hs->btn[0];
      }
      hs->sig[2 * j] = sig[bidx[j]].real();
      hs->sig[2 * j + 1] = sig[bidx[j]].imag();
    }
    HIPCHECK(hipMemcpyAsync(w.Sh, hs, sizeof(ShScalars), hipMemcpyHostToDevice, h->st));
    // x_{-1} and r_{-1} = b - (sigma I - A) x_{-1} per shift (eq. minusXR before the projection)
    for (int j = 0; j < Sb; ++j) {
      const int s = bidx[j];
      HIPCHECK(hipMemcpyAsync(bcol(w.X, j, h), Xc + (size_t)s * n, n * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
      HIPCHECK(hipMemcpyAsync(bcol(w.Xt, j, h), Xtc + (size_t)s * n, n * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
      h->shifted = true;
      h->shift = sig[s];
      launch_residual<cd, M>(h->st, view_A<M>(h), bcol_of(s), bcol(w.X, j, h), bcol(w.R, j, h));
      launch_residual<cd, M>(h->st, view_AH<M>(h), ccol_of(s), bcol(w.Xt, j, h), bcol(w.Rt, j, h));
      h->shifted = false;
      launch_fill_zero<cd>(h->st, bcol(w.P[0], j, h), (size_t)n);
      launch_fill_zero<cd>(h->st, bcol(w.Pt[0], j, h), (size_t)n);
    }
    const int nb3 = sh_blocks(n), nbe = sh_sub_blocks(n);
    ColList BUl{}, BUtl{};
    for (int j = 0; j < k2; ++j) {
      BUl.p[j] = bcol(w.BU, j, h);
      BUtl.p[j] = bcol(w.BUt, j, h);
    }
    // Gram operands: [U~, A^H U~]^H [r..] and [U, A U]^H [r~..] at the start;
    // in every iteration [U~, A^H U~, p~..]^H [z..] and [U, A U]^H [z~.., p~..]
    // (p~ is the direction buffer the iteration writes, which alternates)
    std::vector<const void *> Xg, Yr, Xz[2], Yz[2];
    for (int j = 0; j < k2; ++j) Xg.push_back(bcol(w.BUt, j, h));
    for (int j = 0; j < k2; ++j) Xg.push_back(bcol(w.BU, j, h));
    for (int j = 0; j < Sb; ++j) Yr.push_back(bcol(w.R, j, h));
    for (int j = 0; j < Sb; ++j) Yr.push_back(bcol(w.Rt, j, h));
    for (int c = 0; c < 2; ++c) {
      for (int j = 0; j < k2; ++j) Xz[c].push_back(bcol(w.BUt, j, h));
      for (int j = 0; j < Sb; ++j) Xz[c].push_back(bcol(w.Pt[1 - c], j, h));
      for (int j = 0; j < k2; ++j) Xz[c].push_back(bcol(w.BU, j, h));
      for (int j = 0; j < Sb; ++j) Yz[c].push_back(bcol(w.Z, j, h));
      for (int j = 0; j < Sb; ++j) Yz[c].push_back(bcol(w.Zt, j, h));
      for (int j = 0; j < Sb; ++j) Yz[c].push_back(bcol(w.Pt[1 - c], j, h));
    }
    const int g1 = (k2 + Sb) * Sb;  // second Gram of an iteration
    if (k > 0) {
      // eq. minusXR: g = C~'^H r_{-1}; x += U' g, r -= C' g (dual likewise)
      TRY(shift_gram2(h, Xg, Yr, k2, Sb, k2, k2, Sb, Sb));
      launch_sh_coef(h->st, Sb, w.G, Sb, k2 * Sb, Sb, w.Sh, w.Co, w.Y, w.Yt, w.Yx, w.Yxt, 1, w.rec, 0);
      launch_sh_sub(h->st, n, BUl, k2, w.Y, Sb, w.R, w.R, ld, nbe);
      launch_sh_sub(h->st, n, BUtl, k2, w.Yt, Sb, w.Rt, w.Rt, ld, nbe);
      launch_sh_sub(h->st, n, BUl, k, w.Yx, Sb, w.X, w.X, ld, nbe);
      launch_sh_sub(h->st, n, BUtl, k, w.Yxt, Sb, w.Xt, w.Xt, ld, nbe);
    }
    launch_sh2(h->st, n, ld, Sb, w.X, w.Xt, w.R, w.Rt, nullptr, nullptr, nullptr, nullptr, w.BU, w.BUt, 0,
               w.Y, w.Yt, w.Sh, w.P3, nb3, 0);
    HIPCHECK(hipGetLastError());
    // iterations: chunks of 8, two in flight, one scalar download per chunk
    int launched = 0, pc = 0, slot = 0;
    const int chunk = h->opt.chunk > 0 ? h->opt.chunk : 8;
    std::deque<int> flight;
    bool all_done = false;
    while (true) {
      while (!all_done && flight.size() < 2 && launched < h->opt.maxit) {
        const int cnt = std::min(chunk, h->opt.maxit - launched);
        for (int t = 0; t < cnt; ++t) {
          const int it = launched + 1;
          launch_sh_state(h->st, Sb, w.P3, nb3, w.Sh, w.rec, it, it == 1 ? 1 : 0);
          launch_sh1<M>(h->st, view_A<M>(h), view_AH<M>(h), ld, w.R, w.Rt, w.P[pc], w.Pt[pc],
                        w.P[1 - pc], w.Pt[1 - pc], w.Z, w.Zt, w.Sh);
          TRY(shift_gram2(h, Xz[pc], Yz[pc], k2 + Sb, Sb, k2 + Sb, k2, Sb, 2 * Sb));
          launch_sh_coef(h->st, Sb, w.G, Sb, g1, 2 * Sb, w.Sh, w.Co, w.Y, w.Yt, w.Yx, w.Yxt, 0, w.rec, it);
          launch_sh2(h->st, n, ld, Sb, w.X, w.Xt, w.R, w.Rt, w.P[1 - pc], w.Pt[1 - pc], w.Z, w.Zt, w.BU, w.BUt,
                     k2, w.Y, w.Yt, w.Sh, w.P3, nb3, 1);
          pc = 1 - pc;
          ++launched;
        }
        // the chunk's final stopping test writes every shift's done flag into
        // host slot 1 itself; the two chunks in flight share the slot: the
        // device's flags only become set, so a read after the older chunk's
        // event sees that chunk's flags or newer ones
        launch_sh_state(h->st, Sb, w.P3, nb3, w.Sh, w.rec, launched + 1, 0, w.hShd + 1);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipEventRecord(w.ev[slot], h->st));
        flight.push_back(slot);
        slot = 1 - slot;
      }
      if (flight.empty()) break;
      const int sl = flight.front();
      flight.pop_front();
      HIPCHECK(hipEventSynchronize(w.ev[sl]));
      // every shift stopped (the device's all_done flag lags the last stopping test)
      bool every = true;
      for (int j = 0; j < Sb; ++j) every = every && w.hSh[1].done[j];
      if (every) all_done = true;
      if (all_done) {
        while (!flight.empty()) {
          HIPCHECK(hipEventSynchronize(w.ev[flight.front()]));
          flight.pop_front();
        }
        break;
      }
    }
    TRY(sync(h));
    HIPCHECK(hipMemcpy(&w.hSh[1], w.Sh, sizeof(ShScalars), hipMemcpyDeviceToHost));
    // Algorithm 2 step 7: x -= U' zeta_c, x~ -= U~' zeta~_c
    if (k > 0) {
      launch_sh_coef(h->st, Sb, w.G, Sb, g1, 2 * Sb, w.Sh, w.Co, w.Y, w.Yt, w.Yx, w.Yxt, 2, w.rec, 0);
      launch_sh_sub(h->st, n, BUl, k, w.Yx, Sb, w.X, w.X, ld, nbe);
      launch_sh_sub(h->st, n, BUtl, k, w.Yxt, Sb, w.Xt, w.Xt, ld, nbe);
    }
    HIPCHECK(hipEventRecord(ev1, h->st));
    HIPCHECK(hipEventSynchronize(ev1));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, ev0, ev1));
    const ShScalars &fs = w.hSh[1];
    for (int j = 0; j < Sb; ++j) {
      const int s = bidx[j];
      HIPCHECK(hipMemcpyAsync(Xc + (size_t)s * n, bcol(w.X, j, h), n * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
      HIPCHECK(hipMemcpyAsync(Xtc + (size_t)s * n, bcol(w.Xt, j, h), n * sizeof(cd), hipMemcpyDeviceToDevice, h->st));
      // true residuals
      h->shifted = true;
      h->shift = sig[s];
      launch_residual<cd, M>(h->st, view_A<M>(h), bcol_of(s), bcol(w.X, j, h), (cd *)h->t1);
      launch_residual<cd, M>(h->st, view_AH<M>(h), ccol_of(s), bcol(w.Xt, j, h), (cd *)h->t2);
      h->shifted = false;
      TRY(host_dots<cd>(h, (cd *)h->t1, (cd *)h->t1, (cd *)h->t2, (cd *)h->t2, nullptr, nullptr, d));
      rbicg_stats &st = stats[s];
      st.relres = std::sqrt(std::fabs(d[0].real())) / hs->bn[j];
      st.relres_dual = std::sqrt(std::fabs(d[1].real())) / hs->btn[j];
      st.iters = fs.done[j] ? fs.iter[j] : launched;
      const int dst = fs.done[j] ? fs.status[j] : ST_MAXIT;
      const bool ok = dst == ST_CONVERGED && st.relres <= tol && st.relres_dual <= tol;
      st.status = ok ? RBICG_OK : (dst == ST_BREAKDOWN ? RBICG_BREAKDOWN : RBICG_NOT_CONVERGED);
      st.k_used = fs.p[j];
      st.time_ms = ms;
    }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  // the update shift: a single pair with its own cycle-wise recycle update
  if (u0 >= 0) {
    h->shifted = true;
    h->shift = sig[u0];
    int rc = 0;
    if (k > 0) rc = install_recycle<cd, M>(h, w.BU, w.BUt, k);
    else h->ksys = 0;
    if (rc >= 0)
      rc = solve_impl<cd, M>(h, bcol_of(u0), ccol_of(u0), Xc + (size_t)u0 * n, Xtc + (size_t)u0 * n, tol,
                             &stats[u0]);
    h->shifted = false;
    if (rc < 0) return rc;
  }
  int worst = RBICG_OK;
  for (int s = 0; s < S; ++s)
    if (stats[s].status != RBICG_OK) worst = stats[s].status < 0 ? stats[s].status : (worst < 0 ? worst : stats[s].status);
  return worst;
}

template <class F>
int dispatch(rbicg_s *h, F &&f) {
  if (h->vkind == 0) return f((double *)nullptr, (double *)nullptr);
  if (h->vkind == 2) return f((float *)nullptr, (float *)nullptr);
  if (h->mat_complex) return f((cd *)nullptr, (cd *)nullptr);
  return f((cd *)nullptr, (double *)nullptr);
}

int alloc_workspace(rbicg_s *h) {
  HIPCHECK(hipStreamCreateWithFlags(&h->jst, hipStreamNonBlocking));
  HIPCHECK(hipEventCreateWithFlags(&h->jev, hipEventDisableTiming));
  const size_t vbytes = (size_t)h->ld * h->vb;
  void **vecs[] = {&h->r, &h->rt, &h->p[0], &h->p[1], &h->pt[0], &h->pt[1], &h->z, &h->zt,
                   &h->t1, &h->t2, &h->xs0, &h->xts0};
  for (void **v : vecs) TRY(dalloc(h, v, vbytes));
  const size_t kb = vbytes * std::max(1, h->kcap);
  void **bases[] = {&h->U, &h->Ut, &h->C, &h->Ct, &h->Ua, &h->Uta, &h->Ca, &h->Cta,
                    &h->Uc[0], &h->Utc[0], &h->Cc[0], &h->Ctc[0],
                    &h->Uc[1], &h->Utc[1], &h->Cc[1], &h->Ctc[1]};
  for (void **v : bases) TRY(dalloc(h, v, kb));
  if (h->kcap > 0 && h->opt.update) {
    TRY(dalloc(h, &h->R, 2 * vbytes * h->scap));
    TRY(dalloc(h, &h->Rt, 2 * vbytes * (h->scap + 2)));
    TRY(dalloc(h, &h->Z, 2 * vbytes * (h->scap + 1)));
    TRY(dalloc(h, &h->Zt, 2 * vbytes * (h->scap + 1)));
  }
  if (h->vkind == 2) {
    TRY(dalloc(h, (void **)&h->r64, (size_t)h->ld * sizeof(double)));
    TRY(dalloc(h, (void **)&h->rt64, (size_t)h->ld * sizeof(double)));
    TRY(dalloc(h, (void **)&h->d64, (size_t)h->ld * sizeof(double)));
    TRY(dalloc(h, (void **)&h->dt64, (size_t)h->ld * sizeof(double)));
    TRY(dalloc(h, (void **)&h->b32, (size_t)h->ld * sizeof(float)));
    TRY(dalloc(h, (void **)&h->bt32, (size_t)h->ld * sizeof(float)));
    TRY(dalloc(h, (void **)&h->d32, (size_t)h->ld * sizeof(float)));
    TRY(dalloc(h, (void **)&h->dt32, (size_t)h->ld * sizeof(float)));
  }
  TRY(dalloc(h, (void **)&h->S, sizeof(Scalars)));
  HIPCHECK(hipMemset(h->S, 0, sizeof(Scalars)));
  h->logcap = h->opt.maxit + 2;
  TRY(dalloc(h, (void **)&h->log, (size_t)h->logcap * LOG_STRIDE * sizeof(double)));
  if (h->opt.pencil_setup && h->kcap > 0 && h->opt.update && h->vkind != 2) {
    h->zstride = 2 * h->kcap * (h->vkind == 1 ? 2 : 1);
    TRY(dalloc(h, (void **)&h->zlog, (size_t)h->logcap * h->zstride * sizeof(double)));
    HIPCHECK(hipHostMalloc((void **)&h->hzlog, (size_t)(h->scap + 1) * h->zstride * sizeof(double),
                           hipHostMallocDefault));
  }
  h->nb = iter_grid(h->n);
  if (h->opt.blocks > 0) {
    if (h->opt.blocks < iter_grid_min(h->n))
      return rbicg_fail(RBICG_EINVAL, "blocks=%d too few for n=%d (at least %d)", h->opt.blocks, h->n,
                        iter_grid_min(h->n));
    h->nb = h->opt.blocks;
  }
  TRY(dalloc(h, (void **)&h->partial, (size_t)h->nb * 4 * KMAXD * sizeof(double)));
  TRY(dalloc(h, (void **)&h->P1, (size_t)h->nb * (6 * KMAXD + 2) * sizeof(double)));
  TRY(dalloc(h, (void **)&h->P3, (size_t)h->nb * 8 * sizeof(double)));
  const int wx = std::max(2 * h->kcap, h->kcap + h->scap + 1);
  const int wy = std::max(2 * h->kcap, 2 * (h->kcap + h->scap) + 1);
  const int w = std::max(wx, wy);
  h->gpart_bytes = (size_t)gram_chunks(h->n) * wx * 128 * 2 * sizeof(double);
  TRY(dalloc(h, (void **)&h->gpart, h->gpart_bytes));
  TRY(dalloc(h, (void **)&h->Gd, (size_t)wx * wy * 2 * sizeof(double)));
  h->gram_cap = (size_t)wx * wy;
  TRY(dalloc(h, (void **)&h->Wd, 6 * RBICG_WSLOT * sizeof(cd)));
  if (h->opt.profile) {
    const int nev = 8 * std::max(8, h->opt.chunk);
    h->pev.resize(nev);
    // timing-only events: no system-scope fence (cache writeback and
    // invalidation) when they are recorded, so that a bracket holds the
    // kernel and not a flush the untimed launches never pay; the chunk's
    // synchronizing event, recorded after them, orders their read-back
    for (auto &e : h->pev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  HIPCHECK(hipHostMalloc((void **)&h->hS, 2 * sizeof(Scalars), hipHostMallocDefault));
  HIPCHECK(hipHostGetDevicePointer((void **)&h->hSd, h->hS, 0));
  for (auto &e : h->sev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHECK(hipHostMalloc((void **)&h->hG, (size_t)wx * wy * 2 * sizeof(double), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&h->hW, 6 * RBICG_WSLOT * sizeof(cd), hipHostMallocDefault));
  (void)w;
  HIPCHECK(hipHostMalloc((void **)&h->hlog, (size_t)(h->scap + 2) * LOG_STRIDE * sizeof(double), hipHostMallocDefault));
  return 0;
}

int build_matrix(const rbicg_csr *A, const rbicg_csr *AH, rbicg_mat_s *m) {
  HostCsr hA, hAH;
  TRY(read_csr(A, hA));
  if (AH) {
    TRY(read_csr(AH, hAH));
    if (hAH.n != hA.n) return rbicg_fail(RBICG_EINVAL, "A^H size mismatch");
  } else {
    hAH = conj_transpose(hA);
  }
  m->n = hA.n;
  m->complex_vals = hA.complex_vals || hAH.complex_vals;
  const int kind = m->complex_vals ? 1 : 0;
  TRY(upload_sell(hA, kind, m->A));
  TRY(upload_sell(hAH, kind, m->AH));
  TRY(share_pattern(hA, hAH, m->A, m->AH));
  return 0;
}

int attach_matrix(rbicg_s *h, rbicg_mat_s *m, bool own) {
  if (!m) return rbicg_fail(RBICG_EINVAL, "null matrix");
  if (m->n != h->n) return rbicg_fail(RBICG_EINVAL, "matrix size %d does not match handle n=%d", m->n, h->n);
  if (m->complex_vals && h->vkind != 1) return rbicg_fail(RBICG_EINVAL, "complex matrix needs a RBICG_C128 handle");
  if (h->vkind == 2) {
    TRY(m->A.make_f32(h->st));
    TRY(m->AH.make_f32(h->st));
  }
  if (h->own_mat && h->mat && h->mat != m) {
    h->mat->A.release();
    h->mat->AH.release();
    delete h->mat;
  }
  h->mat = m;
  h->own_mat = own;
  h->mat_complex = m->complex_vals;
  return 0;
}

int set_matrix(rbicg_s *h, const rbicg_csr *A, const rbicg_csr *AH) {
  rbicg_mat_s *m = new rbicg_mat_s();
  int rc = build_matrix(A, AH, m);
  if (rc >= 0) rc = attach_matrix(h, m, true);
  if (rc < 0) {
    m->A.release();
    m->AH.release();
    delete m;
  }
  return rc;
}

}  // namespace

// ====================================================================== C ABI
static int check_opts(const rbicg_opts *opt);
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
  o->profile = 0;
  o->stall_window = 0;
  o->pencil_setup = 0;
  o->blocks = 0;
}

extern "C" int rbicg_create(const rbicg_csr *A, const rbicg_csr *AH, const rbicg_opts *opt,
                            rbicg_handle *out) {
  if (!A || !opt || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  TRY(check_opts(opt));
  if (A->n <= 0) return rbicg_fail(RBICG_EINVAL, "n must be positive");
  rbicg_s *h = new rbicg_s();
  h->opt = *opt;
  h->n = A->n;
  h->ld = (A->n + 255) / 256 * 256;
  h->st = (hipStream_t)opt->stream;
  h->vkind = opt->prec == RBICG_C128 ? 1 : (opt->prec == RBICG_F32_IN_F64_OUT ? 2 : 0);
  h->vb = h->vkind == 1 ? 16 : (h->vkind == 2 ? 4 : 8);
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

extern "C" int rbicg_matrix_create(const rbicg_csr *A, const rbicg_csr *AH, rbicg_matrix *out) {
  if (!A || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  rbicg_mat_s *m = new rbicg_mat_s();
  const int rc = build_matrix(A, AH, m);
  if (rc < 0) {
    m->A.release();
    m->AH.release();
    delete m;
    return rc;
  }
  *out = m;
  return RBICG_OK;
}

namespace {
// Same sliced-ELL layout (sizes, slice pointers and column indices).
int same_layout(const DevSell &a, const DevSell &b) {
  if (a.n != b.n || a.nslices != b.nslices || a.nnzpad != b.nnzpad)
    return rbicg_fail(RBICG_EINVAL, "E and A have different sparsity layouts");
  std::vector<int> x(a.nslices + 1), y(a.nslices + 1);
  HIPCHECK(hipMemcpy(x.data(), a.sliceptr, x.size() * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(y.data(), b.sliceptr, y.size() * sizeof(int), hipMemcpyDeviceToHost));
  if (x != y) return rbicg_fail(RBICG_EINVAL, "E and A have different sparsity layouts");
  x.resize(a.nnzpad);
  y.resize(a.nnzpad);
  if (a.nnzpad) {
    HIPCHECK(hipMemcpy(x.data(), a.col, a.nnzpad * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(y.data(), b.col, a.nnzpad * sizeof(int), hipMemcpyDeviceToHost));
  }
  if (x != y) return rbicg_fail(RBICG_EINVAL, "E must be given on A's sparsity pattern");
  return 0;
}

// A complex sliced-ELL matrix with src's layout (values uninitialized).  If
// src borrows its layout, d borrows that of owner (the new matrix's own A).
int alloc_like(const DevSell &src, DevSell &d, const DevSell *owner = nullptr) {
  d.n = src.n;
  d.nslices = src.nslices;
  d.nnzpad = src.nnzpad;
  d.nnz = src.nnz;
  d.vbytes = 16;
  if (src.borrowed && owner) {
    d.sliceptr = owner->sliceptr;
    d.col = owner->col;
    d.borrowed = true;
    HIPCHECK(hipMalloc(&d.val, std::max<size_t>(src.nnzpad, 1) * sizeof(cd)));
    return 0;
  }
  HIPCHECK(hipMalloc((void **)&d.sliceptr, (size_t)(src.nslices + 1) * sizeof(int)));
  HIPCHECK(hipMalloc((void **)&d.col, std::max<size_t>(src.nnzpad, 1) * sizeof(int)));
  HIPCHECK(hipMalloc(&d.val, std::max<size_t>(src.nnzpad, 1) * sizeof(cd)));
  HIPCHECK(hipMemcpy(d.sliceptr, src.sliceptr, (size_t)(src.nslices + 1) * sizeof(int), hipMemcpyDeviceToDevice));
  if (src.nnzpad)
    HIPCHECK(hipMemcpy(d.col, src.col, src.nnzpad * sizeof(int), hipMemcpyDeviceToDevice));
  return 0;
}
}  // namespace

extern "C" int rbicg_matrix_pencil(rbicg_matrix A, rbicg_matrix E, const double *alpha,
                                   const double *beta, void *stream, rbicg_matrix *out) {
  if (!A || !E || !alpha || !beta || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (A->n != E->n) return rbicg_fail(RBICG_EINVAL, "E is %d x %d, A is %d x %d", E->n, E->n, A->n, A->n);
  hipStream_t st = (hipStream_t)stream;
  rbicg_mat_s *m = *out;
  if (!m) {
    TRY(same_layout(A->A, E->A));
    TRY(same_layout(A->AH, E->AH));
    m = new rbicg_mat_s();
    m->n = A->n;
    m->complex_vals = true;
    m->pencil_a = A;
    m->pencil_e = E;
    int rc = alloc_like(A->A, m->A);
    if (rc >= 0) rc = alloc_like(A->AH, m->AH, &m->A);
    if (rc < 0) {
      m->A.release();
      m->AH.release();
      delete m;
      return rc;
    }
    *out = m;
  } else if (m->pencil_a != A || m->pencil_e != E) {
    return rbicg_fail(RBICG_EINVAL, "out is not a pencil of these matrices");
  }
  const cd al = {alpha[0], alpha[1]}, be = {beta[0], beta[1]};
  // alpha E + beta A and its conjugate transpose conj(alpha) E^H + conj(beta) A^H
  launch_pencil(st, m->A.nnzpad, A->A.val, A->A.vbytes == 16, E->A.val, E->A.vbytes == 16, al, be,
                (cd *)m->A.val);
  launch_pencil(st, m->AH.nnzpad, A->AH.val, A->AH.vbytes == 16, E->AH.val, E->AH.vbytes == 16,
                cd{al.x, -al.y}, cd{be.x, -be.y}, (cd *)m->AH.val);
  HIPCHECK(hipGetLastError());
  return RBICG_OK;
}

// ------------------------------------------- split ILU(0), red-black
// Host set-up of the red-black ILU(0) split preconditioner (the transforms
// run in precond.hip): two-colouring, pivots, the black block
// M_B = (D_B - A_BR D_R^{-1} A_RB) S_B^{-1} of the split-preconditioned
// operator, and the device data of the transforms.
struct rbicg_rbilu_s {
  int n = 0, nb = 0;
  bool complex_vals = false;
  RbDev dev;
  RbRefresh ref;                  // device maps of rbicg_rbilu_refresh
  std::vector<int> rowptr, col;   // A's pattern, for the refresh's check
  rbicg_mat_s *black = nullptr;   // M_B and M_B^H (owned)
  void *cR = nullptr;  // n-long scratch of the right-hand-side transform
  std::vector<void *> allocs;
  ~rbicg_rbilu_s() {
    for (void *p : allocs) (void)hipFree(p);
    if (black) {
      black->A.release();
      black->AH.release();
      delete black;
    }
  }
};

namespace {
template <class T>
int rb_upload(rbicg_rbilu_s *P, const void **dst, const T *src, size_t count) {
  void *p = nullptr;
  HIPCHECK(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
  P->allocs.push_back(p);
  if (count) HIPCHECK(hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice));
  *dst = p;
  return 0;
}

// values as the device type: double (real matrices) or interleaved complex
std::vector<double> rb_values(const std::vector<cplx> &v, bool cplxv) {
  std::vector<double> o(cplxv ? 2 * v.size() : v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    if (cplxv) {
      o[2 * i] = v[i].real();
      o[2 * i + 1] = v[i].imag();
    } else {
      o[i] = v[i].real();
    }
  }
  return o;
}

int rb_upload_vals(rbicg_rbilu_s *P, const void **dst, const std::vector<cplx> &v) {
  const std::vector<double> o = rb_values(v, P->complex_vals);
  return rb_upload(P, dst, o.data(), o.size());
}
}  // namespace

extern "C" int rbicg_rbilu_create(const rbicg_csr *A, rbicg_rbilu *out, rbicg_matrix *black,
                                  int32_t *nb) {
  if (!A || !out || !black || !nb) return rbicg_fail(RBICG_EINVAL, "null argument");
  HostCsr hA;
  TRY(read_csr(A, hA));
  const int n = hA.n;
  std::vector<int> amap;
  const HostCsr hAH = conj_transpose_map(hA, &amap);
  std::vector<cplx> d(n, cplx(0.0, 0.0));
  for (int i = 0; i < n; ++i)
    for (int e = hA.rowptr[i]; e < hA.rowptr[i + 1]; ++e)
      if (hA.col[e] == i) d[i] += hA.val[e];
  for (int i = 0; i < n; ++i)
    if (d[i] == cplx(0.0, 0.0)) return rbicg_fail(RBICG_EINVAL, "zero diagonal entry in row %d", i);
  // two-colouring of the off-diagonal graph of A + A^T (breadth first; each
  // component starts red at its lowest index)
  std::vector<int> color(n, -1), queue;
  queue.reserve(n);
  for (int s0 = 0; s0 < n; ++s0) {
    if (color[s0] >= 0) continue;
    color[s0] = 0;
    queue.assign(1, s0);
    for (size_t q = 0; q < queue.size(); ++q) {
      const int i = queue[q];
      for (const HostCsr *M : {(const HostCsr *)&hA, &hAH})
        for (int e = M->rowptr[i]; e < M->rowptr[i + 1]; ++e) {
          const int j = M->col[e];
          if (j == i) continue;
          if (color[j] < 0) {
            color[j] = 1 - color[i];
            queue.push_back(j);
          } else if (color[j] == color[i]) {
            return rbicg_fail(RBICG_EINVAL, "the off-diagonal graph of A is not two-colourable");
          }
        }
    }
  }
  std::vector<int> bidx(n, -1), blist;
  for (int i = 0; i < n; ++i)
    if (color[i] == 1) {
      bidx[i] = (int)blist.size();
      blist.push_back(i);
    }
  const int nbk = (int)blist.size();
  if (nbk == 0) return rbicg_fail(RBICG_EINVAL, "no black unknowns");
  // rows of S = D_B - A_BR D_R^{-1} A_RB (black numbering), then S_B = diag(S)
  HostCsr hS;
  hS.n = nbk;
  hS.complex_vals = hA.complex_vals;
  hS.rowptr.assign(nbk + 1, 0);
  std::vector<cplx> acc(nbk, cplx(0.0, 0.0));
  std::vector<int> mark(nbk, -1), cols;
  for (int bi = 0; bi < nbk; ++bi) {
    const int i = blist[bi];
    cols.clear();
    auto touch = [&](int bj) {
      if (mark[bj] != bi) {
        mark[bj] = bi;
        acc[bj] = cplx(0.0, 0.0);
        cols.push_back(bj);
      }
    };
    touch(bi);
    acc[bi] += d[i];
    for (int e = hA.rowptr[i]; e < hA.rowptr[i + 1]; ++e) {
      const int k = hA.col[e];
      if (k == i) continue;
      const cplx f = hA.val[e] / d[k];
      for (int g = hA.rowptr[k]; g < hA.rowptr[k + 1]; ++g) {
        const int j = hA.col[g];
        if (j == k) continue;
        touch(bidx[j]);
        acc[bidx[j]] -= f * hA.val[g];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int bj : cols) {
      hS.col.push_back(bj);
      hS.val.push_back(acc[bj]);
    }
    hS.rowptr[bi + 1] = (int)hS.col.size();
  }
  std::vector<cplx> sb(nbk, cplx(0.0, 0.0));
  for (int bi = 0; bi < nbk; ++bi)
    for (int e = hS.rowptr[bi]; e < hS.rowptr[bi + 1]; ++e)
      if (hS.col[e] == bi) sb[bi] = hS.val[e];
  for (int bi = 0; bi < nbk; ++bi)
    if (sb[bi] == cplx(0.0, 0.0)) return rbicg_fail(RBICG_EINVAL, "zero ILU(0) pivot at unknown %d", blist[bi]);
  for (size_t e = 0; e < hS.col.size(); ++e) hS.val[e] /= sb[hS.col[e]];
  // the black block, resident with its conjugate transpose
  rbicg_mat_s *m = new rbicg_mat_s();
  m->n = nbk;
  m->complex_vals = hS.complex_vals;
  std::vector<int> smap;
  const HostCsr hSH = conj_transpose_map(hS, &smap);
  const std::vector<int> sidx = sell_index(hS), shidx = sell_index(hSH);
  std::vector<int> msell(hS.col.size()), mhsell(hS.col.size());
  for (size_t e = 0; e < hS.col.size(); ++e) {
    msell[e] = sidx[e];
    mhsell[e] = shidx[smap[e]];
  }
  int rc = upload_sell(hS, m->complex_vals ? 1 : 0, m->A);
  if (rc >= 0) rc = upload_sell(hSH, m->complex_vals ? 1 : 0, m->AH);
  if (rc >= 0) rc = share_pattern(hS, hSH, m->A, m->AH);
  if (rc < 0) {
    m->A.release();
    m->AH.release();
    delete m;
    return rc;
  }
  // device data of the transforms
  rbicg_rbilu_s *P = new rbicg_rbilu_s();
  P->n = n;
  P->nb = nbk;
  P->complex_vals = hA.complex_vals;
  P->dev.n = n;
  P->dev.nb = nbk;
  rc = rb_upload(P, (const void **)&P->dev.rp, hA.rowptr.data(), hA.rowptr.size());
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->dev.ci, hA.col.data(), hA.col.size());
  if (rc >= 0) rc = rb_upload_vals(P, &P->dev.av, hA.val);
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->dev.hrp, hAH.rowptr.data(), hAH.rowptr.size());
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->dev.hci, hAH.col.data(), hAH.col.size());
  if (rc >= 0) rc = rb_upload_vals(P, &P->dev.hv, hAH.val);
  if (rc >= 0) rc = rb_upload_vals(P, &P->dev.d, d);
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->dev.bidx, bidx.data(), bidx.size());
  if (rc >= 0) rc = rb_upload_vals(P, &P->dev.sb, sb);
  if (rc >= 0) {
    const std::vector<cplx> zero(n, cplx(0.0, 0.0));
    const void *z = nullptr;
    rc = rb_upload_vals(P, &z, zero);
    P->cR = const_cast<void *>(z);
  }
  // maps of the device refresh
  P->ref.nnzm = (int)hS.col.size();
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->ref.amap, amap.data(), amap.size());
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->ref.blist, blist.data(), blist.size());
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->ref.mrp, hS.rowptr.data(), hS.rowptr.size());
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->ref.mci, hS.col.data(), hS.col.size());
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->ref.msell, msell.data(), msell.size());
  if (rc >= 0) rc = rb_upload(P, (const void **)&P->ref.mhsell, mhsell.data(), mhsell.size());
  P->ref.mval = m->A.val;
  P->ref.mhval = m->AH.val;
  P->rowptr = hA.rowptr;
  P->col = hA.col;
  P->black = m;
  if (rc < 0) {
    delete P;
    return rc;
  }
  *out = P;
  *black = m;
  *nb = nbk;
  return RBICG_OK;
}

extern "C" int rbicg_rbilu_refresh(rbicg_rbilu P, const rbicg_csr *A_next, void *stream) {
  if (!P || !A_next) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (A_next->n != P->n || A_next->nnz != (int64_t)P->col.size() ||
      (A_next->values_complex != 0) != P->complex_vals)
    return rbicg_fail(RBICG_EINVAL, "A_next does not match the preconditioner's matrix");
  hipStream_t st = (hipStream_t)stream;
  const size_t nnz = P->col.size();
  bool same;
  if (A_next->on_device) {
    std::vector<int> rp(P->n + 1), ci(nnz);
    HIPCHECK(hipMemcpy(rp.data(), A_next->rowptr, rp.size() * sizeof(int), hipMemcpyDeviceToHost));
    if (nnz) HIPCHECK(hipMemcpy(ci.data(), A_next->colind, nnz * sizeof(int), hipMemcpyDeviceToHost));
    same = rp == P->rowptr && ci == P->col;
  } else {
    same = std::memcmp(A_next->rowptr, P->rowptr.data(), P->rowptr.size() * sizeof(int)) == 0 &&
           (nnz == 0 || std::memcmp(A_next->colind, P->col.data(), nnz * sizeof(int)) == 0);
  }
  if (!same)
    return rbicg_fail(RBICG_EINVAL, "A_next's sparsity pattern differs from the preconditioner's");
  const size_t vb = P->complex_vals ? sizeof(cd) : sizeof(double);
  if (nnz)
    HIPCHECK(hipMemcpyAsync(const_cast<void *>(P->dev.av), A_next->values, nnz * vb,
                            A_next->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (P->complex_vals) launch_rb_refresh<cd>(st, P->dev, P->ref);
  else launch_rb_refresh<double>(st, P->dev, P->ref);
  HIPCHECK(hipGetLastError());
  return RBICG_OK;
}

extern "C" int rbicg_rbilu_refresh_values(rbicg_rbilu P, const void *values, void *stream) {
  if (!P || !values) return rbicg_fail(RBICG_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const size_t nnz = P->col.size();
  const size_t vb = P->complex_vals ? sizeof(cd) : sizeof(double);
  if (nnz)
    HIPCHECK(hipMemcpyAsync(const_cast<void *>(P->dev.av), values, nnz * vb,
                            hipMemcpyDeviceToDevice, st));
  if (P->complex_vals) launch_rb_refresh<cd>(st, P->dev, P->ref);
  else launch_rb_refresh<double>(st, P->dev, P->ref);
  HIPCHECK(hipGetLastError());
  return RBICG_OK;
}

extern "C" int rbicg_rbilu_rhs(rbicg_rbilu P, const void *b, const void *bt, void *bB, void *btB,
                               void *stream) {
  if (!P || !b || !bt || !bB || !btB) return rbicg_fail(RBICG_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (P->complex_vals)
    launch_rb_rhs<cd>(st, P->dev, (const cd *)b, (const cd *)bt, (cd *)bB, (cd *)btB, (cd *)P->cR);
  else
    launch_rb_rhs<double>(st, P->dev, (const double *)b, (const double *)bt, (double *)bB,
                          (double *)btB, (double *)P->cR);
  HIPCHECK(hipGetLastError());
  return RBICG_OK;
}

extern "C" int rbicg_rbilu_solution(rbicg_rbilu P, const void *b, const void *bt, const void *yB,
                                    const void *ytB, void *x, void *xt, void *stream) {
  if (!P || !b || !bt || !yB || !ytB || !x || !xt) return rbicg_fail(RBICG_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (P->complex_vals)
    launch_rb_solution<cd>(st, P->dev, (const cd *)b, (const cd *)bt, (const cd *)yB,
                           (const cd *)ytB, (cd *)x, (cd *)xt);
  else
    launch_rb_solution<double>(st, P->dev, (const double *)b, (const double *)bt,
                               (const double *)yB, (const double *)ytB, (double *)x, (double *)xt);
  HIPCHECK(hipGetLastError());
  return RBICG_OK;
}

extern "C" int rbicg_rbilu_destroy(rbicg_rbilu P) {
  if (!P) return RBICG_OK;
  (void)hipDeviceSynchronize();
  delete P;
  return RBICG_OK;
}

// ------------------------------------------------------ split ILUT
namespace {
int ilu_alloc(rbicg_ilu_s *P, void **dst, size_t bytes) {
  void *p = nullptr;
  HIPCHECK(hipMalloc(&p, std::max<size_t>(bytes, 1)));
  P->allocs.push_back(p);
  *dst = p;
  return 0;
}

int ilu_put(rbicg_ilu_s *P, void **dst, const void *src, size_t bytes) {
  TRY(ilu_alloc(P, dst, bytes));
  if (bytes) HIPCHECK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return 0;
}

int ilu_put_vals(rbicg_ilu_s *P, void **dst, const std::vector<ilut::cplx> &v) {
  std::vector<double> o(P->complex_vals ? 2 * v.size() : v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    if (P->complex_vals) {
      o[2 * i] = v[i].real();
      o[2 * i + 1] = v[i].imag();
    } else {
      o[i] = v[i].real();
    }
  }
  return ilu_put(P, dst, o.data(), o.size() * sizeof(double));
}

// One factor on the device: its strictly triangular entries, the diagonal
// (with_diag) and the level order padded to whole waves.
int ilu_factor_upload(rbicg_ilu_s *P, const ilut::Csr &T, bool lower, bool with_diag,
                      rbicg_ilu_s::Tri &out) {
  const int n = T.n;
  ilut::Csr S;
  S.n = n;
  S.rp.assign(1, 0);
  std::vector<ilut::cplx> d(n, ilut::cplx(1.0, 0.0));
  for (int i = 0; i < n; ++i) {
    for (int e = T.rp[i]; e < T.rp[i + 1]; ++e) {
      const int j = T.ci[e];
      if (j == i) {
        d[i] = T.v[e];
      } else {
        S.ci.push_back(j);
        S.v.push_back(T.v[e]);
      }
    }
    S.rp.push_back((int)S.ci.size());
  }
  std::vector<int> order;
  out.levels = ilut::levels(S, lower, 64, order);
  out.len = (int)order.size();
  out.nnz = (int64_t)S.ci.size();
  TRY(ilu_put(P, (void **)&out.order, order.data(), order.size() * sizeof(int)));
  TRY(ilu_put(P, (void **)&out.rp, S.rp.data(), S.rp.size() * sizeof(int)));
  TRY(ilu_put(P, (void **)&out.ci, S.ci.data(), S.ci.size() * sizeof(int)));
  TRY(ilu_put_vals(P, &out.v, S.v));
  if (with_diag) TRY(ilu_put_vals(P, &out.diag, d));
  return 0;
}
}  // namespace

extern "C" int rbicg_ilut_create(const rbicg_csr *A, double droptol, int32_t fill, double permtol,
                                 rbicg_ilu *out) {
  if (!A || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (!(droptol >= 0.0)) return rbicg_fail(RBICG_EINVAL, "droptol must be >= 0");
  if (!(permtol >= 0.0)) return rbicg_fail(RBICG_EINVAL, "permtol must be >= 0");
  HostCsr hA;
  TRY(read_csr(A, hA));
  ilut::Csr a, L, U;
  a.n = hA.n;
  a.rp = hA.rowptr;
  a.ci = hA.col;
  a.v = hA.val;
  std::string msg;
  std::vector<int> perm;
  const int frc = permtol > 0.0 ? ilut::factor_pivoted(a, droptol, fill, permtol, L, U, perm, msg)
                                : ilut::factor(a, droptol, fill, L, U, msg);
  if (frc < 0) return rbicg_fail(RBICG_EINVAL, "%s", msg.c_str());
  std::unique_ptr<rbicg_ilu_s> P(new rbicg_ilu_s());
  P->n = hA.n;
  P->complex_vals = hA.complex_vals;
  for (int j = 0; j < (int)perm.size(); ++j) P->moved += perm[j] != j ? 1 : 0;
  if (P->moved > 0) {  // the permutation and its inverse, only when columns moved
    std::vector<int> pos(perm.size());
    for (int j = 0; j < (int)perm.size(); ++j) pos[perm[j]] = j;
    TRY(ilu_put(P.get(), (void **)&P->perm, perm.data(), perm.size() * sizeof(int)));
    TRY(ilu_put(P.get(), (void **)&P->pos, pos.data(), pos.size() * sizeof(int)));
  }
  // L: unit lower; U: upper with its diagonal; L^H unit upper; U^H lower
  // with the conjugated diagonal
  TRY(ilu_factor_upload(P.get(), L, true, false, P->L));
  TRY(ilu_factor_upload(P.get(), U, false, true, P->U));
  TRY(ilu_factor_upload(P.get(), ilut::conj_transpose(L), false, false, P->LH));
  TRY(ilu_factor_upload(P.get(), ilut::conj_transpose(U), true, true, P->UH));
  const size_t n = (size_t)P->n;
  for (auto &w : P->ws) {
    for (void *&q : w.q) TRY(ilu_alloc(P.get(), &q, n * sizeof(cd)));
    TRY(ilu_alloc(P.get(), (void **)&w.counter, sizeof(int)));
  }
  TRY(ilu_alloc(P.get(), (void **)&P->err, sizeof(int)));
  HIPCHECK(hipMemset(P->err, 0, sizeof(int)));
  HIPCHECK(hipDeviceSynchronize());
  *out = P.release();
  return RBICG_OK;
}

extern "C" int rbicg_ilu_attach(rbicg_handle h, rbicg_ilu P) {
  if (!h) return rbicg_fail(RBICG_EINVAL, "null handle");
  if (P) {
    if (P->n != h->n || P->complex_vals != h->mat->complex_vals)
      return rbicg_fail(RBICG_EINVAL, "the preconditioner does not match the handle's matrix");
    if (h->vkind == 2) return rbicg_fail(RBICG_EINVAL, "split preconditioning needs an FP64 or complex handle");
    if (h->batch) return rbicg_fail(RBICG_EINVAL, "a batched handle cannot be preconditioned");
  }
  h->ilu = P;
  return RBICG_OK;
}

namespace {
// x = T1^{-1} b, x2 = T2^{-1} b2 on the rhs/solution workspace
template <class V>
int ilu_two_solves(rbicg_ilu P, int f1, const void *b, void *x, int f2, const void *b2, void *x2,
                   hipStream_t st) {
  rbicg_ilu_s::Ws &w = P->ws[2];
  bool done = false;
  if constexpr (std::is_same<V, cd>::value) {  // complex factors need complex vectors
    if (P->complex_vals) {
      ilu_trsv<V, cd>(st, P, w, f1, (const V *)b, (V *)x, f2, (const V *)b2, (V *)x2, nullptr);
      done = true;
    }
  }
  if (!done)
    ilu_trsv<V, double>(st, P, w, f1, (const V *)b, (V *)x, f2, (const V *)b2, (V *)x2, nullptr);
  HIPCHECK(hipGetLastError());
  return RBICG_OK;
}

int ilu_transform(rbicg_ilu P, int f1, const void *b, void *x, int f2, const void *b2, void *x2,
                  int32_t complex_vectors, void *stream) {
  if (!P || !b || !b2 || !x || !x2) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (b == x || b2 == x2) return rbicg_fail(RBICG_EINVAL, "input and output must not alias");
  if (P->complex_vals && !complex_vectors)
    return rbicg_fail(RBICG_EINVAL, "a complex preconditioner needs complex vectors");
  hipStream_t st = (hipStream_t)stream;
  return complex_vectors ? ilu_two_solves<cd>(P, f1, b, x, f2, b2, x2, st)
                         : ilu_two_solves<double>(P, f1, b, x, f2, b2, x2, st);
}

// out[i] = in[map[i]] (ILUTP's column permutation)
int ilu_permute(rbicg_ilu P, const void *in, const int *map, void *out, int32_t complex_vectors,
                hipStream_t st) {
  if (P->complex_vals && !complex_vectors)
    return rbicg_fail(RBICG_EINVAL, "a complex preconditioner needs complex vectors");
  if (complex_vectors) launch_gather<cd>(st, P->n, (const cd *)in, map, (cd *)out);
  else launch_gather<double>(st, P->n, (const double *)in, map, (double *)out);
  HIPCHECK(hipGetLastError());
  return RBICG_OK;
}
}  // namespace

extern "C" int rbicg_ilu_rhs(rbicg_ilu P, const void *b, const void *bt, void *bh, void *ch,
                             int32_t complex_vectors, void *stream) {
  if (!P || !bt) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (!P->perm)  // L^{-1} b, U^{-H} b~
    return ilu_transform(P, 0, b, bh, 3, bt, ch, complex_vectors, stream);
  // L^{-1} b, U^{-H} Q^T b~ with (Q^T b~)[j] = b~[perm[j]]
  void *q = P->ws[2].q[0];
  TRY(ilu_permute(P, bt, P->perm, q, complex_vectors, (hipStream_t)stream));
  return ilu_transform(P, 0, b, bh, 3, q, ch, complex_vectors, stream);
}

extern "C" int rbicg_ilu_solution(rbicg_ilu P, const void *y, const void *yt, void *x, void *xt,
                                  int32_t complex_vectors, void *stream) {
  if (!P || !x) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (!P->perm)  // U^{-1} y, L^{-H} y~
    return ilu_transform(P, 1, y, x, 2, yt, xt, complex_vectors, stream);
  // Q U^{-1} y with (Q t)[c] = t[pos[c]], L^{-H} y~
  void *q = P->ws[2].q[0];
  TRY(ilu_transform(P, 1, y, q, 2, yt, xt, complex_vectors, stream));
  return ilu_permute(P, q, P->pos, x, complex_vectors, (hipStream_t)stream);
}

extern "C" int rbicg_ilu_set_waves(rbicg_ilu P, int32_t waves) {
  if (!P) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (waves < 4 || waves > 65536) return rbicg_fail(RBICG_EINVAL, "waves=%d out of range [4, 65536]", waves);
  P->waves = waves;
  return RBICG_OK;
}

extern "C" int rbicg_ilu_info(rbicg_ilu P, int64_t *info) {
  if (!P || !info) return rbicg_fail(RBICG_EINVAL, "null argument");
  int e = 0;
  HIPCHECK(hipDeviceSynchronize());
  HIPCHECK(hipMemcpy(&e, P->err, sizeof(int), hipMemcpyDeviceToHost));
  info[0] = P->n;
  info[1] = P->L.nnz;
  info[2] = P->U.nnz + P->n;
  info[3] = P->L.levels;
  info[4] = P->U.levels;
  info[5] = e ? 1 : 0;
  info[6] = P->complex_vals ? 1 : 0;
  info[7] = P->moved;
  return RBICG_OK;
}

extern "C" int rbicg_ilu_destroy(rbicg_ilu P) {
  if (!P) return RBICG_OK;
  (void)hipDeviceSynchronize();
  delete P;
  return RBICG_OK;
}

extern "C" int rbicg_matrix_destroy(rbicg_matrix m) {
  if (!m) return RBICG_OK;
  (void)hipDeviceSynchronize();
  m->A.release();
  m->AH.release();
  delete m;
  return RBICG_OK;
}

extern "C" int rbicg_matrix_info(rbicg_matrix m, int64_t *info) {
  if (!m || !info) return rbicg_fail(RBICG_EINVAL, "null argument");
  info[0] = m->n;
  info[1] = m->A.nnz;
  info[2] = (int64_t)m->A.nnzpad;
  info[3] = m->AH.borrowed ? 1 : 0;
  info[4] = m->complex_vals ? 1 : 0;
  return RBICG_OK;
}

int rbicg_matrix_views(rbicg_matrix m, MatViews *out) {
  if (!m || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  out->n = m->n;
  out->complex_vals = m->complex_vals ? 1 : 0;
  out->shared_pattern = m->AH.borrowed ? 1 : 0;
  out->nnz = m->A.nnz;
  if (m->complex_vals) {
    out->Ac = m->A.view<cd>();
    out->AHc = m->AH.view<cd>();
  } else {
    out->A = m->A.view<double>();
    out->AH = m->AH.view<double>();
  }
  return RBICG_OK;
}

static int check_opts(const rbicg_opts *opt) {
  if (opt->k < 0 || opt->k > RBICG_KMAX) return rbicg_fail(RBICG_EINVAL, "k must be in [0, %d]", RBICG_KMAX);
  if (opt->s < 2 || opt->s + opt->k + 1 > 128)
    return rbicg_fail(RBICG_EINVAL, "cycle length s=%d out of range", opt->s);
  if (opt->maxit < 1) return rbicg_fail(RBICG_EINVAL, "maxit must be positive");
  if (opt->chunk < 0 || opt->chunk > 256) return rbicg_fail(RBICG_EINVAL, "chunk out of range");
  if (opt->stall_window < 0) return rbicg_fail(RBICG_EINVAL, "stall_window must be >= 0");
  if (opt->pencil_setup != 0 && opt->pencil_setup != 1)
    return rbicg_fail(RBICG_EINVAL, "pencil_setup must be 0 or 1");
  if (opt->blocks < 0 || opt->blocks > 4096) return rbicg_fail(RBICG_EINVAL, "blocks must be in [0, 4096]");
  if (opt->prec != RBICG_F64 && opt->prec != RBICG_C128 && opt->prec != RBICG_F32_IN_F64_OUT)
    return rbicg_fail(RBICG_EINVAL, "unknown precision mode %d", (int)opt->prec);
  if (opt->prec == RBICG_F32_IN_F64_OUT && (!(opt->inner_tol > 0) || opt->inner_tol >= 1 || opt->max_outer < 1))
    return rbicg_fail(RBICG_EINVAL, "FP32-inner mode needs 0 < inner_tol < 1 and max_outer >= 1");
  return 0;
}

extern "C" int rbicg_create_on(rbicg_matrix A, const rbicg_opts *opt, rbicg_handle *out) {
  if (!A || !opt || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  TRY(check_opts(opt));
  rbicg_s *h = new rbicg_s();
  h->opt = *opt;
  h->n = A->n;
  h->ld = (A->n + 255) / 256 * 256;
  h->st = (hipStream_t)opt->stream;
  h->vkind = opt->prec == RBICG_C128 ? 1 : (opt->prec == RBICG_F32_IN_F64_OUT ? 2 : 0);
  h->vb = h->vkind == 1 ? 16 : (h->vkind == 2 ? 4 : 8);
  h->kcap = opt->k;
  h->scap = opt->s;
  int rc = attach_matrix(h, A, false);
  if (rc >= 0) rc = alloc_workspace(h);
  if (rc < 0) {
    rbicg_destroy(h);
    return rc;
  }
  *out = h;
  return RBICG_OK;
}

extern "C" int rbicg_update_recycle_on(rbicg_handle h, rbicg_matrix A_next) {
  if (!h) return rbicg_fail(RBICG_EINVAL, "null handle");
  if (A_next) TRY(attach_matrix(h, A_next, false));
  return rbicg_update_recycle(h, nullptr, nullptr);
}

extern "C" int rbicg_profile(rbicg_handle h, int32_t reset, double *out) {
  if (!h || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  for (int k = 0; k < 2; ++k) {
    out[2 * k] = h->prof_ms[k];
    out[2 * k + 1] = (double)h->prof_n[k];
  }
  double kb[2];
  kernel_bytes(h, h->ksys, kb);
  out[4] = kb[0];
  out[5] = kb[0] + kb[1];
  for (int kk = 0; kk < 2; ++kk) out[6 + kk] = h->prof_bytes[kk];
  for (int kk = 0; kk < 5; ++kk) out[8 + kk] = h->prof_cyc[kk];
  if (reset) {
    for (int kk = 0; kk < 2; ++kk) {
      h->prof_ms[kk] = 0;
      h->prof_n[kk] = 0;
      h->prof_bytes[kk] = 0;
    }
    for (int kk = 0; kk < 5; ++kk) h->prof_cyc[kk] = 0;
  }
  return RBICG_OK;
}

extern "C" int rbicg_destroy(rbicg_handle h) {
  if (!h) return RBICG_OK;
  if (h->st) (void)hipStreamSynchronize(h->st);
  else (void)hipDeviceSynchronize();
  if (h->jst) {
    (void)hipStreamSynchronize(h->jst);
    (void)hipStreamDestroy(h->jst);
  }
  if (h->jev) (void)hipEventDestroy(h->jev);
  delete h->sw;
  h->sw = nullptr;
  if (h->h64) {
    rbicg_destroy(h->h64);
    h->h64 = nullptr;
  }
  if (h->own_mat && h->mat) {
    h->mat->A.release();
    h->mat->AH.release();
    delete h->mat;
  }
  for (hipEvent_t e : h->pev) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->sev)
    if (e) (void)hipEventDestroy(e);
  for (void *p : h->allocs) (void)hipFree(p);
  if (h->hS) (void)hipHostFree(h->hS);
  if (h->hG) (void)hipHostFree(h->hG);
  if (h->hW) (void)hipHostFree(h->hW);
  if (h->hlog) (void)hipHostFree(h->hlog);
  if (h->hzlog) (void)hipHostFree(h->hzlog);
  delete h;
  return RBICG_OK;
}

extern "C" int rbicg_solve_dual(rbicg_handle h, const void *b, const void *bt, void *x, void *xt,
                                double tol, rbicg_stats *st) {
  if (!h || !b || !bt || !x || !xt) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (!(tol > 0)) return rbicg_fail(RBICG_EINVAL, "tol must be positive");
  if (h->vkind == 2)
    return solve_mixed(h, (const double *)b, (const double *)bt, (double *)x, (double *)xt, tol, st);
  return dispatch(h, [&](auto *vp, auto *mp) {
    using V = std::remove_pointer_t<decltype(vp)>;
    using M = std::remove_pointer_t<decltype(mp)>;
    return solve_impl<V, M>(h, (const V *)b, (const V *)bt, (V *)x, (V *)xt, tol, st);
  });
}

extern "C" int rbicg_solve_sequence(rbicg_handle h, int32_t nsys, const rbicg_matrix *mats,
                                    const void *const *b, const void *const *bt, void *const *x,
                                    void *const *xt, int32_t zero_init, double tol, rbicg_stats *st) {
  if (!h || nsys < 0 || (nsys > 0 && (!mats || !b || !bt || !x || !xt)))
    return rbicg_fail(RBICG_EINVAL, "null argument");
  int worst = RBICG_OK;
  for (int j = 0; j < nsys; ++j) {
    if (!mats[j]) return rbicg_fail(RBICG_EINVAL, "system %d: null matrix", j);
    if (j > 0 || mats[j] != h->mat) TRY(rbicg_update_recycle_on(h, mats[j]));
    if (zero_init) {  // a fill kernel (no memset node), doubles at the boundary
      if (!x[j] || !xt[j]) return rbicg_fail(RBICG_EINVAL, "system %d: null vector", j);
      const size_t words = (size_t)h->n * (h->vkind == 1 ? 2 : 1);
      launch_fill_zero<double>(h->st, (double *)x[j], words);
      launch_fill_zero<double>(h->st, (double *)xt[j], words);
      HIPCHECK(hipGetLastError());
    }
    rbicg_stats one{};
    const int rc = rbicg_solve_dual(h, b[j], bt[j], x[j], xt[j], tol, &one);
    if (st) st[j] = one;
    if (rc < 0) return rc;
    if (rc != RBICG_OK && worst == RBICG_OK) worst = rc;
  }
  return worst;
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
  if (h->ilu) return rbicg_fail(RBICG_EINVAL, "not with a split preconditioner attached");
  if (!(tol > 0)) return rbicg_fail(RBICG_EINVAL, "tol must be positive");
  void *x = nullptr, *xt = nullptr;
  if (h->vkind == 2) {
    // FP64 solution vectors around the FP32-inner solve; FP64 correction term
    const size_t bytes = (size_t)h->ld * sizeof(double);
    HIPCHECK(hipMalloc(&x, bytes));
    if (hipMalloc(&xt, bytes) != hipSuccess) {
      (void)hipFree(x);
      return rbicg_fail(RBICG_ENOMEM, "hipMalloc failed");
    }
    auto run = [&]() -> int {
      launch_fill_zero<double>(h->st, (double *)x, (size_t)h->n);
      launch_fill_zero<double>(h->st, (double *)xt, (size_t)h->n);
      const int r1 = solve_mixed(h, (const double *)w, (const double *)u, (double *)x, (double *)xt, tol, st);
      if (r1 < 0 && r1 != RBICG_BREAKDOWN) return r1;
      launch_residual<double, double>(h->st, h->mat->A.view<double>(), (const double *)w, (const double *)x, h->r64);
      launch_residual<double, double>(h->st, h->mat->AH.view<double>(), (const double *)u, (const double *)xt, h->rt64);
      cplx dd[3];
      TRY(host_dots<double>(h, (const double *)u, (const double *)x, (const double *)xt, h->r64, h->r64, h->r64, dd));
      const double rnorm = std::sqrt(std::fabs(dd[2].real()));
      ((double *)value)[0] = dd[0].real() + dd[1].real();
      TRY(host_dots<double>(h, h->rt64, h->rt64, nullptr, nullptr, nullptr, nullptr, dd));
      if (err_est) *err_est = rnorm * std::sqrt(std::fabs(dd[0].real()));
      return r1;
    };
    const int rc = run();
    (void)hipFree(x);
    (void)hipFree(xt);
    return rc;
  }
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
    launch_residual<V, M>(h->st, view_A<M>(h), (const V *)w, (const V *)x, (V *)h->t1);
    launch_residual<V, M>(h->st, view_AH<M>(h), (const V *)u, (const V *)xt, (V *)h->t2);
    cplx dd[3];
    TRY(host_dots<V>(h, (const V *)u, (const V *)x, (const V *)xt, (const V *)h->t1,
                     (const V *)h->t1, (const V *)h->t1, dd));
    const double vr = dd[0].real() + dd[1].real(), vi = dd[0].imag() + dd[1].imag();
    const double rnorm = std::sqrt(std::fabs(dd[2].real()));
    TRY(host_dots<V>(h, (const V *)h->t2, (const V *)h->t2, nullptr, nullptr, nullptr, nullptr, dd));
    const double rtnorm = std::sqrt(std::fabs(dd[0].real()));
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
  if (!h || !sigma || !b || !c || !X || !Xt || !st) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (h->ilu) return rbicg_fail(RBICG_EINVAL, "not with a split preconditioner attached");
  if (h->vkind != 1) return rbicg_fail(RBICG_EINVAL, "shifted solves need a RBICG_C128 handle");
  if (S < 1 || S > SHMAX) return rbicg_fail(RBICG_EINVAL, "S=%d out of range [1, %d]", S, SHMAX);
  if (!(tol > 0)) return rbicg_fail(RBICG_EINVAL, "tol must be positive");
  if (h->mat_complex)
    return solve_shifted_impl<cd>(h, S, sigma, (const cd *)b, (const cd *)c, (cd *)X, (cd *)Xt, tol, update_from, st);
  return solve_shifted_impl<double>(h, S, sigma, (const cd *)b, (const cd *)c, (cd *)X, (cd *)Xt, tol, update_from, st);
}

// u_i^H A^{-1} w_i for i < S in one batched solve (see rbicg.h).
template <class M>
int bilinear_batch_impl(rbicg_s *h, int S, const cd *U, const cd *W, double tol, double *values,
                        double *err_est, rbicg_stats *st, cd *X, cd *Xt) {
  const int n = h->n;
  // sigma = 0: the shifted solves take (0 I - A) X = W, (0 I - A)^H X~ = U,
  // so X = -A^{-1} W and X~ = -A^{-H} U
  std::vector<double> zero(2 * (size_t)S, 0.0);
  int rc = solve_shifted_impl<M>(h, S, zero.data(), W, U, X, Xt, tol, -1, st, (size_t)n);
  if (rc < 0 && rc != RBICG_BREAKDOWN) return rc;
  h->shifted = true;
  h->shift = 0.0;
  for (int i = 0; i < S; ++i) {
    const cd *u = U + (size_t)i * n, *w = W + (size_t)i * n;
    const cd *x = X + (size_t)i * n, *xt = Xt + (size_t)i * n;
    // r = w - (0 I - A) x = w - A y and r~ = u - A^H y~ with y = -x, y~ = -x~:
    // the value u^H y + y~^H r = -(u^H x + x~^H r) (its error r~^H A^{-1} r is
    // quadratic in the residuals, Sec. 1)
    launch_residual<cd, M>(h->st, view_A<M>(h), w, x, (cd *)h->t1);
    launch_residual<cd, M>(h->st, view_AH<M>(h), u, xt, (cd *)h->t2);
    cplx d[3];
    int r2 = host_dots<cd>(h, u, x, xt, (const cd *)h->t1, (const cd *)h->t1, (const cd *)h->t1, d);
    if (r2 < 0) {
      h->shifted = false;
      return r2;
    }
    const cplx v = -(d[0] + d[1]);
    values[2 * i] = v.real();
    values[2 * i + 1] = v.imag();
    const double rn = std::sqrt(std::fabs(d[2].real()));
    r2 = host_dots<cd>(h, (const cd *)h->t2, (const cd *)h->t2, nullptr, nullptr, nullptr, nullptr, d);
    if (r2 < 0) {
      h->shifted = false;
      return r2;
    }
    if (err_est) err_est[i] = rn * std::sqrt(std::fabs(d[0].real()));
  }
  h->shifted = false;
  return rc;
}

extern "C" int rbicg_batch_attach(rbicg_handle h, rbicg_batch b) {
  if (!h) return rbicg_fail(RBICG_EINVAL, "null handle");
  if (b && h->ilu) return rbicg_fail(RBICG_EINVAL, "a preconditioned handle cannot be batched");
  h->batch = b;
  return RBICG_OK;
}

extern "C" int rbicg_bilinear_batch(rbicg_handle h, int32_t S, const void *U, const void *W, double tol,
                                    double *values, double *err_est, rbicg_stats *st) {
  if (!h || !U || !W || !values || !st) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (h->ilu) return rbicg_fail(RBICG_EINVAL, "not with a split preconditioner attached");
  if (h->vkind != 1) return rbicg_fail(RBICG_EINVAL, "batched bilinear forms need a RBICG_C128 handle");
  if (S < 1 || S > SHMAX) return rbicg_fail(RBICG_EINVAL, "S=%d out of range [1, %d]", S, SHMAX);
  if (!(tol > 0)) return rbicg_fail(RBICG_EINVAL, "tol must be positive");
  // solution buffers: the library's own (n x S each), freed before return
  cd *X = nullptr, *Xt = nullptr;
  const size_t bytes = (size_t)h->n * S * sizeof(cd);
  HIPCHECK(hipMalloc((void **)&X, bytes));
  if (hipMalloc((void **)&Xt, bytes) != hipSuccess) {
    (void)hipFree(X);
    return rbicg_fail(RBICG_ENOMEM, "hipMalloc(%zu) failed", bytes);
  }
  launch_fill_zero<cd>(h->st, X, (size_t)h->n * S);
  launch_fill_zero<cd>(h->st, Xt, (size_t)h->n * S);
  const int rc = h->mat_complex
                     ? bilinear_batch_impl<cd>(h, S, (const cd *)U, (const cd *)W, tol, values, err_est, st, X, Xt)
                     : bilinear_batch_impl<double>(h, S, (const cd *)U, (const cd *)W, tol, values, err_est, st, X, Xt);
  (void)hipStreamSynchronize(h->st);
  (void)hipFree(X);
  (void)hipFree(Xt);
  return rc;
}

extern "C" int rbicg_project(rbicg_handle h, int32_t m, const void *X, const void *Xt, const void *b,
                             const void *c, double *Ar, double *Er, double *br, double *cr) {
  if (!h || !X || !Xt || !Ar || !Er) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (h->ilu) return rbicg_fail(RBICG_EINVAL, "not with a split preconditioner attached");
  if (h->vkind != 1) return rbicg_fail(RBICG_EINVAL, "projection needs a RBICG_C128 handle");
  if (m < 1 || m > 32) return rbicg_fail(RBICG_EINVAL, "m=%d out of range [1, 32]", m);
  if ((b == nullptr) != (c == nullptr) || (b && (!br || !cr)))
    return rbicg_fail(RBICG_EINVAL, "b and c (with br, cr) must be given together");
  const int n = h->n, nb = b ? 2 : 0;
  // n x (m + 2) scratch: A X, then copies of b and c as extra Gram columns
  cd *AX = nullptr;
  HIPCHECK(hipMalloc((void **)&AX, (size_t)n * (m + 2) * sizeof(cd)));
  int rc = 0;
  {
    if (h->mat_complex)
      launch_spmm<cd, cd>(h->st, h->mat->A.view<cd>(), (const cd *)X, AX, n, m);
    else
      launch_spmm<cd, double>(h->st, h->mat->A.view<double>(), (const cd *)X, AX, n, m);
    if (b) {
      (void)hipMemcpyAsync(AX + (size_t)m * n, b, (size_t)n * sizeof(cd), hipMemcpyDeviceToDevice, h->st);
      (void)hipMemcpyAsync(AX + (size_t)(m + 1) * n, c, (size_t)n * sizeof(cd), hipMemcpyDeviceToDevice, h->st);
    }
    // G1 = Xt^H [A X, X, b]  (m x (2m + 1)),  G2 = X^H c  (m x 1)
    std::vector<const void *> Xl, Yl;
    for (int j = 0; j < m; ++j) Xl.push_back((const cd *)Xt + (size_t)j * n);
    for (int j = 0; j < m; ++j) Yl.push_back(AX + (size_t)j * n);
    for (int j = 0; j < m; ++j) Yl.push_back((const cd *)X + (size_t)j * n);
    if (b) Yl.push_back(AX + (size_t)m * n);
    const int my = (int)Yl.size();
    const int gy = gram_group(m, 1);
    rc = gram_enqueue<cd>(h, Xl, Yl);
    if (rc >= 0) rc = sync(h);
    if (rc >= 0) {
      const std::vector<cplx> G = gram_parse(h->hG, m, my, gy);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          const cplx a = G[(size_t)i * my + j], e = G[(size_t)i * my + m + j];
          Ar[2 * (i + (size_t)j * m)] = a.real();
          Ar[2 * (i + (size_t)j * m) + 1] = a.imag();
          Er[2 * (i + (size_t)j * m)] = e.real();
          Er[2 * (i + (size_t)j * m) + 1] = e.imag();
        }
      if (b)
        for (int i = 0; i < m; ++i) {
          const cplx v = G[(size_t)i * my + 2 * m];
          br[2 * i] = v.real();
          br[2 * i + 1] = v.imag();
        }
    }
    if (rc >= 0 && nb) {
      std::vector<const void *> Xc, Yc{AX + (size_t)(m + 1) * n};
      for (int j = 0; j < m; ++j) Xc.push_back((const cd *)X + (size_t)j * n);
      const int gy2 = gram_group(m, 1);
      rc = gram_enqueue<cd>(h, Xc, Yc);
      if (rc >= 0) rc = sync(h);
      if (rc >= 0) {
        const std::vector<cplx> G = gram_parse(h->hG, m, 1, gy2);
        for (int i = 0; i < m; ++i) {
          cr[2 * i] = G[i].real();
          cr[2 * i + 1] = G[i].imag();
        }
      }
    }
  }
  const hipError_t e = hipFree(AX);
  if (rc < 0) return rc;
  if (e != hipSuccess) return rbicg_fail(RBICG_EHIP, "hipFree: %s", hipGetErrorString(e));
  return RBICG_OK;
}
