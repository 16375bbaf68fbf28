// rbicg_solve_dual_noalloc: plain BiCG (Algorithm 1, i.e. Algorithm 2 with an
// empty recycle space) on a resident matrix, for callers that cannot allocate.
// Every buffer beyond the caller's inputs and outputs -- work vectors,
// per-block partial sums, the scalar block, the per-iteration log -- lives in
// one file-scope device array, `scratch`, of fixed size.  The kernels and the
// order of their launches are those of rbicg_solve_dual on a k = 0 handle, so
// the two give the same iterates for the same inputs and options.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>

#include "device.h"
#include "errors.h"
#include "kernels.h"
#include "matviews.h"
#include "rbicg.h"

#define NA_HIPCHECK(call)                                                                \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return rbicg_fail(RBICG_EHIP, "%s failed at %s:%d: %s", #call, __FILE__, __LINE__, \
                        hipGetErrorString(e_));                                          \
  } while (0)

#define NA_TRY(call)         \
  do {                       \
    int rc_ = (call);        \
    if (rc_ < 0) return rc_; \
  } while (0)

// Size of the scratch array (RBICG_NOALLOC_SCRATCH_BYTES in rbicg.h): eight
// work vectors of at most 2 MiB each (n * bytes per element <= 2 MiB after
// padding to 256 elements), the partial sums of at most 256 blocks, two scalar
// blocks and a log of at most RBICG_NOALLOC_MAXIT + 2 iterations.
static_assert(RBICG_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256");
static __device__ __align__(256) char scratch[RBICG_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on each device, looked up once per device (with
// that device current) on the first call there.  In host code the array's own
// name is not a device address; only these pointers are passed to kernels.
constexpr int NA_MAXDEV = 64;
std::mutex g_na_mu;
char *g_na_ptr[NA_MAXDEV] = {};

int scratch_on_current_device(char **out) {
  int dev = -1;
  NA_HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NA_MAXDEV) return rbicg_fail(RBICG_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void *p = nullptr;
    NA_HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return rbicg_fail(RBICG_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_na_ptr[dev] = (char *)p;
  }
  *out = g_na_ptr[dev];
  return 0;
}

constexpr size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Carving of the scratch array for one call.
template <class V>
struct NaLayout {
  Scalars *S = nullptr, *out = nullptr;
  double *partial = nullptr, *P1 = nullptr, *P3 = nullptr, *log = nullptr;
  V *r = nullptr, *rt = nullptr, *p[2] = {}, *pt[2] = {}, *z = nullptr, *zt = nullptr;
  size_t bytes = 0;
  void carve(char *base, int ld, int nb, int maxit) {
    size_t off = 0;
    auto take = [&](size_t b) {
      char *q = base ? base + off : nullptr;
      off += al256(b);
      return q;
    };
    S = (Scalars *)take(sizeof(Scalars));
    out = (Scalars *)take(sizeof(Scalars));
    partial = (double *)take((size_t)nb * 4 * KMAXD * sizeof(double));
    P1 = (double *)take((size_t)nb * (6 * KMAXD + 2) * sizeof(double));
    P3 = (double *)take((size_t)nb * 8 * sizeof(double));
    log = (double *)take((size_t)(maxit + 2) * LOG_STRIDE * sizeof(double));
    V **vecs[] = {&r, &rt, &p[0], &p[1], &pt[0], &pt[1], &z, &zt};
    for (V **v : vecs) *v = (V *)take((size_t)ld * sizeof(V));
    bytes = off;
  }
};

int na_pull(hipStream_t st, Scalars *host, const Scalars *dev) {
  NA_HIPCHECK(hipMemcpyAsync(host, dev, sizeof(Scalars), hipMemcpyDeviceToHost, st));
  NA_HIPCHECK(hipStreamSynchronize(st));
  return 0;
}

template <class V, class M>
int na_solve(const MatViews &mv, const Sell<M> &A, const Sell<M> &AH, const rbicg_opts &o,
             hipStream_t st, char *base, const V *b, const V *bt, V *x, V *xt, double tol,
             rbicg_stats *stp) {
  const auto t0 = std::chrono::steady_clock::now();
  const int n = mv.n, ld = (n + 255) / 256 * 256, nb = iter_grid(n);
  NaLayout<V> L;
  L.carve(nullptr, ld, nb, o.maxit);
  if ((size_t)ld * sizeof(V) > ((size_t)2 << 20) || L.bytes > (size_t)RBICG_NOALLOC_SCRATCH_BYTES)
    return rbicg_fail(RBICG_EINVAL,
                      "n=%d (%zu bytes per padded vector, %zu scratch bytes in all) is beyond the "
                      "no-allocation limits: at most 2 MiB per vector and %d scratch bytes",
                      n, (size_t)ld * sizeof(V), L.bytes, RBICG_NOALLOC_SCRATCH_BYTES);
  L.carve(base, ld, nb, o.maxit);
  constexpr int nd = sizeof(V) == 16 ? 2 : 1;
  Scalars hs;  // host copy of the scalar block (pageable; every copy is waited for)
  int total = 0, restarts = 0, reseeds = 0, status = ST_MAXIT;
  double relres = NAN, relres_dual = NAN, bn = 0.0, btn = 0.0;
  bool first = true;
  while (true) {
    // eq. minusXR with an empty recycle space: r_{-1} = b - A x, r~ likewise;
    // on the first pass also ||b||, ||b~|| and the unprojected ||r||, ||r~||
    if (first) launch_dots<V>(st, nb, n, b, b, bt, bt, nullptr, nullptr, L.partial, L.S->red + 16);
    launch_residual<V, M>(st, A, b, x, L.r);
    launch_residual<V, M>(st, AH, bt, xt, L.rt);
    if (first) launch_dots<V>(st, nb, n, L.r, L.r, L.rt, L.rt, nullptr, nullptr, L.partial, L.S->red + 24);
    launch_init_p3<V>(st, nb, n, L.r, L.rt, L.P3);
    launch_fin_red(st, L.P3, nb, 2 + nd, L.S->red);
    NA_HIPCHECK(hipGetLastError());
    NA_TRY(na_pull(st, &hs, L.S));
    double rn = std::sqrt(std::fabs(hs.red[0])), rtn = std::sqrt(std::fabs(hs.red[1]));
    std::complex<double> rho(hs.red[2], nd == 2 ? hs.red[3] : 0.0);
    // Algorithm 1 step 3 (as Algorithm 2): re-seed x~ if (r_0, r~_0) vanishes
    while (std::abs(rho) <= 1e-14 * rn * rtn && rn > 0 && reseeds < 3) {
      launch_reseed<V>(st, xt, (size_t)n, (unsigned long long)(o.seed + reseeds));
      launch_residual<V, M>(st, AH, bt, xt, L.rt);
      if (first)
        launch_dots<V>(st, nb, n, L.rt, L.rt, nullptr, nullptr, nullptr, nullptr, L.partial,
                       L.S->red + 24 + nd);
      launch_init_p3<V>(st, nb, n, L.r, L.rt, L.P3);
      launch_fin_red(st, L.P3, nb, 2 + nd, L.S->red);
      NA_TRY(na_pull(st, &hs, L.S));
      rn = std::sqrt(std::fabs(hs.red[0]));
      rtn = std::sqrt(std::fabs(hs.red[1]));
      rho = std::complex<double>(hs.red[2], nd == 2 ? hs.red[3] : 0.0);
      ++reseeds;
    }
    if (first) {
      bn = std::sqrt(std::fabs(hs.red[16]));
      btn = std::sqrt(std::fabs(hs.red[16 + nd]));
      if (bn == 0.0) bn = std::sqrt(std::fabs(hs.red[24]));
      if (btn == 0.0) btn = std::sqrt(std::fabs(hs.red[24 + nd]));
      if (bn == 0.0) bn = 1.0;
      if (btn == 0.0) btn = 1.0;
    }
    first = false;
    const int run_start = total;
    std::memset(&hs, 0, sizeof(Scalars));
    hs.tol = tol;
    hs.bn = bn;
    hs.btn = btn;
    hs.iter = total;
    hs.maxit = o.maxit;
    hs.stag_base = total;
    const bool conv0 = rn <= tol * bn && rtn <= tol * btn;
    hs.done = conv0 ? 1 : 0;
    hs.status = conv0 ? ST_CONVERGED : ST_RUNNING;
    if (total >= o.maxit && !conv0) {
      hs.done = 1;
      hs.status = ST_MAXIT;
    }
    NA_HIPCHECK(hipMemcpyAsync(L.S, &hs, sizeof(Scalars), hipMemcpyHostToDevice, st));
    NA_HIPCHECK(hipStreamSynchronize(st));
    launch_fill_zero<V>(st, L.p[0], (size_t)n);
    launch_fill_zero<V>(st, L.pt[0], (size_t)n);
    int pc = 0, launched = total, done = hs.done, dev_status = hs.status, completed = total;
    const int chunk_def = o.chunk > 0 ? o.chunk : 8;
    while (!done && launched < o.maxit) {
      const int chunk = std::min(chunk_def, o.maxit - launched);
      for (int c = 0; c < chunk; ++c) {
        const int it = launched + 1;
        V *pn = L.p[1 - pc], *ptn = L.pt[1 - pc];
        launch_it1<V, M>(st, nb, A, AH, L.r, L.p[pc], L.rt, L.pt[pc], pn, ptn, L.z, L.zt, nullptr,
                         nullptr, 0, ld, nullptr, nullptr, nullptr, nullptr, L.P3, L.P1, L.S, L.log,
                         it, it == run_start + 1 ? 1 : 0, 0);
        launch_it2<V>(st, nb, n, x, xt, L.r, L.rt, pn, ptn, L.z, L.zt, nullptr, nullptr, 0, ld, L.P1,
                      L.P3, L.S, L.log, it, 0);
        pc = 1 - pc;
        ++launched;
      }
      // stopping test of the chunk's last iteration, its outcome into L.out
      launch_itfin<V>(st, nb, L.P3, L.S, L.log, launched + 1, launched == run_start ? 1 : 0, L.out);
      NA_HIPCHECK(hipGetLastError());
      Scalars sc;
      NA_TRY(na_pull(st, &sc, L.out));
      if (sc.done) {
        done = 1;
        dev_status = sc.status;
        completed = sc.iter;
      } else {
        completed = launched;
      }
    }
    if (!done) {
      completed = launched;
      dev_status = ST_MAXIT;
    }
    total = completed;
    status = dev_status;
    // true residuals b - A x, b~ - A^H x~ (z, z~ are free now)
    launch_residual<V, M>(st, A, b, x, L.z);
    launch_residual<V, M>(st, AH, bt, xt, L.zt);
    launch_dots<V>(st, nb, n, L.z, L.z, L.zt, L.zt, nullptr, nullptr, L.partial, L.S->red);
    NA_HIPCHECK(hipGetLastError());
    NA_TRY(na_pull(st, &hs, L.S));
    const double tr = std::sqrt(std::fabs(hs.red[0])), trt = std::sqrt(std::fabs(hs.red[nd]));
    relres = tr / bn;
    relres_dual = trt / btn;
    const bool true_ok = tr <= tol * bn && trt <= tol * btn;
    if (status == ST_CONVERGED && !true_ok && restarts < o.max_restarts && total < o.maxit) {
      ++restarts;
      continue;
    }
    if (status == ST_CONVERGED && !true_ok) status = ST_MAXIT;
    break;
  }
  rbicg_stats s{};
  s.status = (status == ST_CONVERGED || status == ST_STAGNATED)
                 ? RBICG_OK
                 : (status == ST_BREAKDOWN ? RBICG_BREAKDOWN : RBICG_NOT_CONVERGED);
  s.iters = total;
  s.restarts = restarts;
  s.reseeds = reseeds;
  s.k_used = 0;
  s.relres = relres;
  s.relres_dual = relres_dual;
  s.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // algorithmic bytes of the two iteration kernels with an empty recycle space
  const double ba = mv.complex_vals ? 16.0 : 8.0, nnz = (double)mv.nnz, vb = (double)sizeof(V);
  const double ix = mv.shared_pattern ? 1.0 : 2.0;
  s.alg_bytes = (2.0 * nnz * ba + ix * (4.0 * nnz + 4.0 * (n + 1.0)) + 20.0 * n * vb) * total;
  if (stp) *stp = s;
  return s.status;
}

}  // namespace

extern "C" int rbicg_solve_dual_noalloc(rbicg_matrix A, const rbicg_opts *opt, const void *b,
                                        const void *bt, void *x, void *xt, double tol,
                                        rbicg_stats *st) {
  if (!A || !opt || !b || !bt || !x || !xt) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (!(tol > 0)) return rbicg_fail(RBICG_EINVAL, "tol must be positive");
  if (opt->k != 0) return rbicg_fail(RBICG_EINVAL, "the no-allocation solve is plain BiCG: opts.k must be 0");
  if (opt->prec != RBICG_F64 && opt->prec != RBICG_C128)
    return rbicg_fail(RBICG_EINVAL, "the no-allocation solve takes RBICG_F64 or RBICG_C128");
  if (opt->maxit < 1 || opt->maxit > RBICG_NOALLOC_MAXIT)
    return rbicg_fail(RBICG_EINVAL, "maxit must be in [1, %d] for the no-allocation solve", RBICG_NOALLOC_MAXIT);
  if (opt->chunk < 0 || opt->chunk > 256) return rbicg_fail(RBICG_EINVAL, "chunk out of range");
  if (opt->max_restarts < 0) return rbicg_fail(RBICG_EINVAL, "max_restarts must be >= 0");
  MatViews mv;
  NA_TRY(rbicg_matrix_views(A, &mv));
  if (mv.complex_vals && opt->prec != RBICG_C128)
    return rbicg_fail(RBICG_EINVAL, "a complex matrix needs RBICG_C128");
  char *base = nullptr;
  NA_TRY(scratch_on_current_device(&base));
  hipStream_t s = (hipStream_t)opt->stream;
  if (opt->prec == RBICG_F64)
    return na_solve<double, double>(mv, mv.A, mv.AH, *opt, s, base, (const double *)b,
                                    (const double *)bt, (double *)x, (double *)xt, tol, st);
  if (mv.complex_vals)
    return na_solve<cd, cd>(mv, mv.Ac, mv.AHc, *opt, s, base, (const cd *)b, (const cd *)bt,
                            (cd *)x, (cd *)xt, tol, st);
  return na_solve<cd, double>(mv, mv.A, mv.AH, *opt, s, base, (const cd *)b, (const cd *)bt,
                              (cd *)x, (cd *)xt, tol, st);
}
