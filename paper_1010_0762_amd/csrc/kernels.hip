// gfx950 kernels of the RBiCG hot path (Algorithm 2) and of the cycle-end
// recycle-space computations (Sec. 4).
//
// One iteration of Algorithm 2 is three launches, each ending in a grid-wide
// reduction finished by the last block to arrive (ticket counter, fixed
// summation order, so results are deterministic):
//   k_iter_spmv    p = r + beta p, p~ = r~ + conj(beta) p~ (own rows written,
//                  gathered rows recomputed on the fly), z = A p and
//                  z~ = A^H p~ from the two sliced-ELL matrices (no atomics),
//                  and the restriction zeta = C~^H z, zeta~ = C^H z~;
//   k_iter_expand  q = z - C zeta, q~ = z~ - C~ zeta~, sigma = (p~, q),
//                  alpha = rho / sigma, zeta_c += alpha zeta, ...;
//   k_iter_update  x += alpha p, x~ += conj(alpha) p~, r -= alpha q,
//                  r~ -= conj(alpha) q~, ||r||, ||r~||, rho' = (r~, r), the
//                  stopping test and beta = rho' / rho.
// Every launch first reads the device 'done' flag and returns at once after
// convergence, so the host may enqueue iterations ahead of the test.
//
// Vector storage type V is double, float (FP32-inner mode; every element
// operation is done in double and rounded once when stored) or cd (complex).
// Matrix value type M is double, float or cd.  Reductions accumulate in
// double.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace {

// ------------------------------------------------------------------ types
template <class V> struct Ar { using T = double; };
template <> struct Ar<cd> { using T = cd; };

__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cd operator*(double a, cd b) { return {a * b.x, a * b.y}; }
__device__ __forceinline__ cd operator*(cd a, double b) { return {a.x * b, a.y * b}; }
__device__ __forceinline__ cd &operator+=(cd &a, cd b) { a.x += b.x; a.y += b.y; return a; }
__device__ __forceinline__ cd &operator-=(cd &a, cd b) { a.x -= b.x; a.y -= b.y; return a; }

__device__ __forceinline__ double up(float v) { return (double)v; }
__device__ __forceinline__ double up(double v) { return v; }
__device__ __forceinline__ cd up(cd v) { return v; }

template <class V> __device__ __forceinline__ V down(typename Ar<V>::T v);
template <> __device__ __forceinline__ float down<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ double down<double>(double v) { return v; }
template <> __device__ __forceinline__ cd down<cd>(cd v) { return v; }

__device__ __forceinline__ double cj(double a) { return a; }
__device__ __forceinline__ cd cj(cd a) { return {a.x, -a.y}; }

template <class T> __device__ __forceinline__ T zero();
template <> __device__ __forceinline__ double zero<double>() { return 0.0; }
template <> __device__ __forceinline__ cd zero<cd>() { return {0.0, 0.0}; }

template <class T> __device__ __forceinline__ T sc(cd v);
template <> __device__ __forceinline__ double sc<double>(cd v) { return v.x; }
template <> __device__ __forceinline__ cd sc<cd>(cd v) { return v; }

__device__ __forceinline__ cd tocd(double v) { return {v, 0.0}; }
__device__ __forceinline__ cd tocd(cd v) { return v; }

template <class T> struct ND { static constexpr int v = 1; };
template <> struct ND<cd> { static constexpr int v = 2; };
__device__ __forceinline__ double comp(double v, int) { return v; }
__device__ __forceinline__ double comp(cd v, int i) { return i ? v.y : v.x; }

__device__ __forceinline__ double abs2(double v) { return v * v; }
__device__ __forceinline__ double abs2(cd v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ bool isfin(double v) { return isfinite(v); }
__device__ __forceinline__ bool isfin(cd v) { return isfinite(v.x) && isfinite(v.y); }

__device__ __forceinline__ cd cdiv(cd a, cd b) {
  double d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double ld_coherent(const double *p) {
  unsigned long long v = __hip_atomic_load((unsigned long long *)p, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)v);
}

// Block partial of one value: every wave reduces its lanes, wave sums go to
// lds[wave * stride + idx].
__device__ __forceinline__ void wave_put(double *lds, int stride, int idx, double v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[(threadIdx.x >> 6) * stride + idx] = v;
}

// Sum the 4 wave slots of nv values in a fixed order and store the block
// partial (caller synchronizes before).
__device__ __forceinline__ void block_store(const double *lds, int stride, int nv,
                                            double *partial) {
  for (int t = threadIdx.x; t < nv; t += RBICG_BLOCK) {
    double s = lds[t] + lds[stride + t] + lds[2 * stride + t] + lds[3 * stride + t];
    partial[(size_t)blockIdx.x * nv + t] = s;
  }
}

// Grid arrival: true in the last block to finish.  Partials written before
// the call are visible to that block afterwards.
__device__ __forceinline__ bool arrive_last(unsigned *ticket, unsigned nblocks) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(ticket, 1u);
    s_last = (prev == nblocks - 1);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

// Last block: out[t] = sum over blocks of partial[b*nv + t], summed in a fixed
// order (groups of blocks, then the groups in order).  nv <= 256.
__device__ void grid_finish(const double *partial, int nv, int nblocks, double *tmp,
                            double *out, unsigned *ticket) {
  const int G = (nv >= RBICG_BLOCK) ? 1 : RBICG_BLOCK / nv;
  const int t = threadIdx.x;
  const int j = t % nv, g = t / nv;
  if (g < G && t < G * nv) {
    double s = 0.0;
    for (int b = g; b < nblocks; b += G) s += ld_coherent(&partial[(size_t)b * nv + j]);
    tmp[g * nv + j] = s;
  }
  __syncthreads();
  for (int u = t; u < nv; u += RBICG_BLOCK) {
    double s = 0.0;
    for (int gg = 0; gg < G; ++gg) s += tmp[gg * nv + u];
    out[u] = s;
  }
  __syncthreads();
  if (t == 0) atomicExch(ticket, 0u);
}

template <class T> __device__ __forceinline__ void put(double *lds, int stride, int idx, T v) {
#pragma unroll
  for (int c = 0; c < ND<T>::v; ++c) wave_put(lds, stride, idx * ND<T>::v + c, comp(v, c));
}
template <class T> __device__ __forceinline__ T get(const double *v, int idx);
template <> __device__ __forceinline__ double get<double>(const double *v, int idx) { return v[idx]; }
template <> __device__ __forceinline__ cd get<cd>(const double *v, int idx) {
  return {v[2 * idx], v[2 * idx + 1]};
}

// Restriction partials: out_j = sum_rows conj(B[j]) u, out2_j = sum conj(B2[j]) u2
// (j < k); values go to LDS slots [0, k) and [k, 2k) (times ND).
template <class V, class T>
__device__ __forceinline__ void restrict_pair(int row, int n, T u, T u2, const V *B,
                                              const V *B2, int k, int ld, double *lds,
                                              int stride) {
  for (int j = 0; j < k; ++j) {
    T a = zero<T>(), b = zero<T>();
    if (row < n) {
      a = cj(up(B[(size_t)j * ld + row])) * u;
      b = cj(up(B2[(size_t)j * ld + row])) * u2;
    }
    put<T>(lds, stride, j, a);
    put<T>(lds, stride, k + j, b);
  }
}

// ------------------------------------------------------------ SpMV helpers
template <class V, class M, class T>
__device__ __forceinline__ T spmv_dir(const Sell<M> &A, int row, const V *r, const V *p, T beta) {
  const int slice = row >> 6, lane = row & 63;
  const int beg = A.sliceptr[slice], end = A.sliceptr[slice + 1];
  T acc = zero<T>();
  for (int e = beg + lane; e < end; e += RBICG_WAVE) {
    const int c = A.col[e];
    const T pc = up(down<V>(up(r[c]) + beta * up(p[c])));
    acc += up(A.val[e]) * pc;
  }
  return acc;
}

template <class V, class M, class T>
__device__ __forceinline__ T spmv_plain(const Sell<M> &A, int row, const V *x) {
  const int slice = row >> 6, lane = row & 63;
  const int beg = A.sliceptr[slice], end = A.sliceptr[slice + 1];
  T acc = zero<T>();
  for (int e = beg + lane; e < end; e += RBICG_WAVE) acc += up(A.val[e]) * up(x[A.col[e]]);
  return acc;
}

}  // namespace

// ===================================================================== kernels
template <class V, class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_iter_spmv(
    Sell<M> A, Sell<M> AH, const V *__restrict__ r, const V *__restrict__ p,
    const V *__restrict__ rt, const V *__restrict__ pt, V *__restrict__ pn, V *__restrict__ ptn,
    V *__restrict__ z, V *__restrict__ zt, const V *__restrict__ C, const V *__restrict__ Ct,
    int k, int ld, V *capR, V *capRt, V *capZ, V *capZt, double *partial, Scalars *S) {
  using T = typename Ar<V>::T;
  if (S->done) return;
  __shared__ double lds[4 * 4 * KMAXD];
  __shared__ double tmp[RBICG_BLOCK];
  __shared__ double res[4 * KMAXD];
  const int n = A.n;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  const T beta = sc<T>(S->beta);
  const T betac = cj(beta);
  T zz = zero<T>(), zzt = zero<T>();
  if (row < n) {
    const V rv = r[row], rtv = rt[row];
    pn[row] = down<V>(up(rv) + beta * up(p[row]));
    ptn[row] = down<V>(up(rtv) + betac * up(pt[row]));
    zz = up(down<V>(spmv_dir<V, M, T>(A, row, r, p, beta)));
    zzt = up(down<V>(spmv_dir<V, M, T>(AH, row, rt, pt, betac)));
    z[row] = down<V>(zz);
    zt[row] = down<V>(zzt);
    if (capR) {
      capR[row] = rv;
      capRt[row] = rtv;
      capZ[row] = down<V>(zz);
      capZt[row] = down<V>(zzt);
    }
  }
  if (k == 0) return;
  const int nv = 2 * k * ND<T>::v;
  const int stride = 4 * KMAXD;
  restrict_pair<V, T>(row, n, zz, zzt, Ct, C, k, ld, lds, stride);
  __syncthreads();
  block_store(lds, stride, nv, partial);
  if (arrive_last(&S->tickets[0], gridDim.x)) {
    grid_finish(partial, nv, gridDim.x, tmp, res, &S->tickets[0]);
    for (int j = threadIdx.x; j < k; j += RBICG_BLOCK) {
      S->zeta[j] = tocd(get<T>(res, j));
      S->zetat[j] = tocd(get<T>(res, k + j));
    }
  }
}

template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_iter_expand(
    int n, const V *__restrict__ z, const V *__restrict__ zt, const V *__restrict__ C,
    const V *__restrict__ Ct, int k, int ld, const V *__restrict__ ptn, V *__restrict__ q,
    V *__restrict__ qt, double *partial, Scalars *S) {
  using T = typename Ar<V>::T;
  if (S->done) return;
  __shared__ double lds[4 * 2];
  __shared__ double tmp[RBICG_BLOCK];
  __shared__ double res[2];
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  T part = zero<T>();
  if (row < n) {
    T s = zero<T>(), st = zero<T>();
    for (int j = 0; j < k; ++j) {
      s += up(C[(size_t)j * ld + row]) * sc<T>(S->zeta[j]);
      st += up(Ct[(size_t)j * ld + row]) * sc<T>(S->zetat[j]);
    }
    T qq = up(z[row]);
    T qqt = up(zt[row]);
    if (k > 0) {
      qq = up(down<V>(qq - s));
      qqt = up(down<V>(qqt - st));
      q[row] = down<V>(qq);
      qt[row] = down<V>(qqt);
    }
    part = cj(up(ptn[row])) * qq;
  }
  put<T>(lds, 2, 0, part);
  __syncthreads();
  block_store(lds, 2, ND<T>::v, partial);
  if (arrive_last(&S->tickets[1], gridDim.x)) {
    grid_finish(partial, ND<T>::v, gridDim.x, tmp, res, &S->tickets[1]);
    if (threadIdx.x == 0) {
      const T sigma = get<T>(res, 0);
      S->sigma = tocd(sigma);
      if (abs2(sigma) == 0.0 || !isfin(sigma)) {
        S->done = 1;
        S->status = ST_BREAKDOWN;
        S->alpha = tocd(zero<T>());
      } else {
        const cd a = cdiv(S->rho, tocd(sigma));
        S->alpha = a;
        const T al = sc<T>(a);
        for (int j = 0; j < k; ++j) {
          S->zeta_c[j] = tocd(sc<T>(S->zeta_c[j]) + al * sc<T>(S->zeta[j]));
          S->zetat_c[j] = tocd(sc<T>(S->zetat_c[j]) + cj(al) * sc<T>(S->zetat[j]));
        }
      }
    }
  }
}

template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_iter_update(
    int n, V *__restrict__ x, V *__restrict__ xt, V *__restrict__ r, V *__restrict__ rt,
    const V *__restrict__ pn, const V *__restrict__ ptn, const V *__restrict__ q,
    const V *__restrict__ qt, double *partial, Scalars *S, double *log) {
  using T = typename Ar<V>::T;
  if (S->done) return;
  __shared__ double lds[4 * 4];
  __shared__ double tmp[RBICG_BLOCK];
  __shared__ double res[4];
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  const T al = sc<T>(S->alpha);
  const T alc = cj(al);
  double rr = 0.0, rtrt = 0.0;
  T rho = zero<T>();
  if (row < n) {
    x[row] = down<V>(up(x[row]) + al * up(pn[row]));
    xt[row] = down<V>(up(xt[row]) + alc * up(ptn[row]));
    const T rv = up(down<V>(up(r[row]) - al * up(q[row])));
    const T rtv = up(down<V>(up(rt[row]) - alc * up(qt[row])));
    r[row] = down<V>(rv);
    rt[row] = down<V>(rtv);
    rr = abs2(rv);
    rtrt = abs2(rtv);
    rho = cj(rtv) * rv;
  }
  wave_put(lds, 4, 0, rr);
  wave_put(lds, 4, 1, rtrt);
#pragma unroll
  for (int c = 0; c < ND<T>::v; ++c) wave_put(lds, 4, 2 + c, comp(rho, c));
  __syncthreads();
  const int nv = 2 + ND<T>::v;
  block_store(lds, 4, nv, partial);
  if (arrive_last(&S->tickets[2], gridDim.x)) {
    grid_finish(partial, nv, gridDim.x, tmp, res, &S->tickets[2]);
    if (threadIdx.x == 0) {
      const double rn = sqrt(res[0]), rtn = sqrt(res[1]);
      const T rho_new = get<T>(res + 2, 0);
      const int it = S->iter + 1;
      S->iter = it;
      S->rn = rn;
      S->rtn = rtn;
      double *L = log + (size_t)(S->log_base + it) * LOG_STRIDE;
      L[0] = S->alpha.x; L[1] = S->alpha.y;
      L[2] = S->beta.x; L[3] = S->beta.y;
      const cd rn_c = tocd(rho_new);
      L[4] = rn_c.x; L[5] = rn_c.y;
      L[6] = rn; L[7] = rtn;
      const bool conv = rn <= S->tol * S->bn && rtn <= S->tol * S->btn;
      if (conv) {
        S->done = 1;
        S->status = ST_CONVERGED;
      } else if (abs2(rho_new) == 0.0 || !isfin(rho_new) || !isfinite(rn) || !isfinite(rtn)) {
        S->done = 1;
        S->status = ST_BREAKDOWN;
      } else {
        if (it >= S->maxit) {
          S->done = 1;
          S->status = ST_MAXIT;
        }
        S->beta = cdiv(rn_c, S->rho);
        S->rho = rn_c;
      }
      if (conv) S->rho = rn_c;
    }
  }
}

// r_out = b - A x (x may be null -> r_out = b)
template <class V, class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_residual(Sell<M> A, const V *b, const V *x,
                                                          V *out) {
  using T = typename Ar<V>::T;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (row >= A.n) return;
  T v = up(b[row]);
  if (x) v = v - spmv_plain<V, M, T>(A, row, x);
  out[row] = down<V>(v);
}

// Y[:, c] = A X[:, c] for c = blockIdx.y
template <class V, class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_spmm(Sell<M> A, const V *X, V *Y, int ld) {
  using T = typename Ar<V>::T;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (row >= A.n) return;
  const size_t off = (size_t)blockIdx.y * ld;
  Y[off + row] = down<V>(spmv_plain<V, M, T>(A, row, X + off));
}

// out_j = sum conj(B[j]) u, out2_j = sum conj(B2[j]) u2 into S->g, S->gt
template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_restrict(int n, const V *u, const V *B,
                                                          const V *u2, const V *B2, int k,
                                                          int ld, double *partial, Scalars *S) {
  using T = typename Ar<V>::T;
  __shared__ double lds[4 * 4 * KMAXD];
  __shared__ double tmp[RBICG_BLOCK];
  __shared__ double res[4 * KMAXD];
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  const T a = row < n ? up(u[row]) : zero<T>();
  const T b = row < n ? up(u2[row]) : zero<T>();
  const int stride = 4 * KMAXD;
  restrict_pair<V, T>(row, n, a, b, B, B2, k, ld, lds, stride);
  __syncthreads();
  const int nv = 2 * k * ND<T>::v;
  block_store(lds, stride, nv, partial);
  if (arrive_last(&S->tickets[3], gridDim.x)) {
    grid_finish(partial, nv, gridDim.x, tmp, res, &S->tickets[3]);
    for (int j = threadIdx.x; j < k; j += RBICG_BLOCK) {
      S->g[j] = tocd(get<T>(res, j));
      S->gt[j] = tocd(get<T>(res, k + j));
    }
  }
}

// x += sign * sum_j U[j] coef[j]; x2 += sign2 * sum_j U2[j] coef2[j]  (two pairs)
// mode 0: coefficients g/gt ; mode 1: zeta_c / zetat_c
template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_expand2(int n, V *x, const V *U, double sx,
                                                         V *r, const V *C, double sr, V *xt,
                                                         const V *Ut, double sxt, V *rt,
                                                         const V *Ct, double srt, int k, int ld,
                                                         int mode, const Scalars *S) {
  using T = typename Ar<V>::T;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (row >= n) return;
  const cd *c1 = mode ? S->zeta_c : S->g;
  const cd *c2 = mode ? S->zetat_c : S->gt;
  T a = zero<T>(), b = zero<T>(), c = zero<T>(), d = zero<T>();
  for (int j = 0; j < k; ++j) {
    const T g1 = sc<T>(c1[j]), g2 = sc<T>(c2[j]);
    const size_t o = (size_t)j * ld + row;
    if (x) a += up(U[o]) * g1;
    if (r) b += up(C[o]) * g1;
    if (xt) c += up(Ut[o]) * g2;
    if (rt) d += up(Ct[o]) * g2;
  }
  if (x) x[row] = down<V>(up(x[row]) + sx * a);
  if (r) r[row] = down<V>(up(r[row]) + sr * b);
  if (xt) xt[row] = down<V>(up(xt[row]) + sxt * c);
  if (rt) rt[row] = down<V>(up(rt[row]) + srt * d);
}

// Up to three dot products (a_i, b_i) = sum conj(a_i) b_i written (as cd) to
// S->red[2i], S->red[2i+1].
template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_dots(int n, const V *a0, const V *b0,
                                                      const V *a1, const V *b1, const V *a2,
                                                      const V *b2, double *partial,
                                                      Scalars *S) {
  using T = typename Ar<V>::T;
  __shared__ double lds[4 * 8];
  __shared__ double tmp[RBICG_BLOCK];
  __shared__ double res[8];
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  T d0 = zero<T>(), d1 = zero<T>(), d2 = zero<T>();
  if (row < n) {
    if (a0) d0 = cj(up(a0[row])) * up(b0[row]);
    if (a1) d1 = cj(up(a1[row])) * up(b1[row]);
    if (a2) d2 = cj(up(a2[row])) * up(b2[row]);
  }
  put<T>(lds, 8, 0, d0);
  put<T>(lds, 8, 1, d1);
  put<T>(lds, 8, 2, d2);
  __syncthreads();
  const int nv = 3 * ND<T>::v;
  block_store(lds, 8, nv, partial);
  if (arrive_last(&S->tickets[4], gridDim.x)) {
    grid_finish(partial, nv, gridDim.x, tmp, res, &S->tickets[4]);
    if (threadIdx.x == 0)
      for (int i = 0; i < 3; ++i) {
        const cd v = tocd(get<T>(res, i));
        S->red[2 * i] = v.x;
        S->red[2 * i + 1] = v.y;
      }
  }
}

template <class V>
__global__ void k_fill_zero(V *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i < n) p[i] = V{};
}

// SplitMix64 re-seed vector, entries uniform in [-1, 1): counter i uses
// state seed + (i+1)*gamma; complex entries take counters 2i and 2i+1.
__device__ __forceinline__ double smix_uniform(unsigned long long seed, unsigned long long ctr) {
  unsigned long long z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}
template <class V> __device__ V reseed_val(unsigned long long seed, size_t i);
template <> __device__ double reseed_val<double>(unsigned long long seed, size_t i) {
  return smix_uniform(seed, i);
}
template <> __device__ float reseed_val<float>(unsigned long long seed, size_t i) {
  return (float)smix_uniform(seed, i);
}
template <> __device__ cd reseed_val<cd>(unsigned long long seed, size_t i) {
  return {smix_uniform(seed, 2 * i), smix_uniform(seed, 2 * i + 1)};
}
template <class V>
__global__ void k_reseed(V *x, size_t n, unsigned long long seed) {
  const size_t i = (size_t)blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i < n) x[i] = reseed_val<V>(seed, i);
}

// ----------------------------------------------------- cycle-end kernels
// Gram partials G[i][j] = sum_rows conj(X_i) Y_j over a chunk of rows; tiles of
// 16 x 16 outputs per block, 64-row slabs staged in LDS.
template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_gram(int n, ColList X, int mx, ColList Y,
                                                      int my, int rows_per_chunk,
                                                      double *partial) {
  using T = typename Ar<V>::T;
  constexpr int TL = 16, SL = 64;
  __shared__ T xs[TL][SL + 1];
  __shared__ T ys[TL][SL + 1];
  const int tilesy = (my + TL - 1) / TL;
  const int ti = blockIdx.y / tilesy, tj = blockIdx.y % tilesy;
  const int i = threadIdx.x / TL, j = threadIdx.x % TL;
  const int gi = ti * TL + i, gj = tj * TL + j;
  const int r0 = blockIdx.x * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  T acc = zero<T>();
  for (int base = r0; base < r1; base += SL) {
    // load slab: 16 columns x 64 rows for X and Y (256 threads, 4 loads each)
    for (int t = threadIdx.x; t < TL * SL; t += RBICG_BLOCK) {
      const int c = t / SL, rr = t % SL, row = base + rr;
      const int cx = ti * TL + c, cy = tj * TL + c;
      xs[c][rr] = (row < r1 && cx < mx) ? up(((const V *)X.p[cx])[row]) : zero<T>();
      ys[c][rr] = (row < r1 && cy < my) ? up(((const V *)Y.p[cy])[row]) : zero<T>();
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < SL; ++rr) acc += cj(xs[i][rr]) * ys[j][rr];
    __syncthreads();
  }
  if (gi < mx && gj < my) {
    const cd v = tocd(acc);
    double *o = partial + ((size_t)blockIdx.x * mx * my + (size_t)gi * my + gj) * 2;
    o[0] = v.x;
    o[1] = v.y;
  }
}

// G = sum over chunks of the partials (fixed order); G is mx x my complex,
// stored row-major by (i, j) as in the partials.
__global__ void k_gram_reduce(const double *partial, int nchunks, int count, double *G) {
  const int t = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (t >= count) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += partial[(size_t)c * count + t];
  G[t] = s;
}

// Y[:, c] = sum_l X_l W[l, c] (W: m x p complex, column-major), c < p.
template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_tsgemm(int n, ColList X, int m, const cd *W,
                                                        int p, V *Y, int ld) {
  using T = typename Ar<V>::T;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (row >= n) return;
  constexpr int CB = 8;
  for (int c0 = 0; c0 < p; c0 += CB) {
    T acc[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) acc[u] = zero<T>();
    for (int l = 0; l < m; ++l) {
      const T xv = up(((const V *)X.p[l])[row]);
#pragma unroll
      for (int u = 0; u < CB; ++u)
        if (c0 + u < p) acc[u] += xv * sc<T>(W[(size_t)(c0 + u) * m + l]);
    }
#pragma unroll
    for (int u = 0; u < CB; ++u)
      if (c0 + u < p) Y[(size_t)(c0 + u) * ld + row] = down<V>(acc[u]);
  }
}

// =============================================================== launchers
namespace {
inline unsigned nblk(size_t n) { return (unsigned)((n + RBICG_BLOCK - 1) / RBICG_BLOCK); }
}

template <class V, class M>
void launch_iter_spmv(hipStream_t st, const Sell<M> &A, const Sell<M> &AH, const V *r,
                      const V *p, const V *rt, const V *pt, V *pn, V *ptn, V *z, V *zt,
                      const V *C, const V *Ct, int k, int ld, V *capR, V *capRt, V *capZ,
                      V *capZt, double *partial, Scalars *S) {
  hipLaunchKernelGGL((k_iter_spmv<V, M>), dim3(nblk(A.n)), dim3(RBICG_BLOCK), 0, st, A, AH, r,
                     p, rt, pt, pn, ptn, z, zt, C, Ct, k, ld, capR, capRt, capZ, capZt, partial,
                     S);
}
template <class V, class M>
void launch_residual(hipStream_t st, const Sell<M> &A, const V *b, const V *x, V *out) {
  hipLaunchKernelGGL((k_residual<V, M>), dim3(nblk(A.n)), dim3(RBICG_BLOCK), 0, st, A, b, x,
                     out);
}
template <class V, class M>
void launch_spmm(hipStream_t st, const Sell<M> &A, const V *X, V *Y, int ld, int m) {
  if (m <= 0) return;
  hipLaunchKernelGGL((k_spmm<V, M>), dim3(nblk(A.n), m), dim3(RBICG_BLOCK), 0, st, A, X, Y, ld);
}
template <class V>
void launch_iter_expand(hipStream_t st, int n, const V *z, const V *zt, const V *C,
                        const V *Ct, int k, int ld, const V *ptn, V *q, V *qt, double *partial,
                        Scalars *S) {
  hipLaunchKernelGGL((k_iter_expand<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, z, zt, C,
                     Ct, k, ld, ptn, q, qt, partial, S);
}
template <class V>
void launch_iter_update(hipStream_t st, int n, V *x, V *xt, V *r, V *rt, const V *pn,
                        const V *ptn, const V *q, const V *qt, double *partial, Scalars *S,
                        double *log) {
  hipLaunchKernelGGL((k_iter_update<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, x, xt, r,
                     rt, pn, ptn, q, qt, partial, S, log);
}
template <class V>
void launch_restrict(hipStream_t st, int n, const V *u, const V *B, const V *u2, const V *B2,
                     int k, int ld, double *partial, Scalars *S) {
  hipLaunchKernelGGL((k_restrict<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, u, B, u2, B2,
                     k, ld, partial, S);
}
template <class V>
void launch_expand2(hipStream_t st, int n, V *x, const V *U, double sx, V *r, const V *C,
                    double sr, V *xt, const V *Ut, double sxt, V *rt, const V *Ct, double srt,
                    int k, int ld, int mode, const Scalars *S) {
  hipLaunchKernelGGL((k_expand2<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, x, U, sx, r,
                     C, sr, xt, Ut, sxt, rt, Ct, srt, k, ld, mode, S);
}
template <class V>
void launch_dots(hipStream_t st, int n, const V *a0, const V *b0, const V *a1, const V *b1,
                 const V *a2, const V *b2, double *partial, Scalars *S) {
  hipLaunchKernelGGL((k_dots<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, a0, b0, a1, b1,
                     a2, b2, partial, S);
}
template <class V>
void launch_fill_zero(hipStream_t st, V *p, size_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_fill_zero<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, p, n);
}
template <class V>
void launch_reseed(hipStream_t st, V *x, size_t n, unsigned long long seed) {
  hipLaunchKernelGGL((k_reseed<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, x, n, seed);
}
template <class V>
void launch_gram(hipStream_t st, int n, const ColList &X, int mx, const ColList &Y, int my,
                 double *partial, double *G, int nchunks) {
  const int rpc = (int)(((size_t)n + nchunks - 1) / nchunks);
  const int tiles = ((mx + 15) / 16) * ((my + 15) / 16);
  hipLaunchKernelGGL((k_gram<V>), dim3(nchunks, tiles), dim3(RBICG_BLOCK), 0, st, n, X, mx, Y,
                     my, rpc, partial);
  const int count = 2 * mx * my;
  hipLaunchKernelGGL(k_gram_reduce, dim3(nblk(count)), dim3(RBICG_BLOCK), 0, st, partial,
                     nchunks, count, G);
}
template <class V>
void launch_tsgemm(hipStream_t st, int n, const ColList &X, int m, const cd *W, int p, V *Y,
                   int ld) {
  if (p <= 0) return;
  hipLaunchKernelGGL((k_tsgemm<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, X, m, W, p, Y,
                     ld);
}

#define INST_VM(V, M)                                                                        \
  template void launch_iter_spmv<V, M>(hipStream_t, const Sell<M> &, const Sell<M> &,        \
                                       const V *, const V *, const V *, const V *, V *, V *, \
                                       V *, V *, const V *, const V *, int, int, V *, V *,   \
                                       V *, V *, double *, Scalars *);                       \
  template void launch_residual<V, M>(hipStream_t, const Sell<M> &, const V *, const V *,    \
                                      V *);                                                  \
  template void launch_spmm<V, M>(hipStream_t, const Sell<M> &, const V *, V *, int, int);

#define INST_V(V)                                                                            \
  template void launch_iter_expand<V>(hipStream_t, int, const V *, const V *, const V *,     \
                                      const V *, int, int, const V *, V *, V *, double *,    \
                                      Scalars *);                                            \
  template void launch_iter_update<V>(hipStream_t, int, V *, V *, V *, V *, const V *,       \
                                      const V *, const V *, const V *, double *, Scalars *,  \
                                      double *);                                             \
  template void launch_restrict<V>(hipStream_t, int, const V *, const V *, const V *,        \
                                   const V *, int, int, double *, Scalars *);                \
  template void launch_expand2<V>(hipStream_t, int, V *, const V *, double, V *, const V *,  \
                                  double, V *, const V *, double, V *, const V *, double,    \
                                  int, int, int, const Scalars *);                           \
  template void launch_dots<V>(hipStream_t, int, const V *, const V *, const V *, const V *, \
                               const V *, const V *, double *, Scalars *);                   \
  template void launch_fill_zero<V>(hipStream_t, V *, size_t);                               \
  template void launch_reseed<V>(hipStream_t, V *, size_t, unsigned long long);              \
  template void launch_gram<V>(hipStream_t, int, const ColList &, int, const ColList &, int, \
                               double *, double *, int);                                     \
  template void launch_tsgemm<V>(hipStream_t, int, const ColList &, int, const cd *, int, V *, \
                                 int);

INST_VM(double, double)
INST_VM(cd, double)
INST_VM(cd, cd)
INST_VM(float, float)
INST_V(double)
INST_V(cd)
INST_V(float)
