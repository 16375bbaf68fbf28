// gfx950 kernels of the RBiCG hot path (Algorithm 2) and of the cycle-end
// recycle-space computations (Sec. 4).
//
// One iteration i of Algorithm 2 is two launches.  No kernel synchronizes
// its grid: each writes one partial sum per block, and every block of the
// NEXT kernel reduces those partials itself, in a fixed order (so every block
// obtains bit-identical scalars and runs are deterministic; no atomics, no
// fences, no extra launches):
//   k_it1  reduce ||r_{i-1}||^2, ||r~_{i-1}||^2, rho_{i-1} = (r~, r); stopping
//          test; beta_{i-1} = rho_{i-1} / rho_{i-2};
//          p = r + beta p, p~ = r~ + conj(beta) p~ (own rows written, gathered
//          rows recomputed on the fly), z = A p, z~ = A^H p~ from the two
//          sliced-ELL matrices (no atomics), partials of zeta = C~^H z,
//          zeta~ = C^H z~, e = p~^H C and (p~, z);
//   k_it2  reduce them; sigma = (p~, q) for q = z - C zeta is assembled as
//          (p~, z) - e zeta (the same sum by linearity, so q need not exist
//          before sigma); alpha = rho_{i-1} / sigma, zeta_c += alpha zeta,
//          zeta~_c += conj(alpha) zeta~; per row q = z - C zeta,
//          q~ = z~ - C~ zeta~ (kept in registers), x += alpha p,
//          x~ += conj(alpha) p~, r -= alpha q, r~ -= conj(alpha) q~; partials
//          of ||r||^2, ||r~||^2, (r~, r).
// In FP32-storage inner solves (flag rp) k_it1 also forms partials of
// g = C~^H r_{i-1}, g~ = C^H r~_{i-1}; k_it2 re-projects r_{i-1} -= C g,
// r~_{i-1} -= C~ g~ before its update and subtracts g, g~ from zeta_c,
// zeta~_c, which keeps x - U zeta_c consistent.  In exact arithmetic g = 0
// (the recurrences keep r orthogonal to range(C~), Sec. 3.1); in float
// storage the rounding of every update feeds C~^H r, the oblique projector
// amplifies it and the iteration stagnates without this step.
// Block 0 records the scalars of every iteration for the host.  Every launch
// first reads the device 'done' flag and returns at once after the stopping
// test has fired, so the host may enqueue iterations ahead of the test.
//
// Vector storage type V is double, float (FP32-inner mode; every element
// operation is done in double and rounded once when stored) or cd (complex).
// Matrix value type M is double, float or cd.  Reductions accumulate in
// double.
#include <hip/hip_runtime.h>

#include <algorithm>

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
#define IB 1024               // threads per block of the iteration kernels
#define NW (IB / 64)          // waves per block
#define RMAX 8                // rows per thread at most

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// wave sum of v into lds[wave * stride + idx]
__device__ __forceinline__ void wput(double *lds, int stride, int idx, double v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[(threadIdx.x >> 6) * stride + idx] = v;
}
template <class T> __device__ __forceinline__ void put(double *lds, int stride, int idx, T v) {
#pragma unroll
  for (int c = 0; c < ND<T>::v; ++c) wput(lds, stride, idx * ND<T>::v + c, comp(v, c));
}
template <class T> __device__ __forceinline__ T get(const double *v, int idx);
template <> __device__ __forceinline__ double get<double>(const double *v, int idx) { return v[idx]; }
template <> __device__ __forceinline__ cd get<cd>(const double *v, int idx) {
  return {v[2 * idx], v[2 * idx + 1]};
}
template <class T> __device__ __forceinline__ void set(double *v, int idx, T x) {
#pragma unroll
  for (int c = 0; c < ND<T>::v; ++c) v[idx * ND<T>::v + c] = comp(x, c);
}

// Sum over the 64 lanes of a wave of 16 values per lane, by recursive
// halving: at offset o the lanes l and l^o split the values they still hold,
// each keeps one half and adds the partner's copy of it.  After offsets 32,
// 16, 8 and 4 lane l holds value (l >> 2) summed over the 16 lanes that share
// bits 0-1 of l; offsets 1 and 2 complete the sum, so every lane of a quad
// returns the same total.  17 exchanges replace the 16 x 6 of separate wave
// sums, and the independent exchanges of one step issue back to back.  The
// order is fixed, so the bits are reproducible.
template <int H>
__device__ __forceinline__ void halve_step(double (&v)[16], int lane, int o) {
  const bool hi = lane & o;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = hi ? v[i] : v[i + H];
    const double keep = hi ? v[i + H] : v[i];
    v[i] = keep + __shfl_xor(send, o, 64);
  }
}
__device__ __forceinline__ double wave_sum16(double (&v)[16]) {
  const int lane = threadIdx.x & 63;
  halve_step<8>(v, lane, 32);
  halve_step<4>(v, lane, 16);
  halve_step<2>(v, lane, 8);
  halve_step<1>(v, lane, 4);
  double s = v[0];
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  return s;
}

// Block partial: P[block * nv + t] = sum over the waves (fixed order) of the
// wave sums in lds (caller synchronizes before).
__device__ __forceinline__ void bstore(const double *lds, int stride, int nwaves, int nv,
                                       double *P, int bid) {
  for (int t = threadIdx.x; t < nv; t += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += lds[w * stride + t];
    P[(size_t)bid * nv + t] = s;
  }
}

// Whole block: out[t] = sum over nb blocks of P[b * nv + t] (t < nv <= 256) in
// a fixed order; every block that calls it gets the same bits.  tmp holds
// blockDim.x doubles.  Synchronizes before returning.
__device__ __forceinline__ void breduce(const double *P, int nb, int nv, double *tmp,
                                        double *out) {
  const int G = min((int)blockDim.x / nv, 32);
  const int t = threadIdx.x, j = t % nv, g = t / nv;
  if (g < G) {
    // the same sequential sum over b, with 8 loads issued at a time (a
    // load-then-add loop waits out one cache round trip per partial)
    double s = 0.0;
    int b = g;
    for (; b + 7 * G < nb; b += 8 * G) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = P[(size_t)(b + u * G) * nv + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < nb; b += G) s += P[(size_t)b * nv + j];
    tmp[g * nv + j] = s;
  }
  __syncthreads();
  for (int u = t; u < nv; u += blockDim.x) {
    double s = 0.0;
    for (int gg = 0; gg < G; ++gg) s += tmp[gg * nv + u];
    out[u] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double divide(double a, double b) { return a / b; }
__device__ __forceinline__ cd divide(cd a, cd b) { return cdiv(a, b); }

// ------------------------------------------------------------ SpMV helpers
// (sigma I - A) y from A y for a shifted view: sigma y_row - acc
template <class M, class T>
__device__ __forceinline__ T shift_apply(const Sell<M> &A, T acc, T yrow);
template <>
__device__ __forceinline__ double shift_apply<double, double>(const Sell<double> &A, double acc,
                                                              double yrow) {
  return A.shifted ? A.shr * yrow - acc : acc;
}
template <>
__device__ __forceinline__ double shift_apply<float, double>(const Sell<float> &A, double acc,
                                                             double yrow) {
  return A.shifted ? A.shr * yrow - acc : acc;
}
template <>
__device__ __forceinline__ cd shift_apply<double, cd>(const Sell<double> &A, cd acc, cd yrow) {
  return A.shifted ? cd{A.shr, A.shi} * yrow - acc : acc;
}
template <>
__device__ __forceinline__ cd shift_apply<cd, cd>(const Sell<cd> &A, cd acc, cd yrow) {
  return A.shifted ? cd{A.shr, A.shi} * yrow - acc : acc;
}

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
  if (A.shifted) acc = shift_apply<M, T>(A, acc, up(down<V>(up(r[row]) + beta * up(p[row]))));
  return acc;
}

// One row of z = A p with p = r + beta p formed at the gathered columns.  A
// slice of at most 8 entries per row (every stencil here) loads all of the
// row's column indices and values first and then issues all gathers, so that
// up to 24 independent loads per thread are in flight; the sum runs in entry
// order, as in spmv_dir.  Wider slices take spmv_dir.
// Rows wider than 8 entries (e.g. the 19-point black block of the red-black
// preconditioned operator): the same, 8 entries at a time, the sum still in
// entry order.
template <class V, class M, class T>
__device__ __forceinline__ T spmv_dir_groups(const Sell<M> &A, int row, const V *r, const V *p,
                                             T beta, int b0, int w) {
  const int lane = row & 63;
  T a = zero<T>();
  for (int j0 = 0; j0 < w; j0 += 8) {
    int c[8];
    M v[8];
    V g[8], h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j0 + j < w) {
        c[j] = A.col[b0 + lane + RBICG_WAVE * (j0 + j)];
        v[j] = A.val[b0 + lane + RBICG_WAVE * (j0 + j)];
      }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j0 + j < w) {
        g[j] = r[c[j]];
        h[j] = p[c[j]];
      }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j0 + j < w) a += up(v[j]) * up(down<V>(up(g[j]) + beta * up(h[j])));
  }
  if (A.shifted) a = shift_apply<M, T>(A, a, up(down<V>(up(r[row]) + beta * up(p[row]))));
  return a;
}

template <class V, class M, class T>
__device__ __forceinline__ T spmv_dir8(const Sell<M> &A, int row, const V *r, const V *p, T beta) {
  const int slice = row >> 6, lane = row & 63;
  const int b0 = A.sliceptr[slice];
  const int w = (A.sliceptr[slice + 1] - b0) >> 6;
  if (w > 8) {
    // complex matrix values: the per-entry loop (register budget)
    if constexpr (sizeof(M) <= 8) return spmv_dir_groups<V, M, T>(A, row, r, p, beta, b0, w);
    else return spmv_dir<V, M, T>(A, row, r, p, beta);
  }
  int c[8];
  M v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < w) {
      c[j] = A.col[b0 + lane + RBICG_WAVE * j];
      v[j] = A.val[b0 + lane + RBICG_WAVE * j];
    }
  V g[8], h[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < w) {
      g[j] = r[c[j]];
      h[j] = p[c[j]];
    }
  T a = zero<T>();
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < w) a += up(v[j]) * up(down<V>(up(g[j]) + beta * up(h[j])));
  if (A.shifted) a = shift_apply<M, T>(A, a, up(down<V>(up(r[row]) + beta * up(p[row]))));
  return a;
}

// One row of a sliced-ELL matrix of at most 8 entries per row, split into
// phases: the column indices and values, the gathers of r and p at those
// columns, and the sum with p = r + beta p formed at each gathered column (as
// in spmv_dir8).  The first two phases do not depend on beta, so k_it1 issues
// them before it reduces the previous iteration's partials.
template <class V, class M>
struct Row8 {
  int w;
  int c[8];
  M v[8];
  V g[8], h[8];
};
template <class V, class M>
__device__ __forceinline__ void row8_index(const Sell<M> &A, int row, Row8<V, M> &L) {
  const int slice = row >> 6, lane = row & 63;
  const int b0 = A.sliceptr[slice];
  // the 64 lanes of a wave own the 64 rows of one slice (rows are 64-aligned
  // chunks of 1024 plus multiples of the grid's row stride): the width is the
  // same on every active lane, and as a scalar the per-entry tests below
  // become scalar branches instead of per-lane masks
  L.w = __builtin_amdgcn_readfirstlane((A.sliceptr[slice + 1] - b0) >> 6);
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < L.w) {
      L.c[j] = A.col[b0 + lane + RBICG_WAVE * j];
      L.v[j] = A.val[b0 + lane + RBICG_WAVE * j];
    }
}
// The same for a matrix whose slice pointers and column indices are those
// of the matrix P was loaded from (a conjugate transpose that shares the
// pattern): the indices are copied, only the values are loaded.
template <class V, class M>
__device__ __forceinline__ void row8_values(const Sell<M> &A, int row, const Row8<V, M> &P,
                                            Row8<V, M> &L) {
  const int slice = row >> 6, lane = row & 63;
  const int b0 = A.sliceptr[slice];
  L.w = P.w;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < L.w) {
      L.c[j] = P.c[j];
      L.v[j] = A.val[b0 + lane + RBICG_WAVE * j];
    }
}
template <class V, class M>
__device__ __forceinline__ void row8_gather(const V *r, const V *p, Row8<V, M> &L) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < L.w) {
      L.g[j] = r[L.c[j]];
      L.h[j] = p[L.c[j]];
    }
}
template <class V, class M, class T>
__device__ __forceinline__ T row8_sum(const Sell<M> &A, const Row8<V, M> &L, T beta, V rrow,
                                      V prow) {
  T a = zero<T>();
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < L.w) a += up(L.v[j]) * up(down<V>(up(L.g[j]) + beta * up(L.h[j])));
  if (A.shifted) a = shift_apply<M, T>(A, a, up(down<V>(up(rrow) + beta * up(prow))));
  return a;
}

template <class V, class M, class T>
__device__ __forceinline__ T spmv_plain(const Sell<M> &A, int row, const V *x) {
  const int slice = row >> 6, lane = row & 63;
  const int beg = A.sliceptr[slice], end = A.sliceptr[slice + 1];
  T acc = zero<T>();
  // eight entries at a time: their indices and values, then their gathers,
  // are all in flight before the products (summed in entry order)
  for (int e0 = beg + lane; e0 < end; e0 += 8 * RBICG_WAVE) {
    int c[8];
    M v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = e0 + t * RBICG_WAVE;
      c[t] = e < end ? A.col[e] : -1;
      v[t] = e < end ? A.val[e] : M{};
    }
    V xv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) xv[t] = c[t] >= 0 ? x[c[t]] : V{};
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (c[t] >= 0) acc += up(v[t]) * up(xv[t]);
  }
  if (A.shifted) acc = shift_apply<M, T>(A, acc, up(x[row]));
  return acc;
}

// Row chunk of block b of an iteration kernel.  Blocks are dispatched
// round-robin over the 8 XCDs (block b on XCD b mod 8), so b -> (b mod 8)
// nb/8 + b/8 gives each XCD one contiguous range of rows: the neighbour planes
// that its stencil rows gather (rows +-N^2 away) then mostly sit in the same
// XCD's L2 instead of being fetched again by another XCD.
__device__ __forceinline__ int xcd_chunk(int b, int nb) {
  return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

// Stopping test of iteration it-1 and beta_{it-1} (start of iteration it).
// Every block computes the same values; block 0 records them.  Returns false
// (uniformly) when the solve must stop.
template <class T>
__device__ bool it_prologue(const double *P3, int nb, Scalars *S, double *rec, int it, int first,
                            double *tmp, double *red, T &beta, bool block0 = true) {
  constexpr int nv = 2 + ND<T>::v;
  breduce(P3, nb, nv, tmp, red);
  const double rn = sqrt(red[0]), rtn = sqrt(red[1]);
  const T rho = get<T>(red + 2, 0);
  const bool lead = block0 && threadIdx.x == 0;
  double *Rm1 = rec + (size_t)(it - 1) * LOG_STRIDE;
  if (lead) {
    set<T>(Rm1 + 4, 0, rho);
    if (ND<T>::v == 1) Rm1[5] = 0.0;
    Rm1[6] = rn;
    Rm1[7] = rtn;
  }
  int st = ST_RUNNING;
  if (rn <= S->tol * S->bn && rtn <= S->tol * S->btn) st = ST_CONVERGED;
  else if (abs2(rho) == 0.0 || !isfin(rho) || !isfinite(rn) || !isfinite(rtn)) st = ST_BREAKDOWN;
  else if (it > S->maxit) st = ST_MAXIT;
  else if (S->stag_s > 0 && (it - 1 - S->stag_base) % S->stag_s == 0 && it - 1 - S->stag_base >= S->stag_s) {
    // cycle end c of the run: the smallest cycle-end value so far is kept in
    // slot 9 of the cycle-end rows (the host writes that slot only after the run)
    const int s = S->stag_s, base = S->stag_base, c = (it - 1 - base) / s;
    auto h = [&](int cc) {
      const double *R = rec + (size_t)(base + cc * s) * LOG_STRIDE;
      return fmax(R[6] / S->bn, R[7] / S->btn);
    };
    auto best_of = [&](int cc) { return cc == 0 ? h(0) : rec[(size_t)(base + cc * s) * LOG_STRIDE + 9]; };
    const double cur = fmax(rn / S->bn, rtn / S->btn);
    const double best = fmin(best_of(c - 1), cur);
    if (lead) Rm1[9] = best;
    if (cur <= S->stag_lim && cur >= 0.5 * h(c - 1)) st = ST_STAGNATED;
    else if (S->stag_div && c >= S->stag_w && best >= 0.5 * best_of(c - S->stag_w))
      st = best > S->stag_lim ? ST_DIVERGED : ST_STAGNATED;
  }
  if (st != ST_RUNNING) {
    if (lead) {
      S->status = st;
      S->iter = it - 1;
      S->done = 1;
    }
    return false;
  }
  if (first) {
    beta = zero<T>();
  } else {
    beta = divide(rho, get<T>(rec + (size_t)(it - 2) * LOG_STRIDE + 4, 0));
  }
  if (lead) {
    double *R0 = rec + (size_t)it * LOG_STRIDE;
    set<T>(R0 + 2, 0, beta);
    if (ND<T>::v == 1) R0[3] = 0.0;
  }
  return true;
}

// Most doubles of k_it1 partials per block: (3k + 1) values, plus 2k with
// re-projection, times the components of T
#define P1S (6 * KMAXD + 2)

// Restriction partials of one group of GC columns per pass over the block's
// rows (one row per thread): C~_j^H u, C_j^H u~ and, with NPC = 3, the row's
// share of (p~^H C)_j.  All 2 GC column loads of a group are in flight
// together (clamped indices; columns past k are zeroed) and the group's 16
// wave sums share one halving exchange.  The three kinds go to LDS values
// base_a + j, base_b + j, base_e + j.
template <int NPC, class V, class T>
__device__ __forceinline__ void restrict_group(const V *__restrict__ C, const V *__restrict__ Ct,
                                               int k, int ld, size_t rowc, T u, T ut, T cpt,
                                               double *lds, int ls, int base_a, int base_b,
                                               int base_e) {
  constexpr int NDV = ND<T>::v;
  constexpr int GC = 16 / (NPC * NDV);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j0 = 0; j0 < k; j0 += GC) {
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = 0.0;
#pragma unroll
    for (int g = 0; g < GC; ++g) {
      const int j = j0 + g;
      const size_t off = (size_t)(j < k ? j : k - 1) * ld + rowc;
      T ctv = up(Ct[off]), cv = up(C[off]);
      if (j >= k) {
        ctv = zero<T>();
        cv = zero<T>();
      }
      const T a = cj(ctv) * u, b = cj(cv) * ut;
#pragma unroll
      for (int c = 0; c < NDV; ++c) {
        v[g * NDV + c] = comp(a, c);
        v[(GC + g) * NDV + c] = comp(b, c);
      }
      if constexpr (NPC == 3) {
        const T e = cpt * cv;
#pragma unroll
        for (int c = 0; c < NDV; ++c) v[(2 * GC + g) * NDV + c] = comp(e, c);
      }
    }
    const double sum = wave_sum16(v);
    const int id = lane >> 2;
    if ((lane & 3) == 0 && id < NPC * GC * NDV) {
      const int h = id / (GC * NDV), g = (id % (GC * NDV)) / NDV, c = id % NDV, j = j0 + g;
      const int base = h == 0 ? base_a : (h == 1 ? base_b : base_e);
      if (j < k) lds[wv * ls + (base + j) * NDV + c] = sum;
    }
  }
}

}  // namespace

// ===================================================================== kernels
// Body of k_it1 for block bid of the nbl blocks that own the system (the
// whole grid, or one slot of a batched launch); lds holds the wave partials,
// NW rows of ls values (dynamic: sized by the recycle dimension, so that the
// block leaves room on its CU for cycle-end kernels).
template <class V, class M, int RPT>
__device__ __forceinline__ void it1_body(
    Sell<M> A, Sell<M> AH, const V *__restrict__ r, const V *__restrict__ p,
    const V *__restrict__ rt, const V *__restrict__ pt, V *__restrict__ pn, V *__restrict__ ptn,
    V *__restrict__ z, V *__restrict__ zt, const V *__restrict__ C, const V *__restrict__ Ct,
    int k, int ld, V *capR, V *capRt, V *capZ, V *capZt, const double *__restrict__ P3,
    double *__restrict__ P1, Scalars *S, double *rec, int it, int first, int rp, int bid, int nbl,
    double *lds) {
  using T = typename Ar<V>::T;
  rp = sizeof(V) == 4 ? rp : 0;  // re-projection exists for float storage only
  const int ls = (3 * k + 1 + (rp ? 2 * k : 0)) * ND<T>::v;
  __shared__ double tmp[IB];
  __shared__ double red[8];
  const int n = A.n;
  const int stride = nbl * IB;
  const int row0 = xcd_chunk(bid, nbl) * IB + threadIdx.x;
  // one row per thread: the row's own entries, A's indices, values and
  // gathers and A^H's indices and values are loaded before the partials of
  // the previous iteration are reduced (none of them depends on beta)
  Row8<V, M> LA, LB;
  V pre[4] = {};  // r, r~, p, p~ at the row
  bool fast = false;
  // real data (register budget): the same row routine for every row a
  // thread owns; the first row's loads go out before the prologue
  constexpr bool ROWFAST = sizeof(M) <= 8 && sizeof(V) <= 8;
  auto row_loads = [&](int row) {
    pre[0] = r[row];
    pre[1] = rt[row];
    pre[2] = p[row];
    pre[3] = pt[row];
    row8_index(A, row, LA);
    if (AH.col == A.col) row8_values(AH, row, LA, LB);  // uniform branch
    else row8_index(AH, row, LB);
    fast = LA.w <= 8 && LB.w <= 8;
    if (fast) row8_gather(r, p, LA);
  };
  if constexpr (ROWFAST && RPT == 1) {
    if (row0 < n) row_loads(row0);
  } else if constexpr (ROWFAST) {
    if (row0 < n) {
      pre[0] = r[row0];
      pre[1] = rt[row0];
      pre[2] = p[row0];
      pre[3] = pt[row0];
      row8_index(A, row0, LA);
      if (LA.w <= 8) row8_gather(r, p, LA);
    }
  }
  // after the loads above are in flight (a launch past the stopping test
  // reads and discards them)
  if (S->done) return;
  T beta;
  if (!it_prologue<T>(P3, nbl, S, rec, it, first, tmp, red, beta, bid == 0)) return;
  const T betac = cj(beta);
  if constexpr (ROWFAST && RPT > 1) {
    // Several rows per thread: each row in turn, A's indices, values and
    // gathers in flight together, then A^H's (one set of row registers for
    // both, reusing A's indices when A^H shares the pattern); z, z~ and p~ go
    // to memory and the restriction re-reads them (cache hits) column group
    // by column group instead of keeping them in registers per row.  The
    // first row's A loads were issued before the prologue (LA).
    T s0 = zero<T>();
    const bool shared = AH.col == A.col;
#pragma unroll 1
    for (int q = 0; q < RPT; ++q) {
      const int row = row0 + q * stride;
      if (row >= n) break;  // rows grow with q
      if (q > 0) {
        pre[0] = r[row];
        pre[1] = rt[row];
        pre[2] = p[row];
        pre[3] = pt[row];
        row8_index(A, row, LA);
        if (LA.w <= 8) row8_gather(r, p, LA);
      }
      const V rv = pre[0], rtv = pre[1], pv = pre[2], ptv0 = pre[3];
      pn[row] = down<V>(up(rv) + beta * up(pv));
      const V ptv = down<V>(up(rtv) + betac * up(ptv0));
      ptn[row] = ptv;
      const T za = LA.w <= 8 ? row8_sum<V, M, T>(A, LA, beta, rv, pv)
                             : spmv_dir<V, M, T>(A, row, r, p, beta);
      if (shared) row8_values(AH, row, LA, LA);
      else row8_index(AH, row, LA);
      T zb;
      if (LA.w <= 8) {
        row8_gather(rt, pt, LA);
        zb = row8_sum<V, M, T>(AH, LA, betac, rtv, ptv0);
      } else {
        zb = spmv_dir<V, M, T>(AH, row, rt, pt, betac);
      }
      const T zz = up(down<V>(za));
      const T zzt = up(down<V>(zb));
      s0 += cj(up(ptv)) * zz;
      z[row] = down<V>(zz);
      zt[row] = down<V>(zzt);
      if (capR) {
        capR[row] = rv;
        capRt[row] = rtv;
        if (capZ != z) {  // z kept apart from its ring slot
          capZ[row] = down<V>(zz);
          capZt[row] = down<V>(zzt);
        }
      }
    }
    put<T>(lds, ls, 3 * k, s0);
    // restriction: groups of G columns, rows in the same order as above
    constexpr int G = sizeof(V) == 8 ? 4 : 8;
    for (int j0 = 0; j0 < k; j0 += G) {
      T a[G], b[G], e[G], c[G], d[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        a[g] = zero<T>();
        b[g] = zero<T>();
        e[g] = zero<T>();
        c[g] = zero<T>();
        d[g] = zero<T>();
      }
      for (int q = 0; q < RPT; ++q) {
        const int row = row0 + q * stride;
        if (row >= n) break;
        const T zz = up(z[row]), zzt = up(zt[row]), cptv = cj(up(ptn[row]));
        T rv = zero<T>(), rtv = zero<T>();
        if (rp) {
          rv = up(r[row]);
          rtv = up(rt[row]);
        }
        V cb[G], ctb[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const size_t off = (size_t)min(j0 + g, k - 1) * ld + row;
          cb[g] = C[off];
          ctb[g] = Ct[off];
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const T cv = up(cb[g]), ctv = up(ctb[g]);
          a[g] += cj(ctv) * zz;
          b[g] += cj(cv) * zzt;
          e[g] += cptv * cv;
          if (rp) {
            c[g] += cj(ctv) * rv;
            d[g] += cj(cv) * rtv;
          }
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (j0 + g < k) {
          put<T>(lds, ls, j0 + g, a[g]);
          put<T>(lds, ls, k + j0 + g, b[g]);
          put<T>(lds, ls, 2 * k + j0 + g, e[g]);
          if (rp) {
            put<T>(lds, ls, 3 * k + 1 + j0 + g, c[g]);
            put<T>(lds, ls, 4 * k + 1 + j0 + g, d[g]);
          }
        }
    }
    __syncthreads();
    bstore(lds, ls, NW, ls, P1, bid);
    return;
  }
  // per row: z, z~, r_{i-1}, r~_{i-1} and conj(p~) as stored
  T zr[RPT], ztr[RPT], rr_[RPT], rtr_[RPT], cpt[RPT];
  T s0 = zero<T>();
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    zr[q] = zero<T>();
    ztr[q] = zero<T>();
    rr_[q] = zero<T>();
    rtr_[q] = zero<T>();
    cpt[q] = zero<T>();
    const int row = row0 + q * stride;
    if (row < n) {
      const V rv = fast ? pre[0] : r[row], rtv = fast ? pre[1] : rt[row];
      const V pv = fast ? pre[2] : p[row], ptv0 = fast ? pre[3] : pt[row];
      rr_[q] = up(rv);
      rtr_[q] = up(rtv);
      pn[row] = down<V>(up(rv) + beta * up(pv));
      const V ptv = down<V>(up(rtv) + betac * up(ptv0));
      ptn[row] = ptv;
      cpt[q] = cj(up(ptv));
      // one row per thread: the unrolled gathers fit the register budget
      T za, zb;
      if (fast) {
        row8_gather(rt, pt, LB);
        za = row8_sum<V, M, T>(A, LA, beta, rv, pv);
        zb = row8_sum<V, M, T>(AH, LB, betac, rtv, ptv0);
      } else if constexpr (RPT == 1) {
        za = spmv_dir8<V, M, T>(A, row, r, p, beta);
        zb = spmv_dir8<V, M, T>(AH, row, rt, pt, betac);
      } else {
        za = spmv_dir<V, M, T>(A, row, r, p, beta);
        zb = spmv_dir<V, M, T>(AH, row, rt, pt, betac);
      }
      const T zz = up(down<V>(za));
      const T zzt = up(down<V>(zb));
      zr[q] = zz;
      ztr[q] = zzt;
      s0 += cpt[q] * zz;
      z[row] = down<V>(zz);
      zt[row] = down<V>(zzt);
      if (capR) {
        capR[row] = rv;
        capRt[row] = rtv;
        if (capZ != z) {  // z kept apart from its ring slot
          capZ[row] = down<V>(zz);
          capZt[row] = down<V>(zzt);
        }
      }
    }
  }
  // partial layout (values of T): zeta = C~^H z at [0, k), zeta~ = C^H z~ at
  // [k, 2k), e = (p~^H C) at [2k, 3k), (p~, z) at 3k; with rp also
  // g = C~^H r_{i-1} at [3k+1, 4k+1) and g~ = C^H r~_{i-1} at [4k+1, 5k+1).
  // k_it2 assembles sigma = (p~, q) = (p~, z) - e zeta from them.
  put<T>(lds, ls, 3 * k, s0);
  if (k > 0) {
    if constexpr (RPT > 1 || sizeof(M) > 8) {
      // several rows per thread (their loads already overlap) or complex
      // matrix values (register budget): one column at a time
      for (int j = 0; j < k; ++j) {
        T a = zero<T>(), b = zero<T>(), e = zero<T>();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int row = row0 + q * stride;
          if (row < n) {
            const T ctv = up(Ct[(size_t)j * ld + row]), cv = up(C[(size_t)j * ld + row]);
            a += cj(ctv) * zr[q];
            b += cj(cv) * ztr[q];
            e += cpt[q] * cv;
          }
        }
        put<T>(lds, ls, j, a);
        put<T>(lds, ls, k + j, b);
        put<T>(lds, ls, 2 * k + j, e);
      }
      // r_{i-1} read again (cached) rather than held in registers
      for (int j = 0; rp && j < k; ++j) {
        T c = zero<T>(), d = zero<T>();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int row = row0 + q * stride;
          if (row < n) {
            c += cj(up(Ct[(size_t)j * ld + row])) * up(r[row]);
            d += cj(up(C[(size_t)j * ld + row])) * up(rt[row]);
          }
        }
        put<T>(lds, ls, 3 * k + 1 + j, c);
        put<T>(lds, ls, 4 * k + 1 + j, d);
      }
    } else {
      const size_t rowc = row0 < n ? row0 : n - 1;  // rows past n carry zero factors
      restrict_group<3, V, T>(C, Ct, k, ld, rowc, zr[0], ztr[0], cpt[0], lds, ls, 0, k, 2 * k);
      if (rp)
        restrict_group<2, V, T>(C, Ct, k, ld, rowc, rr_[0], rtr_[0], zero<T>(), lds, ls,
                                3 * k + 1, 4 * k + 1, 0);
    }
  }
  __syncthreads();
  bstore(lds, ls, NW, ls, P1, bid);
}

template <class V, class M, int RPT>
__global__ __launch_bounds__(IB) void k_it1(
    Sell<M> A, Sell<M> AH, const V *__restrict__ r, const V *__restrict__ p,
    const V *__restrict__ rt, const V *__restrict__ pt, V *__restrict__ pn, V *__restrict__ ptn,
    V *__restrict__ z, V *__restrict__ zt, const V *__restrict__ C, const V *__restrict__ Ct,
    int k, int ld, V *capR, V *capRt, V *capZ, V *capZt, const double *__restrict__ P3,
    double *__restrict__ P1, Scalars *S, double *rec, int it, int first, int rp) {
  extern __shared__ double lds_dyn[];
  it1_body<V, M, RPT>(A, AH, r, p, rt, pt, pn, ptn, z, zt, C, Ct, k, ld, capR, capRt, capZ, capZt,
                      P3, P1, S, rec, it, first, rp, blockIdx.x, gridDim.x, lds_dyn);
}

// Slot of block blockIdx.x in a batched launch: the last slot s with
// tab[s].b0 <= blockIdx.x (slots in increasing b0, at most RBICG_BATCH_SLOTS;
// a slot's blocks are tab[s].b0 .. tab[s].b0 + tab[s].nb - 1, and the blocks
// up to the next slot's b0 are idle, so that every slot starts on a multiple
// of the XCD count).
template <class A>
__device__ __forceinline__ int batch_slot(const A *tab, int nslot) {
  int s = 0;
  while (s + 1 < nslot && tab[s + 1].b0 <= (int)blockIdx.x) ++s;
  return s;
}

// One iteration's first kernel for several independent systems (one slot
// per system, each with its own matrix, vectors, partials and scalars).
template <class V, class M, int RPT>
__global__ __launch_bounds__(IB) void k_it1_multi(const It1Args<V, M> *__restrict__ tab, int nslot) {
  extern __shared__ double lds_dyn[];
  const It1Args<V, M> &a = tab[batch_slot(tab, nslot)];
  if ((int)blockIdx.x - a.b0 >= a.nb) return;  // alignment gap before the next slot
  it1_body<V, M, RPT>(a.A, a.AH, a.r, a.p, a.rt, a.pt, a.pn, a.ptn, a.z, a.zt, a.C, a.Ct, a.k, a.ld,
                      a.capR, a.capRt, a.capZ, a.capZt, a.P3, a.P1, a.S, a.rec, a.it, a.first, a.rp,
                      (int)blockIdx.x - a.b0, a.nb, lds_dyn);
}

// Reduce the k_it1 partials; sigma = (p~, z) - sum_j e_j zeta_j (= (p~, q));
// alpha = rho_{i-1} / sigma; zeta_c += alpha zeta, zeta~_c += conj(alpha)
// zeta~; per row q = z - C zeta, q~ = z~ - C~ zeta~ (not stored),
// x += alpha p, x~ += conj(alpha) p~, r -= alpha q, r~ -= conj(alpha) q~;
// partials of ||r||^2, ||r~||^2, (r~, r).  With rp set (FP32 storage) first
// r_{i-1} -= C g, r~_{i-1} -= C~ g~ (re-projection, each rounded to storage
// as a stored intermediate would be) and zeta_c -= g, zeta~_c -= g~.
template <class V>
__device__ __forceinline__ void it2_body(int n, V *__restrict__ x, V *__restrict__ xt,
                                         V *__restrict__ r, V *__restrict__ rt,
                                         const V *__restrict__ pn, const V *__restrict__ ptn,
                                         const V *__restrict__ z, const V *__restrict__ zt,
                                         const V *__restrict__ C, const V *__restrict__ Ct,
                                         int k, int ld, const double *__restrict__ P1,
                                         double *__restrict__ P3, Scalars *S, double *rec,
                                         int it, int rp, double *zlog, int zstride, int bid, int nbl) {
  using T = typename Ar<V>::T;
  rp = sizeof(V) == 4 ? rp : 0;  // re-projection exists for float storage only
  __shared__ double lds[NW * 4];
  __shared__ double tmp[IB];
  __shared__ double zl[P1S];
  // The first row's streams (and its first KPF columns of C, C~) do not
  // depend on the scalars: their loads are issued before the partials are
  // reduced, so that the reduction runs under their latency.
  constexpr int KPF = 4;
  const int stride = nbl * IB;
  const int row0 = xcd_chunk(bid, nbl) * IB + threadIdx.x;
  V f[8] = {};
  V fc[KPF] = {}, fct[KPF] = {};
  if (row0 < n) {
    f[0] = z[row0];
    f[1] = zt[row0];
    f[2] = r[row0];
    f[3] = rt[row0];
    f[4] = x[row0];
    f[5] = xt[row0];
    f[6] = pn[row0];
    f[7] = ptn[row0];
#pragma unroll
    for (int j = 0; j < KPF; ++j)
      if (j < k) {
        fc[j] = C[(size_t)j * ld + row0];
        fct[j] = Ct[(size_t)j * ld + row0];
      }
  }
  if (S->done) return;  // after the loads above are in flight
  const int nv1 = (3 * k + 1 + (rp ? 2 * k : 0)) * ND<T>::v;
  breduce(P1, nbl, nv1, tmp, zl);
  T sigma = get<T>(zl, 3 * k);
  for (int j = 0; j < k; ++j) sigma -= get<T>(zl, 2 * k + j) * get<T>(zl, j);
  const bool lead = bid == 0 && threadIdx.x == 0;
  double *Ri = rec + (size_t)it * LOG_STRIDE;
  if (abs2(sigma) == 0.0 || !isfin(sigma)) {
    if (lead) {
      S->status = ST_BREAKDOWN;
      S->iter = it - 1;
      S->done = 1;
    }
    return;
  }
  const T al = divide(get<T>(rec + (size_t)(it - 1) * LOG_STRIDE + 4, 0), sigma);
  const T alc = cj(al);
  if (lead) {
    set<T>(Ri, 0, al);
    if (ND<T>::v == 1) Ri[1] = 0.0;
    Ri[8] = comp(sigma, 0);
    for (int j = 0; j < k; ++j) {
      T u = get<T>(S->zc, j) + al * get<T>(zl, j);
      T ut = get<T>(S->zc, k + j) + alc * get<T>(zl, k + j);
      if (rp) {
        u = u - get<T>(zl, 3 * k + 1 + j);
        ut = ut - get<T>(zl, 4 * k + 1 + j);
      }
      set<T>(S->zc, j, u);
      set<T>(S->zc, k + j, ut);
    }
    // the restrictions zeta_i, zeta~_i of this iteration, for the cycle-end
    // set-up of Sec. 4.4 (B_j from A r_{i-1} = z_i - beta_{i-1} z_{i-1})
    if (zlog) {
      double *zr = zlog + (size_t)it * zstride;
      for (int j = 0; j < 2 * k; ++j) set<T>(zr, j, get<T>(zl, j));
    }
  }
  double rr = 0.0, rtrt = 0.0;
  T rho = zero<T>();
  // several rows per thread: the next row's streams are loaded while this
  // row is computed
  V fn[8] = {};
  for (int row = row0; row < n; row += stride) {
    const bool pre = row == row0;
    if (!pre) {
#pragma unroll
      for (int u = 0; u < 8; ++u) f[u] = fn[u];
    }
    const int nxt = row + stride;
    if (nxt < n) {
      fn[0] = z[nxt];
      fn[1] = zt[nxt];
      fn[2] = r[nxt];
      fn[3] = rt[nxt];
      fn[4] = x[nxt];
      fn[5] = xt[nxt];
      fn[6] = pn[nxt];
      fn[7] = ptn[nxt];
    }
    T qq = up(f[0]), qqt = up(f[1]);
    T rv = up(f[2]), rtv = up(f[3]);
    if (k > 0) {
      T s = zero<T>(), st = zero<T>(), g = zero<T>(), gt = zero<T>();
      auto acc = [&](int j, T cv, T ctv) {
        s += cv * get<T>(zl, j);
        st += ctv * get<T>(zl, k + j);
        if (rp) {
          g += cv * get<T>(zl, 3 * k + 1 + j);
          gt += ctv * get<T>(zl, 4 * k + 1 + j);
        }
      };
      int j = 0;
      if (pre) {
#pragma unroll
        for (int u = 0; u < KPF; ++u)
          if (u < k) acc(u, up(fc[u]), up(fct[u]));
        j = min(KPF, k);
      }
      // the rest in groups whose loads are all issued before the sums
      // (clamped indices; the sums run in column order)
      constexpr int GE = sizeof(V) == 16 ? 4 : 8;
      for (; j < k; j += GE) {
        V cb[GE], ctb[GE];
#pragma unroll
        for (int u = 0; u < GE; ++u) {
          const size_t off = (size_t)min(j + u, k - 1) * ld + row;
          cb[u] = C[off];
          ctb[u] = Ct[off];
        }
#pragma unroll
        for (int u = 0; u < GE; ++u)
          if (j + u < k) acc(j + u, up(cb[u]), up(ctb[u]));
      }
      qq = up(down<V>(qq - s));
      qqt = up(down<V>(qqt - st));
      if (rp) {
        rv = up(down<V>(rv - g));
        rtv = up(down<V>(rtv - gt));
      }
    }
    x[row] = down<V>(up(f[4]) + al * up(f[6]));
    xt[row] = down<V>(up(f[5]) + alc * up(f[7]));
    rv = up(down<V>(rv - al * qq));
    rtv = up(down<V>(rtv - alc * qqt));
    r[row] = down<V>(rv);
    rt[row] = down<V>(rtv);
    rr += abs2(rv);
    rtrt += abs2(rtv);
    rho += cj(rtv) * rv;
  }
  wput(lds, 4, 0, rr);
  wput(lds, 4, 1, rtrt);
#pragma unroll
  for (int c = 0; c < ND<T>::v; ++c) wput(lds, 4, 2 + c, comp(rho, c));
  __syncthreads();
  bstore(lds, 4, NW, 2 + ND<T>::v, P3, bid);
}

template <class V>
__global__ __launch_bounds__(IB) void k_it2(int n, V *__restrict__ x, V *__restrict__ xt,
                                            V *__restrict__ r, V *__restrict__ rt,
                                            const V *__restrict__ pn, const V *__restrict__ ptn,
                                            const V *__restrict__ z, const V *__restrict__ zt,
                                            const V *__restrict__ C, const V *__restrict__ Ct,
                                            int k, int ld, const double *__restrict__ P1,
                                            double *__restrict__ P3, Scalars *S, double *rec,
                                            int it, int rp, double *zlog, int zstride) {
  it2_body<V>(n, x, xt, r, rt, pn, ptn, z, zt, C, Ct, k, ld, P1, P3, S, rec, it, rp, zlog, zstride,
              blockIdx.x, gridDim.x);
}

template <class V>
__global__ __launch_bounds__(IB) void k_it2_multi(const It2Args<V> *__restrict__ tab, int nslot) {
  const It2Args<V> &a = tab[batch_slot(tab, nslot)];
  if ((int)blockIdx.x - a.b0 >= a.nb) return;  // alignment gap before the next slot
  it2_body<V>(a.n, a.x, a.xt, a.r, a.rt, a.pn, a.ptn, a.z, a.zt, a.C, a.Ct, a.k, a.ld, a.P1, a.P3, a.S,
              a.rec, a.it, a.rp, a.zlog, a.zstride, (int)blockIdx.x - a.b0, a.nb);
}

// Stopping test after the last launched iteration (one block).
template <class V>
__global__ __launch_bounds__(IB) void k_itfin(const double *__restrict__ P3, int nb,
                                              Scalars *S, double *rec, int it, int first,
                                              Scalars *hs) {
  using T = typename Ar<V>::T;
  __shared__ double tmp[IB];
  __shared__ double red[8];
  // one block; only its thread 0 (the prologue's lead) writes S->done, after
  // the prologue's barriers, so every wave reads the same value here
  if (!S->done) {
    T beta;
    (void)it_prologue<T>(P3, nb, S, rec, it, first, tmp, red, beta);
  }
  // the stopping test's outcome straight into the host's slot (mapped host
  // memory, read after the event recorded behind this launch completes)
  if (threadIdx.x == 0) {
    hs->done = S->done;
    hs->status = S->status;
    hs->iter = S->iter;
  }
}

// ------------------------------------------------- split preconditioning
// Iteration with the split-preconditioned operator A^ = L^{-1} A U^{-1}
// (ILUT factors): k_it1's work in three steps, because A^ p needs whole
// triangular solves between the SpMV and the restriction:
//   k_op_dir    prologue (stopping test, beta) and p = r + beta p,
//               p~ = r~ + conj(beta) p~ (cycle captures of r_{i-1}, r~_{i-1});
//   A^ p, A^^H p~ by k_sptrsv (U, L^H) / k_spmv / k_sptrsv (L, U^H);
//   k_op_restr  the partials k_it2 reads: zeta = C~^H z, zeta~ = C^H z~,
//               p~^H C and (p~, z) (cycle captures of z, z~).
template <class V>
__global__ __launch_bounds__(IB) void k_op_dir(int n, const V *__restrict__ r,
                                               const V *__restrict__ p, const V *__restrict__ rt,
                                               const V *__restrict__ pt, V *__restrict__ pn,
                                               V *__restrict__ ptn, V *capR, V *capRt,
                                               const double *__restrict__ P3, Scalars *S,
                                               double *rec, int it, int first) {
  using T = typename Ar<V>::T;
  __shared__ double tmp[IB];
  __shared__ double red[8];
  if (S->done) return;
  T beta;
  if (!it_prologue<T>(P3, gridDim.x, S, rec, it, first, tmp, red, beta, blockIdx.x == 0)) return;
  const T betac = cj(beta);
  const int stride = gridDim.x * IB;
  for (int row = xcd_chunk(blockIdx.x, gridDim.x) * IB + threadIdx.x; row < n; row += stride) {
    const V rv = r[row], rtv = rt[row];
    pn[row] = down<V>(up(rv) + beta * up(p[row]));
    ptn[row] = down<V>(up(rtv) + betac * up(pt[row]));
    if (capR) {
      capR[row] = rv;
      capRt[row] = rtv;
    }
  }
}

template <class V>
__global__ __launch_bounds__(IB) void k_op_restr(int n, const V *__restrict__ z,
                                                 const V *__restrict__ zt,
                                                 const V *__restrict__ ptn,
                                                 const V *__restrict__ C, const V *__restrict__ Ct,
                                                 int k, int ld, V *capZ, V *capZt,
                                                 double *__restrict__ P1, const Scalars *S) {
  using T = typename Ar<V>::T;
  extern __shared__ double lds[];
  if (S->done) return;
  const int ls = (3 * k + 1) * ND<T>::v;
  const int stride = gridDim.x * IB;
  const int row0 = xcd_chunk(blockIdx.x, gridDim.x) * IB + threadIdx.x;
  T s0 = zero<T>();
  for (int row = row0; row < n; row += stride) {
    const V zz = z[row], zzt = zt[row];
    s0 += cj(up(ptn[row])) * up(zz);
    if (capZ) {
      capZ[row] = zz;
      capZt[row] = zzt;
    }
  }
  put<T>(lds, ls, 3 * k, s0);
  constexpr int G = sizeof(V) == 16 ? 2 : 4;
  for (int j0 = 0; j0 < k; j0 += G) {
    T a[G], b[G], e[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      a[g] = zero<T>();
      b[g] = zero<T>();
      e[g] = zero<T>();
    }
    for (int row = row0; row < n; row += stride) {
      const T zz = up(z[row]), zzt = up(zt[row]), cptv = cj(up(ptn[row]));
      V cb[G], ctb[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const size_t off = (size_t)min(j0 + g, k - 1) * ld + row;
        cb[g] = C[off];
        ctb[g] = Ct[off];
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const T cv = up(cb[g]), ctv = up(ctb[g]);
        a[g] += cj(ctv) * zz;
        b[g] += cj(cv) * zzt;
        e[g] += cptv * cv;
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (j0 + g < k) {
        put<T>(lds, ls, j0 + g, a[g]);
        put<T>(lds, ls, k + j0 + g, b[g]);
        put<T>(lds, ls, 2 * k + j0 + g, e[g]);
      }
  }
  __syncthreads();
  bstore(lds, ls, NW, ls, P1, blockIdx.x);
}

// 1 / d as the vector type (d real or complex)
template <class T> __device__ __forceinline__ T inv_as(double d);
template <> __device__ __forceinline__ double inv_as<double>(double d) { return 1.0 / d; }
template <> __device__ __forceinline__ cd inv_as<cd>(double d) { return cd{1.0 / d, 0.0}; }
template <class T> __device__ __forceinline__ T inv_as(cd d);
template <> __device__ __forceinline__ cd inv_as<cd>(cd d) { return cdiv(cd{1.0, 0.0}, d); }

// y = A x (sliced ELL, one row per thread); nothing after the stopping test.
template <class V, class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_spmv(Sell<M> A, const V *__restrict__ x,
                                                      V *__restrict__ y, const Scalars *S) {
  using T = typename Ar<V>::T;
  if (S && S->done) return;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (row < A.n) y[row] = down<V>(spmv_plain<V, M, T>(A, row, x));
}

// Triangular solves T x = b by level schedule, without barriers between
// levels, two independent solves per launch (the primal and the dual
// direction of one step of A^ p / A^^H p~).  Work unit: a chunk of 64
// consecutive positions of a solve's order (one wave; order lists the rows
// level by level, each level padded with -1 to whole chunks, so a chunk's
// rows never depend on each other).  A fixed number of waves take chunks from
// a counter, the two solves' chunks interleaved; a row waits only for rows of
// earlier chunks of its solve, which were taken earlier by waves that are
// running, so the waits end.  Keeping the number of waves near the width of a
// few levels (rather than one wave per chunk) keeps the polling traffic to
// the frontier.  The values carry their own readiness: x is first filled with
// TRSV_PENDING (k_trsv_pending), a signalling NaN that no arithmetic produces
// (operations return quiet NaNs); a row polls each value it needs with
// device-coherent 64-bit loads until it differs from the sentinel (a complex
// value is two such words, each polled) and publishes its own with
// device-coherent stores: the polled word is the datum, so neither flags nor
// cache invalidations are needed.  The wait is bounded: past SPIN_MAX polls,
// or once another row has set *err, the row sets *err and goes on (the caller
// reports an error).
#define SPIN_MAX (1 << 22)
#define TRSV_PENDING 0x7FF4C0DE5E471E00ULL
#define TRSV_QNAN 0x7FF8000000000000ULL

// x0 (n0 values) and x1 (n1; may be absent) to the sentinel, the chunk
// counter to zero
template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_trsv_pending(int n0, V *x0, int n1, V *x1,
                                                              int *counter, const Scalars *S) {
  constexpr int NWD = sizeof(V) / 8;
  if (S && S->done) return;
  const int i = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i == 0) *counter = 0;
  if (i < n0) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(x0) + (size_t)i * NWD;
#pragma unroll
    for (int c = 0; c < NWD; ++c) w[c] = TRSV_PENDING;
  }
  if (x1 && i < n1) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(x1) + (size_t)i * NWD;
#pragma unroll
    for (int c = 0; c < NWD; ++c) w[c] = TRSV_PENDING;
  }
}

// One row of T x = b (row < 0: padding, nothing to do).
template <class V, class M>
__device__ __forceinline__ void trsv_row(const TriDev<M> &Tm, const V *__restrict__ b, V *x,
                                         int row, int *err) {
  using T = typename Ar<V>::T;
  constexpr int NWD = sizeof(V) / 8;
  if (row < 0) return;
  unsigned long long *xw = reinterpret_cast<unsigned long long *>(x);
  T acc = up(b[row]);
  for (int e = Tm.rp[row]; e < Tm.rp[row + 1]; ++e) {
    const unsigned long long *src = xw + (size_t)Tm.ci[e] * NWD;
    unsigned long long wv[NWD];
#pragma unroll
    for (int c = 0; c < NWD; ++c) {
      int spins = 0;
      while ((wv[c] = __hip_atomic_load(src + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ==
             TRSV_PENDING) {
        // past the bound, or once any row has given up: stop waiting
        if (++spins > SPIN_MAX ||
            ((spins & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    V xv;
    __builtin_memcpy(&xv, wv, sizeof(V));
    acc -= up(Tm.v[e]) * up(xv);
  }
  if (Tm.diag) acc = acc * inv_as<T>(up(Tm.diag[row]));
  const V out = down<V>(acc);
  unsigned long long ow[NWD];
  __builtin_memcpy(ow, &out, sizeof(V));
#pragma unroll
  for (int c = 0; c < NWD; ++c) {
    if (ow[c] == TRSV_PENDING) ow[c] = TRSV_QNAN;  // an input that carried the sentinel itself
    __hip_atomic_store(xw + (size_t)row * NWD + c, ow[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ns = 1 or 2 solves (T0, b0, x0) and (T1, b1, x1); len of both a multiple of 64
template <class V, class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_sptrsv(TriDev<M> T0, const V *__restrict__ b0,
                                                        V *x0, TriDev<M> T1,
                                                        const V *__restrict__ b1, V *x1, int ns,
                                                        int *counter, const Scalars *S, int *err) {
  if (S && S->done) return;
  const int lane = threadIdx.x & 63;
  const int nc0 = T0.len >> 6, nc1 = ns > 1 ? T1.len >> 6 : 0;
  const int both = 2 * min(nc0, nc1), total = nc0 + nc1;
  while (true) {
    int c = 0;
    if (lane == 0) c = __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c = __builtin_amdgcn_readfirstlane(c);
    if (c >= total) break;
    // interleave the two solves while both have chunks left
    bool first;
    int lc;
    if (c < both) {
      first = (c & 1) == 0;
      lc = c >> 1;
    } else {
      first = nc0 > nc1;
      lc = (c - both) + (both >> 1);
    }
    if (first) trsv_row<V, M>(T0, b0, x0, T0.order[lc * 64 + lane], err);
    else trsv_row<V, M>(T1, b1, x1, T1.order[lc * 64 + lane], err);
  }
}

// y = A x with optional index maps: row j computes A's row orow[j] (NULL:
// j) and reads x at gmap[c] for column c (NULL: c).  With ILUTP's column
// permutation Q (A Q)(:, j) = A(:, perm[j]): y = A (Q t) is gmap = pos
// (column -> position), y = Q^T (A^H v) is orow = perm.  Nothing after the
// stopping test.
template <class V, class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_spmv_perm(Sell<M> A, const V *__restrict__ x,
                                                           V *__restrict__ y,
                                                           const int *__restrict__ gmap,
                                                           const int *__restrict__ orow,
                                                           const Scalars *S) {
  using T = typename Ar<V>::T;
  if (S && S->done) return;
  const int j = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (j >= A.n) return;
  const int row = orow ? orow[j] : j;
  const int slice = row >> 6, lane = row & 63;
  const int beg = A.sliceptr[slice], end = A.sliceptr[slice + 1];
  T acc = zero<T>();
  for (int e = beg + lane; e < end; e += RBICG_WAVE) {
    const int c = A.col[e];
    acc += up(A.val[e]) * up(x[gmap ? gmap[c] : c]);
  }
  if (A.shifted) acc = shift_apply<M, T>(A, acc, up(x[gmap ? gmap[row] : row]));
  y[j] = down<V>(acc);
}

// out[i] = in[map[i]]
template <class V>
__global__ void k_gather(int n, const V *__restrict__ in, const int *__restrict__ map,
                         V *__restrict__ out) {
  const int i = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i < n) out[i] = in[map[i]];
}

// out = b - t (out may be t)
template <class V>
__global__ void k_rsub(int n, const V *__restrict__ b, const V *t, V *out) {
  using T = typename Ar<V>::T;
  const int i = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i < n) out[i] = down<V>(up(b[i]) - up(t[i]));
}

// k_itfin for several systems: block s is slot s's stopping test.
template <class V>
__global__ __launch_bounds__(IB) void k_itfin_multi(const ItfinArgs *__restrict__ tab) {
  using T = typename Ar<V>::T;
  __shared__ double tmp[IB];
  __shared__ double red[8];
  const ItfinArgs &a = tab[blockIdx.x];
  if (!a.S->done) {
    T beta;
    (void)it_prologue<T>(a.P3, a.nb, a.S, a.rec, a.it, a.first, tmp, red, beta, true);
  }
  if (threadIdx.x == 0) {
    a.hs->done = a.S->done;
    a.hs->status = a.S->status;
    a.hs->iter = a.S->iter;
  }
}

// P3-layout partials (||r||^2, ||r~||^2, (r~, r)) of the initial residuals.
template <class V>
__global__ __launch_bounds__(IB) void k_init_p3(int n, const V *__restrict__ r,
                                                const V *__restrict__ rt, double *P3) {
  using T = typename Ar<V>::T;
  __shared__ double lds[NW * 4];
  const int stride = gridDim.x * IB;
  double rr = 0.0, rtrt = 0.0;
  T rho = zero<T>();
  for (int row = blockIdx.x * IB + threadIdx.x; row < n; row += stride) {
    const T rv = up(r[row]), rtv = up(rt[row]);
    rr += abs2(rv);
    rtrt += abs2(rtv);
    rho += cj(rtv) * rv;
  }
  wput(lds, 4, 0, rr);
  wput(lds, 4, 1, rtrt);
#pragma unroll
  for (int c = 0; c < ND<T>::v; ++c) wput(lds, 4, 2 + c, comp(rho, c));
  __syncthreads();
  bstore(lds, 4, NW, 2 + ND<T>::v, P3, blockIdx.x);
}

// Up to three dot products (a_i, b_i) as block partials (3 * ND values).
template <class V>
__global__ __launch_bounds__(IB) void k_dots(int n, const V *a0, const V *b0, const V *a1,
                                             const V *b1, const V *a2, const V *b2, double *P) {
  using T = typename Ar<V>::T;
  __shared__ double lds[NW * 8];
  const int stride = gridDim.x * IB;
  T d0 = zero<T>(), d1 = zero<T>(), d2 = zero<T>();
  for (int row = blockIdx.x * IB + threadIdx.x; row < n; row += stride) {
    if (a0) d0 += cj(up(a0[row])) * up(b0[row]);
    if (a1) d1 += cj(up(a1[row])) * up(b1[row]);
    if (a2) d2 += cj(up(a2[row])) * up(b2[row]);
  }
  put<T>(lds, 8, 0, d0);
  put<T>(lds, 8, 1, d1);
  put<T>(lds, 8, 2, d2);
  __syncthreads();
  bstore(lds, 8, NW, 3 * ND<T>::v, P, blockIdx.x);
}

// Restriction partials: [B^H u (k values), B2^H u2 (k values)].
template <class V>
__global__ __launch_bounds__(IB) void k_restrict(int n, const V *u, const V *B, const V *u2,
                                                 const V *B2, int k, int ld, double *P) {
  using T = typename Ar<V>::T;
  __shared__ double lds[NW * 4 * KMAXD];
  const int stride = gridDim.x * IB;
  const int ls = 4 * KMAXD;
  for (int j = 0; j < k; ++j) {
    T a = zero<T>(), b = zero<T>();
    for (int row = blockIdx.x * IB + threadIdx.x; row < n; row += stride) {
      a += cj(up(B[(size_t)j * ld + row])) * up(u[row]);
      b += cj(up(B2[(size_t)j * ld + row])) * up(u2[row]);
    }
    put<T>(lds, ls, j, a);
    put<T>(lds, ls, k + j, b);
  }
  __syncthreads();
  bstore(lds, ls, NW, 2 * k * ND<T>::v, P, blockIdx.x);
}

// One block: out[t] = fixed-order sum of the nb block partials.
__global__ __launch_bounds__(IB) void k_fin_red(const double *P, int nb, int nv, double *out) {
  __shared__ double tmp[IB];
  __shared__ double res[4 * KMAXD];
  breduce(P, nb, nv, tmp, res);
  for (int t = threadIdx.x; t < nv; t += IB) out[t] = res[t];
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


// x += sx * U c1; r += sr * C c1; xt += sxt * Ut c2; rt += srt * Ct c2 with
// coefficients coef = [c1 (k values), c2 (k values)] (doubles, ND per value).
template <class V>
__global__ __launch_bounds__(RBICG_BLOCK) void k_expand2(int n, V *x, const V *U, double sx,
                                                         V *r, const V *C, double sr, V *xt,
                                                         const V *Ut, double sxt, V *rt,
                                                         const V *Ct, double srt, int k, int ld,
                                                         const double *coef) {
  using T = typename Ar<V>::T;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (row >= n) return;
  T a = zero<T>(), b = zero<T>(), c = zero<T>(), d = zero<T>();
  for (int j = 0; j < k; ++j) {
    const T g1 = get<T>(coef, j), g2 = get<T>(coef, k + j);
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
// FP32-inner mode: round FP64 data to float storage, and accumulate a float
// correction into an FP64 vector (x += sgn d, sgn = +-1, computed in double).
__global__ void k_d2f(const double *__restrict__ in, float *__restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}
template <class S>
__global__ void k_add_to_d(double *__restrict__ x, const S *__restrict__ d, double sgn, size_t n) {
  const size_t i = (size_t)blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i < n) x[i] += sgn * (double)d[i];
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

// Values of the pencil alpha E + beta A on a shared sliced-ELL layout (the
// shifted operators sigma E - A of Algorithm 3 with E != I).  a, e: real
// (acplx / ecplx = 0) or complex entries; padding entries are zero in both.
__global__ void k_pencil(size_t m, const void *a, int acplx, const void *e, int ecplx, cd alpha,
                         cd beta, cd *out) {
  const size_t i = (size_t)blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i >= m) return;
  const cd av = acplx ? ((const cd *)a)[i] : cd{((const double *)a)[i], 0.0};
  const cd ev = ecplx ? ((const cd *)e)[i] : cd{((const double *)e)[i], 0.0};
  out[i] = alpha * ev + beta * av;
}

// ----------------------------------------------------- cycle-end kernels
// Load through a pointer known to point at device global memory (pointers
// read back from LDS tables would otherwise produce flat loads).
template <class V>
__device__ __forceinline__ V gload(const V *p, size_t i) {
  return ((const __attribute__((address_space(1))) V *)p)[i];
}
template <>
__device__ __forceinline__ cd gload<cd>(const cd *p, size_t i) {
  const __attribute__((address_space(1))) double *q =
      (const __attribute__((address_space(1))) double *)p + 2 * i;
  return cd{q[0], q[1]};
}

// FP64 MFMA 16x16x4 (one wave): A operand A[i][kk] in lane i + 16 kk, B operand
// B[kk][j] in lane j + 16 kk, accumulator D[i][j] in lane j + 16 (i % 4),
// register i / 4.
typedef double d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

#define GRAM_MAXT 9        // output tiles per wave (at most 36 tiles of 16 x 16)
#define TS_PC(JT) (16 * (JT) + 2)  // LDS row stride (doubles) of W in k_tsgemm_mfma
#define GRAM_BLOCK 256

// Gram partials over a chunk of rows: G[i][j] = sum conj(X_i) Y_j for every
// (i < mx <= 128, j < my), one complex (re, im) per entry.  Each block reads its
// rows of every column once, in slabs of SR rows staged in LDS (column stride
// SR + 2 doubles keeps the MFMA operand reads free of bank conflicts), double
// buffered: the next slab's loads are in flight while the MFMAs consume the
// current one.  All 16 x 16 output tiles of the block accumulate on MFMA.
// With gridDim.y = 2 the launch holds two independent Grams: blocks with
// blockIdx.y = 1 contract X[x1, x1 + mx1) against Y[y1, y1 + my1) and write
// their entries after the mx x my entries of the first in each chunk's
// partial row.
template <class V, int SR, int GRAM_NLD, int MAXT>
__global__ __launch_bounds__(GRAM_BLOCK) void k_gram_mfma(int n, ColList X, int mx, ColList Y,
                                                          int my, int rows_per_chunk,
                                                          double *partial, int same, int x1,
                                                          int mx1, int y1, int my1) {
  constexpr int ndv = sizeof(V) == 16 ? 2 : 1;
  constexpr int PC = SR + 2;
  extern __shared__ double sm[];
  const size_t tot = (size_t)mx * my + (gridDim.y > 1 ? (size_t)mx1 * my1 : 0);
  size_t base = 0;
  int xo = 0, yo = 0;
  if (blockIdx.y == 1) {
    base = (size_t)mx * my;
    xo = x1;
    yo = y1;
    mx = mx1;
    my = my1;
    same = 0;
  }
  const int mxp = (mx + 15) / 16 * 16, myp = (my + 15) / 16 * 16;
  // same: Y is X (a Hermitian Gram); its columns are staged once
  const int ncol = same ? mxp : mxp + myp;
  const size_t bufsz = (size_t)ndv * ncol * PC;
  const int TY = myp / 16, T = (mxp / 16) * TY;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nval = ncol * SR;
  d4 acc[MAXT][ndv];
#pragma unroll
  for (int t = 0; t < MAXT; ++t)
#pragma unroll
    for (int c = 0; c < ndv; ++c) acc[t][c] = d4{0.0, 0.0, 0.0, 0.0};
  const int r0 = blockIdx.x * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  const int nslabs = (r1 - r0 + SR - 1) / SR;
  double pre[GRAM_NLD][ndv];
  // Each thread's (column, row-in-slab) pairs are the same for every slab:
  // resolve the column pointers once (a per-lane index into the pointer list
  // would otherwise make every data load wait for a pointer load first).
  const V *colp[GRAM_NLD];
  int rrs[GRAM_NLD];
#pragma unroll
  for (int t = 0; t < GRAM_NLD; ++t) {
    const int idx = threadIdx.x + t * GRAM_BLOCK;
    const int c = idx / SR;
    rrs[t] = idx % SR;
    const bool isx = c < mxp;
    const int cc = isx ? c : c - mxp;
    colp[t] = (idx < nval && cc < (isx ? mx : my)) ? (const V *)(isx ? X.p[xo + cc] : Y.p[yo + cc])
                                                   : nullptr;
  }
  // global -> registers for slab `sl`
  auto load = [&](int sl) {
    const int base = r0 + sl * SR;
#pragma unroll
    for (int t = 0; t < GRAM_NLD; ++t) {
      const int row = base + rrs[t];
      double vr = 0.0, vi = 0.0;
      if (colp[t] && row < r1) {
        const V v = colp[t][row];
        if constexpr (ndv == 2) {
          vr = ((const cd &)v).x;
          vi = ((const cd &)v).y;
        } else {
          vr = (double)v;
        }
      }
      pre[t][0] = vr;
      if constexpr (ndv == 2) pre[t][ndv - 1] = vi;
    }
  };
  // registers -> LDS buffer b: layout [part][column][PC] with X columns first
  auto store = [&](int b) {
    double *buf = sm + (size_t)b * bufsz;
#pragma unroll
    for (int t = 0; t < GRAM_NLD; ++t) {
      const int idx = threadIdx.x + t * GRAM_BLOCK;
      if (idx < nval) {
        const int c = idx / SR, rr = idx % SR;
        buf[(size_t)c * PC + rr] = pre[t][0];
        if constexpr (ndv == 2) buf[(size_t)ncol * PC + (size_t)c * PC + rr] = pre[t][ndv - 1];
      }
    }
  };
  if (nslabs > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int sl = 0; sl < nslabs; ++sl) {
    if (sl + 1 < nslabs) load(sl + 1);
    const double *buf = sm + (size_t)(sl & 1) * bufsz;
    // k-steps outside, tiles inside: consecutive MFMAs feed different
    // accumulators, so they issue back to back instead of waiting out the
    // latency of a dependent chain
#pragma unroll
    for (int kk = 0; kk < SR; kk += 4) {
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        const int tile = w + 4 * t;
        if (tile < T) {
          const int ti = tile / TY, tj = tile % TY;
          const double *xa = buf + (size_t)(ti * 16 + li) * PC + lk;
          const double *yb = buf + (size_t)((same ? 0 : mxp) + tj * 16 + li) * PC + lk;
          const double ar = xa[kk], br = yb[kk];
          if constexpr (ndv == 1) {
            acc[t][0] = mfma(ar, br, acc[t][0]);
          } else {
            const double ai = xa[(size_t)ncol * PC + kk], bi = yb[(size_t)ncol * PC + kk];
            // conj(x) y = (xr yr + xi yi) + i (xr yi - xi yr)
            acc[t][0] = mfma(ar, br, acc[t][0]);
            acc[t][0] = mfma(ai, bi, acc[t][0]);
            acc[t][ndv - 1] = mfma(ar, bi, acc[t][ndv - 1]);
            acc[t][ndv - 1] = mfma(-ai, br, acc[t][ndv - 1]);
          }
        }
      }
    }
    if (sl + 1 < nslabs) store((sl + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int tile = w + 4 * t;
    if (tile < T) {
      const int ti = tile / TY, tj = tile % TY;
      const int gj = tj * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = ti * 16 + lk + 4 * v;
        if (gi < mx && gj < my) {
          // real data: one double per entry (the reduction fills in Im = 0)
          double *o = partial + ((size_t)blockIdx.x * tot + base + (size_t)gi * my + gj) * ndv;
          o[0] = acc[t][0][v];
          if constexpr (ndv == 2) o[1] = acc[t][ndv - 1][v];
        }
      }
    }
  }
}

// G = sum over chunks of the partials (fixed order); G is mx x my complex,
// stored row-major by (i, j) as in the partials.  real: the partials hold
// count real values and G[2t], G[2t + 1] = (sum, 0).
template <int L>
__global__ __launch_bounds__(256) void k_gram_reduce(const double *partial, int nchunks, int count,
                                                     double *G, int real) {
  // L lanes per entry, each summing every L-th chunk in two chains; the L
  // sums are then added pairwise in a fixed order, so the bits do not depend
  // on timing
  __shared__ double sub[256];
  const int e = blockIdx.x * (256 / L) + threadIdx.x / L, sl = threadIdx.x % L;
  double s0 = 0.0, s1 = 0.0;
  if (e < count) {
    int c = sl;
    // four steps' loads issued together, added in the same order
    for (; c + 7 * L < nchunks; c += 8 * L) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(c + u * L) * count + e];
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        s0 += v[u];
        s1 += v[u + 1];
      }
    }
    for (; c + L < nchunks; c += 2 * L) {
      s0 += partial[(size_t)c * count + e];
      s1 += partial[(size_t)(c + L) * count + e];
    }
    if (c < nchunks) s0 += partial[(size_t)c * count + e];
  }
  sub[threadIdx.x] = s0 + s1;
  __syncthreads();
#pragma unroll
  for (int h = L / 2; h >= 1; h /= 2) {
    if (sl < h) sub[threadIdx.x] += sub[threadIdx.x + h];
    __syncthreads();
  }
  if (sl == 0 && e < count) {
    const double sum = sub[threadIdx.x];
    if (real) {
      G[2 * (size_t)e] = sum;
      G[2 * (size_t)e + 1] = 0.0;
    } else {
      G[e] = sum;
    }
  }
}

// Tall-skinny product Y[:, c] = sum_l X_l W[l, c] (W: m x p complex,
// column-major; p <= 64) computed as Y^T = W^T X^T on MFMA so that both the X
// loads and the Y stores are contiguous 16-row segments.  Each wave owns 16
// rows.
template <class V, int JT>
__global__ __launch_bounds__(256) void k_tsgemm_mfma(int n, ColList X, int m, const cd *W, int p,
                                                     V *Y, int ld) {
  constexpr int ndv = sizeof(V) == 16 ? 2 : 1;
  constexpr int PC = TS_PC(JT);  // LDS row stride of W (padded against bank conflicts)
  __shared__ const V *cols[RBICG_MAXCOLS];
  // W rows of one batch (up to 64 input columns), Re then Im planes:
  // wl[(part * 64 + kk) * PC + c] = W(c, k0 + kk), zero outside m x p
  extern __shared__ double wl[];
  for (int t = threadIdx.x; t < m; t += 256) cols[t] = (const V *)X.p[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = (blockIdx.x * 4 + w) * 16;
  // a wave past n loads nothing but still takes part in the block's barriers
  const bool live = row0 < n;
  // rows past n (within the columns' padded length) feed only output rows
  // that are not stored
  const int row = row0 + li;
  d4 acc[JT][ndv];
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int c = 0; c < ndv; ++c) acc[t][c] = d4{0.0, 0.0, 0.0, 0.0};
  // batches of up to four 16-column steps: the batch's X loads are issued
  // together (column pointers from LDS, clamped indices), W's rows of the
  // batch are staged in LDS meanwhile, then the MFMAs run in the order of
  // one step after another
#pragma unroll 1
  for (int k0 = 0; k0 < m; k0 += 64) {
    const int ks = min(4, (m - k0 + 15) / 16);
    double xr[4][4], xi[4][4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xr[sp][u] = 0.0;
        xi[sp][u] = 0.0;
        if (live && sp < ks) {
          const int kc = min(k0 + 16 * sp + 4 * u + lk, m - 1);
          const V v = gload(cols[kc], row);
          if constexpr (ndv == 2) {
            xr[sp][u] = ((const cd &)v).x;
            xi[sp][u] = ((const cd &)v).y;
          } else {
            xr[sp][u] = (double)v;
          }
        }
      }
    if (k0 > 0) __syncthreads();  // the previous batch's reads of wl are done
    for (int e = threadIdx.x; e < 64 * 16 * JT; e += 256) {
      const int kk = e / (16 * JT), c = e % (16 * JT);
      const int kcol = k0 + kk;
      const bool in = kcol < m && c < p;
      const cd wv = in ? W[(size_t)c * m + kcol] : cd{0.0, 0.0};
      wl[kk * PC + c] = wv.x;
      if constexpr (ndv == 2) wl[(64 + kk) * PC + c] = wv.y;
    }
    __syncthreads();
    if (live) {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        if (sp < ks) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < JT; ++t) {
              const int e = (16 * sp + 4 * u + lk) * PC + t * 16 + li;
              const double wr = wl[e];
              if constexpr (ndv == 1) {
                acc[t][0] = mfma(wr, xr[sp][u], acc[t][0]);  // real bases take Re W
              } else {
                // (W^T X^T): re = wr xr - wi xi, im = wr xi + wi xr
                const double wi = wl[64 * PC + e];
                acc[t][0] = mfma(wr, xr[sp][u], acc[t][0]);
                acc[t][0] = mfma(-wi, xi[sp][u], acc[t][0]);
                acc[t][1] = mfma(wr, xi[sp][u], acc[t][1]);
                acc[t][1] = mfma(wi, xr[sp][u], acc[t][1]);
              }
            }
        }
      }
    }
  }
  if (!live || row >= n) return;
#pragma unroll
  for (int t = 0; t < JT; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = t * 16 + lk + 4 * v;
      if (c < p) {
        if constexpr (ndv == 2) {
          cd o;
          o.x = acc[t][0][v];
          o.y = acc[t][1][v];
          ((cd *)Y)[(size_t)c * ld + row] = o;
        } else {
          Y[(size_t)c * ld + row] = (V)acc[t][0][v];
        }
      }
    }
  }
}

// Y[:, c] = A X[:, c] for the 8 columns c = 8 blockIdx.y + (0..7) (< m):
// the matrix is read once per 8 columns.
template <class V, class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_spmm8(Sell<M> A, const V *X, V *Y, int ld,
                                                       int m) {
  using T = typename Ar<V>::T;
  const int row = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (row >= A.n) return;
  const int c0 = blockIdx.y * 8;
  const int nc = min(8, m - c0);
  T acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = zero<T>();
  const int slice = row >> 6, lane = row & 63;
  const int beg = A.sliceptr[slice], end = A.sliceptr[slice + 1];
  // eight entries at a time: indices and values first, then per column the
  // eight gathers together, then the products (in entry order per column)
  for (int e0 = beg + lane; e0 < end; e0 += 8 * RBICG_WAVE) {
    int c[8];
    M v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = e0 + t * RBICG_WAVE;
      c[t] = e < end ? A.col[e] : -1;
      v[t] = e < end ? A.val[e] : M{};
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < nc) {
        const V *Xc = X + (size_t)(c0 + j) * ld;
        V xv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) xv[t] = c[t] >= 0 ? Xc[c[t]] : V{};
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (c[t] >= 0) acc[j] += up(v[t]) * up(xv[t]);
      }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < nc) {
      if (A.shifted) acc[j] = shift_apply<M, T>(A, acc[j], up(X[(size_t)(c0 + j) * ld + row]));
      Y[(size_t)(c0 + j) * ld + row] = down<V>(acc[j]);
    }
}

// ========================================================= shifted pairs
// Batched IRKA-style pairs (sigma_s I - A) x_s = b, (sigma_s I - A)^H x~_s = c
// for S shifts sharing one recycle space (Algorithm 3 steps 2-3 with E = I).
// The batch vectors are n x S column-major (leading dimension ld), one column
// per shift.  One iteration of Algorithm 2 for all shifts is five launches:
//   k_sh_state one block per shift: the stopping test of the previous
//              iteration from the k_sh2 partials and beta_s;
//   k_sh1      p_s = r_s + beta_s p_s and z_s = sigma_s p_s - A p_s (dual:
//              conj(beta_s), conj(sigma_s), A^H); one block per (row block,
//              side) for all shifts, the matrix row read once;
//   Gram       [U~, A^H U~, p~_1..p~_S]^H [z_1..z_S] and [U, A U]^H
//              [z~_1..z~_S, p~_1..p~_S] (k_gram_mfma, both in one launch: FP64
//              MFMA contractions of the shared bases against all shifts);
//   k_sh_coef  one block per shift: zeta_s = K_s w_s, y_s = L_s zeta_s (and
//              the dual), sigma_s = (p~_s, q_s) = (p~_s, z_s) - (p~_s^H
//              [U, A U]) y_s, alpha_s and the zeta_c updates;
//   k_sh2      per row q_s = z_s - [U, A U] y_s and q~_s (in registers, never
//              stored), the x, x~, r, r~ updates and the partials of ||r_s||,
//              ||r~_s||, (r~_s, r_s).
// Shifts that have stopped are skipped.  Per-shift scalars are logged per
// iteration in rec[(it * SHMAX + s) * SH_LOG + ...]; k_sh2 writes its
// partials to P3[(s * nb + block) * 4 + i].

// Block s: stopping test of iteration it-1 and beta_{it-1} for shift s of the
// batch (act1, beta for k_sh1); records them in rec and, when the shift
// stops, its status.  Also the final test after the last launched iteration;
// that launch (hs != null) also writes every shift's done flag into the
// host's slot hs (mapped host memory, read after the event behind it).
__global__ __launch_bounds__(RBICG_BLOCK) void k_sh_state(const double *__restrict__ P3, int nb,
                                                          ShScalars *Sh, double *rec, int it,
                                                          int first, ShScalars *hs) {
  __shared__ double tmp[RBICG_BLOCK];
  __shared__ double red[4];
  const int s = blockIdx.x;
  if (Sh->done[s]) {  // only this block writes done[s] in this launch
    if (threadIdx.x == 0) {
      Sh->act1[s] = 0;
      if (hs) hs->done[s] = 1;
    }
    return;
  }
  breduce(P3 + (size_t)s * nb * 4, nb, 4, tmp, red);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(red[0]), rtn = sqrt(red[1]);
  const cd rho = {red[2], red[3]};
  double *Rm1 = rec + ((size_t)(it - 1) * SHMAX + s) * SH_LOG;
  Rm1[4] = rho.x;
  Rm1[5] = rho.y;
  Rm1[6] = rn;
  Rm1[7] = rtn;
  int st = ST_RUNNING;
  if (rn <= Sh->tol * Sh->bn[s] && rtn <= Sh->tol * Sh->btn[s]) st = ST_CONVERGED;
  else if (abs2(rho) == 0.0 || !isfin(rho) || !isfinite(rn) || !isfinite(rtn)) st = ST_BREAKDOWN;
  else if (it > Sh->maxit) st = ST_MAXIT;
  if (st != ST_RUNNING) {
    Sh->status[s] = st;
    Sh->iter[s] = it - 1;
    Sh->done[s] = 1;
    Sh->act1[s] = 0;
    if (hs) hs->done[s] = 1;
    return;
  }
  if (hs) hs->done[s] = 0;
  cd b = {0.0, 0.0};
  if (!first) {
    const double *Rm2 = rec + ((size_t)(it - 2) * SHMAX + s) * SH_LOG;
    b = cdiv(rho, cd{Rm2[4], Rm2[5]});
  }
  double *R0 = rec + ((size_t)it * SHMAX + s) * SH_LOG;
  R0[2] = b.x;
  R0[3] = b.y;
  Sh->beta[2 * s] = b.x;
  Sh->beta[2 * s + 1] = b.y;
  Sh->act1[s] = 1;
}

// Block b of k_sh1 -> (row block, side).  With nrb a multiple of 8 the blocks
// of one XCD (b mod 8) cover one contiguous range of row blocks, both sides.
__device__ __forceinline__ void sh1_block(int b, int nrb, int &rb, int &side) {
  if ((nrb & 7) == 0) {
    const int i = b >> 3;
    rb = (b & 7) * (nrb >> 3) + (i >> 1);
    side = i & 1;
  } else {
    rb = b >> 1;
    side = b & 1;
  }
}

// One row of (sigma I - A) (r + beta p) for two shifts at once from the row's
// column byte offsets co and values v (w <= 8 entries): all gathers of both
// shifts are issued before the sums (entry order, as spmv_dir).
template <class M>
__device__ __forceinline__ void sh1_pair(int w, const unsigned (&co)[8], const M (&v)[8],
                                         const char *ra, const char *pa, const char *rb_,
                                         const char *pb, unsigned roff, cd ba, cd bb, cd sa,
                                         cd sb, cd &pna, cd &za, cd &pnb, cd &zb) {
  cd ga[8], ha[8], gb[8], hb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < w) {
      ga[j] = *(const cd *)(ra + co[j]);
      ha[j] = *(const cd *)(pa + co[j]);
      gb[j] = *(const cd *)(rb_ + co[j]);
      hb[j] = *(const cd *)(pb + co[j]);
    }
  const cd ra0 = *(const cd *)(ra + roff), pa0 = *(const cd *)(pa + roff);
  const cd rb0 = *(const cd *)(rb_ + roff), pb0 = *(const cd *)(pb + roff);
  cd acca = {0.0, 0.0}, accb = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < w) {
      acca += up(v[j]) * (ga[j] + ba * ha[j]);
      accb += up(v[j]) * (gb[j] + bb * hb[j]);
    }
  pna = ra0 + ba * pa0;
  pnb = rb0 + bb * pb0;
  za = sa * pna - acca;
  zb = sb * pnb - accb;
}

template <class M>
__global__ __launch_bounds__(RBICG_BLOCK) void k_sh1(Sell<M> A, Sell<M> AH, int ld,
                                                     const cd *__restrict__ R,
                                                     const cd *__restrict__ Rt,
                                                     const cd *__restrict__ P,
                                                     const cd *__restrict__ Pt, cd *__restrict__ Pn,
                                                     cd *__restrict__ Ptn, cd *__restrict__ Z,
                                                     cd *__restrict__ Zt, const ShScalars *Sh,
                                                     int nrb) {
  __shared__ cd bet[SHMAX], sgs[SHMAX];
  __shared__ int acts[SHMAX];
  if (Sh->all_done) return;
  const int S = Sh->S;
  int rb, side;
  sh1_block(blockIdx.x, nrb, rb, side);
  const bool primal = side == 0;
  if (threadIdx.x < S) {
    const int s = threadIdx.x;
    acts[s] = Sh->act1[s];
    const cd b = {Sh->beta[2 * s], Sh->beta[2 * s + 1]};
    bet[s] = primal ? b : cj(b);
    sgs[s] = cd{Sh->sig[2 * s], primal ? Sh->sig[2 * s + 1] : -Sh->sig[2 * s + 1]};
  }
  __syncthreads();
  const Sell<M> &Am = primal ? A : AH;
  const int row = rb * RBICG_BLOCK + threadIdx.x;
  if (row >= Am.n) return;
  const char *rbase = (const char *)(primal ? R : Rt), *pbase = (const char *)(primal ? P : Pt);
  char *pnbase = (char *)(primal ? Pn : Ptn), *zbase = (char *)(primal ? Z : Zt);
  const size_t colb = (size_t)ld * sizeof(cd);
  // byte offsets of the row and of its columns (ld * 9 * 16 < 2^32)
  const unsigned roff = (unsigned)row * (unsigned)sizeof(cd);
  const int slice = row >> 6, lane = row & 63;
  const int b0 = Am.sliceptr[slice];
  const int w = (Am.sliceptr[slice + 1] - b0) >> 6;
  unsigned co[8];
  M v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    co[j] = 0;
    v[j] = M{};
    if (j < w) {
      co[j] = (unsigned)Am.col[b0 + lane + RBICG_WAVE * j] * (unsigned)sizeof(cd);
      v[j] = Am.val[b0 + lane + RBICG_WAVE * j];
    }
  }
  for (int s0 = 0; s0 < S; s0 += 2) {
    const int sb = min(s0 + 1, S - 1);
    const int aa = __builtin_amdgcn_readfirstlane(acts[s0]);
    const int ab = s0 + 1 < S ? __builtin_amdgcn_readfirstlane(acts[sb]) : 0;
    if (!aa && !ab) continue;
    // an inactive shift of the pair reads the other one's columns (cache
    // hits) and stores nothing
    const int ca = aa ? s0 : sb, cb = ab ? sb : s0;
    const size_t oa = ca * colb, ob = cb * colb;
    cd pna, za, pnb, zb;
    if (w <= 8) {
      sh1_pair<M>(w, co, v, rbase + oa, pbase + oa, rbase + ob, pbase + ob, roff, bet[ca],
                  bet[cb], sgs[ca], sgs[cb], pna, za, pnb, zb);
    } else {
      const cd *ra = (const cd *)(rbase + oa), *pa = (const cd *)(pbase + oa);
      const cd *rbv = (const cd *)(rbase + ob), *pbv = (const cd *)(pbase + ob);
      pna = ra[row] + bet[ca] * pa[row];
      pnb = rbv[row] + bet[cb] * pbv[row];
      za = sgs[ca] * pna - spmv_dir<cd, M, cd>(Am, row, ra, pa, bet[ca]);
      zb = sgs[cb] * pnb - spmv_dir<cd, M, cd>(Am, row, rbv, pbv, bet[cb]);
    }
    if (aa) {
      *(cd *)(pnbase + oa + roff) = pna;
      *(cd *)(zbase + oa + roff) = za;
    }
    if (ab) {
      *(cd *)(pnbase + ob + roff) = pnb;
      *(cd *)(zbase + ob + roff) = zb;
    }
  }
}

// One block per shift s of the batch.  G holds two Grams: G0 (rows of ld0
// entries) = [U~, A^H U~, p~..]^H [z..] (iteration) or [U~, A^H U~]^H [r..]
// (start), and from entry g1 on G1 (rows of ld1 entries) = [U, A U]^H
// [z~.., p~..] or [U, A U]^H [r~..].
//   mode 0 (iteration): zeta = K w, zeta~ = Kt w~ with w = G0[:k2, s],
//     w~ = G1[:, s]; y = L zeta, y~ = Lt zeta~; sigma = G0[k2 + s, s]
//     - sum_j conj(G1[j, S + s]) y_j (= (p~, z) - (p~^H [U, A U]) y);
//     alpha = rho_{it-1} / sigma;
//     zeta_c += alpha zeta, zeta~_c += conj(alpha) zeta~; act/alpha for k_sh2.
//   mode 1 (start): g = K w; Y = L g and
//     Yx = -T g (x += U' g, r -= C' g).
//   mode 2 (finish): Yx = T zeta_c (x -= U zeta_c).
// Y, Yt: k2 x S column-major; Yx, Yxt: (k2/2) x S column-major.
__global__ __launch_bounds__(256) void k_sh_coef(const double *__restrict__ G, int ld0, int g1,
                                                 int ld1, ShScalars *Sh,
                                                 const ShCoef *__restrict__ Co,
                                                 cd *Y, cd *Yt, cd *Yx, cd *Yxt, int mode,
                                                 double *rec, int it) {
  __shared__ cd zs[2][KSH];
  __shared__ cd ys[2 * KSH];
  __shared__ cd alsh;
  __shared__ int flag;
  const int s = blockIdx.x, S = Sh->S, k2 = Sh->k2, k = k2 / 2;
  if (mode == 0) {
    if (threadIdx.x == 0) flag = Sh->done[s];
    __syncthreads();
    if (flag) {
      if (threadIdx.x == 0) Sh->act[s] = 0;
      return;
    }
  }
  const int p = Sh->p[s];
  // zeta (or g, or zeta_c) of both sides
  for (int t = threadIdx.x; t < 2 * KSH; t += blockDim.x) {
    const int side = t / KSH, l = t % KSH;
    cd v = {0.0, 0.0};
    if (l < p) {
      if (mode == 2) {
        const double *zc = side ? Sh->zct[s] : Sh->zc[s];
        v = cd{zc[2 * l], zc[2 * l + 1]};
      } else {
        // 8 terms at a time, their loads issued together (a term-by-term
        // loop waits out one cache round trip per term)
        const double *Km = side ? Co->Kt[s] : Co->K[s];
        for (int j0 = 0; j0 < k2; j0 += 8) {
          cd kv[8], gv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = min(j0 + u, k2 - 1);
            const size_t gi = side ? (size_t)g1 + (size_t)j * ld1 + s : (size_t)j * ld0 + s;
            kv[u] = cd{Km[2 * (l * k2 + j)], Km[2 * (l * k2 + j) + 1]};
            gv[u] = cd{G[2 * gi], G[2 * gi + 1]};
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (j0 + u < k2) v += kv[u] * gv[u];
        }
      }
    }
    zs[side][l] = v;
  }
  __syncthreads();
  if (mode != 2)
    for (int t = threadIdx.x; t < 2 * k2; t += blockDim.x) {
      const int side = t / k2, j = t % k2;
      const double *Lm = side ? Co->Lt[s] : Co->L[s];
      cd v = {0.0, 0.0};
      for (int l = 0; l < p; ++l)
        v += cd{Lm[2 * (j * p + l)], Lm[2 * (j * p + l) + 1]} * zs[side][l];
      (side ? Yt : Y)[(size_t)s * k2 + j] = v;
      if (!side) ys[j] = v;
    }
  if (mode != 0) {
    const double sg = mode == 1 ? -1.0 : 1.0;
    for (int t = threadIdx.x; t < 2 * k; t += blockDim.x) {
      const int side = t / k, i = t % k;
      const double *Tm = side ? Co->Tt[s] : Co->T[s];
      cd v = {0.0, 0.0};
      for (int l = 0; l < p; ++l)
        v += cd{Tm[2 * (i * p + l)], Tm[2 * (i * p + l) + 1]} * zs[side][l];
      (side ? Yxt : Yx)[(size_t)s * k + i] = sg * v;
    }
    return;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    cd c = {0.0, 0.0};
    for (int j = threadIdx.x; j < k2; j += 64) {
      const size_t gi = (size_t)g1 + (size_t)j * ld1 + S + s;
      c += cj(cd{G[2 * gi], G[2 * gi + 1]}) * ys[j];
    }
    c.x = wave_sum(c.x);
    c.y = wave_sum(c.y);
    if (threadIdx.x == 0) {
      const size_t gd = (size_t)(k2 + s) * ld0 + s;
      const cd sigma = {G[2 * gd] - c.x, G[2 * gd + 1] - c.y};
      int a = 0;
      cd al = {0.0, 0.0};
      if (abs2(sigma) == 0.0 || !isfin(sigma)) {
        Sh->status[s] = ST_BREAKDOWN;
        Sh->iter[s] = it - 1;
        Sh->done[s] = 1;
      } else {
        const double *Rm1 = rec + ((size_t)(it - 1) * SHMAX + s) * SH_LOG;
        al = cdiv(cd{Rm1[4], Rm1[5]}, sigma);
        a = 1;
        double *R0 = rec + ((size_t)it * SHMAX + s) * SH_LOG;
        R0[0] = al.x;
        R0[1] = al.y;
      }
      Sh->act[s] = a;
      Sh->alpha[2 * s] = al.x;
      Sh->alpha[2 * s + 1] = al.y;
      flag = a;
      alsh = al;
    }
  }
  __syncthreads();
  if (!flag) return;
  for (int t = threadIdx.x; t < 2 * p; t += blockDim.x) {
    const int side = t / p, l = t % p;
    const cd a = side ? cj(alsh) : alsh;
    double *zc = side ? Sh->zct[s] : Sh->zc[s];
    const cd v = cd{zc[2 * l], zc[2 * l + 1]} + a * zs[side][l];
    zc[2 * l] = v.x;
    zc[2 * l + 1] = v.y;
  }
}

// Out[:, c] = Zin[:, c] - sum_l X_l W[l, c] for c < p <= 16 (W: m x p complex,
// column-major), on FP64 MFMA (Y^T = W^T X^T, one wave per 16 rows, waves
// stride over the row tiles).  Out may alias Zin.  Used at the start and the
// end of a batched solve.
__global__ __launch_bounds__(256) void k_sh_sub(int n, ColList X, int m, const cd *W, int p,
                                                const cd *Zin, cd *Out, int ld) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ntiles = (n + 15) / 16;
  for (int tile = blockIdx.x * 4 + w; tile < ntiles; tile += gridDim.x * 4) {
    const int row = tile * 16 + li;
    d4 ar = d4{0.0, 0.0, 0.0, 0.0}, ai = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < m; k0 += 4) {
      const int kcol = k0 + lk;
      double xr = 0.0, xi = 0.0;
      if (kcol < m && row < n) {
        const cd v = ((const cd *)X.p[kcol])[row];
        xr = v.x;
        xi = v.y;
      }
      const int c = li;
      double wr = 0.0, wi = 0.0;
      if (kcol < m && c < p) {
        const cd wv = W[(size_t)c * m + kcol];
        wr = wv.x;
        wi = wv.y;
      }
      ar = mfma(wr, xr, ar);
      ar = mfma(-wi, xi, ar);
      ai = mfma(wr, xi, ai);
      ai = mfma(wi, xr, ai);
    }
    if (row < n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = lk + 4 * v;
        if (c < p) {
          const size_t o = (size_t)c * ld + row;
          const cd z = Zin[o];
          Out[o] = cd{z.x - ar[v], z.y - ai[v]};
        }
      }
    }
  }
}

// k_sh2 for the NS shifts [s0, s0 + NS) of the batch.  With upd set, per row
// and shift q = z - [U, A U] y and q~ = z~ - [U~, A^H U~] y~ (the bases are
// n x k2 column-major with leading dimension ld at Bb, Btb; each basis row
// is read once for all NS shifts; y, y~ are staged in LDS), then for the
// shifts still active x += alpha p, x~ += conj(alpha) p~, r -= alpha q,
// r~ -= conj(alpha) q~.  Then (also with upd = 0, the start of a solve)
// partials of ||r||^2, ||r~||^2, (r~, r) into P3[(s * gridDim.x + block) * 4
// + i].  Blocks stride over the row blocks of 256 rows, XCD-contiguous.
// Every load is unconditional, so that the compiler keeps them all in flight:
// an inactive shift reads the row of an active one (a cache hit) and its
// results are dropped; basis columns past k2 read column k2 - 1 again and
// meet zero coefficients.
template <int NS>
__global__ __launch_bounds__(RBICG_BLOCK) void k_sh2(
    int n, int ld, int s0, cd *__restrict__ X, cd *__restrict__ Xt, cd *__restrict__ R,
    cd *__restrict__ Rt, const cd *__restrict__ Pn, const cd *__restrict__ Ptn,
    const cd *__restrict__ Z, const cd *__restrict__ Zt, const cd *__restrict__ Bb,
    const cd *__restrict__ Btb, int k2, const cd *__restrict__ Y, const cd *__restrict__ Yt,
    ShScalars *Sh, double *__restrict__ P3, int upd) {
  constexpr int GB = 8;  // basis columns per load group
  __shared__ double lds[(RBICG_BLOCK / 64) * 4 * NS];
  __shared__ cd ysh[2][NS][2 * KSH];
  __shared__ cd als[NS];
  __shared__ int acts[NS];
  const int kpad = (k2 + 2 * GB - 1) / (2 * GB) * (2 * GB);  // <= 2 KSH
  if (threadIdx.x < NS) {
    const int s = s0 + threadIdx.x;
    const int on = upd ? Sh->act[s] : 0;
    acts[threadIdx.x] = on;
    als[threadIdx.x] = on ? cd{Sh->alpha[2 * s], Sh->alpha[2 * s + 1]} : cd{0.0, 0.0};
  }
  if (upd)
    for (int i = threadIdx.x; i < 2 * NS * kpad; i += blockDim.x) {
      const int side = i / (NS * kpad), t = (i / kpad) % NS, j = i % kpad;
      ysh[side][t][j] = j < k2 ? (side ? Yt : Y)[(size_t)(s0 + t) * k2 + j] : cd{0.0, 0.0};
    }
  if (upd && s0 == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    // every shift's state of this iteration is final here
    int all = 1;
    for (int s = 0; s < Sh->S; ++s) all &= Sh->done[s];
    if (all) Sh->all_done = 1;
  }
  __syncthreads();
  // block-uniform flags and 32-bit byte offsets (the host checks
  // (9 ld) * 16 < 2^32): shift t of an array at base + s0 ld + toff[t]
  const unsigned ldb = (unsigned)ld * (unsigned)sizeof(cd);
  int on[NS], tfirst = -1;
  unsigned toff[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    on[t] = __builtin_amdgcn_readfirstlane(acts[t]);
    if (on[t] && tfirst < 0) tfirst = t;
  }
#pragma unroll
  for (int t = 0; t < NS; ++t) toff[t] = (unsigned)(on[t] ? t : (tfirst < 0 ? 0 : tfirst)) * ldb;
  double a[NS][4];
#pragma unroll
  for (int t = 0; t < NS; ++t) a[t][0] = a[t][1] = a[t][2] = a[t][3] = 0.0;
  const int nrb = (n + RBICG_BLOCK - 1) / RBICG_BLOCK, nb = gridDim.x;
  for (int rb = xcd_chunk(blockIdx.x, nb); rb < nrb; rb += nb) {
    const int row = rb * RBICG_BLOCK + threadIdx.x;
    if (row >= n) continue;
    const unsigned boff = (unsigned)row * (unsigned)sizeof(cd);
    cd rn[NS], rtn[NS];
    auto side_pass = [&](const int side, cd(&out)[NS]) {
      char *xb = (char *)((side ? Xt : X) + (size_t)s0 * ld);
      char *rbs = (char *)((side ? Rt : R) + (size_t)s0 * ld);
      if (!upd) {
#pragma unroll
        for (int t = 0; t < NS; ++t) out[t] = *(const cd *)(rbs + boff + (unsigned)t * ldb);
        return;
      }
      if (tfirst < 0) {
#pragma unroll
        for (int t = 0; t < NS; ++t) out[t] = cd{0.0, 0.0};
        return;
      }
      const char *pb = (const char *)((side ? Ptn : Pn) + (size_t)s0 * ld);
      const char *zb = (const char *)((side ? Zt : Z) + (size_t)s0 * ld);
      const cd *bb = side ? Btb : Bb;
      cd q[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) q[t] = *(const cd *)(zb + boff + toff[t]);
      cd b0[GB], b1[GB];
      auto load_group = [&](cd(&g)[GB], int j0) {
#pragma unroll
        for (int u = 0; u < GB; ++u)
          g[u] = *(const cd *)((const char *)(bb + (size_t)min(j0 + u, k2 - 1) * ld) + boff);
      };
      auto use_group = [&](const cd(&g)[GB], int j0) {
#pragma unroll
        for (int u = 0; u < GB; ++u)
#pragma unroll
          for (int t = 0; t < NS; ++t) q[t] -= g[u] * ysh[side][t][j0 + u];
      };
      if (k2 > 0) {
        load_group(b0, 0);
        for (int j0 = 0; j0 < kpad; j0 += 2 * GB) {
          load_group(b1, j0 + GB);
          use_group(b0, j0);
          load_group(b0, j0 + 2 * GB);
          use_group(b1, j0 + GB);
        }
      }
      cd ro[NS], xo[NS], po[NS];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        ro[t] = *(const cd *)(rbs + boff + toff[t]);
        xo[t] = *(const cd *)(xb + boff + toff[t]);
        po[t] = *(const cd *)(pb + boff + toff[t]);
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const cd al = side ? cj(als[t]) : als[t];
        const cd xn = xo[t] + al * po[t], rn_ = ro[t] - al * q[t];
        out[t] = on[t] ? rn_ : cd{0.0, 0.0};
        if (on[t]) {
          *(cd *)(xb + boff + toff[t]) = xn;
          *(cd *)(rbs + boff + toff[t]) = rn_;
        }
      }
    };
    side_pass(0, rn);
    side_pass(1, rtn);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      a[t][0] += abs2(rn[t]);
      a[t][1] += abs2(rtn[t]);
      const cd rho = cj(rtn[t]) * rn[t];
      a[t][2] += rho.x;
      a[t][3] += rho.y;
    }
  }
  // wave sums, 16 values at a time (lane 4i holds value i of its group)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c0 = 0; c0 < 4 * NS; c0 += 16) {
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = c0 + i < 4 * NS ? a[(c0 + i) / 4][(c0 + i) % 4] : 0.0;
    const double sum = wave_sum16(v);
    const int id = c0 + (lane >> 2);
    if ((lane & 3) == 0 && id < 4 * NS) lds[wv * 4 * NS + id] = sum;
  }
  __syncthreads();
  if (threadIdx.x < 4 * NS) {
    double t = 0.0;
    for (int w = 0; w < RBICG_BLOCK / 64; ++w) t += lds[w * 4 * NS + threadIdx.x];
    P3[((size_t)(s0 + threadIdx.x / 4) * nb + blockIdx.x) * 4 + threadIdx.x % 4] = t;
  }
}

// =============================================================== launchers
namespace {
inline unsigned nblk(size_t n) { return (unsigned)((n + RBICG_BLOCK - 1) / RBICG_BLOCK); }
}

bool iter_one_row(int n, int nb) { return (size_t)nb * IB >= (size_t)n; }

int iter_grid_min(int n) { return std::max(1, (n + IB * RMAX - 1) / (IB * RMAX)); }
int iter_grid(int n) {
  const int a = (n + IB - 1) / IB;
  const int b = (n + IB * RMAX - 1) / (IB * RMAX);
  return std::max(1, std::max(std::min(a, 256), b));
}

template <class V, class M>
void launch_it1(hipStream_t st, int nb, const Sell<M> &A, const Sell<M> &AH, const V *r,
                const V *p, const V *rt, const V *pt, V *pn, V *ptn, V *z, V *zt, const V *C,
                const V *Ct, int k, int ld, V *capR, V *capRt, V *capZ, V *capZt,
                const double *P3, double *P1, Scalars *S, double *rec, int it, int first, int rp) {
  // one row per thread when the grid covers the rows, else up to RMAX
  const int ndv = sizeof(V) == 16 ? 2 : 1;
  const int rpv = sizeof(V) == 4 ? rp : 0;
  const size_t lds = (size_t)NW * (3 * k + 1 + (rpv ? 2 * k : 0)) * ndv * sizeof(double);
  if ((size_t)nb * IB >= (size_t)A.n)
    hipLaunchKernelGGL((k_it1<V, M, 1>), dim3(nb), dim3(IB), lds, st, A, AH, r, p, rt, pt, pn, ptn,
                       z, zt, C, Ct, k, ld, capR, capRt, capZ, capZt, P3, P1, S, rec, it, first, rp);
  else
    hipLaunchKernelGGL((k_it1<V, M, RMAX>), dim3(nb), dim3(IB), lds, st, A, AH, r, p, rt, pt, pn,
                       ptn, z, zt, C, Ct, k, ld, capR, capRt, capZ, capZt, P3, P1, S, rec, it, first,
                       rp);
}
template <class V>
void launch_op_dir(hipStream_t st, int nb, int n, const V *r, const V *p, const V *rt, const V *pt,
                   V *pn, V *ptn, V *capR, V *capRt, const double *P3, Scalars *S, double *rec,
                   int it, int first) {
  hipLaunchKernelGGL((k_op_dir<V>), dim3(nb), dim3(IB), 0, st, n, r, p, rt, pt, pn, ptn, capR,
                     capRt, P3, S, rec, it, first);
}
template <class V>
void launch_op_restr(hipStream_t st, int nb, int n, const V *z, const V *zt, const V *ptn,
                     const V *C, const V *Ct, int k, int ld, V *capZ, V *capZt, double *P1,
                     const Scalars *S) {
  const size_t lds = it1_lds_bytes<V>(k, 0);
  hipLaunchKernelGGL((k_op_restr<V>), dim3(nb), dim3(IB), lds, st, n, z, zt, ptn, C, Ct, k, ld,
                     capZ, capZt, P1, S);
}
template <class V, class M>
void launch_spmv(hipStream_t st, const Sell<M> &A, const V *x, V *y, const Scalars *S) {
  hipLaunchKernelGGL((k_spmv<V, M>), dim3(nblk(A.n)), dim3(RBICG_BLOCK), 0, st, A, x, y, S);
}
template <class V, class M>
void launch_sptrsv(hipStream_t st, const TriDev<M> &T0, const V *b0, V *x0, const TriDev<M> *T1,
                   const V *b1, V *x1, int *counter, int waves, const Scalars *S, int *err) {
  const int ns = T1 ? 2 : 1;
  const long chunks = (long)(T0.len >> 6) + (T1 ? (T1->len >> 6) : 0);
  if (chunks == 0) return;
  const int n1 = T1 ? T1->n : 0;
  hipLaunchKernelGGL((k_trsv_pending<V>), dim3(nblk(std::max(T0.n, n1))), dim3(RBICG_BLOCK), 0, st,
                     T0.n, x0, n1, T1 ? x1 : nullptr, counter, S);
  const int w = (int)std::min<long>(chunks, std::max(4, waves));
  const int blocks = (w + 3) / 4;  // four waves per block
  hipLaunchKernelGGL((k_sptrsv<V, M>), dim3(blocks), dim3(RBICG_BLOCK), 0, st, T0, b0, x0,
                     T1 ? *T1 : T0, b1, x1, ns, counter, S, err);
}
template <class V, class M>
void launch_spmv_perm(hipStream_t st, const Sell<M> &A, const V *x, V *y, const int *gmap,
                      const int *orow, const Scalars *S) {
  hipLaunchKernelGGL((k_spmv_perm<V, M>), dim3(nblk(A.n)), dim3(RBICG_BLOCK), 0, st, A, x, y, gmap,
                     orow, S);
}
template <class V>
void launch_gather(hipStream_t st, int n, const V *in, const int *map, V *out) {
  if (n > 0) hipLaunchKernelGGL((k_gather<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, in, map, out);
}
template <class V>
void launch_rsub(hipStream_t st, int n, const V *b, const V *t, V *out) {
  hipLaunchKernelGGL((k_rsub<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, b, t, out);
}
template <class V>
size_t it1_lds_bytes(int k, int rp) {
  const int ndv = sizeof(V) == 16 ? 2 : 1;
  const int rpv = sizeof(V) == 4 ? rp : 0;
  return (size_t)NW * (3 * k + 1 + (rpv ? 2 * k : 0)) * ndv * sizeof(double);
}
template <class V, class M>
void launch_it1_multi(hipStream_t st, const It1Args<V, M> *dtab, int nslot, int nblocks,
                      size_t lds_bytes, bool rpt1) {
  if (rpt1)
    hipLaunchKernelGGL((k_it1_multi<V, M, 1>), dim3(nblocks), dim3(IB), lds_bytes, st, dtab, nslot);
  else
    hipLaunchKernelGGL((k_it1_multi<V, M, RMAX>), dim3(nblocks), dim3(IB), lds_bytes, st, dtab,
                       nslot);
}
template <class V>
void launch_it2_multi(hipStream_t st, const It2Args<V> *dtab, int nslot, int nblocks) {
  hipLaunchKernelGGL((k_it2_multi<V>), dim3(nblocks), dim3(IB), 0, st, dtab, nslot);
}
template <class V>
void launch_itfin_multi(hipStream_t st, const ItfinArgs *dtab, int nslot) {
  hipLaunchKernelGGL((k_itfin_multi<V>), dim3(nslot), dim3(IB), 0, st, dtab);
}

// The same launches as kernel nodes of a HIP graph, each after `last`
// (nullptr: a root), which then becomes the new node.
namespace {
hipError_t add_node(hipGraph_t g, hipGraphNode_t &last, void *fn, dim3 grid, size_t lds,
                    void **args) {
  hipKernelNodeParams p{};
  p.func = fn;
  p.gridDim = grid;
  p.blockDim = dim3(IB);
  p.sharedMemBytes = (unsigned)lds;
  p.kernelParams = args;
  p.extra = nullptr;
  hipGraphNode_t node = nullptr;
  const hipError_t e = hipGraphAddKernelNode(&node, g, last ? &last : nullptr, last ? 1 : 0, &p);
  if (e == hipSuccess) last = node;
  return e;
}
}  // namespace
template <class V, class M>
hipError_t graph_it1_multi(hipGraph_t g, hipGraphNode_t &last, const It1Args<V, M> *dtab, int nslot,
                           int nblocks, size_t lds_bytes, bool rpt1) {
  void *args[] = {(void *)&dtab, (void *)&nslot};
  void *fn = rpt1 ? reinterpret_cast<void *>(&k_it1_multi<V, M, 1>)
                  : reinterpret_cast<void *>(&k_it1_multi<V, M, RMAX>);
  return add_node(g, last, fn, dim3(nblocks), lds_bytes, args);
}
template <class V>
hipError_t graph_it2_multi(hipGraph_t g, hipGraphNode_t &last, const It2Args<V> *dtab, int nslot,
                           int nblocks) {
  void *args[] = {(void *)&dtab, (void *)&nslot};
  return add_node(g, last, reinterpret_cast<void *>(&k_it2_multi<V>), dim3(nblocks), 0, args);
}
template <class V>
hipError_t graph_itfin_multi(hipGraph_t g, hipGraphNode_t &last, const ItfinArgs *dtab, int nslot) {
  void *args[] = {(void *)&dtab};
  return add_node(g, last, reinterpret_cast<void *>(&k_itfin_multi<V>), dim3(nslot), 0, args);
}
template <class V>
void launch_it2(hipStream_t st, int nb, int n, V *x, V *xt, V *r, V *rt, const V *pn,
                const V *ptn, const V *z, const V *zt, const V *C, const V *Ct, int k, int ld,
                const double *P1, double *P3, Scalars *S, double *rec, int it, int rp,
                double *zlog, int zstride) {
  hipLaunchKernelGGL((k_it2<V>), dim3(nb), dim3(IB), 0, st, n, x, xt, r, rt, pn, ptn, z, zt, C,
                     Ct, k, ld, P1, P3, S, rec, it, rp, zlog, zstride);
}
template <class V>
void launch_itfin(hipStream_t st, int nb, const double *P3, Scalars *S, double *rec, int it,
                  int first, Scalars *hs) {
  hipLaunchKernelGGL((k_itfin<V>), dim3(1), dim3(IB), 0, st, P3, nb, S, rec, it, first, hs);
}
template <class V>
void launch_init_p3(hipStream_t st, int nb, int n, const V *r, const V *rt, double *P3) {
  hipLaunchKernelGGL((k_init_p3<V>), dim3(nb), dim3(IB), 0, st, n, r, rt, P3);
}
template <class V>
void launch_dots(hipStream_t st, int nb, int n, const V *a0, const V *b0, const V *a1,
                 const V *b1, const V *a2, const V *b2, double *P, double *out) {
  hipLaunchKernelGGL((k_dots<V>), dim3(nb), dim3(IB), 0, st, n, a0, b0, a1, b1, a2, b2, P);
  hipLaunchKernelGGL(k_fin_red, dim3(1), dim3(IB), 0, st, P, nb, sizeof(V) == 16 ? 6 : 3, out);
}
template <class V>
void launch_restrict(hipStream_t st, int nb, int n, const V *u, const V *B, const V *u2,
                     const V *B2, int k, int ld, double *P, double *out) {
  hipLaunchKernelGGL((k_restrict<V>), dim3(nb), dim3(IB), 0, st, n, u, B, u2, B2, k, ld, P);
  const int nv = 2 * k * (sizeof(V) == 16 ? 2 : 1);
  hipLaunchKernelGGL(k_fin_red, dim3(1), dim3(IB), 0, st, P, nb, nv, out);
}
void launch_fin_red(hipStream_t st, const double *P, int nb, int nv, double *out) {
  hipLaunchKernelGGL(k_fin_red, dim3(1), dim3(IB), 0, st, P, nb, nv, out);
}
template <class V, class M>
void launch_residual(hipStream_t st, const Sell<M> &A, const V *b, const V *x, V *out) {
  hipLaunchKernelGGL((k_residual<V, M>), dim3(nblk(A.n)), dim3(RBICG_BLOCK), 0, st, A, b, x,
                     out);
}
template <class V, class M>
void launch_spmm(hipStream_t st, const Sell<M> &A, const V *X, V *Y, int ld, int m) {
  if (m <= 0) return;
  hipLaunchKernelGGL((k_spmm8<V, M>), dim3(nblk(A.n), (m + 7) / 8), dim3(RBICG_BLOCK), 0, st, A,
                     X, Y, ld, m);
}
template <class V>
void launch_expand2(hipStream_t st, int n, V *x, const V *U, double sx, V *r, const V *C,
                    double sr, V *xt, const V *Ut, double sxt, V *rt, const V *Ct, double srt,
                    int k, int ld, const double *coef) {
  hipLaunchKernelGGL((k_expand2<V>), dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, n, x, U, sx, r,
                     C, sr, xt, Ut, sxt, rt, Ct, srt, k, ld, coef);
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
void launch_d2f(hipStream_t st, const double *in, float *out, size_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_d2f, dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, in, out, n);
}
void launch_add_f2d(hipStream_t st, double *x, const float *d, double sgn, size_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_add_to_d<float>, dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, x, d, sgn, n);
}
void launch_add_d2d(hipStream_t st, double *x, const double *d, double sgn, size_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_add_to_d<double>, dim3(nblk(n)), dim3(RBICG_BLOCK), 0, st, x, d, sgn, n);
}
// two chunks per CU at full size (the per-block slab loop is latency-bound)
// Row chunks of a Gram: at least 128 rows each, at most 512 chunks (two per
// CU), so that a short basis still gives every CU a block.
int gram_chunks(int n) { return std::max(1, std::min(512, (n + 127) / 128)); }

int gram_group(int mx, int complex_vals) {
  const int TX = (mx + 15) / 16;
  int g = std::min(128, (4 * GRAM_MAXT / TX) * 16);
  // the short-slab variant holds up to 282 (real) / 266 (complex) columns
  const int mxp = TX * 16;
  const int lim = (complex_vals ? 266 : 282) / 16 * 16;
  g = std::min(g, lim - mxp);
  return std::max(16, g);
}

template <class V>
void launch_gram2(hipStream_t st, int n, const ColList &X, int mx, const ColList &Y, int my, int x1,
                  int mx1, int y1, int my1, double *partial, double *G, int nchunks) {
  constexpr int ndv = sizeof(V) == 16 ? 2 : 1;
  const int two = mx1 > 0 && my1 > 0;
  const int rpc = (int)(((size_t)n + nchunks - 1) / nchunks);
  const int mxp = (std::max(mx, two ? mx1 : 0) + 15) / 16 * 16;
  const int myp = (std::max(my, two ? my1 : 0) + 15) / 16 * 16;
  bool same = !two && mx == my;
  for (int c = 0; same && c < mx; ++c) same = X.p[c] == Y.p[c];
  const int ncol = same ? mxp : mxp + myp;
  // Slabs of 64 rows, else 32, else 16: the widest whose columns fit 18
  // prefetch slots per thread and whose two LDS buffers leave room for a
  // second block on the CU (a block waits out one slab load at a time, so
  // wider slabs mean fewer round trips; the rows still enter every
  // accumulator in the same order, so the sums do not change).
  auto fits = [&](int r) {
    return (size_t)ncol * r <= 18 * GRAM_BLOCK &&
           2 * (size_t)ncol * (r + 2) * ndv * sizeof(double) <= GRAM_LDS_BYTES / 2;
  };
  const bool wide = fits(64);
  const bool big = fits(32);
  const int sr = wide ? 64 : big ? 32 : 16;
  const size_t lds = 2 * (size_t)ncol * (sr + 2) * ndv * sizeof(double);
  const dim3 grid(nchunks, two ? 2 : 1);
  // at most one 16 x 16 output tile per wave (skinny products): a variant
  // with one accumulator tile and 16-row slabs, small enough in registers
  // and LDS for several blocks per CU
  const int tiles = (mxp / 16) * (myp / 16);
  if (tiles <= 4 && ncol * 16 <= 8 * GRAM_BLOCK) {
    const size_t lds1 = 2 * (size_t)ncol * (16 + 2) * ndv * sizeof(double);
    hipLaunchKernelGGL((k_gram_mfma<V, 16, 8, 1>), grid, dim3(GRAM_BLOCK), lds1, st, n, X, mx, Y,
                       my, rpc, partial, same ? 1 : 0, x1, mx1, y1, my1);
  } else if (wide) {
    hipLaunchKernelGGL((k_gram_mfma<V, 64, 18, GRAM_MAXT>), grid, dim3(GRAM_BLOCK), lds, st, n, X,
                       mx, Y, my, rpc, partial, same ? 1 : 0, x1, mx1, y1, my1);
  } else if (big) {
    hipLaunchKernelGGL((k_gram_mfma<V, 32, 18, GRAM_MAXT>), grid, dim3(GRAM_BLOCK), lds, st, n, X,
                       mx, Y, my, rpc, partial, same ? 1 : 0, x1, mx1, y1, my1);
  } else {
    hipLaunchKernelGGL((k_gram_mfma<V, 16, 18, GRAM_MAXT>), grid, dim3(GRAM_BLOCK), lds, st, n, X,
                       mx, Y, my, rpc, partial, same ? 1 : 0, x1, mx1, y1, my1);
  }
  const int count = ndv * (mx * my + (two ? mx1 * my1 : 0));
  // few entries: 32 lanes per entry, so that the reduction still spreads
  // over the chip
  if (count < 8192)
    hipLaunchKernelGGL(k_gram_reduce<32>, dim3((count + 7) / 8), dim3(256), 0, st, partial, nchunks,
                       count, G, ndv == 1 ? 1 : 0);
  else
    hipLaunchKernelGGL(k_gram_reduce<8>, dim3((count + 31) / 32), dim3(256), 0, st, partial,
                       nchunks, count, G, ndv == 1 ? 1 : 0);
}
template <class V>
void launch_gram(hipStream_t st, int n, const ColList &X, int mx, const ColList &Y, int my,
                 double *partial, double *G, int nchunks) {
  launch_gram2<V>(st, n, X, mx, Y, my, 0, 0, 0, 0, partial, G, nchunks);
}
template <class V>
void launch_tsgemm(hipStream_t st, int n, const ColList &X, int m, const cd *W, int p, V *Y,
                   int ld) {
  if (p <= 0) return;
  const unsigned nb = (unsigned)((n + 63) / 64);
  const int jt = (p + 15) / 16;  // p <= KMAXD = 64
  // W's rows of one batch of 64 input columns in LDS (Re, and Im for complex
  // bases): at most 2 x 64 x 66 doubles
  const size_t lds = (sizeof(V) == 16 ? 2 : 1) * 64 * (size_t)TS_PC(jt) * sizeof(double);
  if (jt == 1)
    hipLaunchKernelGGL((k_tsgemm_mfma<V, 1>), dim3(nb), dim3(256), lds, st, n, X, m, W, p, Y, ld);
  else if (jt == 2)
    hipLaunchKernelGGL((k_tsgemm_mfma<V, 2>), dim3(nb), dim3(256), lds, st, n, X, m, W, p, Y, ld);
  else if (jt == 3)
    hipLaunchKernelGGL((k_tsgemm_mfma<V, 3>), dim3(nb), dim3(256), lds, st, n, X, m, W, p, Y, ld);
  else
    hipLaunchKernelGGL((k_tsgemm_mfma<V, 4>), dim3(nb), dim3(256), lds, st, n, X, m, W, p, Y, ld);
}

void launch_pencil(hipStream_t st, size_t m, const void *a, int acplx, const void *e, int ecplx,
                   cd alpha, cd beta, cd *out) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_pencil, dim3((unsigned)nblk(m)), dim3(RBICG_BLOCK), 0, st, m, a, acplx, e,
                     ecplx, alpha, beta, out);
}

// ------------------------------------------------------- shifted launchers
int sh_blocks(int n) { return std::max(1, std::min(1024, (int)nblk((size_t)n))); }
int sh_sub_blocks(int n) { return std::max(1, std::min(256, ((n + 15) / 16 + 3) / 4)); }

void launch_sh_state(hipStream_t st, int S, const double *P3, int nb3, ShScalars *Sh, double *rec,
                     int it, int first, ShScalars *hs) {
  hipLaunchKernelGGL(k_sh_state, dim3(S), dim3(RBICG_BLOCK), 0, st, P3, nb3, Sh, rec, it, first,
                     hs);
}
template <class M>
void launch_sh1(hipStream_t st, const Sell<M> &A, const Sell<M> &AH, int ld, const cd *R,
                const cd *Rt, const cd *P, const cd *Pt, cd *Pn, cd *Ptn, cd *Z, cd *Zt,
                const ShScalars *Sh) {
  const int nrb = std::max(1, (int)nblk((size_t)A.n));
  hipLaunchKernelGGL((k_sh1<M>), dim3((unsigned)nrb * 2), dim3(RBICG_BLOCK), 0, st, A, AH, ld, R,
                     Rt, P, Pt, Pn, Ptn, Z, Zt, Sh, nrb);
}
void launch_sh_coef(hipStream_t st, int S, const double *G, int ld0, int g1, int ld1,
                    ShScalars *Sh, const ShCoef *Co, cd *Y, cd *Yt, cd *Yx, cd *Yxt, int mode,
                    double *rec, int it) {
  hipLaunchKernelGGL(k_sh_coef, dim3(S), dim3(256), 0, st, G, ld0, g1, ld1, Sh, Co, Y, Yt, Yx, Yxt,
                     mode, rec, it);
}
void launch_sh_sub(hipStream_t st, int n, const ColList &X, int m, const cd *W, int p,
                   const cd *Zin, cd *Out, int ld, int nbe) {
  hipLaunchKernelGGL(k_sh_sub, dim3(nbe), dim3(256), 0, st, n, X, m, W, p, Zin, Out, ld);
}
void launch_sh2(hipStream_t st, int n, int ld, int S, cd *X, cd *Xt, cd *R, cd *Rt, const cd *Pn,
                const cd *Ptn, const cd *Z, const cd *Zt, const cd *B, const cd *Bt, int k2,
                const cd *Y, const cd *Yt, ShScalars *Sh, double *P3, int nb, int upd) {
  for (int s0 = 0; s0 < S; s0 += 8) {
#define SH2(NS)                                                                               \
  case NS:                                                                                    \
    hipLaunchKernelGGL((k_sh2<NS>), dim3(nb), dim3(RBICG_BLOCK), 0, st, n, ld, s0, X, Xt, R, Rt, \
                       Pn, Ptn, Z, Zt, B, Bt, k2, Y, Yt, Sh, P3, upd);                         \
    break;
    switch (std::min(8, S - s0)) {
      SH2(1) SH2(2) SH2(3) SH2(4) SH2(5) SH2(6) SH2(7) SH2(8)
    }
#undef SH2
  }
}
template void launch_sh1<double>(hipStream_t, const Sell<double> &, const Sell<double> &, int,
                                 const cd *, const cd *, const cd *, const cd *, cd *, cd *,
                                 cd *, cd *, const ShScalars *);
template void launch_sh1<cd>(hipStream_t, const Sell<cd> &, const Sell<cd> &, int, const cd *,
                             const cd *, const cd *, const cd *, cd *, cd *, cd *, cd *,
                             const ShScalars *);

#define INST_VM(V, M)                                                                        \
  template void launch_it1<V, M>(hipStream_t, int, const Sell<M> &, const Sell<M> &,         \
                                 const V *, const V *, const V *, const V *, V *, V *, V *,  \
                                 V *, const V *, const V *, int, int, V *, V *, V *, V *,    \
                                 const double *, double *, Scalars *, double *, int, int,    \
                                 int);                                                       \
  template void launch_residual<V, M>(hipStream_t, const Sell<M> &, const V *, const V *,    \
                                      V *);                                                  \
  template void launch_spmm<V, M>(hipStream_t, const Sell<M> &, const V *, V *, int, int);      \
  template void launch_it1_multi<V, M>(hipStream_t, const It1Args<V, M> *, int, int, size_t, \
                                       bool);                                                 \
  template hipError_t graph_it1_multi<V, M>(hipGraph_t, hipGraphNode_t &, const It1Args<V, M> *, \
                                            int, int, size_t, bool);                          \
  template void launch_spmv<V, M>(hipStream_t, const Sell<M> &, const V *, V *,              \
                                  const Scalars *);                                           \
  template void launch_spmv_perm<V, M>(hipStream_t, const Sell<M> &, const V *, V *,         \
                                       const int *, const int *, const Scalars *);

#define INST_V(V)                                                                            \
  template size_t it1_lds_bytes<V>(int, int);                                                \
  template void launch_op_dir<V>(hipStream_t, int, int, const V *, const V *, const V *,     \
                                 const V *, V *, V *, V *, V *, const double *, Scalars *,   \
                                 double *, int, int);                                         \
  template void launch_op_restr<V>(hipStream_t, int, int, const V *, const V *, const V *,   \
                                   const V *, const V *, int, int, V *, V *, double *,       \
                                   const Scalars *);                                          \
  template void launch_rsub<V>(hipStream_t, int, const V *, const V *, V *);                 \
  template void launch_gather<V>(hipStream_t, int, const V *, const int *, V *);             \
  template void launch_it2_multi<V>(hipStream_t, const It2Args<V> *, int, int);              \
  template void launch_itfin_multi<V>(hipStream_t, const ItfinArgs *, int);                  \
  template hipError_t graph_it2_multi<V>(hipGraph_t, hipGraphNode_t &, const It2Args<V> *, int, \
                                         int);                                                 \
  template hipError_t graph_itfin_multi<V>(hipGraph_t, hipGraphNode_t &, const ItfinArgs *, int); \
  template void launch_it2<V>(hipStream_t, int, int, V *, V *, V *, V *, const V *,          \
                              const V *, const V *, const V *, const V *, const V *, int, int, \
                              const double *, double *, Scalars *, double *, int, int,       \
                              double *, int);                                                \
  template void launch_itfin<V>(hipStream_t, int, const double *, Scalars *, double *, int,  \
                                int, Scalars *);                                             \
  template void launch_init_p3<V>(hipStream_t, int, int, const V *, const V *, double *);    \
  template void launch_dots<V>(hipStream_t, int, int, const V *, const V *, const V *,       \
                               const V *, const V *, const V *, double *, double *);         \
  template void launch_restrict<V>(hipStream_t, int, int, const V *, const V *, const V *,   \
                                   const V *, int, int, double *, double *);                 \
  template void launch_expand2<V>(hipStream_t, int, V *, const V *, double, V *, const V *,  \
                                  double, V *, const V *, double, V *, const V *, double,    \
                                  int, int, const double *);                                 \
  template void launch_fill_zero<V>(hipStream_t, V *, size_t);                               \
  template void launch_reseed<V>(hipStream_t, V *, size_t, unsigned long long);              \
  template void launch_gram2<V>(hipStream_t, int, const ColList &, int, const ColList &, int,  \
                                int, int, int, int, double *, double *, int);                \
  template void launch_gram<V>(hipStream_t, int, const ColList &, int, const ColList &, int, \
                               double *, double *, int);                                     \
  template void launch_tsgemm<V>(hipStream_t, int, const ColList &, int, const cd *, int, V *, \
                                 int);

INST_VM(double, double)
INST_VM(cd, double)
INST_VM(cd, cd)
INST_VM(float, float)
// triangular solves: FP64 words only (real and complex vectors)
template void launch_sptrsv<double, double>(hipStream_t, const TriDev<double> &, const double *,
                                            double *, const TriDev<double> *, const double *,
                                            double *, int *, int, const Scalars *, int *);
template void launch_sptrsv<cd, double>(hipStream_t, const TriDev<double> &, const cd *, cd *,
                                        const TriDev<double> *, const cd *, cd *, int *, int,
                                        const Scalars *, int *);
template void launch_sptrsv<cd, cd>(hipStream_t, const TriDev<cd> &, const cd *, cd *,
                                    const TriDev<cd> *, const cd *, cd *, int *, int,
                                    const Scalars *, int *);
INST_V(double)
INST_V(cd)
INST_V(float)
