// Split ILU(0) preconditioning in red-black ordering: the transforms of the
// right-hand sides and of the solutions between a dual pair A x = b,
// A^H x~ = b~ and the black block of its split-preconditioned form.
//
// With the unknowns coloured red/black so that every off-diagonal entry of A
// joins two colours, d = diag(A) and S_B the ILU(0) pivots of the black
// unknowns (d_i - sum_k a_ik a_ki / d_k), the split-preconditioned pair is
// block diagonal with an identity red block (Sec. 6 preconditions every
// system this way, with ILUT); the transforms are
//   b^_B[i]  = b_i - sum_k a_ik b_k / d_k                      (i black, k red)
//   c^_R[k]  = b~_k / conj(d_k),  c^_B[i] = (b~_i - sum_k (A^H)_ik c^_R[k]) / conj(S_B[i])
//   x_B[i]   = y_B[i] / S_B[i],   x_R[k] = (b_k - sum_j a_kj x_B[j]) / d_k
//   x~_B[i]  = y~_B[i],           x~_R[k] = c^_R[k] - sum_j (A^H)_kj x~_B[j] / conj(d_k)
// Each is one pass over CSR rows of A or A^H, one thread per unknown; they
// run once per solve.
#include "kernels.h"

namespace {
__device__ __forceinline__ double conjv(double a) { return a; }
__device__ __forceinline__ cd conjv(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ double mulv(double a, double b) { return a * b; }
__device__ __forceinline__ cd mulv(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ double subv(double a, double b) { return a - b; }
__device__ __forceinline__ cd subv(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double addv(double a, double b) { return a + b; }
__device__ __forceinline__ cd addv(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double divv(double a, double b) { return a / b; }
__device__ __forceinline__ cd divv(cd a, cd b) {
  const double s = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / s, (a.y * b.x - a.x * b.y) / s};
}
template <class V> __device__ __forceinline__ V zerov() { return V{}; }
}  // namespace

// b^_B (black rows) and c^_R (red rows, full-length scratch cR)
template <class V>
__global__ void k_rb_rhs1(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                          const V *__restrict__ av, const V *__restrict__ d,
                          const int *__restrict__ bidx, const V *__restrict__ b,
                          const V *__restrict__ bt, V *__restrict__ bB, V *__restrict__ cR) {
  const int i = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int bi = bidx[i];
  if (bi < 0) {
    cR[i] = divv(bt[i], conjv(d[i]));
    return;
  }
  V s = b[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int k = ci[e];
    if (k != i) s = subv(s, mulv(av[e], divv(b[k], d[k])));
  }
  bB[bi] = s;
}

// c^_B (black rows) from c^_R and the rows of A^H
template <class V>
__global__ void k_rb_rhs2(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                          const V *__restrict__ hv, const int *__restrict__ bidx,
                          const V *__restrict__ sb, const V *__restrict__ bt,
                          const V *__restrict__ cR, V *__restrict__ cB) {
  const int i = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int bi = bidx[i];
  if (bi < 0) return;
  V s = bt[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int k = ci[e];
    if (k != i) s = subv(s, mulv(hv[e], cR[k]));
  }
  cB[bi] = divv(s, conjv(sb[bi]));
}

// black unknowns of x and x~
template <class V>
__global__ void k_rb_sol1(int n, const int *__restrict__ bidx, const V *__restrict__ sb,
                          const V *__restrict__ yB, const V *__restrict__ ytB, V *__restrict__ x,
                          V *__restrict__ xt) {
  const int i = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int bi = bidx[i];
  if (bi < 0) return;
  x[i] = divv(yB[bi], sb[bi]);
  xt[i] = ytB[bi];
}

// red unknowns of x and x~ from the black ones
template <class V>
__global__ void k_rb_sol2(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                          const V *__restrict__ av, const int *__restrict__ hrp,
                          const int *__restrict__ hci, const V *__restrict__ hv,
                          const V *__restrict__ d, const int *__restrict__ bidx,
                          const V *__restrict__ b, const V *__restrict__ bt, V *__restrict__ x,
                          V *__restrict__ xt) {
  const int k = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (k >= n || bidx[k] >= 0) return;
  V s = b[k], t = zerov<V>();
  for (int e = rp[k]; e < rp[k + 1]; ++e) {
    const int j = ci[e];
    if (j != k) s = subv(s, mulv(av[e], x[j]));
  }
  for (int e = hrp[k]; e < hrp[k + 1]; ++e) {
    const int j = hci[e];
    if (j != k) t = addv(t, mulv(hv[e], xt[j]));
  }
  const V dc = conjv(d[k]);
  x[k] = divv(s, d[k]);
  xt[k] = divv(subv(bt[k], t), dc);
}

namespace {
inline unsigned rb_blocks(int n) { return (unsigned)((n + RBICG_BLOCK - 1) / RBICG_BLOCK); }
}

template <class V>
void launch_rb_rhs(hipStream_t st, const RbDev &P, const V *b, const V *bt, V *bB, V *cB, V *cR) {
  hipLaunchKernelGGL((k_rb_rhs1<V>), dim3(rb_blocks(P.n)), dim3(RBICG_BLOCK), 0, st, P.n, P.rp,
                     P.ci, (const V *)P.av, (const V *)P.d, P.bidx, b, bt, bB, cR);
  hipLaunchKernelGGL((k_rb_rhs2<V>), dim3(rb_blocks(P.n)), dim3(RBICG_BLOCK), 0, st, P.n, P.hrp,
                     P.hci, (const V *)P.hv, P.bidx, (const V *)P.sb, bt, (const V *)cR, cB);
}

template <class V>
void launch_rb_solution(hipStream_t st, const RbDev &P, const V *b, const V *bt, const V *yB,
                        const V *ytB, V *x, V *xt) {
  hipLaunchKernelGGL((k_rb_sol1<V>), dim3(rb_blocks(P.n)), dim3(RBICG_BLOCK), 0, st, P.n, P.bidx,
                     (const V *)P.sb, yB, ytB, x, xt);
  hipLaunchKernelGGL((k_rb_sol2<V>), dim3(rb_blocks(P.n)), dim3(RBICG_BLOCK), 0, st, P.n, P.rp,
                     P.ci, (const V *)P.av, P.hrp, P.hci, (const V *)P.hv, (const V *)P.d, P.bidx,
                     b, bt, x, xt);
}

template void launch_rb_rhs<double>(hipStream_t, const RbDev &, const double *, const double *,
                                    double *, double *, double *);
template void launch_rb_rhs<cd>(hipStream_t, const RbDev &, const cd *, const cd *, cd *, cd *,
                                cd *);
template void launch_rb_solution<double>(hipStream_t, const RbDev &, const double *,
                                         const double *, const double *, const double *, double *,
                                         double *);
template void launch_rb_solution<cd>(hipStream_t, const RbDev &, const cd *, const cd *,
                                     const cd *, const cd *, cd *, cd *);
