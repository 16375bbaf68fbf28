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
// run once per solve.  For a new matrix on the same pattern the values of
// A^H, the diagonal, the black pivots and the Schur block are recomputed on
// the device (k_rbr_*), so that a sequence needs one host set-up.
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

// ---- device refresh for new values of A on the same pattern ----
// (the sums run in the order of the host set-up: the diagonal first, then
// the red neighbours k of i in row order, each term (a_ik / d_k) a_kj)

template <class V>
__device__ __forceinline__ V rb_entry(const int *__restrict__ rp, const int *__restrict__ ci,
                                      const V *__restrict__ av, int k, int j) {
  V v = zerov<V>();
  for (int e = rp[k]; e < rp[k + 1]; ++e)
    if (ci[e] == j) v = addv(v, av[e]);
  return v;
}

// A^H values and the diagonal
template <class V>
__global__ void k_rbr_prep(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const V *__restrict__ av, const int *__restrict__ amap,
                           V *__restrict__ hv, V *__restrict__ d) {
  const int i = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (i >= n) return;
  V s = zerov<V>();
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    hv[amap[e]] = conjv(av[e]);
    if (ci[e] == i) s = addv(s, av[e]);
  }
  d[i] = s;
}

// black pivots S_B = d_i - sum_k (a_ik / d_k) a_ki
template <class V>
__global__ void k_rbr_pivot(int nb, const int *__restrict__ blist, const int *__restrict__ rp,
                            const int *__restrict__ ci, const V *__restrict__ av,
                            const V *__restrict__ d, V *__restrict__ sb) {
  const int bi = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (bi >= nb) return;
  const int i = blist[bi];
  V s = d[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int k = ci[e];
    if (k == i) continue;
    s = subv(s, mulv(divv(av[e], d[k]), rb_entry(rp, ci, av, k, i)));
  }
  sb[bi] = s;
}

// M_B entries (d_i delta_ij - sum_k (a_ik / d_k) a_kj) / S_B[j] into the
// sliced-ELL values of M_B and (conjugated) of M_B^H
template <class V>
__global__ void k_rbr_schur(int nb, const int *__restrict__ blist, const int *__restrict__ mrp,
                            const int *__restrict__ mci, const int *__restrict__ rp,
                            const int *__restrict__ ci, const V *__restrict__ av,
                            const V *__restrict__ d, const V *__restrict__ sb,
                            const int *__restrict__ msell, const int *__restrict__ mhsell,
                            V *__restrict__ mval, V *__restrict__ mhval) {
  const int bi = blockIdx.x * RBICG_BLOCK + threadIdx.x;
  if (bi >= nb) return;
  const int i = blist[bi];
  for (int e = mrp[bi]; e < mrp[bi + 1]; ++e) {
    const int bj = mci[e], j = blist[bj];
    V v = bj == bi ? d[i] : zerov<V>();
    for (int g = rp[i]; g < rp[i + 1]; ++g) {
      const int k = ci[g];
      if (k == i) continue;
      v = subv(v, mulv(divv(av[g], d[k]), rb_entry(rp, ci, av, k, j)));
    }
    v = divv(v, sb[bj]);
    mval[msell[e]] = v;
    mhval[mhsell[e]] = conjv(v);
  }
}

namespace {
inline unsigned rb_blocks(int n) { return (unsigned)((n + RBICG_BLOCK - 1) / RBICG_BLOCK); }
}

template <class V>
void launch_rb_refresh(hipStream_t st, const RbDev &P, const RbRefresh &R) {
  V *hv = (V *)const_cast<void *>(P.hv), *d = (V *)const_cast<void *>(P.d);
  V *sb = (V *)const_cast<void *>(P.sb);
  const V *av = (const V *)P.av;
  hipLaunchKernelGGL((k_rbr_prep<V>), dim3(rb_blocks(P.n)), dim3(RBICG_BLOCK), 0, st, P.n, P.rp,
                     P.ci, av, R.amap, hv, d);
  hipLaunchKernelGGL((k_rbr_pivot<V>), dim3(rb_blocks(P.nb)), dim3(RBICG_BLOCK), 0, st, P.nb,
                     R.blist, P.rp, P.ci, av, (const V *)d, sb);
  hipLaunchKernelGGL((k_rbr_schur<V>), dim3(rb_blocks(P.nb)), dim3(RBICG_BLOCK), 0, st, P.nb,
                     R.blist, R.mrp, R.mci, P.rp, P.ci, av, (const V *)d, (const V *)sb, R.msell,
                     R.mhsell, (V *)R.mval, (V *)R.mhval);
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
template void launch_rb_refresh<double>(hipStream_t, const RbDev &, const RbRefresh &);
template void launch_rb_refresh<cd>(hipStream_t, const RbDev &, const RbRefresh &);
