// Host-side launchers of the RBiCG kernels (definitions in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"

#define RBICG_MAXCOLS 160

// Column pointer list passed by value as a kernel argument.
struct ColList {
  const void *p[RBICG_MAXCOLS];
};

// Blocks of the iteration kernels for n rows (at most 8 rows per thread).
int iter_grid(int n);
// fewest blocks that cover n rows (RMAX rows per thread)
int iter_grid_min(int n);
// whether nb iteration blocks cover n rows with one row per thread
bool iter_one_row(int n, int nb);

template <class V, class M>
void launch_it1(hipStream_t st, int nb, const Sell<M> &A, const Sell<M> &AH, const V *r,
                const V *p, const V *rt, const V *pt, V *pn, V *ptn, V *z, V *zt, const V *C,
                const V *Ct, int k, int ld, V *capR, V *capRt, V *capZ, V *capZt,
                const double *P3, double *P1, Scalars *S, double *rec, int it, int first,
                int rp);
template <class V>
void launch_it2(hipStream_t st, int nb, int n, V *x, V *xt, V *r, V *rt, const V *pn,
                const V *ptn, const V *z, const V *zt, const V *C, const V *Ct, int k, int ld,
                const double *P1, double *P3, Scalars *S, double *rec, int it, int rp,
                double *zlog = nullptr, int zstride = 0);
template <class V>
void launch_itfin(hipStream_t st, int nb, const double *P3, Scalars *S, double *rec, int it,
                  int first, Scalars *hs);

// ---- split preconditioning by triangular factors (ILUT) ----
// A triangular factor for k_sptrsv: the strictly triangular part in CSR (rp,
// ci, v over the n rows), the diagonal (NULL: unit), and the level-scheduled
// row order (len entries, -1 padding; levels padded to whole waves).
template <class M>
struct TriDev {
  int n, len;
  const int *order, *rp, *ci;
  const M *v, *diag;
};
template <class V>
void launch_op_dir(hipStream_t st, int nb, int n, const V *r, const V *p, const V *rt, const V *pt,
                   V *pn, V *ptn, V *capR, V *capRt, const double *P3, Scalars *S, double *rec,
                   int it, int first);
template <class V>
void launch_op_restr(hipStream_t st, int nb, int n, const V *z, const V *zt, const V *ptn,
                     const V *C, const V *Ct, int k, int ld, V *capZ, V *capZt, double *P1,
                     const Scalars *S);
// y = A x; S may be NULL (else nothing happens after the stopping test)
template <class V, class M>
void launch_spmv(hipStream_t st, const Sell<M> &A, const V *x, V *y, const Scalars *S);
// T0 x0 = b0 and, when T1 is given, T1 x1 = b1 (see k_sptrsv): two launches
// (x0, x1 marked pending and the counter cleared, then the solves on `waves`
// waves); V double or complex; b must alias neither x
template <class V, class M>
void launch_sptrsv(hipStream_t st, const TriDev<M> &T0, const V *b0, V *x0, const TriDev<M> *T1,
                   const V *b1, V *x1, int *counter, int waves, const Scalars *S, int *err);
template <class V>
void launch_rsub(hipStream_t st, int n, const V *b, const V *t, V *out);
// y = A x with optional row map (row j computes A's row orow[j]) and gather
// map (x read at gmap[c]); see k_spmv_perm
template <class V, class M>
void launch_spmv_perm(hipStream_t st, const Sell<M> &A, const V *x, V *y, const int *gmap,
                      const int *orow, const Scalars *S);
// out[i] = in[map[i]]
template <class V>
void launch_gather(hipStream_t st, int n, const V *in, const int *map, V *out);

// ---- batched launches: several independent systems ("slots") per launch ----
#define RBICG_BATCH_SLOTS 16
// Arguments of one slot of k_it1_multi / k_it2_multi: those of launch_it1 /
// launch_it2 for that system, and the slot's first block b0 and block count
// nb (slots in increasing b0, contiguous).
template <class V, class M>
struct It1Args {
  Sell<M> A, AH;
  const V *r, *p, *rt, *pt;
  V *pn, *ptn, *z, *zt;
  const V *C, *Ct;
  int k, ld;
  V *capR, *capRt, *capZ, *capZt;
  const double *P3;
  double *P1;
  Scalars *S;
  double *rec;
  int it, first, rp;
  int b0, nb;
};
template <class V>
struct It2Args {
  int n;
  V *x, *xt, *r, *rt;
  const V *pn, *ptn, *z, *zt, *C, *Ct;
  int k, ld;
  const double *P1;
  double *P3;
  Scalars *S;
  double *rec;
  int it, rp;
  double *zlog;
  int zstride;
  int b0, nb;
};
struct ItfinArgs {
  const double *P3;
  int nb;
  Scalars *S;
  double *rec;
  int it, first;
  Scalars *hs;
};
// dtab: device arrays of nslot entries; nblocks = sum of the slots' nb; rpt1:
// every slot covers its rows with one row per thread (else RMAX rows)
template <class V, class M>
void launch_it1_multi(hipStream_t st, const It1Args<V, M> *dtab, int nslot, int nblocks,
                      size_t lds_bytes, bool rpt1);
template <class V>
void launch_it2_multi(hipStream_t st, const It2Args<V> *dtab, int nslot, int nblocks);
template <class V>
void launch_itfin_multi(hipStream_t st, const ItfinArgs *dtab, int nslot);
// the same three launches as kernel nodes of a graph, chained after `last`
template <class V, class M>
hipError_t graph_it1_multi(hipGraph_t g, hipGraphNode_t &last, const It1Args<V, M> *dtab, int nslot,
                           int nblocks, size_t lds_bytes, bool rpt1);
template <class V>
hipError_t graph_it2_multi(hipGraph_t g, hipGraphNode_t &last, const It2Args<V> *dtab, int nslot,
                           int nblocks);
template <class V>
hipError_t graph_itfin_multi(hipGraph_t g, hipGraphNode_t &last, const ItfinArgs *dtab, int nslot);
// dynamic LDS bytes of k_it1 for recycle dimension k (and re-projection rp)
template <class V>
size_t it1_lds_bytes(int k, int rp);
template <class V>
void launch_init_p3(hipStream_t st, int nb, int n, const V *r, const V *rt, double *P3);
// dots (a_i, b_i), i < 3, reduced into out[0 .. 3*ND)
template <class V>
void launch_dots(hipStream_t st, int nb, int n, const V *a0, const V *b0, const V *a1,
                 const V *b1, const V *a2, const V *b2, double *P, double *out);
// [B^H u, B2^H u2] reduced into out[0 .. 2*k*ND)
template <class V>
void launch_restrict(hipStream_t st, int nb, int n, const V *u, const V *B, const V *u2,
                     const V *B2, int k, int ld, double *P, double *out);
void launch_fin_red(hipStream_t st, const double *P, int nb, int nv, double *out);
template <class V, class M>
void launch_residual(hipStream_t st, const Sell<M> &A, const V *b, const V *x, V *out);
template <class V, class M>
void launch_spmm(hipStream_t st, const Sell<M> &A, const V *X, V *Y, int ld, int m);
template <class V>
void launch_expand2(hipStream_t st, int n, V *x, const V *U, double sx, V *r, const V *C,
                    double sr, V *xt, const V *Ut, double sxt, V *rt, const V *Ct, double srt,
                    int k, int ld, const double *coef);
template <class V>
void launch_fill_zero(hipStream_t st, V *p, size_t n);
template <class V>
void launch_reseed(hipStream_t st, V *x, size_t n, unsigned long long seed);
// out = (float)in; x += sgn (double)d (FP32-inner mode)
void launch_d2f(hipStream_t st, const double *in, float *out, size_t n);
void launch_add_f2d(hipStream_t st, double *x, const float *d, double sgn, size_t n);
void launch_add_d2d(hipStream_t st, double *x, const double *d, double sgn, size_t n);
// row chunks (blocks) of the Gram kernel for n rows
int gram_chunks(int n);
// Gram kernel: LDS budget per block (gfx950 has 160 KB per CU)
#define GRAM_LDS_BYTES 153600
// widest column group of Y per Gram launch for mx columns of X
int gram_group(int mx, int complex_vals);
// G = X^H Y for mx, my <= 192 columns (complex (re, im) row-major by (i, j))
template <class V>
void launch_gram(hipStream_t st, int n, const ColList &X, int mx, const ColList &Y, int my,
                 double *partial, double *G, int nchunks);
// Two Grams in one launch: G = [X[0, mx)^H Y[0, my), X[x1, x1 + mx1)^H
// Y[y1, y1 + my1)], each row-major, the second after the first (mx1 = 0:
// launch_gram).  partial holds nchunks (mx my + mx1 my1) entries.
template <class V>
void launch_gram2(hipStream_t st, int n, const ColList &X, int mx, const ColList &Y, int my, int x1,
                  int mx1, int y1, int my1, double *partial, double *G, int nchunks);
template <class V>
void launch_tsgemm(hipStream_t st, int n, const ColList &X, int m, const cd *W, int p, V *Y,
                   int ld);

// out[i] = alpha e[i] + beta a[i] over m sliced-ELL entries (a, e real or complex)
void launch_pencil(hipStream_t st, size_t m, const void *a, int acplx, const void *e, int ecplx,
                   cd alpha, cd beta, cd *out);

// ---- batched shifted pairs (see kernels.hip) ----
int sh_blocks(int n);      // blocks of k_sh2 (partials of P3)
int sh_sub_blocks(int n);  // blocks of k_sh_sub
void launch_sh_state(hipStream_t st, int S, const double *P3, int nb3, ShScalars *Sh, double *rec,
                     int it, int first, ShScalars *hs = nullptr);
template <class M>
void launch_sh1(hipStream_t st, const Sell<M> &A, const Sell<M> &AH, int ld, const cd *R,
                const cd *Rt, const cd *P, const cd *Pt, cd *Pn, cd *Ptn, cd *Z, cd *Zt,
                const ShScalars *Sh);
void launch_sh_coef(hipStream_t st, int S, const double *G, int ld0, int g1, int ld1,
                    ShScalars *Sh, const ShCoef *Co, cd *Y, cd *Yt, cd *Yx, cd *Yxt, int mode,
                    double *rec, int it);
void launch_sh_sub(hipStream_t st, int n, const ColList &X, int m, const cd *W, int p,
                   const cd *Zin, cd *Out, int ld, int nbe);
// B, Bt: n x k2 column-major bases (leading dimension ld); ld * 9 * 16 < 2^32
void launch_sh2(hipStream_t st, int n, int ld, int S, cd *X, cd *Xt, cd *R, cd *Rt, const cd *Pn,
                const cd *Ptn, const cd *Z, const cd *Zt, const cd *B, const cd *Bt, int k2,
                const cd *Y, const cd *Yt, ShScalars *Sh, double *P3, int nb, int upd);

// ---- split ILU(0) preconditioning in red-black ordering (precond.hip) ----
// Device data of a preconditioner: CSR rows of A (rp, ci, av) and of A^H
// (hrp, hci, hv), the diagonal d of A, the black index of each unknown
// (bidx, -1 for red) and the black ILU(0) pivots sb (length nb); values are
// double or complex (cd) as the matrix.
struct RbDev {
  int n = 0, nb = 0;
  const int *rp = nullptr, *ci = nullptr, *hrp = nullptr, *hci = nullptr, *bidx = nullptr;
  const void *av = nullptr, *hv = nullptr, *d = nullptr, *sb = nullptr;
};
// Maps of the device refresh (new values of A on the same pattern): amap[e]
// the A^H entry of A's entry e, blist the original index of each black
// unknown, M_B's CSR pattern (mrp, mci, black numbering; nnzm entries) and
// the sliced-ELL positions of its entries in M_B (msell) and M_B^H (mhsell),
// whose value arrays are mval, mhval.
struct RbRefresh {
  int nnzm = 0;
  const int *amap = nullptr, *blist = nullptr, *mrp = nullptr, *mci = nullptr;
  const int *msell = nullptr, *mhsell = nullptr;
  void *mval = nullptr, *mhval = nullptr;
};
// from P.av (new values of A): A^H values, d, the black pivots and M_B
template <class V>
void launch_rb_refresh(hipStream_t st, const RbDev &P, const RbRefresh &R);
// b^_B, c^_B (length nb) from b, b~ (length n); cR: n-long scratch
template <class V>
void launch_rb_rhs(hipStream_t st, const RbDev &P, const V *b, const V *bt, V *bB, V *cB, V *cR);
// x, x~ (length n) from the black solutions y_B, y~_B and b, b~
template <class V>
void launch_rb_solution(hipStream_t st, const RbDev &P, const V *b, const V *bt, const V *yB,
                        const V *ytB, V *x, V *xt);
