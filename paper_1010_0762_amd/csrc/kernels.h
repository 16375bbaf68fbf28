// Host-side launchers of the RBiCG kernels (definitions in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"

#define RBICG_MAXCOLS 160

// Column pointer list passed by value as a kernel argument.
struct ColList {
  const void *p[RBICG_MAXCOLS];
};

template <class V, class M>
void launch_iter_spmv(hipStream_t st, const Sell<M> &A, const Sell<M> &AH, const V *r,
                      const V *p, const V *rt, const V *pt, V *pn, V *ptn, V *z, V *zt,
                      const V *C, const V *Ct, int k, int ld, V *capR, V *capRt, V *capZ,
                      V *capZt, double *partial, Scalars *S);
template <class V, class M>
void launch_residual(hipStream_t st, const Sell<M> &A, const V *b, const V *x, V *out);
template <class V, class M>
void launch_spmm(hipStream_t st, const Sell<M> &A, const V *X, V *Y, int ld, int m);
template <class V>
void launch_iter_expand(hipStream_t st, int n, const V *z, const V *zt, const V *C,
                        const V *Ct, int k, int ld, const V *ptn, V *q, V *qt, double *partial,
                        Scalars *S);
template <class V>
void launch_iter_update(hipStream_t st, int n, V *x, V *xt, V *r, V *rt, const V *pn,
                        const V *ptn, const V *q, const V *qt, double *partial, Scalars *S,
                        double *log);
template <class V>
void launch_restrict(hipStream_t st, int n, const V *u, const V *B, const V *u2, const V *B2,
                     int k, int ld, double *partial, Scalars *S);
template <class V>
void launch_expand2(hipStream_t st, int n, V *x, const V *U, double sx, V *r, const V *C,
                    double sr, V *xt, const V *Ut, double sxt, V *rt, const V *Ct, double srt,
                    int k, int ld, int mode, const Scalars *S);
template <class V>
void launch_dots(hipStream_t st, int n, const V *a0, const V *b0, const V *a1, const V *b1,
                 const V *a2, const V *b2, double *partial, Scalars *S);
template <class V>
void launch_fill_zero(hipStream_t st, V *p, size_t n);
template <class V>
void launch_reseed(hipStream_t st, V *x, size_t n, unsigned long long seed);
template <class V>
void launch_gram(hipStream_t st, int n, const ColList &X, int mx, const ColList &Y, int my,
                 double *partial, double *G, int nchunks);
template <class V>
void launch_tsgemm(hipStream_t st, int n, const ColList &X, int m, const cd *W, int p, V *Y,
                   int ld);
