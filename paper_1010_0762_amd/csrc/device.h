// Device-side types shared by the RBiCG kernels and the runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RBICG_BLOCK 256
#define RBICG_WAVE 64
#define KMAXD 64

// complex double, interleaved (re, im) -- the layout of the C ABI
struct cd {
  double x, y;
};

// Per-handle scalar block in device memory.  Vectors of k complex or real
// values are stored as doubles (ND = 1 or 2 per value): zc holds
// [zeta_c | zeta~_c], gbuf holds host-requested restrictions, red the
// results of host-requested dot products.
struct Scalars {
  double tol, bn, btn;
  int iter, done, status, maxit;
  // Cycle-end guards.  At every stag_s-th iteration of the run that started
  // after iteration stag_base (a cycle end), with the relative residual
  // max(||r||/||b||, ||r~||/||b~||) now (cur) and at the previous cycle end
  // (prev): stop as stagnated if cur <= stag_lim and cur >= prev / 2; with
  // stag_div set, from cycle stag_w on, stop when the smallest cycle-end
  // value has not halved over the last stag_w cycles (diverged if it is above
  // stag_lim, else stagnated).  stag_s = 0: off.  FP32-inner solves use
  // stag_w = 2 and stag_lim = sqrt(inner tol); solves with a recycle space
  // and opts.stall_window = w > 0 use stag_w = w and stag_lim = 0 (the stall
  // guard).
  int stag_s, stag_div, stag_w, stag_base;
  double stag_lim;
  double zc[4 * KMAXD];
  double gbuf[4 * KMAXD];
  double red[32];
};

// status codes written by the kernels
#define ST_RUNNING 0
#define ST_CONVERGED 1
#define ST_MAXIT 2
#define ST_BREAKDOWN 3
#define ST_STAGNATED 4
#define ST_DIVERGED 5

// Wave-sliced ELL: rows grouped in slices of 64 (one wavefront, one row per
// lane); entry j of row r sits at sliceptr[r/64] + j*64 + r%64.  Padding
// entries point at their own row with value 0.
//
// A view may carry a shift: with shifted = 1 it stands for sigma I - A
// (sigma = shr + i shi), applied by the kernels on the fly, so the shifted
// systems of IRKA (Algorithm 3) need no second matrix.
template <class M>
struct Sell {
  int n;
  int nslices;
  const int *sliceptr;  // nslices + 1 offsets (multiples of 64)
  const int *col;
  const M *val;
  int shifted;
  double shr, shi;
};

#define LOG_STRIDE 10

// ---------------------------------------------------------------- shifts
// Batched shifted pairs (sigma_i I - A) x_i = b, (sigma_i I - A)^H x~_i = c:
// per-shift scalars and small per-shift data of one sweep.
#define SHMAX 16   // shifts per batch
#define KSH 32     // recycle dimension in the shifted path (2k basis columns <= 64)
#define SH_LOG 8   // per shift per iteration: alpha (re, im), beta (re, im), rho (re, im), ||r||, ||r~||

struct ShScalars {
  double tol;
  int S, k2, maxit, all_done;
  int done[SHMAX], status[SHMAX], iter[SHMAX], p[SHMAX];
  double bn[SHMAX], btn[SHMAX];
  double sig[2 * SHMAX];
  // per shift: beta and whether the iteration goes on (act1, from the
  // stopping test), alpha and whether it updates (act, after sigma)
  double beta[2 * SHMAX], alpha[2 * SHMAX];
  int act1[SHMAX], act[SHMAX];
  // per shift: the running zeta_c, zeta~_c (complex, p_sigma entries)
  double zc[SHMAX][2 * KSH], zct[SHMAX][2 * KSH];
};

// Per-shift coefficient matrices of a sweep (complex, interleaved):
//   K  (p x 2k, row-major)  zeta  = K w,   w  = [U~, A^H U~]^H z
//   Kt (p x 2k, row-major)  zeta~ = Kt w~, w~ = [U, A U]^H z~
//   L  (2k x p, row-major)  y  = L zeta:   q  = z  - [U, A U] y
//   Lt (2k x p, row-major)  y~ = Lt zeta~: q~ = z~ - [U~, A^H U~] y~
//   T  (k x p, row-major)   x  -= U (T zeta_c),  Tt likewise for x~
#define SH_MAT (2 * KSH * KSH)  // complex entries reserved per matrix
struct ShCoef {
  double K[SHMAX][2 * SH_MAT], Kt[SHMAX][2 * SH_MAT];
  double L[SHMAX][2 * SH_MAT], Lt[SHMAX][2 * SH_MAT];
  double T[SHMAX][2 * SH_MAT], Tt[SHMAX][2 * SH_MAT];
};
