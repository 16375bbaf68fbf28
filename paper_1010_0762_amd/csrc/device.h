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
// values are stored as doubles (ND = 1 or 2 per value): zbuf holds
// [zeta_i | zeta~_i] of the current iteration, zc holds [zeta_c | zeta~_c],
// gbuf holds host-requested restrictions, red the results of host-requested
// dot products.
struct Scalars {
  double tol, bn, btn;
  int iter, done, status, maxit;
  // FP32-inner solves: at every stag_s-th iteration, when the relative
  // residual max(||r||/||b||, ||r~||/||b~||) is not below the one stag_s
  // iterations earlier, stop as stagnated if it is <= stag_lim, or (with
  // stag_div set: a recycle space is in use) as diverged if, from the second
  // cycle on, it is not below the initial one (stag_s = 0: off)
  int stag_s, stag_div;
  double stag_lim;
  double zbuf[4 * KMAXD];
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
template <class M>
struct Sell {
  int n;
  int nslices;
  const int *sliceptr;  // nslices + 1 offsets (multiples of 64)
  const int *col;
  const M *val;
};

#define LOG_STRIDE 10
