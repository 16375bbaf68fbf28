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

// Per-handle scalar block in device memory.  Complex slots hold real values
// in .x with .y = 0 for real problems.
struct Scalars {
  cd rho, beta, alpha, sigma;
  double rn, rtn, bn, btn, tol;
  int iter, done, status, maxit;
  int log_base, pad0, pad1, pad2;
  unsigned tickets[16];
  cd zeta[KMAXD], zetat[KMAXD], zeta_c[KMAXD], zetat_c[KMAXD], g[KMAXD], gt[KMAXD];
  double red[32];
};

// status codes written by the kernels
#define ST_RUNNING 0
#define ST_CONVERGED 1
#define ST_MAXIT 2
#define ST_BREAKDOWN 3

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
