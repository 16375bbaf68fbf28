// Kernel views of a resident matrix, for the library's translation units that
// do not own the matrix type (the matrix object is defined in runtime.hip).
#pragma once
#include <stdint.h>

#include "device.h"
#include "rbicg.h"

struct MatViews {
  int n = 0;
  int complex_vals = 0;   // 1: values are interleaved complex doubles
  int shared_pattern = 0; // 1: A^H keeps A's slice pointers and column indices
  int64_t nnz = 0;
  Sell<double> A{}, AH{};  // valid when complex_vals == 0
  Sell<cd> Ac{}, AHc{};    // valid when complex_vals == 1
};

// Fill *out for a matrix made by rbicg_matrix_create (or rbicg_matrix_pencil).
int rbicg_matrix_views(rbicg_matrix m, MatViews *out);
