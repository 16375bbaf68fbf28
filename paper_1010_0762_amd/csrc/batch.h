// Batched launches of the iteration kernels of several solves (continuous
// batching): every solve attached to a batch hands its chunk of iterations to
// the batch instead of launching it; the batch launches the chunks of all
// solves that are ready together, one k_it1_multi and one k_it2_multi per
// iteration and one k_itfin_multi at the end, on its own stream.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.h"
#include "rbicg.h"

// Value and matrix types of a slot (one kernel instantiation per kind).
enum BatchKind { BK_F64 = 0, BK_C128_REAL_A = 1, BK_C128 = 2, BK_F32 = 3, BK_KINDS = 4 };

// One solve's chunk: len iterations, their It1Args / It2Args (as bytes of the
// kind's argument types), and the chunk's final stopping test.
struct BatchChunk {
  int kind = 0;
  bool one_row = true;   // the system's rows are covered with one row per thread
  int nb = 0;            // blocks of the system
  size_t lds = 0;        // dynamic LDS bytes of its k_it1
  int len = 0;
  std::vector<char> it1, it2;
  ItfinArgs fin{};
  hipStream_t st = nullptr;  // the solve's stream: the chunk runs after its prior work
};

// The calling solve is iterating (enter) / done iterating (leave); the batch
// launches without waiting once every iterating solve has handed in a chunk.
void batch_enter(rbicg_batch b);
void batch_leave(rbicg_batch b);
// Hand in a chunk; returns once the chunk's launches are enqueued, with c.st
// ordered after them.  Thread safe.
int batch_submit(rbicg_batch b, BatchChunk &c);
