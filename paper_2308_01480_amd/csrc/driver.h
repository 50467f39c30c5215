// Internal interface between the forward sweep (sweep.hip) and the gradient driver
// (grad.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace ttr {

// Forward state kept for the reverse sweep of the gradient entry (device memory).
struct ModeTape {
  double* Q;      // m x w Krylov basis (regular modes), float64
  double* Yall;   // m x w, A A^T Q (regular modes), float64
  double* T;      // (q+1) blocks of s x s: Q_j = P_j T_j, T_j = E R_j^{-1}
  double* U;      // e x e eigenvectors (of M, A A^T or A^T A), columns by decreasing value
  double* lam;    // e eigenvalues
  int* ints;      // [0..q]: kept columns per block, [q+1]: valid Ritz / singular directions
  void* carry;    // C_k (r x n, carry dtype)
};

// The sweep of Algorithm 3; with `tapes` (one per mode k = 1..d-1) the forward state is
// kept and every carry gets its own buffer.
int sweep(const void* x, const Plan& pl, uint64_t seed, double* const* cores, char* ws, hipStream_t st,
          const ModeTape* tapes);

// Streaming (||X - Xhat||^2, ||X||^2, ||Xhat||_inf) of float64 cores (host array of device
// pointers) into out3; ws holds tt_error_ws_bytes(d, dims, ranks) bytes.
hipError_t tt_error_run(const void* x, int x_dtype, int d, const int64_t* dims, const int64_t* ranks,
                        const double* const* cores, double* out3, char* ws, hipStream_t st);

}  // namespace ttr
