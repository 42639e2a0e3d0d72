// Internal interface of the state upload kernels (state_io.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "amr_internal.hpp"

namespace amr {

struct StateIO {
  // Interior cells of `count` patches from primitive values: patch pids[b]
  // reads prim[src[b] ...], var-major (rho, u_1..u_d, p) over n_l^d cells;
  // ghost cells are left as they are
  static void set_prim(const DevMesh& m, double* U, const double* prim, const long long* src,
                       const int* pids, int count, double gm1, hipStream_t s);
};

}  // namespace amr
