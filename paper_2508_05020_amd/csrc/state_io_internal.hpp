// Internal interface of the state upload kernels (state_io.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "amr_internal.hpp"

namespace amr {

struct StateIO {
  // bytes of the per-device staging array of the upload that allocates nothing
  static constexpr size_t kScratchBytes = size_t(32) << 20;
  // device address of that array on the current device (looked up once per
  // device; the current device must be the one the caller launches on)
  static hipError_t noalloc_scratch(void** out);
  // Interior cells of `count` patches from primitive values: patch pids[b]
  // reads prim[src[b] ...], var-major (rho, u_1..u_d, p) over n_l^d cells;
  // ghost cells are left as they are
  static void set_prim(const DevMesh& m, double* U, const double* prim, const long long* src,
                       const int* pids, int count, double gm1, hipStream_t s);
};

}  // namespace amr
