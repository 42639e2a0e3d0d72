// Internal interface of the diagnostic kernels (diag.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "amr_internal.hpp"

namespace amr {

struct Diagnostics {
  // velocity-gradient tensor and density-gradient magnitude at the interior
  // cells of the listed leaf patches (ghosts filled); out holds d*d + 1
  // planes of `plane` doubles in the cell layout of one state variable
  static void velocity_gradient(const DevMesh& m, const double* U, const int* leaves, int count,
                                double* out, long long plane, hipStream_t s);
};

}  // namespace amr
