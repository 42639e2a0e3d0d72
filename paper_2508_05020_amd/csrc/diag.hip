// Velocity-gradient diagnostic: at every interior cell of a leaf patch,
// G[i][j] = (u_i(x + h e_j) - u_i(x - h e_j)) / (2h) with u_i = m_i / rho,
// and the density-gradient magnitude S = |grad rho| by the same differences
// (the quantity a numerical Schlieren image is drawn from).  The paper's
// fusion listing (§4.1) shows the task that writes this region with its body
// elided; second-order central differences on the cell's own level are the
// reading taken here.  Memory-bound: (d + 1) values read at 2d neighbours,
// d*d + 1 written per cell.
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

#include "device_common.hpp"
#include "diag_internal.hpp"

namespace amr {
namespace {

template <int D>
__global__ __launch_bounds__(256) void k_velocity_gradient(DevMesh m, const double* __restrict__ U,
                                                           const int* __restrict__ leaves, int count,
                                                           double* __restrict__ out, long long plane) {
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    const int pid = leaves[b];
    const int l = m.level[pid];
    const LevelC& L = m.lv[l];
    const int n = L.n, f = L.full;
    const int vs = var_stride<D>(f);
    const double* P = U + patch_base(m, pid, l);
    // cell layout of one variable: the patch's box at its state offset / nvar
    double* O = out + (L.pool_off + (long long)(pid - L.pid_base) * L.stride) / m.nvar;
    const double two_h = 2.0 * L.h;
    long long step[3] = {1, f, (long long)f * f};
    int ncell = n;
    if constexpr (D >= 2) ncell *= n;
    if constexpr (D >= 3) ncell *= n;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
      const int x = c % n;
      const int y = D >= 2 ? (c / n) % n : 0;
      const int z = D >= 3 ? c / (n * n) : 0;
      const long long o = box_off<D>(f, x + NG, y + NG, z + NG);
      double gr[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const long long op = o + step[j], om = o - step[j];
        const double rp = P[op], rm = P[om];
        gr[j] = (rp - rm) / two_h;
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const double up = P[(1 + i) * vs + op] / rp;
          const double um = P[(1 + i) * vs + om] / rm;
          O[(long long)(i * D + j) * plane + o] = (up - um) / two_h;
        }
      }
      double s2 = gr[0] * gr[0];
      if constexpr (D >= 2) s2 = s2 + gr[1] * gr[1];
      if constexpr (D >= 3) s2 = s2 + gr[2] * gr[2];
      O[(long long)(D * D) * plane + o] = sqrt(s2);
    }
  }
}

}  // namespace

void Diagnostics::velocity_gradient(const DevMesh& m, const double* U, const int* leaves, int count,
                                    double* out, long long plane, hipStream_t s) {
  if (count <= 0) return;
  const int blocks = count < 65535 ? count : 65535;
  if (m.dim == 1)
    hipLaunchKernelGGL(k_velocity_gradient<1>, dim3(blocks), dim3(64), 0, s, m, U, leaves, count, out,
                       plane);
  else if (m.dim == 2)
    hipLaunchKernelGGL(k_velocity_gradient<2>, dim3(blocks), dim3(256), 0, s, m, U, leaves, count,
                       out, plane);
  else
    hipLaunchKernelGGL(k_velocity_gradient<3>, dim3(blocks), dim3(256), 0, s, m, U, leaves, count,
                       out, plane);
}

}  // namespace amr
