// Primitive-to-conservative upload of patch interiors: m_j = rho u_j and
// E = p / (gamma - 1) + rho |u|^2 / 2 (Eq. (4), (6)), one block per patch.
// Memory-bound: (d + 2) doubles read and written per cell.  Contraction is
// off so that every value is the one a host conversion in the same order
// produces.
#include <hip/hip_runtime.h>

#include <mutex>

#pragma clang fp contract(off)

#include "device_common.hpp"
#include "state_io_internal.hpp"

namespace amr {
namespace {

// Staging memory of the upload that allocates nothing: every GPU the library
// runs on holds one copy of this array until the process ends.  Host code
// must not pass `scratch` itself to a kernel (in host code the name is a
// host-side stand-in): it uses the device address hipGetSymbolAddress gives
// for the current device, resolved once per device by noalloc_scratch().
static __device__ __align__(256) unsigned char scratch[StateIO::kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

template <int D>
__global__ __launch_bounds__(256) void k_set_prim(DevMesh m, double* __restrict__ U,
                                                  const double* __restrict__ prim,
                                                  const long long* __restrict__ src,
                                                  const int* __restrict__ pids, int count,
                                                  double gm1) {
  constexpr int NV = D + 2;
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    const int pid = pids[b];
    const int l = m.level[pid];
    const LevelC& L = m.lv[l];
    const int n = L.n, f = L.full;
    const int vs = var_stride<D>(f);
    double* P = U + patch_base(m, pid, l);
    const double* S = prim + src[b];
    int ncell = n;
    if constexpr (D >= 2) ncell *= n;
    if constexpr (D >= 3) ncell *= n;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
      const int x = c % n;
      const int y = D >= 2 ? (c / n) % n : 0;
      const int z = D >= 3 ? c / (n * n) : 0;
      const int off = box_off<D>(f, x + NG, y + NG, z + NG);
      const double rho = S[c];
      double uu = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double u = S[(long long)(1 + j) * ncell + c];
        uu = (j == 0) ? u * u : uu + u * u;
        P[(1 + j) * vs + off] = rho * u;
      }
      const double p = S[(long long)(D + 1) * ncell + c];
      P[off] = rho;
      P[(NV - 1) * vs + off] = p / gm1 + 0.5 * rho * uu;
    }
  }
}

}  // namespace

hipError_t StateIO::noalloc_scratch(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

void StateIO::set_prim(const DevMesh& m, double* U, const double* prim, const long long* src,
                       const int* pids, int count, double gm1, hipStream_t s) {
  if (count <= 0) return;
  const int blocks = count < 65536 ? count : 65536;
  switch (m.dim) {
    case 1:
      hipLaunchKernelGGL(k_set_prim<1>, dim3(blocks), dim3(64), 0, s, m, U, prim, src, pids,
                         count, gm1);
      break;
    case 2:
      hipLaunchKernelGGL(k_set_prim<2>, dim3(blocks), dim3(256), 0, s, m, U, prim, src, pids,
                         count, gm1);
      break;
    default:
      hipLaunchKernelGGL(k_set_prim<3>, dim3(blocks), dim3(256), 0, s, m, U, prim, src, pids,
                         count, gm1);
      break;
  }
}

}  // namespace amr
