// Device helpers shared by the HIP kernels of libamr: patch-pool
// addressing, physical-boundary mapping, same-level cell lookup through the
// level maps, MC-limited prolongation, the CFL rate of a cell, a block-wide
// maximum, and the XCD-contiguous block-to-work-item mapping.
//
// Included by the .hip sources only, after their fp-contract pragma.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "amr_internal.hpp"

namespace amr {
namespace {


constexpr int NG = kNG;

__device__ __forceinline__ int bc_map(int g, int N, int periodic) {
  if (periodic) {
    g %= N;
    return g < 0 ? g + N : g;
  }
  return g < 0 ? 0 : (g >= N ? N - 1 : g);
}

template <int D>
__device__ __forceinline__ int box_off(int full, int x, int y, int z) {
  // offsets inside one patch fit 32 bits, and the factors 24 (one full-rate
  // 24-bit multiply-add each instead of 64-bit products)
  if constexpr (D == 1) return x;
  if constexpr (D == 2) return __mul24(y, full) + x;
  return __mul24(__mul24(z, full) + y, full) + x;
}

template <int D>
__device__ __forceinline__ int var_stride(int full) {
  if constexpr (D == 1) return full;
  if constexpr (D == 2) return __mul24(full, full);
  return __mul24(__mul24(full, full), full);
}

__device__ __forceinline__ long long patch_base(const DevMesh& m, int pid, int l) {
  return m.lv[l].pool_off + (long long)(pid - m.lv[l].pid_base) * m.lv[l].stride;
}

template <int D>
__device__ __forceinline__ int map_at(const DevMesh& m, int l, const int q[3]) {
  const LevelC& L = m.lv[l];
  int idx = q[0];
  if constexpr (D >= 2) idx += L.np * q[1];
  if constexpr (D >= 3) idx += L.np * L.np * q[2];
  return m.map[L.map_off + idx];
}

// Conserved values of the level-l cell at in-domain global index g.
template <int D>
__device__ bool fetch_cell(const DevMesh& m, const double* __restrict__ U, int l,
                           const int g[3], double out[D + 2]) {
  const LevelC& L = m.lv[l];
  int q[3] = {0, 0, 0}, c[3] = {0, 0, 0};
  for (int j = 0; j < D; ++j) {
    q[j] = g[j] / L.n;
    c[j] = g[j] - q[j] * L.n;
  }
  const int pid = map_at<D>(m, l, q);
  if (pid < 0) return false;
  const double* P = U + patch_base(m, pid, l);
  const int off = box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG);
  const int vs = var_stride<D>(L.full);
#pragma unroll
  for (int v = 0; v < D + 2; ++v) out[v] = P[v * vs + off];
  return true;
}

// Pressure from conserved values in the reference operation order:
// u_j = m_j / rho, ke = 0.5 * (m_x u_x + m_y u_y + m_z u_z), p = (gamma-1)(E - ke).
template <int D>
__device__ __forceinline__ double pressure_exact(const double* u, double gm1) {
  const double rho = u[0];
  double ke = u[1] * (u[1] / rho);
#pragma unroll
  for (int j = 1; j < D; ++j) ke = ke + u[1 + j] * (u[1 + j] / rho);
  ke = 0.5 * ke;
  return gm1 * (u[D + 1] - ke);
}

// Conservative MC-limited linear prolongation of the level-lf cell at mapped
// global index g from level lf-1.  Slopes are dropped when any of the 2^D
// children of the coarse cell would have rho <= 0 or p <= 0.
template <int D>
__device__ bool prolong_cell(const DevMesh& m, const double* __restrict__ U, int lf,
                             const int g[3], double out[D + 2]) {
  constexpr int NV = D + 2;
  constexpr int NS = 2 * D + 1;  // coarse stencil: centre, then (+1, -1) per direction
  const int lc = lf - 1;
  const LevelC& C = m.lv[lc];
  int gc[3] = {0, 0, 0};
  double sig[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < D; ++j) {
    gc[j] = g[j] >> 1;
    sig[j] = (g[j] & 1) ? 1.0 : -1.0;
  }
  // all map lookups first, then all loads, so the latencies overlap
  int pids[NS];
  long long offs[NS];
  const int vs = var_stride<D>(C.full);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    int gs[3] = {gc[0], gc[1], gc[2]};
    if (s > 0) {
      const int j = (s - 1) >> 1;
      gs[j] = bc_map(gc[j] + (((s - 1) & 1) ? -1 : 1), C.cells, m.periodic[j]);
    }
    int q[3] = {0, 0, 0}, c[3] = {0, 0, 0};
    for (int j = 0; j < D; ++j) {
      q[j] = gs[j] / C.n;
      c[j] = gs[j] - q[j] * C.n;
    }
    pids[s] = map_at<D>(m, lc, q);
    offs[s] = box_off<D>(C.full, c[0] + NG, c[1] + NG, c[2] + NG);
  }
  bool found = true;
#pragma unroll
  for (int s = 0; s < NS; ++s) found &= pids[s] >= 0;
  if (!found) return false;
  double val[NS][NV];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double* P = U + patch_base(m, pids[s], lc) + offs[s];
#pragma unroll
    for (int v = 0; v < NV; ++v) val[s][v] = P[v * vs];
  }
  const double* phi = val[0];
  double sl[D][NV];
#pragma unroll
  for (int j = 0; j < D; ++j) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double a = val[1 + 2 * j][v] - phi[v];
      const double b = phi[v] - val[2 + 2 * j][v];
      const bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
      const double mag = fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b));
      sl[j][v] = same ? copysign(mag, a) : 0.0;
    }
  }
  bool bad = false;
  for (int c = 0; c < (1 << D); ++c) {
    double ch[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double x = phi[v];
      for (int j = 0; j < D; ++j) x = x + (((c >> j) & 1) ? 0.25 : -0.25) * sl[j][v];
      ch[v] = x;
    }
    const double p = pressure_exact<D>(ch, m.gm1);
    if (!(ch[0] > 0.0 && p > 0.0)) bad = true;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double x = phi[v];
    for (int j = 0; j < D; ++j) x = x + (sig[j] * 0.25) * (bad ? 0.0 : sl[j][v]);
    out[v] = x;
  }
  return true;
}

// CFL rate of one cell, sum_j (|u_j| + c) / h with c = sqrt(gamma p / rho),
// as the IEEE bits of a non-negative double (order-preserving as an
// unsigned integer); NaN maps to the largest value so that it propagates.
template <int D>
__device__ __forceinline__ unsigned long long cell_rate_bits(const double* u, const DevMesh& m,
                                                             double h) {
  const double rho = u[0];
  double uj[D];
#pragma unroll
  for (int j = 0; j < D; ++j) uj[j] = u[1 + j] / rho;
  double ke = u[1] * uj[0];
#pragma unroll
  for (int j = 1; j < D; ++j) ke = ke + u[1 + j] * uj[j];
  ke = 0.5 * ke;
  const double p = m.gm1 * (u[D + 1] - ke);
  const double c = sqrt(m.gamma * p / rho);
  double s = fabs(uj[0]) + c;
#pragma unroll
  for (int j = 1; j < D; ++j) s = s + (fabs(uj[j]) + c);
  const double r = s / h;
  if (!(r >= 0.0)) return 0x7ff8000000000000ull;
  return (unsigned long long)__double_as_longlong(r);
}

// block-wide max of per-thread values, then one 64-bit atomic max
__device__ __forceinline__ void block_max_atomic(unsigned long long best,
                                                 unsigned long long* __restrict__ lam) {
  __shared__ unsigned long long red[16];
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(best, off);
    best = o > best ? o : best;
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) b = red[k] > b ? red[k] : b;
    if (b) atomicMax(lam, b);
  }
}

// Work item of this block.  Workgroups are dealt to the chip's XCDs in
// turn (block b runs on XCD b mod kXcds) and each XCD has its own L2: XCD x
// takes the contiguous items [x per, (x + 1) per), per = ceil(count /
// kXcds), in dispatch order, so tiles of one patch and of neighbouring
// patches (the list is in brick order), which read each other's cells as
// halos, share an L2.  The grid holds at least kXcds per blocks; it may hold
// more (a launch recorded for a longer list), and a block without an item
// gets -1.
__device__ __forceinline__ int xcd_item(int count) {
  const int per = (count + kXcds - 1) / kXcds;
  const int k = (int)blockIdx.x / kXcds;
  const int item = ((int)blockIdx.x % kXcds) * per + k;
  return (k < per && item < count) ? item : -1;
}

}  // namespace
}  // namespace amr
