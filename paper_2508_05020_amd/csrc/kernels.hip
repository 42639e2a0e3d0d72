// HIP kernels of libamr for gfx950 (CDNA4, wave64).
//
// Every kernel works on the patch pools described in amr_internal.hpp: a
// patch of level l stores nvar * (n_l + 8)^dim doubles, var-major, x fastest,
// with 4 ghost layers.  Work lists (pids or (pid, tile) pairs) are device
// arrays built by the host after each regrid, so one launch covers the
// patches of every level.
//
// Floating-point contract: every kernel disables implicit contraction and
// writes its fused multiply-adds out with fma(), so that a cell's operation
// sequence is fixed by the source and identical in every kernel variant (tile
// shape, fused or explicit halo, per-patch or batched launch).  The
// prolongation, restriction, tag and time-step paths use the operation order
// of the definitions they implement (no fma), so that integer decisions (tags,
// positivity switches) are taken on the same values as the FP64 reference.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "amr_internal.hpp"

// no implicit contraction anywhere in this file (see the header comment)
#pragma clang fp contract(off)

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
__device__ __forceinline__ long long box_off(int full, int x, int y, int z) {
  if constexpr (D == 1) return x;
  if constexpr (D == 2) return (long long)y * full + x;
  return ((long long)z * full + y) * full + x;
}

template <int D>
__device__ __forceinline__ long long var_stride(int full) {
  if constexpr (D == 1) return full;
  if constexpr (D == 2) return (long long)full * full;
  return (long long)full * full * full;
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
  const long long off = box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG);
  const long long vs = var_stride<D>(L.full);
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
  const long long vs = var_stride<D>(C.full);
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

// ---------------------------------------------------------------------------
// ghost fill
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_fill(DevMesh m, double* __restrict__ U,
                                              const int* __restrict__ list, int count,
                                              int* __restrict__ err, int coarse_only) {
  constexpr int NV = D + 2;
  if ((int)blockIdx.x >= count) return;
  const int pid = list[blockIdx.x];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, full = L.full;
  const long long vs = var_stride<D>(full);
  double* P = U + patch_base(m, pid, l);
  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  const int total = (int)vs;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int b[3] = {idx % full, 0, 0};
    if constexpr (D >= 2) b[1] = (idx / full) % full;
    if constexpr (D >= 3) b[2] = idx / (full * full);
    bool ghost = false;
    int g[3] = {0, 0, 0};
    for (int j = 0; j < D; ++j) {
      const int c = b[j] - NG;
      ghost |= (c < 0) || (c >= n);
      g[j] = bc_map(pc[j] * n + c, L.cells, m.periodic[j]);
    }
    if (!ghost) continue;
    double val[NV];
    bool ok = fetch_cell<D>(m, U, l, g, val);
    if (ok && coarse_only) continue;
    if (!ok) ok = (l > 0) && prolong_cell<D>(m, U, l, g, val);
    if (!ok) {
      err[0] = 1;
      for (int v = 0; v < NV; ++v) val[v] = __builtin_nan("");
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) P[v * vs + idx] = val[v];
  }
}

// Ghost cells without a same-level source: one work item per (leaf, ghost
// region), region = neighbour offset r in {-1,0,1}^D coded as
// (r0+1) + 3 (r1+1) + 9 (r2+1); the host lists only regions whose source
// position (after the physical-boundary clamp) holds no same-level patch, so
// every cell of the region is prolonged from level l-1.
template <int D, int NT>
__global__ __launch_bounds__(NT) void k_fill_cf(DevMesh m, double* __restrict__ U,
                                                const int* __restrict__ list, int count,
                                                int* __restrict__ err) {
  constexpr int NV = D + 2;
  if ((int)blockIdx.x >= count) return;
  const int pid = list[2 * blockIdx.x];
  const int code = list[2 * blockIdx.x + 1];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, full = L.full;
  const long long vs = var_stride<D>(full);
  double* P = U + patch_base(m, pid, l);
  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  int start[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  int total = 1;
  for (int j = 0; j < D; ++j) {
    const int r = (j == 0 ? code : (j == 1 ? code / 3 : code / 9)) % 3 - 1;
    start[j] = r < 0 ? -NG : (r == 0 ? 0 : n);
    ext[j] = r == 0 ? n : NG;
    total *= ext[j];
  }
  for (int idx = threadIdx.x; idx < total; idx += NT) {
    int c[3] = {start[0] + idx % ext[0], 0, 0};
    if constexpr (D >= 2) c[1] = start[1] + (idx / ext[0]) % ext[1];
    if constexpr (D >= 3) c[2] = start[2] + idx / (ext[0] * ext[1]);
    int g[3] = {0, 0, 0};
    for (int j = 0; j < D; ++j) g[j] = bc_map(pc[j] * n + c[j], L.cells, m.periodic[j]);
    double val[NV];
    const bool ok = (l > 0) && prolong_cell<D>(m, U, l, g, val);
    if (!ok) {
      err[0] = 1;
      for (int v = 0; v < NV; ++v) val[v] = __builtin_nan("");
    }
    const long long off = box_off<D>(full, c[0] + NG, c[1] + NG, c[2] + NG);
#pragma unroll
    for (int v = 0; v < NV; ++v) P[v * vs + off] = val[v];
  }
}

// Work item of this block when the grid is a whole number of groups of kXcds
// blocks.  Workgroups are dealt to the chip's XCDs in turn (block b runs on
// XCD b mod kXcds), and each XCD has its own L2; the mapping gives every XCD
// one contiguous run of the work list, so tiles of one patch and of
// neighbouring patches (the list is in level, z, y, x order), which read
// each other's cells as halos, share an L2.
__device__ __forceinline__ int xcd_item(int count) {
  const int per_xcd = (int)gridDim.x / kXcds;
  return ((int)blockIdx.x % kXcds) * per_xcd + (int)blockIdx.x / kXcds;
}

// ---------------------------------------------------------------------------
// fused right-hand side + SSP-RK3 stage on (pid, tile) work items
// ---------------------------------------------------------------------------

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (relative error near one ulp); used where correct rounding is not required.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Nonlinear WENO5-JS combination of three candidates from their smoothness
// indicators.  The weights alpha_k / sum(alpha) with alpha_k = d_k / t_k,
// t_k = (eps + beta_k)^2 and d = (1, 10, 5)/16 are evaluated as cross
// products, so one division serves all three.  Inputs are scaled: candidates
// by 8, indicators and eps by 4; with power-of-two factors the scaling is
// exact and only the final 1/8 is applied.
__device__ __forceinline__ double weno_combine(double b0, double b1, double b2, double q0,
                                               double q1, double q2, double eps4) {
  const double e0 = eps4 + b0, e1 = eps4 + b1, e2 = eps4 + b2;
  const double t0 = e0 * e0, t1 = e1 * e1, t2 = e2 * e2;
  const double a0 = t1 * t2;
  const double a1 = 10.0 * (t0 * t2);
  const double a2 = 5.0 * (t0 * t1);
  const double num = fma(a2, q2, fma(a1, q1, a0 * q0));
  return (num * rcp_nr((a0 + a1) + a2)) * 0.125;
}

// WENO5-JS point values on both sides of the edge between v2 and v3 from the
// six nodes v0..v5: the left-biased value from v0..v4 and the right-biased
// value from the mirrored stencil v5..v1.  Candidates: the quadratic through
// three consecutive nodes evaluated at the edge (x8), two of which the sides
// share; indicators (x4): 13/12 (second difference)^2 + 1/4 (first-difference
// form)^2 of the Jiang-Shu definition, with the second differences of the
// two middle windows shared.
__device__ __forceinline__ void weno5_pair(double v0, double v1, double v2, double v3, double v4,
                                           double v5, double eps4, double& L, double& R) {
  const double qa = fma(15.0, v2, fma(-10.0, v1, 3.0 * v0));  // left, nodes v0..v2
  const double qb = fma(3.0, v3, fma(6.0, v2, -v1));          // nodes v1..v3 (both sides)
  const double qc = fma(6.0, v3, fma(3.0, v2, -v4));          // nodes v2..v4 (both sides)
  const double qd = fma(15.0, v3, fma(-10.0, v4, 3.0 * v5));  // right, nodes v3..v5
  const double k0 = fma(-2.0, v1, v0) + v2;
  const double k1 = fma(-2.0, v2, v1) + v3;
  const double k2 = fma(-2.0, v3, v2) + v4;
  const double k3 = fma(-2.0, v4, v3) + v5;
  constexpr double c4 = 4.0 * (13.0 / 12.0);
  const double g0 = c4 * k0, g1 = c4 * k1, g2 = c4 * k2, g3 = c4 * k3;
  const double sl0 = fma(3.0, v2, fma(-4.0, v1, v0));
  const double sl1 = v1 - v3;
  const double sl2 = fma(3.0, v2, fma(-4.0, v3, v4));
  const double sr0 = fma(3.0, v3, fma(-4.0, v4, v5));
  const double sr1 = v4 - v2;
  const double sr2 = fma(3.0, v3, fma(-4.0, v2, v1));
  const double bl0 = fma(g0, k0, sl0 * sl0);
  const double bl1 = fma(g1, k1, sl1 * sl1);
  const double bl2 = fma(g2, k2, sl2 * sl2);
  const double br0 = fma(g3, k3, sr0 * sr0);
  const double br1 = fma(g2, k2, sr1 * sr1);
  const double br2 = fma(g1, k1, sr2 * sr2);
  L = weno_combine(bl0, bl1, bl2, qa, qb, qc, eps4);
  R = weno_combine(br0, br1, br2, qd, qc, qb, eps4);
}

__device__ __forceinline__ double central4(double b, double c, double d, double e) {
  return fma(9.0, c + d, -(b + e)) * 0.0625;
}

template <int D>
struct EdgeState {
  double p, T, u[D];
};

// Conserved state and direction-J flux of an edge state (Eq. (1)-(3), (5)-(7)).
template <int D, int J>
__device__ __forceinline__ void edge_flux(const DevMesh& m, const EdgeState<D>& w,
                                          double U[D + 2], double F[D + 2], double& speed) {
  const double rho = w.p * rcp_nr(w.T);
  double uu = w.u[0] * w.u[0];
#pragma unroll
  for (int i = 1; i < D; ++i) uu = fma(w.u[i], w.u[i], uu);
  const double E = fma(0.5 * rho, uu, w.p * m.igm1);
  U[0] = rho;
  F[0] = rho * w.u[J];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double mi = rho * w.u[i];
    U[1 + i] = mi;
    F[1 + i] = (i == J) ? fma(mi, w.u[J], w.p) : mi * w.u[J];
  }
  U[D + 1] = E;
  F[D + 1] = (E + w.p) * w.u[J];
  speed = sqrt(m.gamma * w.T) + fabs(w.u[J]);
}

template <int D, int TX, int TY, int TZ>
struct TileShape {
  static constexpr int T0 = TX;
  static constexpr int T1 = D >= 2 ? TY : 1;
  static constexpr int T2 = D >= 3 ? TZ : 1;
  static constexpr int NCELL = T0 * T1 * T2;
  static constexpr int ext(int j) {
    return (T0 + (j == 0 ? 8 : 0)) * (T1 + (j == 1 ? 8 : 0)) * (T2 + (j == 2 ? 8 : 0));
  }
  static constexpr int edges(int j) {
    return (T0 + (j == 0 ? 3 : 0)) * (T1 + (j == 1 ? 3 : 0)) * (T2 + (j == 2 ? 3 : 0));
  }
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int EXTMAX = cmax(ext(0), cmax(D >= 2 ? ext(1) : 0, D >= 3 ? ext(2) : 0));
  static constexpr int EDMAX =
      cmax(edges(0), cmax(D >= 2 ? edges(1) : 0, D >= 3 ? edges(2) : 0));
};

// Primitives (p, T, u_j) of one node from its conserved values.
template <int D>
__device__ __forceinline__ void node_primitives(const DevMesh& m, const double* u, double* q) {
  const double r = rcp_nr(u[0]);
  double ke = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double ui = u[1 + i] * r;
    ke = (i == 0) ? u[1] * ui : fma(u[1 + i], ui, ke);
    q[2 + i] = ui;
  }
  const double p = m.gm1 * fma(-0.5, ke, u[D + 1]);
  q[0] = p;
  q[1] = p * r;
}

// Conserved values of a node at patch-local cell c (may lie in the halo):
// from the patch itself, or by the ghost-fill rule when outside the patch.
template <int D, bool FUSE>
__device__ __forceinline__ void node_conserved(const DevMesh& m, const double* __restrict__ Uin,
                                               const double* __restrict__ Pin, int n, int full,
                                               const int c[3], const int pc[3], int l,
                                               double* u) {
  constexpr int NV = D + 2;
  bool inside = true;
  for (int j = 0; j < D; ++j) inside &= (c[j] >= 0 && c[j] < n);
  if (FUSE && !inside) {
    int g[3] = {0, 0, 0};
    for (int j = 0; j < D; ++j) g[j] = bc_map(pc[j] * n + c[j], m.lv[l].cells, m.periodic[j]);
    if (fetch_cell<D>(m, Uin, l, g, u)) return;
    // no same-level source: the prolonged ghost value was written into the
    // patch's own ghost layer by the coarse-ghost fill pass
  }
  const long long vs = var_stride<D>(full);
  const long long off = box_off<D>(full, c[0] + NG, c[1] + NG, c[2] + NG);
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Pin[v * vs + off];
}

// 1D/2D: primitives of the tile plus 4-node halos in every direction
// (corner nodes, used by no stencil, are skipped), loaded once per launch.
template <int D, int TX, int TY, int NT, bool FUSE>
__device__ __forceinline__ void load_union(const DevMesh& m, const double* __restrict__ Uin,
                                           const double* __restrict__ Pin, int n, int full,
                                           const int o[3], const int pc[3], int l, double* sP) {
  constexpr int T0 = TX, T1 = D >= 2 ? TY : 1;
  constexpr int U0 = T0 + 8, U1 = D >= 2 ? T1 + 8 : 1;
  constexpr int NU = U0 * U1;
  constexpr int NQ = D + 2;
  for (int idx = threadIdx.x; idx < NU; idx += NT) {
    const int e0 = idx % U0, e1 = idx / U0;
    const bool hx = e0 < 4 || e0 >= T0 + 4;
    const bool hy = D >= 2 && (e1 < 4 || e1 >= T1 + 4);
    if (hx && hy) continue;
    const int c[3] = {o[0] + e0 - 4, D >= 2 ? o[1] + e1 - 4 : 0, 0};
    double u[D + 2], q[NQ];
    node_conserved<D, FUSE>(m, Uin, Pin, n, full, c, pc, l, u);
    node_primitives<D>(m, u, q);
#pragma unroll
    for (int k = 0; k < NQ; ++k) sP[k * NU + idx] = q[k];
  }
}

template <int D, int TX, int TY, int TZ, int NT, int J, bool FUSE, bool UNION>
__device__ __forceinline__ void stage_direction(const DevMesh& m, const double* __restrict__ Uin,
                                                const double* __restrict__ Pin,
                                                double* __restrict__ frp, int n, int full,
                                                const int o[3], const int pc[3], int l,
                                                double* sP, double* sF,
                                                double acc[][D + 2], double inv_h) {
  using S = TileShape<D, TX, TY, TZ>;
  constexpr int NV = D + 2;
  constexpr int NQ = D + 2;  // interpolated primitives: p, T, u_j
  constexpr int E0 = UNION ? S::T0 + 8 : S::T0 + (J == 0 ? 8 : 0);
  constexpr int E1 = UNION ? (D >= 2 ? S::T1 + 8 : 1) : S::T1 + (J == 1 ? 8 : 0);
  constexpr int E2 = UNION ? 1 : S::T2 + (J == 2 ? 8 : 0);
  constexpr int NEXT = E0 * E1 * E2;
  constexpr int G0 = S::T0 + (J == 0 ? 3 : 0);
  constexpr int G1 = S::T1 + (J == 1 ? 3 : 0);
  constexpr int G2 = S::T2 + (J == 2 ? 3 : 0);
  constexpr int NED = G0 * G1 * G2;
  constexpr int STEP = J == 0 ? 1 : (J == 1 ? E0 : E0 * E1);
  constexpr int CPT = (S::NCELL + NT - 1) / NT;
  const int tid = threadIdx.x;

  // 1. primitives of the tile extended by 4 nodes on both sides along J
  // (the union layout is loaded once by the caller for all directions)
  if constexpr (!UNION) {
    for (int idx = tid; idx < NEXT; idx += NT) {
      const int e0 = idx % E0;
      const int e1 = (idx / E0) % E1;
      const int e2 = idx / (E0 * E1);
      const int c[3] = {o[0] + e0 - (J == 0 ? 4 : 0), o[1] + e1 - (J == 1 ? 4 : 0),
                        o[2] + e2 - (J == 2 ? 4 : 0)};
      double u[NV], q[NQ];
      node_conserved<D, FUSE>(m, Uin, Pin, n, full, c, pc, l, u);
      node_primitives<D>(m, u, q);
#pragma unroll
      for (int k = 0; k < NQ; ++k) sP[k * NEXT + idx] = q[k];
    }
    __syncthreads();
  }

  // 2. Riemann flux at every edge i+1/2, i = o_J-2 .. o_J+T_J
  for (int e = tid; e < NED; e += NT) {
    const int a0 = e % G0;
    const int a1 = (e / G0) % G1;
    const int a2 = e / (G0 * G1);
    // layout index of node i-2 of this edge's window
    int base;
    if constexpr (!UNION) base = a0 + E0 * (a1 + E1 * a2);
    else if constexpr (J == 0) base = (D >= 2 ? (a1 + 4) * E0 : 0) + a0;
    else base = a1 * E0 + (a0 + 4);
    EdgeState<D> wl, wr;
    double lo[NQ], hi[NQ], lv[NQ], rv[NQ];
    const double eps4 = 4.0 * m.eps;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double* col = sP + q * NEXT + base;
      const double v0 = col[0], v1 = col[STEP], v2 = col[2 * STEP];
      const double v3 = col[3 * STEP], v4 = col[4 * STEP], v5 = col[5 * STEP];
      if (m.scheme == AMR_SCHEME_CENTRAL) {
        lv[q] = central4(v1, v2, v3, v4);
        rv[q] = lv[q];
      } else {
        weno5_pair(v0, v1, v2, v3, v4, v5, eps4, lv[q], rv[q]);
      }
      lo[q] = v2;
      hi[q] = v3;
    }
    const bool ok = (lv[0] > 0.0) && (lv[1] > 0.0) && (rv[0] > 0.0) && (rv[1] > 0.0);
    wl.p = ok ? lv[0] : lo[0];
    wl.T = ok ? lv[1] : lo[1];
    wr.p = ok ? rv[0] : hi[0];
    wr.T = ok ? rv[1] : hi[1];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      wl.u[i] = ok ? lv[2 + i] : lo[2 + i];
      wr.u[i] = ok ? rv[2 + i] : hi[2 + i];
    }
    double UL[NV], FL[NV], UR[NV], FR[NV], sl, sr;
    edge_flux<D, J>(m, wl, UL, FL, sl);
    edge_flux<D, J>(m, wr, UR, FR, sr);
    const double S = fmax(sr, sl);
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[v * NED + e] = fma(-S, UR[v] - UL[v], FR[v] + FL[v]);
  }
  __syncthreads();

  // 3. face fluxes G (flux form of Eq. (9)) and their divergence
  const int nface = (D == 1) ? 1 : (D == 2 ? n : n * n);
  constexpr double c24 = 1.0 / 24.0;
  const double half_inv_h = 0.5 * inv_h;
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int cell = tid + cc * NT;
    if (cell >= S::NCELL) break;
    const int t0 = cell % S::T0;
    const int t1 = (cell / S::T0) % S::T1;
    const int t2 = cell / (S::T0 * S::T1);
    const int tj = J == 0 ? t0 : (J == 1 ? t1 : t2);
    // edge-array index of edge (t_J - 2 + k) + 1/2 in the edge box
    int eb;
    constexpr int ESTEP = J == 0 ? 1 : (J == 1 ? G0 : G0 * G1);
    if constexpr (J == 0) eb = G0 * (t1 + G1 * t2);
    else if constexpr (J == 1) eb = t0 + G0 * G1 * t2;
    else eb = t0 + G0 * t1;
    eb += tj * ESTEP;
    const int i = o[J] + tj;
    int tang = 0;
    if constexpr (D == 2) tang = (J == 0) ? (o[1] + t1) : (o[0] + t0);
    if constexpr (D == 3) {
      if constexpr (J == 0) tang = (o[1] + t1) + n * (o[2] + t2);
      else if constexpr (J == 1) tang = (o[0] + t0) + n * (o[2] + t2);
      else tang = (o[0] + t0) + n * (o[1] + t1);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      // edge fluxes are stored doubled (the Rusanov 1/2 is applied here, as
      // 1/2 inv_h, and to the boundary faces; power-of-two scaling is exact)
      const double* F = sF + v * NED + eb;
      const double Fm2 = F[0], Fm1 = F[ESTEP], F0 = F[2 * ESTEP], Fp1 = F[3 * ESTEP];
      const double Gp = fma(-c24, fma(-2.0, F0, Fm1) + Fp1, F0);
      const double Gm = fma(-c24, fma(-2.0, Fm1, Fm2) + F0, Fm1);
      acc[cc][v] = fma(-(Gp - Gm), half_inv_h, acc[cc][v]);
      if (i == 0) frp[((J * 2 + 0) * NV + v) * nface + tang] = 0.5 * Gm;
      if (i == n - 1) frp[((J * 2 + 1) * NV + v) * nface + tang] = 0.5 * Gp;
    }
  }
  __syncthreads();
}

template <int D, int TX, int TY, int TZ, int NT, bool FUSE>
__global__ __launch_bounds__(NT) void k_stage(DevMesh m, int mode, const double* __restrict__ Uin,
                                              const double* Un, double* out,
                                              double* __restrict__ fr,
                                              const int* __restrict__ tiles, int count,
                                              const double* __restrict__ dtp,
                                              unsigned long long* __restrict__ lam_next,
                                              const uint8_t* __restrict__ cfmask) {
  using S = TileShape<D, TX, TY, TZ>;
  constexpr int NV = D + 2;
  constexpr int CPT = (S::NCELL + NT - 1) / NT;
  constexpr bool UNION = D <= 2;
  constexpr int NU = (S::T0 + 8) * (D >= 2 ? S::T1 + 8 : 1);
  __shared__ double sP[(D + 2) * (UNION ? NU : S::EXTMAX)];
  __shared__ double sF[(D + 2) * S::EDMAX];
  const int item = xcd_item(count);
  if (item >= count) return;
  const int pid = tiles[2 * item];
  const int tix = tiles[2 * item + 1];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, full = L.full;
  const int nt0 = n / S::T0, nt1 = n / S::T1;
  const int o[3] = {(tix % nt0) * S::T0, ((tix / nt0) % nt1) * S::T1, (tix / (nt0 * nt1)) * S::T2};
  const long long base = patch_base(m, pid, l);
  const double* Pin = Uin + base;
  double* frp = fr + L.fr_off + (long long)(pid - L.pid_base) * L.fr_stride;
  double acc[CPT][NV];
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[cc][v] = 0.0;

  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  if constexpr (UNION) {
    load_union<D, TX, TY, NT, FUSE>(m, Uin, Pin, n, full, o, pc, l, sP);
    __syncthreads();
  }
  stage_direction<D, TX, TY, TZ, NT, 0, FUSE, UNION>(m, Uin, Pin, frp, n, full, o, pc, l, sP, sF,
                                                     acc, L.inv_h);
  if constexpr (D >= 2)
    stage_direction<D, TX, TY, TZ, NT, 1, FUSE, UNION>(m, Uin, Pin, frp, n, full, o, pc, l, sP,
                                                       sF, acc, L.inv_h);
  if constexpr (D >= 3)
    stage_direction<D, TX, TY, TZ, NT, 2, FUSE, UNION>(m, Uin, Pin, frp, n, full, o, pc, l, sP,
                                                       sF, acc, L.inv_h);

  const long long vs = var_stride<D>(full);
  const double dt = (mode == kModeRHS) ? 0.0 : dtp[0];
  constexpr double c23 = 2.0 / 3.0;
  // next step's CFL rate from the final leaf values; cells on coarse/fine
  // faces are left to the flux-correction kernel, which changes them
  const bool want_rate = lam_next != nullptr && mode == kModeStage3;
  const int fmask = want_rate ? cfmask[pid] : 0;
  unsigned long long best = 0ull;
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int cell = threadIdx.x + cc * NT;
    if (cell >= S::NCELL) break;
    const int t0 = cell % S::T0;
    const int t1 = (cell / S::T0) % S::T1;
    const int t2 = cell / (S::T0 * S::T1);
    const long long off = base + box_off<D>(full, o[0] + t0 + NG, o[1] + t1 + NG, o[2] + t2 + NG);
    double r[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long a = off + v * vs;
      const double Lv = acc[cc][v];
      if (mode == kModeRHS) {
        r[v] = Lv;
      } else if (mode == kModeStage1) {
        r[v] = fma(dt, Lv, Un[a]);
      } else {
        const double un = Un[a];
        const double ui = Uin[a];
        r[v] = fma(mode == kModeStage2 ? 0.25 : c23, fma(dt, Lv, ui) - un, un);
      }
      out[a] = r[v];
    }
    if (want_rate) {
      const int c3[3] = {o[0] + t0, o[1] + t1, o[2] + t2};
      bool on_cf = false;
      for (int j = 0; j < D; ++j)
        on_cf |= ((fmask >> (2 * j)) & 1) && c3[j] == 0 || ((fmask >> (2 * j + 1)) & 1) && c3[j] == n - 1;
      if (!on_cf) {
        const unsigned long long bits = cell_rate_bits<D>(r, m, L.h);
        best = bits > best ? bits : best;
      }
    }
  }
  if (want_rate) block_max_atomic(best, lam_next);
}

// ---------------------------------------------------------------------------
// coarse/fine flux correction: list of (pid, face mask); faces are processed
// in the order x-, x+, y-, y+, z-, z+ so that corner cells see a fixed order
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_reflux(DevMesh m, int mode, double* __restrict__ out,
                                                const double* __restrict__ fr,
                                                const int* __restrict__ list, int count,
                                                const double* __restrict__ dtp, double w,
                                                unsigned long long* __restrict__ lam_next) {
  constexpr int NV = D + 2;
  if ((int)blockIdx.x >= count) return;
  const int pid = list[2 * blockIdx.x];
  const int mask = list[2 * blockIdx.x + 1];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const LevelC& Fv = m.lv[l + 1];
  const int n = L.n, nf = Fv.n, Nf = Fv.cells;
  const int nface = (D == 1) ? 1 : (D == 2 ? n : n * n);
  const int nfface = (D == 1) ? 1 : (D == 2 ? nf : nf * nf);
  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  const double* frc = fr + L.fr_off + (long long)(pid - L.pid_base) * L.fr_stride;
  double* P = out + patch_base(m, pid, l);
  const long long vs = var_stride<D>(L.full);
  const double coef = (mode == kModeRHS) ? L.inv_h : (w * dtp[0]) * L.inv_h;
  for (int f = 0; f < 2 * D; ++f) {
    if (mask & (1 << f)) {
      const int j = f >> 1, side = f & 1;
      int tdim[2] = {0, 0}, nt = 0;
      for (int k = 0; k < D; ++k)
        if (k != j) tdim[nt++] = k;
      int F = 2 * (pc[j] * n + (side ? n : 0));
      int cj;
      if (side) {
        F %= Nf;
        cj = F;
      } else {
        if (F == 0) F = Nf;
        cj = F - 1;
      }
      const int fside = side ? 0 : 1;
      for (int t = threadIdx.x; t < nface; t += blockDim.x) {
        int tl[2] = {0, 0};
        if constexpr (D >= 2) tl[0] = t % n;
        if constexpr (D >= 3) tl[1] = t / n;
        double sub[4][NV];
        const int nsub = 1 << (D - 1);
        bool ok = true;
        for (int s = 0; s < nsub; ++s) {
          int q[3] = {0, 0, 0}, fl[2] = {0, 0};
          q[j] = cj / nf;
          for (int k = 0; k < D - 1; ++k) {
            const int gfc = 2 * (pc[tdim[k]] * n + tl[k]) + ((s >> k) & 1);
            q[tdim[k]] = gfc / nf;
            fl[k] = gfc - q[tdim[k]] * nf;
          }
          const int fpid = map_at<D>(m, l + 1, q);
          if (fpid < 0) {
            ok = false;
            break;
          }
          const double* frf = fr + Fv.fr_off + (long long)(fpid - Fv.pid_base) * Fv.fr_stride;
          const int ft = fl[0] + nf * fl[1];
#pragma unroll
          for (int v = 0; v < NV; ++v) sub[s][v] = frf[((j * 2 + fside) * NV + v) * nfface + ft];
        }
        int c[3] = {0, 0, 0};
        c[j] = side ? n - 1 : 0;
        for (int k = 0; k < D - 1; ++k) c[tdim[k]] = tl[k];
        const long long off = box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG);
        const double sgn = side ? 1.0 : -1.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double avg;
          if constexpr (D == 1) avg = sub[0][v];
          else if constexpr (D == 2) avg = (sub[0][v] + sub[1][v]) * 0.5;
          else avg = ((sub[0][v] + sub[1][v]) + (sub[2][v] + sub[3][v])) * 0.25;
          if (!ok) avg = __builtin_nan("");
          const double gc = frc[((j * 2 + side) * NV + v) * nface + t];
          P[v * vs + off] = fma(coef, sgn * (gc - avg), P[v * vs + off]);
        }
      }
    }
    __syncthreads();
  }
  if (lam_next == nullptr || mode != kModeStage3) return;
  // CFL rate of every corrected cell, from its final value
  unsigned long long best = 0ull;
  for (int f = 0; f < 2 * D; ++f) {
    if (!(mask & (1 << f))) continue;
    const int j = f >> 1, side = f & 1;
    int tdim[2] = {0, 0}, nt = 0;
    for (int k = 0; k < D; ++k)
      if (k != j) tdim[nt++] = k;
    for (int t = threadIdx.x; t < nface; t += blockDim.x) {
      int c[3] = {0, 0, 0};
      c[j] = side ? n - 1 : 0;
      if constexpr (D >= 2) c[tdim[0]] = t % n;
      if constexpr (D >= 3) c[tdim[1]] = t / n;
      const long long off = box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG);
      double u[NV];
      for (int v = 0; v < NV; ++v) u[v] = P[v * vs + off];
      const unsigned long long bits = cell_rate_bits<D>(u, m, L.h);
      best = bits > best ? bits : best;
    }
  }
  block_max_atomic(best, lam_next);
}

// ---------------------------------------------------------------------------
// restriction of one level: list of child pids; pairwise sums in x-fastest
// child order, times 2^-D
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_restrict(DevMesh m, double* __restrict__ U,
                                                  const int* __restrict__ list, int count) {
  constexpr int NV = D + 2;
  if ((int)blockIdx.x >= count) return;
  const int cpid = list[blockIdx.x];
  const int lf = m.level[cpid];
  const int ppid = m.parent[cpid];
  const LevelC& F = m.lv[lf];
  const LevelC& C = m.lv[lf - 1];
  const int h = F.n / 2;
  int o[3] = {0, 0, 0};
  for (int j = 0; j < D; ++j) o[j] = m.coord[3 * cpid + j] * h - m.coord[3 * ppid + j] * C.n;
  const double* Pc = U + patch_base(m, cpid, lf);
  double* Pp = U + patch_base(m, ppid, lf - 1);
  const long long vsf = var_stride<D>(F.full), vsc = var_stride<D>(C.full);
  int total = h;
  if constexpr (D >= 2) total *= h;
  if constexpr (D >= 3) total *= h;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int a = idx % h;
    const int b = D >= 2 ? (idx / h) % h : 0;
    const int c = D >= 3 ? idx / (h * h) : 0;
    const long long dst = box_off<D>(C.full, o[0] + a + NG, o[1] + b + NG, o[2] + c + NG);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double* S = Pc + v * vsf;
      auto at = [&](int x, int y, int z) {
        return S[box_off<D>(F.full, 2 * a + x + NG, 2 * b + y + NG, 2 * c + z + NG)];
      };
      double r;
      if constexpr (D == 1) r = (at(0, 0, 0) + at(1, 0, 0)) * 0.5;
      else if constexpr (D == 2)
        r = ((at(0, 0, 0) + at(1, 0, 0)) + (at(0, 1, 0) + at(1, 1, 0))) * 0.25;
      else
        r = (((at(0, 0, 0) + at(1, 0, 0)) + (at(0, 1, 0) + at(1, 1, 0))) +
             ((at(0, 0, 1) + at(1, 0, 1)) + (at(0, 1, 1) + at(1, 1, 1)))) * 0.125;
      Pp[v * vsc + dst] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// CFL rate: max over leaf cells of sum_j (|u_j| + c) / h, as IEEE bits of a
// non-negative double (order-preserving), reduced with a wave shuffle, LDS and
// one 64-bit atomic max per block
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_max_rate(DevMesh m, const double* __restrict__ U,
                                                  const int* __restrict__ list, int count,
                                                  unsigned long long* __restrict__ lam) {
  constexpr int NV = D + 2;
  unsigned long long best = 0ull;
  if ((int)blockIdx.x < count) {
    const int pid = list[blockIdx.x];
    const int l = m.level[pid];
    const LevelC& L = m.lv[l];
    const int n = L.n;
    const double* P = U + patch_base(m, pid, l);
    const long long vs = var_stride<D>(L.full);
    int total = n;
    if constexpr (D >= 2) total *= n;
    if constexpr (D >= 3) total *= n;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int x = idx % n;
      const int y = D >= 2 ? (idx / n) % n : 0;
      const int z = D >= 3 ? idx / (n * n) : 0;
      const long long off = box_off<D>(L.full, x + NG, y + NG, z + NG);
      double u[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = P[v * vs + off];
      const unsigned long long bits = cell_rate_bits<D>(u, m, L.h);
      best = bits > best ? bits : best;
    }
  }
  block_max_atomic(best, lam);
}

__global__ void k_zero_u64(unsigned long long* p) { p[0] = 0ull; }

__global__ void k_dt_from_rate(const unsigned long long* __restrict__ lam, double cfl,
                               double* __restrict__ dt, unsigned long long* __restrict__ clear) {
  dt[0] = cfl / __longlong_as_double((long long)lam[0]);
  if (clear) clear[0] = 0ull;
}

// ---------------------------------------------------------------------------
// tagging: per leaf, any cell within tag_buffer of the interior with
// |phi+ - phi-| > theta (|phi+| + |phi-|) for phi in {rho, p}, any direction
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void rho_p_at(const DevMesh& m, const double* P, long long vs,
                                         long long off, double& rho, double& p) {
  double u[D + 2];
#pragma unroll
  for (int v = 0; v < D + 2; ++v) u[v] = P[v * vs + off];
  rho = u[0];
  p = pressure_exact<D>(u, m.gm1);
}

template <int D>
__global__ __launch_bounds__(256) void k_tag(DevMesh m, const double* __restrict__ U,
                                             const int* __restrict__ list, int count,
                                             uint8_t* __restrict__ has_tag,
                                             uint8_t* __restrict__ raw) {
  if ((int)blockIdx.x >= count) return;
  const int pid = list[blockIdx.x];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, b = m.tag_buffer, w = n + 2 * b;
  const double* P = U + patch_base(m, pid, l);
  const long long vs = var_stride<D>(L.full);
  int total = w;
  if constexpr (D >= 2) total *= w;
  if constexpr (D >= 3) total *= w;
  int any = 0;
  uint8_t* rp = raw ? raw + L.tag_off + (long long)(pid - L.pid_base) * vs : nullptr;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int c[3] = {idx % w - b, 0, 0};
    if constexpr (D >= 2) c[1] = (idx / w) % w - b;
    if constexpr (D >= 3) c[2] = idx / (w * w) - b;
    bool t = false;
    for (int j = 0; j < D; ++j) {
      int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
      cp[j] += 1;
      cm[j] -= 1;
      double rp_, pp_, rm_, pm_;
      rho_p_at<D>(m, P, vs, box_off<D>(L.full, cp[0] + NG, cp[1] + NG, cp[2] + NG), rp_, pp_);
      rho_p_at<D>(m, P, vs, box_off<D>(L.full, cm[0] + NG, cm[1] + NG, cm[2] + NG), rm_, pm_);
      t |= fabs(rp_ - rm_) > m.theta * (fabs(rp_) + fabs(rm_));
      t |= fabs(pp_ - pm_) > m.theta * (fabs(pp_) + fabs(pm_));
    }
    any |= t;
    if (rp) rp[box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG)] = t ? 1 : 0;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) has_tag[pid] = any ? 1 : 0;
}

template <int D>
__global__ __launch_bounds__(256) void k_cell_tags(DevMesh m, const uint8_t* __restrict__ raw,
                                                   const int* __restrict__ list, int count,
                                                   uint8_t* __restrict__ out) {
  if ((int)blockIdx.x >= count) return;
  const int pid = list[blockIdx.x];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, b = m.tag_buffer;
  const long long vs = var_stride<D>(L.full);
  const uint8_t* rp = raw + L.tag_off + (long long)(pid - L.pid_base) * vs;
  uint8_t* op = out + L.tag_off + (long long)(pid - L.pid_base) * vs;
  int total = n;
  if constexpr (D >= 2) total *= n;
  if constexpr (D >= 3) total *= n;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int x = idx % n;
    const int y = D >= 2 ? (idx / n) % n : 0;
    const int z = D >= 3 ? idx / (n * n) : 0;
    int t = 0;
    for (int dz = (D >= 3 ? -b : 0); dz <= (D >= 3 ? b : 0); ++dz)
      for (int dy = (D >= 2 ? -b : 0); dy <= (D >= 2 ? b : 0); ++dy)
        for (int dx = -b; dx <= b; ++dx)
          t |= rp[box_off<D>(L.full, x + dx + NG, y + dy + NG, z + dz + NG)];
    op[box_off<D>(L.full, x + NG, y + NG, z + NG)] = t ? 1 : 0;
  }
}

// refine request: active leaf below the finest level with a tag;
// coarsen request: patch whose children are all leaves without tags
__global__ void k_requests(DevMesh m, const uint8_t* __restrict__ has_tag,
                           const uint8_t* __restrict__ active_leaf, int nslots,
                           uint8_t* __restrict__ refine, uint8_t* __restrict__ coarsen) {
  const int pid = blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= nslots) return;
  const uint8_t al = active_leaf[pid];  // 0 inactive, 1 leaf, 2 non-leaf
  uint8_t rq = 0, cq = 0;
  if (al == 1) {
    rq = (has_tag[pid] && m.level[pid] < m.nlev - 1) ? 1 : 0;
  } else if (al == 2) {
    // a coarsening candidate (all children leaves) was tagged on its own
    // restricted data as well; it is coarsened only if that is untagged too
    cq = has_tag[pid] ? 0 : 1;
    const int nc = m.nchild[pid];
    for (int k = 0; k < nc; ++k) {
      const int c = m.child[(long long)pid * m.maxc + k];
      if (active_leaf[c] != 1 || has_tag[c]) {
        cq = 0;
        break;
      }
    }
  }
  if (refine) refine[pid] = rq;
  if (coarsen) coarsen[pid] = cq;
}

// prolongation of the interiors of newly created patches of one level
template <int D>
__global__ __launch_bounds__(256) void k_prolong_new(DevMesh m, double* __restrict__ U,
                                                     const int* __restrict__ list, int count,
                                                     int* __restrict__ err) {
  constexpr int NV = D + 2;
  if ((int)blockIdx.x >= count) return;
  const int pid = list[blockIdx.x];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n;
  double* P = U + patch_base(m, pid, l);
  const long long vs = var_stride<D>(L.full);
  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  int total = n;
  if constexpr (D >= 2) total *= n;
  if constexpr (D >= 3) total *= n;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int c[3] = {idx % n, 0, 0};
    if constexpr (D >= 2) c[1] = (idx / n) % n;
    if constexpr (D >= 3) c[2] = idx / (n * n);
    int g[3] = {0, 0, 0};
    for (int j = 0; j < D; ++j) g[j] = pc[j] * n + c[j];
    double val[NV];
    if (!prolong_cell<D>(m, U, l, g, val)) {
      err[0] = 1;
      for (int v = 0; v < NV; ++v) val[v] = __builtin_nan("");
    }
    const long long off = box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG);
#pragma unroll
    for (int v = 0; v < NV; ++v) P[v * vs + off] = val[v];
  }
}

__global__ void k_count_nonzero(const uint8_t* __restrict__ a, int n, int* __restrict__ out) {
  int c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    c += a[i] ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__global__ void k_scatter_int(int* __restrict__ dst, const int* __restrict__ pairs, int npairs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npairs) dst[pairs[2 * i]] = pairs[2 * i + 1];
}

template <int D>
__global__ __launch_bounds__(256) void k_check(DevMesh m, const double* __restrict__ U,
                                               const int* __restrict__ list, int count,
                                               int* __restrict__ bad) {
  constexpr int NV = D + 2;
  if ((int)blockIdx.x >= count) return;
  const int pid = list[blockIdx.x];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n;
  const double* P = U + patch_base(m, pid, l);
  const long long vs = var_stride<D>(L.full);
  int total = n;
  if constexpr (D >= 2) total *= n;
  if constexpr (D >= 3) total *= n;
  int cnt = 0;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int x = idx % n;
    const int y = D >= 2 ? (idx / n) % n : 0;
    const int z = D >= 3 ? idx / (n * n) : 0;
    double u[NV];
    const long long off = box_off<D>(L.full, x + NG, y + NG, z + NG);
    for (int v = 0; v < NV; ++v) u[v] = P[v * vs + off];
    const double p = pressure_exact<D>(u, m.gm1);
    if (!(u[0] > 0.0 && p > 0.0)) ++cnt;
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(bad, cnt);
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
#define AMR_DISPATCH_DIM(dim, KERNEL, GRID, BLOCK, STREAM, ...)                         \
  do {                                                                                  \
    if ((dim) == 1) hipLaunchKernelGGL(KERNEL<1>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); \
    else if ((dim) == 2) hipLaunchKernelGGL(KERNEL<2>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); \
    else hipLaunchKernelGGL(KERNEL<3>, GRID, BLOCK, 0, STREAM, __VA_ARGS__);             \
  } while (0)

void Kernels::fill_cf(const DevMesh& m, double* U, const int* list, int count, int* err,
                      hipStream_t s) {
  if (count <= 0) return;
  switch (m.dim) {
    case 1: k_fill_cf<1, 64><<<count, 64, 0, s>>>(m, U, list, count, err); break;
    case 2: k_fill_cf<2, 64><<<count, 64, 0, s>>>(m, U, list, count, err); break;
    default: k_fill_cf<3, 256><<<count, 256, 0, s>>>(m, U, list, count, err); break;
  }
}

void Kernels::fill(const DevMesh& m, double* U, const int* list, int count, int* err,
                   bool coarse_only, hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_fill, dim3(count), dim3(256), s, m, U, list, count, err,
                   coarse_only ? 1 : 0);
}

// Stage-kernel tile variants: thread counts cover the edges of one
// direction of the tile in one pass (multiples of 64).
static const Kernels::TileVariant kVariants[] = {
    {1, 16, 1, 1, 64}, {1, 8, 1, 1, 64},                                   // 1D
    {2, 16, 16, 1, 320}, {2, 16, 8, 1, 192}, {2, 8, 8, 1, 128},           // 2D
    {3, 8, 8, 8, 704}, {3, 8, 8, 4, 448}, {3, 4, 4, 4, 128},              // 3D
};

int Kernels::num_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

Kernels::TileVariant Kernels::variant(int v) { return kVariants[v]; }

bool Kernels::variant_fits(int v, int dim, const int* n, int nlev) {
  if (v < 0 || v >= num_variants() || kVariants[v].dim != dim) return false;
  const TileVariant& t = kVariants[v];
  for (int l = 0; l < nlev; ++l) {
    if (n[l] % t.tx) return false;
    if (dim >= 2 && n[l] % t.ty) return false;
    if (dim >= 3 && n[l] % t.tz) return false;
  }
  return true;
}

int Kernels::default_variant(int dim, const int* n, int nlev) {
  for (int v = 0; v < num_variants(); ++v)
    if (variant_fits(v, dim, n, nlev)) return v;
  return -1;
}

int Kernels::tiles_per_patch(int v, int n) {
  const TileVariant& t = kVariants[v];
  int r = n / t.tx;
  if (t.dim >= 2) r *= n / t.ty;
  if (t.dim >= 3) r *= n / t.tz;
  return r;
}

void Kernels::stage(const DevMesh& m, int mode, const double* Uin, const double* Un,
                    double* out, double* fr, const int* tiles, int count, const double* dt,
                    bool fuse, unsigned long long* lam_next, const uint8_t* cfmask,
                    hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (count <= 0) return;
  // one block per work item, rounded up to whole groups of kXcds blocks (see
  // xcd_item)
  const int nb = ((count + kXcds - 1) / kXcds) * kXcds;
#define AMR_STAGE_F(D, TX, TY, TZ, NT, F)                                                   \
  do {                                                                                      \
    if (ev0)                                                                                \
      hipExtLaunchKernelGGL((k_stage<D, TX, TY, TZ, NT, F>), dim3(nb), dim3(NT), 0, s, ev0,  \
                            ev1, 0, m, mode, Uin, Un, out, fr, tiles, count, dt, lam_next,  \
                            cfmask);                                                        \
    else                                                                                    \
      hipLaunchKernelGGL((k_stage<D, TX, TY, TZ, NT, F>), dim3(nb), dim3(NT), 0, s, m, mode, \
                         Uin, Un, out, fr, tiles, count, dt, lam_next, cfmask);             \
  } while (0)
#define AMR_STAGE(D, TX, TY, TZ, NT)        \
  do {                                      \
    if (fuse)                               \
      AMR_STAGE_F(D, TX, TY, TZ, NT, true); \
    else                                    \
      AMR_STAGE_F(D, TX, TY, TZ, NT, false);\
  } while (0)
  switch (m.tile) {
    case 0: AMR_STAGE(1, 16, 1, 1, 64); break;
    case 1: AMR_STAGE(1, 8, 1, 1, 64); break;
    case 2: AMR_STAGE(2, 16, 16, 1, 320); break;
    case 3: AMR_STAGE(2, 16, 8, 1, 192); break;
    case 4: AMR_STAGE(2, 8, 8, 1, 128); break;
    case 5: AMR_STAGE(3, 8, 8, 8, 704); break;
    case 6: AMR_STAGE(3, 8, 8, 4, 448); break;
    default: AMR_STAGE(3, 4, 4, 4, 128); break;
  }
#undef AMR_STAGE
#undef AMR_STAGE_F
}

void Kernels::reflux(const DevMesh& m, int mode, double* out, const double* fr,
                     const int* list, int count, const double* dt, double w,
                     unsigned long long* lam_next, hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_reflux, dim3(count), dim3(256), s, m, mode, out, fr, list, count,
                   dt, w, lam_next);
}

void Kernels::restrict_level(const DevMesh& m, double* U, const int* list, int count,
                             hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_restrict, dim3(count), dim3(256), s, m, U, list, count);
}

void Kernels::max_rate(const DevMesh& m, const double* U, const int* list, int count,
                       unsigned long long* lam, hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_max_rate, dim3(count), dim3(256), s, m, U, list, count, lam);
}

void Kernels::zero_u64(unsigned long long* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, p);
}

void Kernels::dt_from_rate(const DevMesh& m, const unsigned long long* lam, double* dt,
                           unsigned long long* clear, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_from_rate, dim3(1), dim3(1), 0, s, lam, m.cfl, dt, clear);
}

void Kernels::tag(const DevMesh& m, const double* U, const int* list, int count,
                  uint8_t* has_tag, uint8_t* raw, hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_tag, dim3(count), dim3(256), s, m, U, list, count, has_tag, raw);
}

void Kernels::cell_tags(const DevMesh& m, const uint8_t* raw, const int* list, int count,
                        uint8_t* out, hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_cell_tags, dim3(count), dim3(256), s, m, raw, list, count, out);
}

void Kernels::requests(const DevMesh& m, const uint8_t* has_tag, const uint8_t* active_leaf,
                       int nslots, uint8_t* refine, uint8_t* coarsen, hipStream_t s) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_requests, dim3((nslots + 255) / 256), dim3(256), 0, s, m, has_tag,
                     active_leaf, nslots, refine, coarsen);
}

void Kernels::prolong_new(const DevMesh& m, double* U, const int* list, int count, int* err,
                          hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_prolong_new, dim3(count), dim3(256), s, m, U, list, count, err);
}

void Kernels::count_nonzero(const uint8_t* a, int n, int* out, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = std::min(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_count_nonzero, dim3(blocks), dim3(256), 0, s, a, n, out);
}

void Kernels::scatter_int(int* dst, const int* pairs, int npairs, hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_scatter_int, dim3((npairs + 255) / 256), dim3(256), 0, s, dst, pairs,
                     npairs);
}

void Kernels::check(const DevMesh& m, const double* U, const int* list, int count, int* bad,
                    hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_check, dim3(count), dim3(256), s, m, U, list, count, bad);
}

}  // namespace amr
