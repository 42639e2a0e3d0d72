// HIP kernels of libamr for gfx950 (CDNA4, wave64), except the fused stage
// kernel (stage.hip): ghost fill, refluxing, restriction, CFL rate, tagging,
// prolongation of new patches, checks.
//
// Every kernel works on the patch pools described in amr_internal.hpp: a
// patch of level l stores nvar * (n_l + 8)^dim doubles, var-major, x fastest,
// with 4 ghost layers.  Work lists (pids or (pid, tile) pairs) are device
// arrays built by the host after each regrid, so one launch covers the
// patches of every level.
//
// Floating-point contract: implicit contraction is disabled; the refluxing
// correction writes its fused multiply-add out with fma().  The
// prolongation, restriction, tag and time-step paths use the operation order
// of the definitions they implement (no fma), so that integer decisions (tags,
// positivity switches) are taken on the same values as the FP64 reference.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <stdexcept>

#include "amr_internal.hpp"

// no implicit contraction anywhere in this file (see the header comment)
#pragma clang fp contract(off)

#include "device_common.hpp"

namespace amr {
namespace {

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
  const int vs = var_stride<D>(full);
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
__device__ __forceinline__ void fill_cf_region(const DevMesh& m, double* __restrict__ U,
                                               const int* __restrict__ list, int item,
                                               int* __restrict__ err) {
  constexpr int NV = D + 2;
  const int pid = list[2 * item];
  const int code = list[2 * item + 1];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, full = L.full;
  const int vs = var_stride<D>(full);
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
    const int off = box_off<D>(full, c[0] + NG, c[1] + NG, c[2] + NG);
#pragma unroll
    for (int v = 0; v < NV; ++v) P[v * vs + off] = val[v];
  }
}

// One block per region.  With `dir` (batched launches) the list is
// list + dir[0] and the count dir[1], read at run time (the grid may hold
// more blocks than regions).
template <int D, int NT>
__global__ __launch_bounds__(NT) void k_fill_cf(DevMesh m,
                                                double* __restrict__ U,
                                                const int* __restrict__ list, int count,
                                                const int* __restrict__ dir,
                                                int* __restrict__ err) {
  if (dir) {
    list += dir[0];
    count = dir[1];
  }
  if ((int)blockIdx.x < count) fill_cf_region<D, NT>(m, U, list, blockIdx.x, err);
}

// The same regions by coarse cell (2D and 3D).  A region's start and extent
// are even in every dimension, so its fine cells come in aligned blocks of
// 2^D, and both cells of an aligned pair have the same coarse cell also
// after the boundary mapping (a periodic wrap of an even cell count keeps
// pairs together; the clamp sends a whole out-of-domain pair to one edge
// cell).  One thread computes the coarse stencil, the MC slopes and the
// positivity test once and forms each of the 2^D fine values as
// prolong_cell does, in the same operation order, so the values are bitwise
// those of the per-fine-cell fill.  A block takes G consecutive regions and
// spreads all their coarse cells over its lanes: a 3D region covers as few
// as 8 coarse cells (a corner).
template <int D, int NT, int G>
__device__ __forceinline__ void fill_cf_coarse_group(const DevMesh& m, double* __restrict__ U,
                                                     const int* __restrict__ list, int count,
                                                     int first, int* __restrict__ err,
                                                     int* s_pid, int* s_code, int* s_pre) {
  constexpr int NV = D + 2, NS = 2 * D + 1, NF = 1 << D;
  if (threadIdx.x < G) {
    const int i = first + (int)threadIdx.x;
    int pid = -1, code = 0, cnt = 0;
    if (i < count) {
      pid = list[2 * i];
      code = list[2 * i + 1];
      const int n = m.lv[m.level[pid]].n;
      cnt = 1;
      for (int j = 0; j < D; ++j) {
        const int r = (j == 0 ? code : (j == 1 ? code / 3 : code / 9)) % 3 - 1;
        cnt *= (r == 0 ? n : NG) / 2;
      }
    }
    s_pid[threadIdx.x] = pid;
    s_code[threadIdx.x] = code;
    s_pre[threadIdx.x + 1] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_pre[0] = 0;
    for (int i = 0; i < G; ++i) s_pre[i + 1] += s_pre[i];
  }
  __syncthreads();
  const int total = s_pre[G];
  for (int idx = threadIdx.x; idx < total; idx += NT) {
    int it = 0;
    while (idx >= s_pre[it + 1]) ++it;
    const int pid = s_pid[it], code = s_code[it];
    const int local = idx - s_pre[it];
    const int l = m.level[pid];
    const LevelC& L = m.lv[l];
    const int n = L.n, full = L.full;
    const int vs = var_stride<D>(full);
    double* P = U + patch_base(m, pid, l);
    int start[3] = {0, 0, 0}, half[3] = {1, 1, 1};
    for (int j = 0; j < D; ++j) {
      const int r = (j == 0 ? code : (j == 1 ? code / 3 : code / 9)) % 3 - 1;
      start[j] = r < 0 ? -NG : (r == 0 ? 0 : n);
      half[j] = (r == 0 ? n : NG) / 2;
    }
    const int k[3] = {local % half[0], (local / half[0]) % half[1], local / (half[0] * half[1])};
    int c0[3] = {0, 0, 0}, gc[3] = {0, 0, 0};
    double sg[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int j = 0; j < D; ++j) {
      const int pcj = m.coord[3 * pid + j];
      c0[j] = start[j] + 2 * k[j];
      const int g0 = bc_map(pcj * n + c0[j], L.cells, m.periodic[j]);
      const int g1 = bc_map(pcj * n + c0[j] + 1, L.cells, m.periodic[j]);
      gc[j] = g0 >> 1;
      sg[j][0] = (g0 & 1) ? 1.0 : -1.0;
      sg[j][1] = (g1 & 1) ? 1.0 : -1.0;
    }
    const int lc = l > 0 ? l - 1 : 0;
    const LevelC& C = m.lv[lc];
    const long long vsc = var_stride<D>(C.full);
    int pids[NS];
    long long offs[NS];
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
      pids[s] = l > 0 ? map_at<D>(m, lc, q) : -1;
      offs[s] = box_off<D>(C.full, c[0] + NG, c[1] + NG, c[2] + NG);
    }
    bool found = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) found &= pids[s] >= 0;
    if (!found) {
      err[0] = 1;
      for (int f = 0; f < NF; ++f) {
        const int off = box_off<D>(full, c0[0] + (f & 1) + NG, c0[1] + ((f >> 1) & 1) + NG,
                                         c0[2] + ((f >> 2) & 1) + NG);
#pragma unroll
        for (int v = 0; v < NV; ++v) P[v * vs + off] = __builtin_nan("");
      }
      continue;
    }
    double val[NS][NV];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double* Q = U + patch_base(m, pids[s], lc) + offs[s];
#pragma unroll
      for (int v = 0; v < NV; ++v) val[s][v] = Q[v * vsc];
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
    for (int c = 0; c < NF; ++c) {
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
    for (int f = 0; f < NF; ++f) {
      const int off = box_off<D>(full, c0[0] + (f & 1) + NG, c0[1] + ((f >> 1) & 1) + NG,
                                       c0[2] + ((f >> 2) & 1) + NG);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double x = phi[v];
        for (int j = 0; j < D; ++j) x = x + (sg[j][(f >> j) & 1] * 0.25) * (bad ? 0.0 : sl[j][v]);
        P[v * vs + off] = x;
      }
    }
  }
}

// Block b takes the group of G regions starting at G b.  With `dir` (batched
// launches) the list and count are read at run time.
template <int D, int NT, int G>
__global__ __launch_bounds__(NT) void k_fill_cf_coarse(DevMesh m,
                                                       double* __restrict__ U,
                                                       const int* __restrict__ list, int count,
                                                       const int* __restrict__ dir,
                                                       int* __restrict__ err) {
  __shared__ int s_pid[G], s_code[G], s_pre[G + 1];
  if (dir) {
    list += dir[0];
    count = dir[1];
  }
  const int first = (int)blockIdx.x * G;
  if (first < count)
    fill_cf_coarse_group<D, NT, G>(m, U, list, count, first, err, s_pid, s_code, s_pre);
}

// ---------------------------------------------------------------------------
// coarse/fine flux correction: list of (pid, face mask); faces are processed
// in the order x-, x+, y-, y+, z-, z+ so that corner cells see a fixed order
// ---------------------------------------------------------------------------
// Correction of the coarse leaf cell c (patch-local) for its c/f face f =
// 2 j + side: coef (G_c - mean of the 2^(D-1) fine sub-face fluxes), signed
// +1 on the high face and -1 on the low face.
template <int D>
__device__ __forceinline__ void face_correct(const DevMesh& m, const double* __restrict__ fr,
                                             const double* __restrict__ frc, int l,
                                             const int pc[3], const int c[3], int f,
                                             double coef, double u[D + 2]) {
  constexpr int NV = D + 2;
  const LevelC& L = m.lv[l];
  const LevelC& Fv = m.lv[l + 1];
  const int n = L.n, nf = Fv.n, Nf = Fv.cells;
  const int nface = (D == 1) ? 1 : (D == 2 ? n : n * n);
  const int nfface = (D == 1) ? 1 : (D == 2 ? nf : nf * nf);
  const int j = f >> 1, side = f & 1;
  // fine cell column adjacent to the face (periodic wrap on the high side,
  // and on the low side of the domain)
  int F = 2 * ((j == 0 ? pc[0] : (j == 1 ? pc[1] : pc[2])) * n + (side ? n : 0));
  int cj;
  if (side) {
    F %= Nf;
    cj = F;
  } else {
    if (F == 0) F = Nf;
    cj = F - 1;
  }
  const int fside = side ? 0 : 1;
  // tangential coordinates of the cell in ascending dimension order (all
  // indexing below is by compile-time constants; j selects)
  int tc[2] = {0, 0}, tp[2] = {0, 0};
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if (d == j) continue;
    const int k = d - (d > j ? 1 : 0);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
      if (kk == k) {
        tc[kk] = c[d];
        tp[kk] = pc[d];
      }
  }
  const int t = (D >= 2 ? tc[0] : 0) + (D >= 3 ? n * tc[1] : 0);
  double sub[4][NV];
  constexpr int nsub = 1 << (D - 1);
  bool ok = true;
#pragma unroll
  for (int s = 0; s < nsub; ++s) {
    int qt[2] = {0, 0}, fl[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {
      const int gfc = 2 * (tp[k] * n + tc[k]) + ((s >> k) & 1);
      qt[k] = gfc / nf;
      fl[k] = gfc - qt[k] * nf;
    }
    // fine patch position: normal component cj / nf, tangential ones qt in
    // ascending dimension order
    int q[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int k = d - (d > j ? 1 : 0);
      const int qtd = (k == 0) ? qt[0] : qt[1];
      q[d] = (d == j) ? cj / nf : qtd;
    }
    const int fpid = map_at<D>(m, l + 1, q);
    ok &= fpid >= 0;
    const double* frf = fr + Fv.fr_off + (long long)((fpid < 0 ? Fv.pid_base : fpid) - Fv.pid_base) * Fv.fr_stride;
    const int ft = fl[0] + nf * fl[1];
#pragma unroll
    for (int v = 0; v < NV; ++v) sub[s][v] = frf[((j * 2 + fside) * NV + v) * nfface + ft];
  }
  const double sgn = side ? 1.0 : -1.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double avg;
    if constexpr (D == 1) avg = sub[0][v];
    else if constexpr (D == 2) avg = (sub[0][v] + sub[1][v]) * 0.5;
    else avg = ((sub[0][v] + sub[1][v]) + (sub[2][v] + sub[3][v])) * 0.25;
    if (!ok) avg = __builtin_nan("");
    const double gc = frc[((j * 2 + side) * NV + v) * nface + t];
    u[v] = fma(coef, sgn * (gc - avg), u[v]);
  }
}

// Refluxing on (leaf, c/f face mask) items.  Every cell on a masked face is
// owned by one thread (the first masked face containing it in the order
// x-, x+, y-, y+, z-, z+), which applies the corrections of all masked faces
// containing the cell in that order; at stage 3 it also feeds the corrected
// cell's CFL rate to the next step's maximum.
template <int D, int NT>
__device__ __forceinline__ void reflux_item(const DevMesh& m, int mode, double* __restrict__ out,
                                            const double* __restrict__ fr,
                                            const int* __restrict__ list, int item,
                                            const double* __restrict__ dtp, double w,
                                            unsigned long long* __restrict__ lam_next) {
  constexpr int NV = D + 2;
  const int pid = list[2 * item];
  const int mask = list[2 * item + 1];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n;
  const int nface = (D == 1) ? 1 : (D == 2 ? n : n * n);
  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  const double* frc = fr + L.fr_off + (long long)(pid - L.pid_base) * L.fr_stride;
  double* P = out + patch_base(m, pid, l);
  const int vs = var_stride<D>(L.full);
  const double coef = (mode == kModeRHS) ? L.inv_h : (w * dtp[0]) * L.inv_h;
  const bool want_rate = lam_next != nullptr && mode == kModeStage3;
  auto on_face = [&](const int c[3], int g) {
    const int j = g >> 1;
    const int cj = (j == 0) ? c[0] : (j == 1 ? c[1] : c[2]);
    return cj == ((g & 1) ? n - 1 : 0);
  };
  unsigned long long best = 0ull;
  for (int it = threadIdx.x; it < 2 * D * nface; it += NT) {
    const int f = it / nface, t = it - f * nface;
    if (!(mask & (1 << f))) continue;
    const int j = f >> 1;
    // cell on face f: normal coordinate 0 or n-1, tangential ones from t in
    // ascending dimension order
    const int t0 = (D >= 2) ? t % n : 0, t1 = (D >= 3) ? t / n : 0;
    int c[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int k = d - (d > j ? 1 : 0);
      c[d] = (d == j) ? ((f & 1) ? n - 1 : 0) : (k == 0 ? t0 : t1);
    }
    bool owned = true;
    for (int g = 0; g < f; ++g) owned &= !((mask & (1 << g)) && on_face(c, g));
    if (!owned) continue;
    // the cell's values stay in registers through all of its corrections
    const int off = box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG);
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = P[v * vs + off];
    for (int g = f; g < 2 * D; ++g)
      if ((mask & (1 << g)) && on_face(c, g)) face_correct<D>(m, fr, frc, l, pc, c, g, coef, u);
#pragma unroll
    for (int v = 0; v < NV; ++v) P[v * vs + off] = u[v];
    if (want_rate) {
      const unsigned long long bits = cell_rate_bits<D>(u, m, L.h);
      best = bits > best ? bits : best;
    }
  }
  if (want_rate) block_max_atomic(best, lam_next);
}

template <int D, int NT>
__global__ __launch_bounds__(NT) void k_reflux(DevMesh m, int mode, double* __restrict__ out,
                                               const double* __restrict__ fr,
                                               const int* __restrict__ list, int count,
                                               const double* __restrict__ dtp, double w,
                                               unsigned long long* __restrict__ lam_next) {
  if ((int)blockIdx.x >= count) return;
  reflux_item<D, NT>(m, mode, out, fr, list, blockIdx.x, dtp, w, lam_next);
}

// Restriction of one child patch into the covered cells of its parent:
// pairwise sums in x, then y, then z order, times 2^-D.
// One covered parent cell (index idx of the h^D cells a child covers): the
// pairwise sum of its 2^D child cells times 2^-D.
template <int D>
__device__ __forceinline__ void restrict_cell(const DevMesh& m, double* __restrict__ U, int cpid,
                                              int ppid, int lf, int h, int idx) {
  constexpr int NV = D + 2;
  const LevelC& F = m.lv[lf];
  const LevelC& C = m.lv[lf - 1];
  int o[3] = {0, 0, 0};
  for (int j = 0; j < D; ++j) o[j] = m.coord[3 * cpid + j] * h - m.coord[3 * ppid + j] * C.n;
  const double* Pc = U + patch_base(m, cpid, lf);
  double* Pp = U + patch_base(m, ppid, lf - 1);
  const long long vsf = var_stride<D>(F.full), vsc = var_stride<D>(C.full);
  const int a = idx % h;
  const int b = D >= 2 ? (idx / h) % h : 0;
  const int c = D >= 3 ? idx / (h * h) : 0;
  const long long dst = box_off<D>(C.full, o[0] + a + NG, o[1] + b + NG, o[2] + c + NG);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double* S = Pc + v * vsf;
    // sum of the x-pair (2a, 2a + 1) of fine row (y, z), read as one 16-byte
    // load: every offset here is even (even patch edges, ghost width 4, pools
    // of whole patches) and the state buffer is 256-byte aligned
    auto xsum = [&](int y, int z) {
      const double2 t = *reinterpret_cast<const double2*>(
          S + box_off<D>(F.full, 2 * a + NG, 2 * b + y + NG, 2 * c + z + NG));
      return t.x + t.y;
    };
    double r;
    if constexpr (D == 1) r = xsum(0, 0) * 0.5;
    else if constexpr (D == 2)
      r = (xsum(0, 0) + xsum(1, 0)) * 0.25;
    else
      r = ((xsum(0, 0) + xsum(1, 0)) + (xsum(0, 1) + xsum(1, 1))) * 0.125;
    Pp[v * vsc + dst] = r;
  }
}

template <int D>
__device__ __forceinline__ int covered_cells(int h) {
  int total = h;
  if constexpr (D >= 2) total *= h;
  if constexpr (D >= 3) total *= h;
  return total;
}

// restriction of patch cpid into its parent, by the whole block
template <int D>
__device__ __forceinline__ void restrict_patch(const DevMesh& m, double* __restrict__ U,
                                               int cpid) {
  const int lf = m.level[cpid];
  const int ppid = m.parent[cpid];
  const int h = m.lv[lf].n / 2;
  const int total = covered_cells<D>(h);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x)
    restrict_cell<D>(m, U, cpid, ppid, lf, h, idx);
}

// restriction of every child of ppid into it, all children's covered cells in
// one loop over the block (children share their level and edge)
template <int D>
__device__ __forceinline__ void restrict_children(const DevMesh& m, double* __restrict__ U,
                                                  int ppid) {
  const int nc = m.nchild[ppid];
  if (nc <= 0) return;
  const int lf = m.level[ppid] + 1;
  const int h = m.lv[lf].n / 2;
  const int per = covered_cells<D>(h);
  for (int idx = threadIdx.x; idx < nc * per; idx += blockDim.x) {
    const int k = idx / per;
    restrict_cell<D>(m, U, m.child[(long long)ppid * m.maxc + k], ppid, lf, h, idx - k * per);
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_restrict(DevMesh m,
                                                  double* __restrict__ U,
                                                  const int* __restrict__ list, int count,
                                                  const int* __restrict__ dir) {
  if (dir) {
    list += dir[0];
    count = dir[1];
  }
  if ((int)blockIdx.x < count) restrict_patch<D>(m, U, list[blockIdx.x]);
}

// After a stage, in one launch: refluxing and the restriction of the two
// finest levels, L-1 into L-2 and L-2 into L-3 (when L-2 >= 1).  Blocks:
//  [0, nref)            reflux items (pid, mask); a level-(L-2) item then
//                       restricts its (corrected) patch into its parent;
//  [nref, +npair)       level-(L-2) patches with children: restrict every
//                       child into the patch, then the patch into its parent;
//  [.., +nsingle)       level-(L-2) leaves without coarse/fine faces:
//                       restrict into the parent.
// Each block's second restriction reads only what the same block wrote
// (block barrier between); the blocks touch disjoint cells otherwise:
// refluxing changes leaf cells, restriction writes non-leaf cells.
template <int D, int NT>
__device__ __forceinline__ void post_block(const DevMesh& m, int mode, double* __restrict__ out,
                                           const double* __restrict__ fr,
                                           const int* __restrict__ rlist, int nref,
                                           const int* __restrict__ plist, int npair,
                                           const int* __restrict__ slist, int nsingle, int lup,
                                           int fine_done, const double* __restrict__ dtp, double w,
                                           unsigned long long* __restrict__ lam_next, int b) {
  if (b < nref) {
    reflux_item<D, NT>(m, mode, out, fr, rlist, b, dtp, w, lam_next);
    const int pid = rlist[2 * b];
    if (lup >= 1 && m.level[pid] == lup) {
      __syncthreads();
      restrict_patch<D>(m, out, pid);
    }
  } else if (b - nref < npair) {
    const int pid = plist[b - nref];
    // the stage kernel has restricted the finest level (the children) itself
    // unless the launch says otherwise
    if (!fine_done) {
      restrict_children<D>(m, out, pid);
      __syncthreads();
    }
    if (lup >= 1) restrict_patch<D>(m, out, pid);
  } else if (b - nref - npair < nsingle) {
    restrict_patch<D>(m, out, slist[b - nref - npair]);
  }
}


// One block per block index.  With `dir` (batched launches) the three lists
// and their counts are read at run time from their directory entries.
template <int D, int NT>
__global__ __launch_bounds__(NT) void k_post(DevMesh m, int mode,
                                             double* __restrict__ out,
                                             const double* __restrict__ fr,
                                             const int* __restrict__ rlist, int nref,
                                             const int* __restrict__ plist, int npair,
                                             const int* __restrict__ slist, int nsingle,
                                             const int* __restrict__ dir,
                                             int lup, int fine_done,
                                             const double* __restrict__ dtp, double w,
                                             unsigned long long* __restrict__ lam_next) {
  if (dir) {
    // the three lists' directory entries, in order; rlist is the list buffer
    const int* buf = rlist;
    rlist = buf + dir[0];
    nref = dir[1];
    plist = buf + dir[2];
    npair = dir[3];
    slist = buf + dir[4];
    nsingle = dir[5];
  }
  post_block<D, NT>(m, mode, out, fr, rlist, nref, plist, npair, slist, nsingle, lup, fine_done,
                    dtp, w, lam_next, blockIdx.x);
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
    const int vs = var_stride<D>(L.full);
    int total = n;
    if constexpr (D >= 2) total *= n;
    if constexpr (D >= 3) total *= n;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int x = idx % n;
      const int y = D >= 2 ? (idx / n) % n : 0;
      const int z = D >= 3 ? idx / (n * n) : 0;
      const int off = box_off<D>(L.full, x + NG, y + NG, z + NG);
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

// rho and p at patch-local cell c of patch P (level l, patch position pc);
// with FUSE a cell outside the patch is read from the same-level patch that
// holds it (neighbour table sN by offset code, periodic wrap and transmissive
// clamp applied), else from P's own ghost layer (prolonged values).
template <int D, bool FUSE>
__device__ __forceinline__ void rho_p_node(const DevMesh& m, const double* __restrict__ U,
                                           const double* __restrict__ P, long long vs, int full,
                                           int n, int l, const int pc[3], const int* sN,
                                           const int c[3], double& rho, double& p) {
  if constexpr (FUSE) {
    bool inside = true;
    for (int j = 0; j < D; ++j) inside &= (c[j] >= 0 && c[j] < n);
    if (!inside) {
      const LevelC& L = m.lv[l];
      int code = 0, loc[3] = {0, 0, 0}, mul = 1;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const int g = bc_map(pc[j] * n + c[j], L.cells, m.periodic[j]);
        const int q = g / n;
        int o = q - pc[j];
        if (o > 1) o -= L.np;
        if (o < -1) o += L.np;
        loc[j] = g - q * n;
        code += (o + 1) * mul;
        mul *= 3;
      }
      const int src = sN[code];
      if (src >= 0) {
        rho_p_at<D>(m, U + patch_base(m, src, l), vs,
                    box_off<D>(full, loc[0] + NG, loc[1] + NG, loc[2] + NG), rho, p);
        return;
      }
    }
  }
  rho_p_at<D>(m, P, vs, box_off<D>(full, c[0] + NG, c[1] + NG, c[2] + NG), rho, p);
}

template <int D, bool FUSE>
__global__ __launch_bounds__(256) void k_tag(DevMesh m, const double* __restrict__ U,
                                             const int* __restrict__ list, int count,
                                             uint8_t* __restrict__ has_tag,
                                             uint8_t* __restrict__ raw, int lds_nodes) {
  if ((int)blockIdx.x >= count) return;
  const int pid = list[blockIdx.x];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, b = m.tag_buffer, w = n + 2 * b;
  const double* P = U + patch_base(m, pid, l);
  const int vs = var_stride<D>(L.full);
  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  // same-level neighbours by offset code (o0+1) + 3 (o1+1) + 9 (o2+1)
  __shared__ int sN[27];
  if constexpr (FUSE) {
    constexpr int NO = D == 1 ? 3 : (D == 2 ? 9 : 27);
    const int t = threadIdx.x;
    if (t < NO) {
      int q[3] = {0, 0, 0};
      bool in = true;
      for (int j = 0; j < D; ++j) {
        const int o = (j == 0 ? t : (j == 1 ? t / 3 : t / 9)) % 3 - 1;
        int v = pc[j] + o;
        if (v < 0 || v >= L.np) {
          if (m.periodic[j]) v = (v + L.np) % L.np;
          else in = false;
        }
        q[j] = v;
      }
      sN[t] = in ? map_at<D>(m, l, q) : -1;
    }
    __syncthreads();
  }
  int total = w;
  if constexpr (D >= 2) total *= w;
  if constexpr (D >= 3) total *= w;
  int any = 0;
  uint8_t* rp = raw ? raw + L.tag_off + (long long)(pid - L.pid_base) * vs : nullptr;
  // rho and p of every node of the box [-b-1, n+b]^D once, in LDS (dynamic,
  // sized on the host for the largest patch edge whose box fits; always in
  // 1D/2D), then the tests read LDS; larger 3D patches compute each cell's
  // neighbours directly below
  const int wn = w + 2;
  int nodes = wn;
  if constexpr (D >= 2) nodes *= wn;
  if constexpr (D >= 3) nodes *= wn;
  if (nodes <= lds_nodes) {
    extern __shared__ double stag[];
    double* sr = stag;
    double* sp = stag + nodes;
    for (int idx = threadIdx.x; idx < nodes; idx += blockDim.x) {
      const int c[3] = {idx % wn - b - 1, D >= 2 ? (idx / wn) % wn - b - 1 : 0,
                        D >= 3 ? idx / (wn * wn) - b - 1 : 0};
      rho_p_node<D, FUSE>(m, U, P, vs, L.full, n, l, pc, sN, c, sr[idx], sp[idx]);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int c0 = idx % w - b;
      const int c1 = D >= 2 ? (idx / w) % w - b : 0;
      const int c2 = D >= 3 ? idx / (w * w) - b : 0;
      const int node = (c0 + b + 1) + (D >= 2 ? (c1 + b + 1) * wn : 0) +
                       (D >= 3 ? (c2 + b + 1) * wn * wn : 0);
      bool t = false;
      for (int j = 0; j < D; ++j) {
        const int st = j == 0 ? 1 : (j == 1 ? wn : wn * wn);
        const double rp_ = sr[node + st], rm_ = sr[node - st];
        const double pp_ = sp[node + st], pm_ = sp[node - st];
        t |= fabs(rp_ - rm_) > m.theta * (fabs(rp_) + fabs(rm_));
        t |= fabs(pp_ - pm_) > m.theta * (fabs(pp_) + fabs(pm_));
      }
      any |= t;
      if (rp) rp[box_off<D>(L.full, c0 + NG, c1 + NG, c2 + NG)] = t ? 1 : 0;
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) has_tag[pid] = any ? 1 : 0;
    return;
  }
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
      rho_p_node<D, FUSE>(m, U, P, vs, L.full, n, l, pc, sN, cp, rp_, pp_);
      rho_p_node<D, FUSE>(m, U, P, vs, L.full, n, l, pc, sN, cm, rm_, pm_);
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
  const int vs = var_stride<D>(L.full);
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
  const int vs = var_stride<D>(L.full);
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
    const int off = box_off<D>(L.full, c[0] + NG, c[1] + NG, c[2] + NG);
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
  const int vs = var_stride<D>(L.full);
  int total = n;
  if constexpr (D >= 2) total *= n;
  if constexpr (D >= 3) total *= n;
  int cnt = 0;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int x = idx % n;
    const int y = D >= 2 ? (idx / n) % n : 0;
    const int z = D >= 3 ? idx / (n * n) : 0;
    double u[NV];
    const int off = box_off<D>(L.full, x + NG, y + NG, z + NG);
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

// Regions per block of the coarse/fine fill launch for this mesh (the
// kernel choice of fill_cf below).
static int fill_cf_per_block(const DevMesh& m) {
  if (m.dim == 1) return 1;
  if (m.dim == 2) {
    int nmax = 0;
    for (int l = 1; l < m.nlev; ++l) nmax = std::max(nmax, m.lv[l].n);
    return nmax <= 16 ? 1 : 2;
  }
  return 4;
}

int Kernels::fill_cf_grid(const DevMesh& m, int count) {
  const int g = fill_cf_per_block(m);
  return (count + g - 1) / g;
}

void Kernels::fill_cf(const DevMesh& m, double* U, const int* list, int count, const int* dir,
                      int* err, hipStream_t s) {
  if (count <= 0) return;
  // one block per region (group of regions)
  auto launch = [&](auto kern, int threads, int per_block) {
    const int nb = (count + per_block - 1) / per_block;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(threads), 0, s, m, U, list, count, dir, err);
  };
  switch (m.dim) {
    case 1: launch(k_fill_cf<1, 64>, 64, 1); break;
    case 2: {
      // refined patches of edge 16 or less: one fine cell per thread (a side
      // region is 4 n = 64 cells); wider ones: by coarse cell, two regions
      // per wave (a side region of a 32^2 patch is 64 coarse cells).  Level 0
      // has no prolonged ghosts.  Per launch on a 3-level 2D hierarchy of
      // base 256^2 with 32/16/16 patches: 7.2 us per fine cell, 10.1 / 8.5 /
      // 11.1 us by coarse cell with 1 / 2 / 8 regions per block; on a
      // 5-level one of base 512^2 with 32^2 patches: 30.3 us per fine cell
      // (128 threads), 34.1 / 25.4 us by coarse cell with 1 / 2 regions per
      // block.
      int nmax = 0;
      for (int l = 1; l < m.nlev; ++l) nmax = std::max(nmax, m.lv[l].n);
      if (nmax <= 16)
        launch(k_fill_cf<2, 64>, 64, 1);
      else
        launch(k_fill_cf_coarse<2, 64, 2>, 64, 2);
      break;
    }
    default:
      // one thread per coarse cell, 4 regions per wave: a region of an 8^3
      // patch covers 8, 16 or 32 coarse cells and one of a 16^3 patch 8 to
      // 128 (per launch on a four-level 3D hierarchy of base 256^3 with
      // 32/16/16/8 patches: 2.12 ms with 4 regions per block, 2.19 with 8,
      // 2.27 with 16)
      launch(k_fill_cf_coarse<3, 64, 4>, 64, 4);
      break;
  }
}

void Kernels::fill(const DevMesh& m, double* U, const int* list, int count, int* err,
                   bool coarse_only, hipStream_t s) {
  if (count <= 0) return;
  AMR_DISPATCH_DIM(m.dim, k_fill, dim3(count), dim3(256), s, m, U, list, count, err,
                   coarse_only ? 1 : 0);
}

void Kernels::reflux(const DevMesh& m, int mode, double* out, const double* fr,
                     const int* list, int count, const double* dt, double w,
                     unsigned long long* lam_next, hipStream_t s) {
  if (count <= 0) return;
  switch (m.dim) {
    case 1: k_reflux<1, 64><<<count, 64, 0, s>>>(m, mode, out, fr, list, count, dt, w, lam_next); break;
    case 2: k_reflux<2, 64><<<count, 64, 0, s>>>(m, mode, out, fr, list, count, dt, w, lam_next); break;
    default: k_reflux<3, 256><<<count, 256, 0, s>>>(m, mode, out, fr, list, count, dt, w, lam_next); break;
  }
}

void Kernels::post(const DevMesh& m, int mode, double* out, const double* fr,
                   const int* rlist, int nref, const int* plist, int npair, const int* slist,
                   int nsingle, const int* dir, int lup, bool fine_done, const double* dt,
                   double w, unsigned long long* lam_next, hipStream_t s) {
  const int nb = nref + npair + nsingle;
  if (nb <= 0) return;
  auto launch = [&](auto kern, int threads) {
    hipLaunchKernelGGL(kern, dim3(nb), dim3(threads), 0, s, m, mode, out, fr, rlist, nref,
                       plist, npair, slist, nsingle, dir, lup, fine_done ? 1 : 0, dt, w,
                       lam_next);
  };
  switch (m.dim) {
    case 1: launch(k_post<1, 64>, 64); break;
    case 2: launch(k_post<2, 256>, 256); break;
    default: launch(k_post<3, 256>, 256); break;
  }
}

void Kernels::restrict_level(const DevMesh& m, double* U, const int* list, int count,
                             const int* dir, hipStream_t s) {
  if (count <= 0) return;
  // one block per child patch, one thread per covered parent cell
  auto launch = [&](auto kern, int threads) {
    const int nb = count;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(threads), 0, s, m, U, list, count, dir);
  };
  switch (m.dim) {
    case 1: launch(k_restrict<1>, 64); break;
    case 2: launch(k_restrict<2>, 64); break;
    default: launch(k_restrict<3>, 256); break;
  }
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
                  uint8_t* has_tag, uint8_t* raw, bool fuse, hipStream_t s) {
  if (count <= 0) return;
  // LDS for rho and p on the box [-b-1, n+b]^D of the largest patch edge
  // (1D/2D), or of the largest edge whose box fits 64 KB (3D)
  int lds_nodes = 0;
  for (int l = 0; l < m.nlev; ++l) {
    const long long wn = (long long)m.lv[l].n + 2 * m.tag_buffer + 2;
    const long long nodes = m.dim == 1 ? wn : (m.dim == 2 ? wn * wn : wn * wn * wn);
    if (m.dim <= 2 || nodes * 2 * (long long)sizeof(double) <= 64 * 1024)
      lds_nodes = std::max<long long>(lds_nodes, nodes);
  }
  const size_t lds = 2 * (size_t)lds_nodes * sizeof(double);
  if (lds > 160 * 1024) throw std::runtime_error("tagging box exceeds LDS");
  if (lds > 64 * 1024) {
    static bool big = false;
    if (!big) {
      big = true;
      (void)hipFuncSetAttribute((const void*)k_tag<1, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipFuncSetAttribute((const void*)k_tag<1, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipFuncSetAttribute((const void*)k_tag<2, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipFuncSetAttribute((const void*)k_tag<2, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
  }
#define AMR_TAG(D)                                                                           \
  do {                                                                                       \
    if (fuse) k_tag<D, true><<<count, 256, lds, s>>>(m, U, list, count, has_tag, raw, lds_nodes); \
    else k_tag<D, false><<<count, 256, lds, s>>>(m, U, list, count, has_tag, raw, lds_nodes);    \
  } while (0)
  if (m.dim == 1) AMR_TAG(1);
  else if (m.dim == 2) AMR_TAG(2);
  else AMR_TAG(3);
#undef AMR_TAG
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
