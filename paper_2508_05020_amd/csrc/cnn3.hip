// Learned refinement predictor (3D): BF16 inputs/weights/activations, FP32
// accumulation on the MFMA units of gfx950.
//
// The network works on tiles of 8^3 output cells, so that one patch of edge
// 8, 16 or 32 is 1, 8 or 64 tiles and every tile's activations fit in LDS.
// Input per tile: normalised (rho, u, v, w, p) on the tile plus a halo of 3
// cells, [14]^3 voxels stored with 8 channels (the last 3 zero) so that the
// 4 consecutive channels an MFMA lane needs are one 8-byte load.  Three valid
// 3x3x3 convolutions 5 -> 8 -> 8 -> 1 with bias, ReLU after the first two,
// give one logit per tile cell.
//
// Convolutions as implicit GEMM on the 16x16x16 MFMA: rows = 16 output
// voxels, columns = output channels (8 of 16 used), K = (tap, input channel)
// with 2 taps x 8 channels per 16-wide chunk, 14 chunks for 27 taps.  Weight
// gradients swap the roles: rows = output channel, columns = (tap of a pair,
// input channel), K = voxels.  Operand layout: see cnn_device.hpp.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "amr_internal.hpp"
#include "cnn_device.hpp"
#include "cnn_internal.hpp"

namespace amr {
namespace {

using namespace cnnd;

constexpr int NG = kNG;
constexpr int T = CNN3_TILE;
constexpr int CH = CNN3_CH;
constexpr int W0 = T + 6, W1 = T + 4, W2 = T + 2;
constexpr int P0 = CNN3_P0, P1 = CNN3_P1, P2 = CNN3_P2, P3 = CNN3_P3;
constexpr int KCH = 14;  // K chunks: taps (2 kc, 2 kc + 1), 8 channels each
// threads per block: the loops stride over the block's waves, so more waves
// shorten a tile's latency (a training batch is only tens of tiles)
constexpr int FWD_THREADS = 512;
constexpr int BWD_THREADS = 1024;

static_assert(CH == 8, "two taps of 8 channels per MFMA K chunk");
static_assert(P1 % 16 == 0, "layer-1 voxels in whole MFMA row blocks");

__device__ __forceinline__ void tap_xyz(int tap, int& tz, int& ty, int& tx) {
  tz = tap / 9;
  ty = (tap / 3) % 3;
  tx = tap % 3;
}

// ---------------------------------------------------------------------------
// gather: normalised BF16 input tiles from the FP64 state (ghosts filled)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cnn3_gather(DevMesh m, const double* __restrict__ U,
                                                     const int* __restrict__ items, int count,
                                                     CnnNorm norm,
                                                     unsigned short* __restrict__ X) {
#pragma clang fp contract(off)
  const long long total = (long long)count * P0;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / P0);
    const int v = (int)(t - (long long)b * P0);
    const int item = items[b];
    const int pid = item / CNN3_MAX_TILES, tile = item - pid * CNN3_MAX_TILES;
    const LevelC& L = m.lv[m.level[pid]];
    const int nt = L.n / T;
    const int tz = tile / (nt * nt), ty = (tile / nt) % nt, tx = tile % nt;
    const int z = v / (W0 * W0), y = (v / W0) % W0, x = v % W0;
    // interior cell coordinates -3 .. n + 2: inside the 4 ghost layers
    const int cz = T * tz + z - 3, cy = T * ty + y - 3, cx = T * tx + x - 3;
    const double* P = U + L.pool_off + (long long)(pid - L.pid_base) * L.stride;
    const long long vs = (long long)L.full * L.full * L.full;
    const long long off = ((long long)(cz + NG) * L.full + (cy + NG)) * L.full + (cx + NG);
    const double rho = P[off], mx = P[vs + off], my = P[2 * vs + off], mz = P[3 * vs + off];
    const double E = P[4 * vs + off];
    const double ux = mx / rho, uy = my / rho, uz = mz / rho;
    double ke = mx * ux;
    ke = ke + my * uy;
    ke = ke + mz * uz;
    ke = 0.5 * ke;
    const double pr = m.gm1 * (E - ke);
    const double f[5] = {rho, ux, uy, uz, pr};
    unsigned short h[8];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const double zc = (f[c] - (double)norm.mean[c]) * (double)norm.istd[c];
      h[c] = f2bf((float)zc);
    }
    h[5] = h[6] = h[7] = 0;
    uint4 o;
    o.x = h[0] | ((unsigned)h[1] << 16);
    o.y = h[2] | ((unsigned)h[3] << 16);
    o.z = h[4] | ((unsigned)h[5] << 16);
    o.w = h[6] | ((unsigned)h[7] << 16);
    reinterpret_cast<uint4*>(X)[(long long)b * P0 + v] = o;
  }
}

// ---------------------------------------------------------------------------
// forward of one tile per block (4 waves); activations in LDS
// ---------------------------------------------------------------------------

// valid 3x3x3 convolution, 8 output channels, from a voxel-major LDS input of
// edge WI with 8 stored channels (CI of them weighted) to edge WI - 2 (bias,
// ReLU, BF16); W layout [8][CI][27].
template <int WI, int CI>
__device__ void conv3(const unsigned short* __restrict__ in, unsigned short* __restrict__ out,
                      unsigned short* __restrict__ gout, const unsigned short* __restrict__ W,
                      const float* __restrict__ bias) {
  constexpr int WO = WI - 2;
  constexpr int P = WO * WO * WO;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int half = kq >> 1, cg = 4 * (kq & 1);
  s4 bop[KCH];
  int toff[KCH];
#pragma unroll
  for (int kc = 0; kc < KCH; ++kc) {
    const int tap = 2 * kc + half;
    int tz, ty, tx;
    tap_xyz(tap, tz, ty, tx);
    toff[kc] = ((tz * WI + ty) * WI + tx) * CH + cg;
    short w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = cg + e;
      w[e] = (i < 8 && tap < 27 && c < CI) ? (short)W[(i * CI + c) * 27 + tap] : (short)0;
    }
    bop[kc] = pack4(w[0], w[1], w[2], w[3]);
  }
  const float bcol = i < 8 ? bias[i] : 0.f;
  constexpr int nblk = (P + 15) / 16;
  for (int blk = wave; blk < nblk; blk += nw) {
    const int p = 16 * blk + i;
    const int pc = p < P ? p : P - 1;
    const int pz = pc / (WO * WO), r = pc - pz * WO * WO;
    const int py = r / WO, px = r - py * WO;
    const unsigned short* base = in + ((pz * WI + py) * WI + px) * CH;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc) {
      const bool ok = kc < KCH - 1 || half == 0;  // tap 27 does not exist
      const s4 a = ok ? load4(base + toff[kc]) : zero4();
      acc = mfma(a, bop[kc], acc);
    }
    if (i < 8) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = 16 * blk + 4 * kq + e;
        if (q < P) {
          float v = acc[e] + bcol;
          v = v > 0.f ? v : 0.f;
          const unsigned short hb = f2bf(v);
          out[q * CH + i] = hb;
          if (gout) gout[q * CH + i] = hb;
        }
      }
    }
  }
}

__global__ __launch_bounds__(FWD_THREADS) void k_cnn3_fwd(int count, const unsigned short* __restrict__ X,
                                                      const unsigned short* __restrict__ Wb,
                                                      const float* __restrict__ params,
                                                      unsigned short* __restrict__ A1,
                                                      unsigned short* __restrict__ A2,
                                                      float* __restrict__ Z) {
  extern __shared__ unsigned short smem[];
  const int b = blockIdx.x;
  if (b >= count) return;
  unsigned short* sx = smem;           // P0 x 8
  unsigned short* s1 = sx + P0 * CH;   // P1 x 8
  unsigned short* s2 = smem;           // P2 x 8, over sx once layer 1 is done
  const uint4* xg = reinterpret_cast<const uint4*>(X) + (long long)b * P0;
  for (int t = threadIdx.x; t < P0; t += blockDim.x) reinterpret_cast<uint4*>(sx)[t] = xg[t];
  __syncthreads();
  conv3<W0, 5>(sx, s1, A1 ? A1 + (long long)b * P1 * CH : nullptr, Wb + CNN3_W1, params + CNN3_B1);
  __syncthreads();
  conv3<W1, 8>(s1, s2, A2 ? A2 + (long long)b * P2 * CH : nullptr, Wb + CNN3_W2, params + CNN3_B2);
  __syncthreads();
  // layer 3 (8 -> 1) on the VALU
  const float b3 = params[CNN3_B3];
  for (int p = threadIdx.x; p < P3; p += blockDim.x) {
    const int pz = p / (T * T), py = (p / T) % T, px = p % T;
    float acc = 0.f;
    for (int tap = 0; tap < 27; ++tap) {
      int tz, ty, tx;
      tap_xyz(tap, tz, ty, tx);
      const uint4 a = *reinterpret_cast<const uint4*>(
          s2 + (((pz + tz) * W2 + (py + ty)) * W2 + (px + tx)) * CH);
      const unsigned int u[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const unsigned short hc = (unsigned short)((u[c >> 1] >> (16 * (c & 1))) & 0xffffu);
        acc += bf2f(hc) * bf2f(Wb[CNN3_W3 + c * 27 + tap]);
      }
    }
    Z[(long long)b * P3 + p] = acc + b3;
  }
}

// ---------------------------------------------------------------------------
// backward of one tile per block: per-tile parameter-gradient partials
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BWD_THREADS) void k_cnn3_bwd(int count, const unsigned short* __restrict__ X,
                                                      const unsigned short* __restrict__ A1,
                                                      const unsigned short* __restrict__ A2,
                                                      const float* __restrict__ G,
                                                      const unsigned short* __restrict__ Wb,
                                                      float* __restrict__ partials) {
  extern __shared__ unsigned short smem[];
  const int b = blockIdx.x;
  if (b >= count) return;
  // the tile's input and saved activations are copied to LDS first (one
  // round of 16-byte loads), so that the reduction loops below read LDS
  unsigned short* dz2 = smem;              // P2 x 8
  unsigned short* dz1 = dz2 + P2 * CH;     // P1 x 8
  unsigned short* a2 = dz1 + P1 * CH;      // P2 x 8
  unsigned short* a1 = a2 + P2 * CH;       // P1 x 8
  unsigned short* x = a1 + P1 * CH;        // P0 x 8
  float* sg = reinterpret_cast<float*>(x + P0 * CH);  // P3 logit gradients
  float* part = partials + (long long)b * CNN3_NPARAM;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int half = kq >> 1, cg = 4 * (kq & 1);

  {
    const uint4* g2 = reinterpret_cast<const uint4*>(A2) + (long long)b * P2;
    const uint4* g1 = reinterpret_cast<const uint4*>(A1) + (long long)b * P1;
    const uint4* g0 = reinterpret_cast<const uint4*>(X) + (long long)b * P0;
    for (int t = tid; t < P2; t += blockDim.x) reinterpret_cast<uint4*>(a2)[t] = g2[t];
    for (int t = tid; t < P1; t += blockDim.x) reinterpret_cast<uint4*>(a1)[t] = g1[t];
    for (int t = tid; t < P0; t += blockDim.x) reinterpret_cast<uint4*>(x)[t] = g0[t];
  }
  for (int p = tid; p < P3; p += blockDim.x) sg[p] = G[(long long)b * P3 + p];
  __syncthreads();

  // --- layer 3: dz2 = relu'(z2) * (W3 (x) g) on the layer-2 grid; dW3, db3
  for (int q = tid; q < P2; q += blockDim.x) {
    const int qz = q / (W2 * W2), qy = (q / W2) % W2, qx = q % W2;
    float acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.f;
    for (int tap = 0; tap < 27; ++tap) {
      int tz, ty, tx;
      tap_xyz(tap, tz, ty, tx);
      const int pz = qz - tz, py = qy - ty, px = qx - tx;
      if (pz < 0 || py < 0 || px < 0 || pz >= T || py >= T || px >= T) continue;
      const float gv = sg[(pz * T + py) * T + px];
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] += bf2f(Wb[CNN3_W3 + c * 27 + tap]) * gv;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bool on = a2[q * CH + c] != 0;  // a2 = relu(z2) in BF16: nonzero iff z2 > 0
      dz2[q * CH + c] = f2bf(on ? acc[c] : 0.f);
    }
  }
  // dW3[c][tap] = sum_p a2[p + tap][c] g[p]; db3 = sum_p g[p]
  for (int k = tid; k < 8 * 27 + 1; k += blockDim.x) {
    float s = 0.f;
    if (k < 8 * 27) {
      const int c = k / 27, tap = k % 27;
      int tz, ty, tx;
      tap_xyz(tap, tz, ty, tx);
      for (int p = 0; p < P3; ++p) {
        const int pz = p / (T * T), py = (p / T) % T, px = p % T;
        s += bf2f(a2[(((pz + tz) * W2 + (py + ty)) * W2 + (px + tx)) * CH + c]) * sg[p];
      }
      part[CNN3_W3 + k] = s;
    } else {
      for (int p = 0; p < P3; ++p) s += sg[p];
      part[CNN3_B3] = s;
    }
  }
  __syncthreads();

  // --- layer 2 weight gradient: dW2[o][c][tap] = sum_p dz2[p][o] a1[p + tap][c]
  // D[i = o][j = 8 tsub + c], tap = 2 tp + tsub; K = layer-2 voxels
  for (int tp = wave; tp < KCH; tp += nw) {
    const int tsub = i >> 3, c = i & 7, tap = 2 * tp + tsub;
    const bool valid = tap < 27;
    int tz = 0, ty = 0, tx = 0;
    if (valid) tap_xyz(tap, tz, ty, tx);
    const int toff = ((tz * W1 + ty) * W1 + tx) * CH + c;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < P2; p0 += 16) {
      short av[4], bv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = p0 + 4 * kq + e;
        av[e] = 0;
        bv[e] = 0;
        if (p < P2) {
          const int pz = p / (W2 * W2), py = (p / W2) % W2, px = p % W2;
          if (i < 8) av[e] = (short)dz2[p * CH + i];
          if (valid) bv[e] = (short)a1[((pz * W1 + py) * W1 + px) * CH + toff];
        }
      }
      acc = mfma(pack4(av[0], av[1], av[2], av[3]), pack4(bv[0], bv[1], bv[2], bv[3]), acc);
    }
    if (valid) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = 4 * kq + e;
        if (o < 8) part[CNN3_W2 + (o * 8 + c) * 27 + tap] = acc[e];
      }
    }
  }
  for (int o = tid; o < 8; o += blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < P2; ++p) s += bf2f(dz2[p * CH + o]);
    part[CNN3_B2 + o] = s;
  }

  // --- layer 2 data gradient: dz1[q][c] = relu'(z1) sum_tap sum_o W2[o][c][tap] dz2[q - tap][o]
  // D[i = voxel][j = c]; K = (tap, o), 2 taps x 8 channels per chunk
  {
    s4 bop[KCH];
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc) {
      const int tap = 2 * kc + half;
      short w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = cg + e;
        w[e] = (i < 8 && tap < 27) ? (short)Wb[CNN3_W2 + (o * 8 + i) * 27 + tap] : (short)0;
      }
      bop[kc] = pack4(w[0], w[1], w[2], w[3]);
    }
    constexpr int nblk = P1 / 16;
    for (int blk = wave; blk < nblk; blk += nw) {
      const int q = 16 * blk + i;
      const int qz = q / (W1 * W1), qy = (q / W1) % W1, qx = q % W1;
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < KCH; ++kc) {
        const int tap = 2 * kc + half;
        s4 a = zero4();
        if (tap < 27) {
          int tz, ty, tx;
          tap_xyz(tap, tz, ty, tx);
          const int sz = qz - tz, sy = qy - ty, sx = qx - tx;
          if (sz >= 0 && sy >= 0 && sx >= 0 && sz < W2 && sy < W2 && sx < W2)
            a = load4(dz2 + ((sz * W2 + sy) * W2 + sx) * CH + cg);
        }
        acc = mfma(a, bop[kc], acc);
      }
      if (i < 8) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int qq = 16 * blk + 4 * kq + e;
          const bool on = a1[qq * CH + i] != 0;
          dz1[qq * CH + i] = f2bf(on ? acc[e] : 0.f);
        }
      }
    }
  }
  __syncthreads();

  // --- layer 1 weight gradient: dW1[o][c][tap] = sum_p dz1[p][o] x[p + tap][c]
  for (int tp = wave; tp < KCH; tp += nw) {
    const int tsub = i >> 3, c = i & 7, tap = 2 * tp + tsub;
    const bool valid = tap < 27 && c < 5;
    int tz = 0, ty = 0, tx = 0;
    if (valid) tap_xyz(tap, tz, ty, tx);
    const int toff = ((tz * W0 + ty) * W0 + tx) * CH + c;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < P1; p0 += 16) {
      short av[4], bv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = p0 + 4 * kq + e;
        const int pz = p / (W1 * W1), py = (p / W1) % W1, px = p % W1;
        av[e] = i < 8 ? (short)dz1[p * CH + i] : (short)0;
        bv[e] = valid ? (short)x[((pz * W0 + py) * W0 + px) * CH + toff] : (short)0;
      }
      acc = mfma(pack4(av[0], av[1], av[2], av[3]), pack4(bv[0], bv[1], bv[2], bv[3]), acc);
    }
    if (valid) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = 4 * kq + e;
        if (o < 8) part[CNN3_W1 + (o * 5 + c) * 27 + tap] = acc[e];
      }
    }
  }
  for (int o = tid; o < 8; o += blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < P1; ++p) s += bf2f(dz1[p * CH + o]);
    part[CNN3_B1 + o] = s;
  }
}

// per-tile refine request: any logit above the threshold flags the tile's patch
__global__ __launch_bounds__(256) void k_cnn3_requests(int count, const float* __restrict__ Z,
                                                       const int* __restrict__ items, float zt,
                                                       uint8_t* __restrict__ flag) {
  const int b = blockIdx.x;
  if (b >= count) return;
  int any = 0;
  for (int p = threadIdx.x; p < P3; p += blockDim.x) any |= Z[(long long)b * P3 + p] > zt;
  any = __syncthreads_or(any);
  // several tiles of one patch may store the same value
  if (threadIdx.x == 0 && any) flag[items[b] / CNN3_MAX_TILES] = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
size_t Cnn3::fwd_lds() { return (size_t)(P0 + P1) * CH * sizeof(unsigned short); }

size_t Cnn3::bwd_lds() {
  return (size_t)(2 * P2 + 2 * P1 + P0) * CH * sizeof(unsigned short) + P3 * sizeof(float);
}

static void allow_large_lds3() {
  static bool done = false;
  if (done) return;
  done = true;
  (void)hipFuncSetAttribute((const void*)k_cnn3_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_cnn3_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
}

void Cnn3::gather(const DevMesh& m, const double* U, const int* items, int count,
                  const CnnNorm& norm, unsigned short* X, hipStream_t s) {
  if (count <= 0) return;
  const long long total = (long long)count * P0;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 65535);
  hipLaunchKernelGGL(k_cnn3_gather, dim3(blocks), dim3(256), 0, s, m, U, items, count, norm, X);
}

void Cnn3::forward(int count, const unsigned short* X, const unsigned short* Wb, const float* params,
                   unsigned short* A1, unsigned short* A2, float* Z, hipStream_t s) {
  if (count <= 0) return;
  allow_large_lds3();
  hipLaunchKernelGGL(k_cnn3_fwd, dim3(count), dim3(FWD_THREADS), fwd_lds(), s, count, X, Wb, params, A1,
                     A2, Z);
}

void Cnn3::backward(int count, const unsigned short* X, const unsigned short* A1,
                    const unsigned short* A2, const float* G, const unsigned short* Wb,
                    float* partials, float* grads, hipStream_t s) {
  if (count <= 0) return;
  allow_large_lds3();
  hipLaunchKernelGGL(k_cnn3_bwd, dim3(count), dim3(BWD_THREADS), bwd_lds(), s, count, X, A1, A2, G, Wb,
                     partials);
  Cnn::reduce(partials, count, CNN3_NPARAM, grads, s);
}

void Cnn3::requests(int count, const float* Z, const int* items, float zt, uint8_t* flag,
                    hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_cnn3_requests, dim3(count), dim3(256), 0, s, count, Z, items, zt, flag);
}

}  // namespace amr
