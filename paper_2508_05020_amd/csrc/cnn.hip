// Learned refinement predictor (2D): BF16 inputs/weights/activations, FP32
// accumulation on the MFMA units of gfx950.
//
// Network per patch of n x n cells: input (rho, u, v, p) normalised, with a
// halo of 3 cells, [n+6]^2 pixels x 4 channels; three valid 3x3
// convolutions 4 -> 16 -> 16 -> 1 with bias, ReLU after the first two;
// output logits on the n x n interior.  Activations are stored pixel-major
// with the channels innermost (HWC), so that the 4 consecutive channels an
// MFMA lane needs are one 8-byte load.
//
// MFMA operand layout: see cnn_device.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "amr_internal.hpp"
#include "cnn_device.hpp"
#include "cnn_internal.hpp"

namespace amr {
namespace {

using namespace cnnd;

constexpr int NG = kNG;

// ---------------------------------------------------------------------------
// gather: normalised BF16 input tiles from the FP64 state (ghosts filled)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cnn_gather(DevMesh m, const double* __restrict__ U,
                                                    const int* __restrict__ pids, int count,
                                                    int n, CnnNorm norm,
                                                    unsigned short* __restrict__ X) {
#pragma clang fp contract(off)
  const int w = n + 6;
  const int P0 = w * w;
  const long long total = (long long)count * P0;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / P0);
    const int p = (int)(t - (long long)b * P0);
    const int pid = pids[b];
    const int l = m.level[pid];
    const LevelC& L = m.lv[l];
    const int y = p / w - 3, x = p % w - 3;
    const double* P = U + L.pool_off + (long long)(pid - L.pid_base) * L.stride;
    const long long vs = (long long)L.full * L.full;
    const long long off = (long long)(y + NG) * L.full + (x + NG);
    const double rho = P[off], mx = P[vs + off], my = P[2 * vs + off], E = P[3 * vs + off];
    const double ux = mx / rho, uy = my / rho;
    double ke = mx * ux;
    ke = ke + my * uy;
    ke = 0.5 * ke;
    const double pr = m.gm1 * (E - ke);
    const double f[4] = {rho, ux, uy, pr};
    unsigned short* o = X + ((long long)b * P0 + p) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double z = (f[c] - (double)norm.mean[c]) * (double)norm.istd[c];
      o[c] = f2bf((float)z);
    }
  }
}

// ---------------------------------------------------------------------------
// fused forward of one patch per block (4 waves); activations in LDS
// ---------------------------------------------------------------------------
constexpr int FWD_THREADS = 256;

// layer-1 B operand (weights) for k-chunk kc: k = (tap, channel), tap = 4 kc + kq
__device__ __forceinline__ s4 w1_operand(const unsigned short* __restrict__ W, int j, int kq, int kc) {
  const int tap = 4 * kc + kq;
  if (tap >= 9) return zero4();
  s4 r;
  // W1 layout [o][c][tap] (o = j)
  r.x = (short)W[(j * 4 + 0) * 9 + tap];
  r.y = (short)W[(j * 4 + 1) * 9 + tap];
  r.z = (short)W[(j * 4 + 2) * 9 + tap];
  r.w = (short)W[(j * 4 + 3) * 9 + tap];
  return r;
}

// layer-2 B operand for tap: B[k = in-channel][j = out-channel] = W2[j][k][tap]
__device__ __forceinline__ s4 w2_operand(const unsigned short* __restrict__ W, int j, int kq, int tap) {
  s4 r;
  r.x = (short)W[(j * 16 + 4 * kq + 0) * 9 + tap];
  r.y = (short)W[(j * 16 + 4 * kq + 1) * 9 + tap];
  r.z = (short)W[(j * 16 + 4 * kq + 2) * 9 + tap];
  r.w = (short)W[(j * 16 + 4 * kq + 3) * 9 + tap];
  return r;
}

// conv 3x3 valid, 16 output channels, from an HWC LDS input of width wi and
// CI channels (4 or 16) to an HWC output of width wo = wi - 2 (bias, ReLU,
// BF16); rows of 16 output pixels per MFMA tile.
template <int CI>
__device__ void conv16(const unsigned short* __restrict__ in, int wi, unsigned short* __restrict__ out,
                       unsigned short* __restrict__ gout, const unsigned short* __restrict__ Wb,
                       const float* __restrict__ bias) {
  const int wo = wi - 2;
  const int P = wo * wo;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  constexpr int KC = CI == 4 ? 3 : 9;  // k-chunks of 16
  s4 bop[KC];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) bop[kc] = CI == 4 ? w1_operand(Wb, i, kq, kc) : w2_operand(Wb, i, kq, kc);
  const float bcol = bias[i];  // D column j = lane % 16
  const int nblk = (P + 15) / 16;
  for (int blk = wave; blk < nblk; blk += nw) {
    // A rows: output pixel p = 16 blk + i (clamped for the tail)
    int p = 16 * blk + i;
    const int pc = p < P ? p : P - 1;
    const int py = pc / wo, px = pc - py * wo;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      s4 a;
      if (CI == 4) {
        const int tap = 4 * kc + kq;
        if (tap < 9) {
          const int ty = tap / 3, tx = tap - 3 * (tap / 3);
          a = load4(in + ((py + ty) * wi + (px + tx)) * 4);
        } else {
          a = zero4();
        }
      } else {
        const int tap = kc;
        const int ty = tap / 3, tx = tap - 3 * (tap / 3);
        a = load4(in + ((py + ty) * wi + (px + tx)) * 16 + 4 * kq);
      }
      acc = mfma(a, bop[kc], acc);
    }
    // D[i'][j]: j = lane % 16, i' = 4 kq + e -> pixel 16 blk + 4 kq + e
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = 16 * blk + 4 * kq + e;
      if (q < P) {
        float v = acc[e] + bcol;
        v = v > 0.f ? v : 0.f;
        const unsigned short h = f2bf(v);
        out[q * 16 + i] = h;
        if (gout) gout[q * 16 + i] = h;
      }
    }
  }
}

__global__ __launch_bounds__(FWD_THREADS) void k_cnn_fwd(int count, int n,
                                                         const unsigned short* __restrict__ X,
                                                         const unsigned short* __restrict__ Wb,
                                                         const float* __restrict__ params,
                                                         unsigned short* __restrict__ A1,
                                                         unsigned short* __restrict__ A2,
                                                         float* __restrict__ Z) {
  extern __shared__ unsigned short smem[];
  const int b = blockIdx.x;
  if (b >= count) return;
  const int w0 = n + 6, w1 = n + 4, w2 = n + 2;
  const int P0 = w0 * w0, P1 = w1 * w1, P2 = w2 * w2;
  unsigned short* sx = smem;                 // P0 x 4
  unsigned short* s1 = sx + P0 * 4;          // P1 x 16
  unsigned short* s2 = s1 + P1 * 16;         // P2 x 16
  const unsigned short* xg = X + (long long)b * P0 * 4;
  for (int t = threadIdx.x; t < P0; t += blockDim.x)
    *reinterpret_cast<uint2*>(sx + 4 * t) = *reinterpret_cast<const uint2*>(xg + 4 * t);
  __syncthreads();
  conv16<4>(sx, w0, s1, A1 ? A1 + (long long)b * P1 * 16 : nullptr, Wb + CNN_W1, params + CNN_B1);
  __syncthreads();
  conv16<16>(s1, w1, s2, A2 ? A2 + (long long)b * P2 * 16 : nullptr, Wb + CNN_W2, params + CNN_B2);
  __syncthreads();
  // layer 3 (16 -> 1) on the VALU
  const int P3 = n * n;
  const float b3 = params[CNN_B3];
  for (int p = threadIdx.x; p < P3; p += blockDim.x) {
    const int py = p / n, px = p - py * n;
    float acc = 0.f;
    for (int tap = 0; tap < 9; ++tap) {
      const int ty = tap / 3, tx = tap % 3;
      const unsigned short* a = s2 + ((py + ty) * w2 + (px + tx)) * 16;
#pragma unroll
      for (int c = 0; c < 16; ++c) acc += bf2f(a[c]) * bf2f(Wb[CNN_W3 + c * 9 + tap]);
    }
    Z[(long long)b * P3 + p] = acc + b3;
  }
}

// ---------------------------------------------------------------------------
// loss: weighted BCE with logits, per-cell gradient, per-block partial sums
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cnn_loss(long long total, const float* __restrict__ Z,
                                                  const uint8_t* __restrict__ Y, float pos_weight,
                                                  float* __restrict__ G, float* __restrict__ partial) {
  __shared__ float red[4];
  float acc = 0.f;
  const float inv = 1.0f / (float)total;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const float z = Z[t];
    const float y = Y[t] ? 1.f : 0.f;
    const float sp_pos = fmaxf(-z, 0.f) + log1pf(expf(-fabsf(z)));  // softplus(-z)
    const float sp_neg = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));   // softplus(z)
    acc += pos_weight * y * sp_pos + (1.f - y) * sp_neg;
    const float s = 1.f / (1.f + expf(-z));
    G[t] = (pos_weight * y * (s - 1.f) + (1.f - y) * s) * inv;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + (red[2] + red[3])) * inv;
}

__global__ void k_cnn_loss_final(const float* __restrict__ partial, int nblocks, float* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < nblocks; ++i) s += partial[i];
    loss[0] = s;
  }
}

// ---------------------------------------------------------------------------
// backward of one patch per block: per-patch parameter-gradient partials
// ---------------------------------------------------------------------------
constexpr int BWD_THREADS = 512;  // the loops stride over the block's waves

__device__ __forceinline__ s4 pick4(const unsigned short* base, int stride) {
  s4 r;
  r.x = (short)base[0];
  r.y = (short)base[stride];
  r.z = (short)base[2 * stride];
  r.w = (short)base[3 * stride];
  return r;
}

__global__ __launch_bounds__(BWD_THREADS) void k_cnn_bwd(int count, int n,
                                                         const unsigned short* __restrict__ X,
                                                         const unsigned short* __restrict__ A1,
                                                         const unsigned short* __restrict__ A2,
                                                         const float* __restrict__ G,
                                                         const unsigned short* __restrict__ Wb,
                                                         float* __restrict__ partials,
                                                         int stage_a1) {
  extern __shared__ unsigned short smem[];
  const int b = blockIdx.x;
  if (b >= count) return;
  const int w0 = n + 6, w1 = n + 4, w2 = n + 2;
  const int P0 = w0 * w0, P1 = w1 * w1, P2 = w2 * w2, P3 = n * n;
  // the patch's input, second activation and logit gradients (and the first
  // activation when LDS allows) are copied to LDS first, so that the
  // reduction loops below read LDS
  unsigned short* dz2 = smem;            // P2 x 16
  unsigned short* dz1 = dz2 + P2 * 16;   // P1 x 16
  unsigned short* sa2 = dz1 + P1 * 16;   // P2 x 16
  unsigned short* sx = sa2 + P2 * 16;    // P0 x 4
  float* sgr = reinterpret_cast<float*>(sx + P0 * 4);            // P3
  unsigned short* sa1 = reinterpret_cast<unsigned short*>(sgr + P3);  // P1 x 16 (stage_a1)
  const unsigned short* a1g = A1 + (long long)b * P1 * 16;
  {
    const uint4* g2 = reinterpret_cast<const uint4*>(A2 + (long long)b * P2 * 16);
    const uint2* g0 = reinterpret_cast<const uint2*>(X + (long long)b * P0 * 4);
    for (int t = threadIdx.x; t < P2 * 2; t += blockDim.x) reinterpret_cast<uint4*>(sa2)[t] = g2[t];
    for (int t = threadIdx.x; t < P0; t += blockDim.x) reinterpret_cast<uint2*>(sx)[t] = g0[t];
    for (int t = threadIdx.x; t < P3; t += blockDim.x) sgr[t] = G[(long long)b * P3 + t];
    if (stage_a1) {
      const uint4* g1 = reinterpret_cast<const uint4*>(a1g);
      for (int t = threadIdx.x; t < P1 * 2; t += blockDim.x) reinterpret_cast<uint4*>(sa1)[t] = g1[t];
    }
  }
  __syncthreads();
  const unsigned short* x = sx;
  const unsigned short* a1 = stage_a1 ? sa1 : a1g;
  const unsigned short* a2 = sa2;
  const float* g = sgr;
  float* part = partials + (long long)b * CNN_NPARAM;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;

  // --- layer 3: dZ2 = relu'(z2) * (W3 (x) G) on the P2 grid; dW3, db3
  for (int q = tid; q < P2; q += blockDim.x) {
    const int qy = q / w2, qx = q - qy * w2;
    float acc[16];
    for (int c = 0; c < 16; ++c) acc[c] = 0.f;
    for (int tap = 0; tap < 9; ++tap) {
      const int py = qy - tap / 3, px = qx - tap % 3;
      if (py < 0 || px < 0 || py >= n || px >= n) continue;
      const float gv = g[py * n + px];
      for (int c = 0; c < 16; ++c) acc[c] += bf2f(Wb[CNN_W3 + c * 9 + tap]) * gv;
    }
    for (int c = 0; c < 16; ++c) {
      const bool on = a2[q * 16 + c] != 0;  // a2 = relu(z2) stored in BF16: > 0 iff z2 > 0
      dz2[q * 16 + c] = f2bf(on ? acc[c] : 0.f);
    }
  }
  // dW3[c][tap] = sum_p a2[p + tap][c] g[p]; db3 = sum_p g[p]  (one thread per (c, tap))
  for (int k = tid; k < 16 * 9 + 1; k += blockDim.x) {
    float s = 0.f;
    if (k < 144) {
      const int c = k / 9, tap = k % 9, ty = tap / 3, tx = tap % 3;
      for (int p = 0; p < P3; ++p) {
        const int py = p / n, px = p - py * n;
        s += bf2f(a2[((py + ty) * w2 + px + tx) * 16 + c]) * g[p];
      }
      part[CNN_W3 + k] = s;
    } else {
      for (int p = 0; p < P3; ++p) s += g[p];
      part[CNN_B3] = s;
    }
  }
  __syncthreads();

  // --- layer 2 weight gradient: dW2[o][c][tap] = sum_p dz2[p][o] a1[p+tap][c]
  // D[i = o][j = c], K = pixels; wave w owns taps w, w + nw, ...
  for (int tap = wave; tap < 9; tap += nw) {
    const int ty = tap / 3, tx = tap % 3;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < P2; p0 += 16) {
      // A[o = i16][k = 4 kq + e] = dz2[p0 + 4kq + e][o]; B[k][c = i16] = a1[p + tap][c]
      s4 a, bb;
      short av[4], bv[4];
      for (int e = 0; e < 4; ++e) {
        const int p = p0 + 4 * kq + e;
        if (p < P2) {
          const int py = p / w2, px = p - py * w2;
          av[e] = (short)dz2[p * 16 + i16];
          bv[e] = (short)a1[((py + ty) * w1 + px + tx) * 16 + i16];
        } else {
          av[e] = 0;
          bv[e] = 0;
        }
      }
      a.x = av[0]; a.y = av[1]; a.z = av[2]; a.w = av[3];
      bb.x = bv[0]; bb.y = bv[1]; bb.z = bv[2]; bb.w = bv[3];
      acc = mfma(a, bb, acc);
    }
    for (int e = 0; e < 4; ++e) {
      const int o = 4 * kq + e, c = i16;
      part[CNN_W2 + (o * 16 + c) * 9 + tap] = acc[e];
    }
  }
  for (int o = tid; o < 16; o += blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < P2; ++p) s += bf2f(dz2[p * 16 + o]);
    part[CNN_B2 + o] = s;
  }

  // --- layer 2 data gradient: dZ1[q][c] = relu'(z1) sum_tap sum_o W2[o][c][tap] dz2[q - tap][o]
  // D[i = pixel][j = c]; A[pixel][k = o] from dz2 at q - tap; B[k = o][j = c] = W2[o][c][tap]
  {
    s4 bop[9];
    for (int tap = 0; tap < 9; ++tap) {
      s4 r;
      r.x = (short)Wb[CNN_W2 + ((4 * kq + 0) * 16 + i16) * 9 + tap];
      r.y = (short)Wb[CNN_W2 + ((4 * kq + 1) * 16 + i16) * 9 + tap];
      r.z = (short)Wb[CNN_W2 + ((4 * kq + 2) * 16 + i16) * 9 + tap];
      r.w = (short)Wb[CNN_W2 + ((4 * kq + 3) * 16 + i16) * 9 + tap];
      bop[tap] = r;
    }
    const int nblk = (P1 + 15) / 16;
    for (int blk = wave; blk < nblk; blk += nw) {
      const int p = 16 * blk + i16;
      const int pc = p < P1 ? p : P1 - 1;
      const int qy = pc / w1, qx = pc - qy * w1;
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int tap = 0; tap < 9; ++tap) {
        const int sy = qy - tap / 3, sx = qx - tap % 3;
        s4 a = zero4();
        if (sy >= 0 && sx >= 0 && sy < w2 && sx < w2) a = load4(dz2 + (sy * w2 + sx) * 16 + 4 * kq);
        acc = mfma(a, bop[tap], acc);
      }
      for (int e = 0; e < 4; ++e) {
        const int q = 16 * blk + 4 * kq + e;
        if (q < P1) {
          const bool on = a1[q * 16 + i16] != 0;
          dz1[q * 16 + i16] = f2bf(on ? acc[e] : 0.f);
        }
      }
    }
  }
  __syncthreads();

  // --- layer 1 weight gradient: dW1[o][c][tap] = sum_p dz1[p][o] x[p + tap][c]
  // D[i = o][j = k'] with k' = 4 tap' + c over 3 chunks of 16 (taps 4 kc .. 4 kc + 3)
  for (int kc = wave; kc < 3; kc += nw) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const int kp = 16 * kc + i16;     // column k' of this lane
    const int tap = kp >> 2, c = kp & 3;
    const int ty = tap / 3, tx = tap % 3;
    for (int p0 = 0; p0 < P1; p0 += 16) {
      short av[4], bv[4];
      for (int e = 0; e < 4; ++e) {
        const int p = p0 + 4 * kq + e;
        if (p < P1) {
          const int py = p / w1, px = p - py * w1;
          av[e] = (short)dz1[p * 16 + i16];
          bv[e] = tap < 9 ? (short)x[((py + ty) * w0 + px + tx) * 4 + c] : (short)0;
        } else {
          av[e] = 0;
          bv[e] = 0;
        }
      }
      s4 a, bb;
      a.x = av[0]; a.y = av[1]; a.z = av[2]; a.w = av[3];
      bb.x = bv[0]; bb.y = bv[1]; bb.z = bv[2]; bb.w = bv[3];
      acc = mfma(a, bb, acc);
    }
    if (tap < 9)
      for (int e = 0; e < 4; ++e) {
        const int o = 4 * kq + e;
        part[CNN_W1 + (o * 4 + c) * 9 + tap] = acc[e];
      }
  }
  for (int o = tid; o < 16; o += blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < P1; ++p) s += bf2f(dz1[p * 16 + o]);
    part[CNN_B1 + o] = s;
  }
}

// deterministic sum of the per-patch partials (fixed order over patches)
__global__ void k_cnn_reduce(const float* __restrict__ partials, int count, int np,
                             float* __restrict__ grads) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  float s = 0.f;
  for (int b = 0; b < count; ++b) s += partials[(long long)b * np + k];
  grads[k] = s;
}

// Adam on FP32 master weights, then the BF16 copy (round to nearest even)
__global__ void k_cnn_adam(float* __restrict__ params, const float* __restrict__ grads,
                           float* __restrict__ m, float* __restrict__ v, float lr, float c1,
                           float c2, int np, unsigned short* __restrict__ Wb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grads[k];
  const float mk = b1 * m[k] + (1.f - b1) * g;
  const float vk = b2 * v[k] + (1.f - b2) * g * g;
  m[k] = mk;
  v[k] = vk;
  const float mh = mk / c1, vh = vk / c2;
  const float p = params[k] - lr * mh / (sqrtf(vh) + eps);
  params[k] = p;
  Wb[k] = f2bf(p);
}

__global__ void k_cnn_to_bf16(const float* __restrict__ params, int np, unsigned short* __restrict__ Wb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < np) Wb[k] = f2bf(params[k]);
}

// per-patch refine request: any logit above the threshold
__global__ __launch_bounds__(256) void k_cnn_requests(int count, int n, const float* __restrict__ Z,
                                                      const int* __restrict__ pids, float zt,
                                                      uint8_t* __restrict__ flag) {
  const int b = blockIdx.x;
  if (b >= count) return;
  int any = 0;
  for (int p = threadIdx.x; p < n * n; p += blockDim.x) any |= Z[(long long)b * n * n + p] > zt;
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flag[pids[b]] = any ? 1 : 0;
}

// MFMA lane-layout check: D = A B for 16x16 BF16 matrices (row-major inputs)
__global__ void k_mfma_selftest(const unsigned short* __restrict__ A, const unsigned short* __restrict__ B,
                                float* __restrict__ D) {
  const int l = threadIdx.x;
  const int i = l & 15, kq = l >> 4;
  s4 a, b;
  a.x = (short)A[i * 16 + 4 * kq + 0];
  a.y = (short)A[i * 16 + 4 * kq + 1];
  a.z = (short)A[i * 16 + 4 * kq + 2];
  a.w = (short)A[i * 16 + 4 * kq + 3];
  b.x = (short)B[(4 * kq + 0) * 16 + i];
  b.y = (short)B[(4 * kq + 1) * 16 + i];
  b.z = (short)B[(4 * kq + 2) * 16 + i];
  b.w = (short)B[(4 * kq + 3) * 16 + i];
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = mfma(a, b, acc);
  for (int e = 0; e < 4; ++e) D[(4 * kq + e) * 16 + i] = acc[e];
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
size_t Cnn::fwd_lds(int n) {
  const int w0 = n + 6, w1 = n + 4, w2 = n + 2;
  return (size_t)(w0 * w0 * 4 + w1 * w1 * 16 + w2 * w2 * 16) * sizeof(unsigned short);
}

// LDS of the backward kernel: dz2, dz1, a2, the input, the logit gradients,
// and a1 when the total stays within the 160 KB of a CU
static size_t bwd_lds_parts(int n, bool with_a1) {
  const size_t P0 = (size_t)(n + 6) * (n + 6), P1 = (size_t)(n + 4) * (n + 4);
  const size_t P2 = (size_t)(n + 2) * (n + 2), P3 = (size_t)n * n;
  size_t bytes = (P2 * 16 + P1 * 16 + P2 * 16 + P0 * 4) * sizeof(unsigned short) + P3 * sizeof(float);
  if (with_a1) bytes += P1 * 16 * sizeof(unsigned short);
  return bytes;
}

static bool bwd_stage_a1(int n) { return bwd_lds_parts(n, true) <= 160 * 1024; }

size_t Cnn::bwd_lds(int n) { return bwd_lds_parts(n, bwd_stage_a1(n)); }

void Cnn::gather(const DevMesh& m, const double* U, const int* pids, int count, int n,
                 const CnnNorm& norm, unsigned short* X, hipStream_t s) {
  if (count <= 0) return;
  const long long total = (long long)count * (n + 6) * (n + 6);
  const int blocks = (int)std::min<long long>((total + 255) / 256, 65535);
  hipLaunchKernelGGL(k_cnn_gather, dim3(blocks), dim3(256), 0, s, m, U, pids, count, n, norm, X);
}

static void allow_large_lds() {
  static bool done = false;
  if (done) return;
  done = true;
  (void)hipFuncSetAttribute((const void*)k_cnn_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_cnn_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
}

void Cnn::forward(int count, int n, const unsigned short* X, const unsigned short* Wb,
                  const float* params, unsigned short* A1, unsigned short* A2, float* Z,
                  hipStream_t s) {
  if (count <= 0) return;
  allow_large_lds();
  hipLaunchKernelGGL(k_cnn_fwd, dim3(count), dim3(FWD_THREADS), fwd_lds(n), s, count, n, X, Wb,
                     params, A1, A2, Z);
}

void Cnn::loss(long long total, const float* Z, const uint8_t* Y, float pos_weight, float* G,
               float* partial, int nblocks, float* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_loss, dim3(nblocks), dim3(256), 0, s, total, Z, Y, pos_weight, G,
                     partial);
  hipLaunchKernelGGL(k_cnn_loss_final, dim3(1), dim3(64), 0, s, partial, nblocks, loss_out);
}

void Cnn::backward(int count, int n, const unsigned short* X, const unsigned short* A1,
                   const unsigned short* A2, const float* G, const unsigned short* Wb,
                   float* partials, float* grads, hipStream_t s) {
  if (count <= 0) return;
  allow_large_lds();
  hipLaunchKernelGGL(k_cnn_bwd, dim3(count), dim3(BWD_THREADS), bwd_lds(n), s, count, n, X, A1, A2,
                     G, Wb, partials, bwd_stage_a1(n) ? 1 : 0);
  reduce(partials, count, CNN_NPARAM, grads, s);
}

void Cnn::reduce(const float* partials, int count, int np, float* grads, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_reduce, dim3((np + 255) / 256), dim3(256), 0, s, partials, count, np,
                     grads);
}

void Cnn::adam(float* params, const float* grads, float* m, float* v, float lr, int t, int np,
               unsigned short* Wb, hipStream_t s) {
  const float c1 = 1.f - powf(0.9f, (float)t);
  const float c2 = 1.f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(k_cnn_adam, dim3((np + 255) / 256), dim3(256), 0, s, params, grads, m, v, lr,
                     c1, c2, np, Wb);
}

void Cnn::to_bf16(const float* params, int np, unsigned short* Wb, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_to_bf16, dim3((np + 255) / 256), dim3(256), 0, s, params, np, Wb);
}

void Cnn::requests(int count, int n, const float* Z, const int* pids, float zt, uint8_t* flag,
                   hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_cnn_requests, dim3(count), dim3(256), 0, s, count, n, Z, pids, zt, flag);
}

void Cnn::mfma_selftest(const unsigned short* A, const unsigned short* B, float* D, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, s, A, B, D);
}

}  // namespace amr
