// Internal interface of the refinement predictor kernels (cnn.hip: 2D,
// cnn3.hip: 3D).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "amr_internal.hpp"

namespace amr {

// Flat parameter layout (FP32 master and BF16 copy share it):
// W1 [16][4][3x3] | b1 [16] | W2 [16][16][3x3] | b2 [16] | W3 [16][3x3] | b3
constexpr int CNN_W1 = 0;
constexpr int CNN_B1 = CNN_W1 + 16 * 4 * 9;
constexpr int CNN_W2 = CNN_B1 + 16;
constexpr int CNN_B2 = CNN_W2 + 16 * 16 * 9;
constexpr int CNN_W3 = CNN_B2 + 16;
constexpr int CNN_B3 = CNN_W3 + 16 * 9;
constexpr int CNN_NPARAM = CNN_B3 + 1;

// 3D network on tiles of 8^3 output cells: input (rho, u, v, w, p) with a
// halo of 3 cells, stored with 8 channels per voxel (the last 3 zero);
// convolutions 5 -> 8 -> 8 -> 1 over 3x3x3 taps (tap = 9 dz + 3 dy + dx).
// W1 [8][5][27] | b1 [8] | W2 [8][8][27] | b2 [8] | W3 [8][27] | b3
constexpr int CNN3_TILE = 8;
constexpr int CNN3_CH = 8;  // stored channels per voxel
constexpr int CNN3_W1 = 0;
constexpr int CNN3_B1 = CNN3_W1 + 8 * 5 * 27;
constexpr int CNN3_W2 = CNN3_B1 + 8;
constexpr int CNN3_B2 = CNN3_W2 + 8 * 8 * 27;
constexpr int CNN3_W3 = CNN3_B2 + 8;
constexpr int CNN3_B3 = CNN3_W3 + 8 * 27;
constexpr int CNN3_NPARAM = CNN3_B3 + 1;
constexpr int CNN3_W0 = CNN3_TILE + 6;  // input tile edge
constexpr int CNN3_P0 = CNN3_W0 * CNN3_W0 * CNN3_W0;
constexpr int CNN3_P1 = (CNN3_TILE + 4) * (CNN3_TILE + 4) * (CNN3_TILE + 4);
constexpr int CNN3_P2 = (CNN3_TILE + 2) * (CNN3_TILE + 2) * (CNN3_TILE + 2);
constexpr int CNN3_P3 = CNN3_TILE * CNN3_TILE * CNN3_TILE;
// a tile item is pid * CNN3_MAX_TILES + tile index (tile = (tz nt + ty) nt + tx)
constexpr int CNN3_MAX_TILES = 64;

struct CnnNorm {
  float mean[5];  // (rho, u, v, p) in 2D, (rho, u, v, w, p) in 3D
  float istd[5];
};

struct Cnn {
  static size_t fwd_lds(int n);
  static size_t bwd_lds(int n);
  static void gather(const DevMesh& m, const double* U, const int* pids, int count, int n,
                     const CnnNorm& norm, unsigned short* X, hipStream_t s);
  static void forward(int count, int n, const unsigned short* X, const unsigned short* Wb,
                      const float* params, unsigned short* A1, unsigned short* A2, float* Z,
                      hipStream_t s);
  static void loss(long long total, const float* Z, const uint8_t* Y, float pos_weight, float* G,
                   float* partial, int nblocks, float* loss_out, hipStream_t s);
  static void backward(int count, int n, const unsigned short* X, const unsigned short* A1,
                       const unsigned short* A2, const float* G, const unsigned short* Wb,
                       float* partials, float* grads, hipStream_t s);
  static void reduce(const float* partials, int count, int np, float* grads, hipStream_t s);
  static void adam(float* params, const float* grads, float* m, float* v, float lr, int t, int np,
                   unsigned short* Wb, hipStream_t s);
  static void to_bf16(const float* params, int np, unsigned short* Wb, hipStream_t s);
  static void requests(int count, int n, const float* Z, const int* pids, float zt,
                       uint8_t* flag, hipStream_t s);
  static void mfma_selftest(const unsigned short* A, const unsigned short* B, float* D,
                            hipStream_t s);
};

// 3D kernels; `items` are tile items (see CNN3_MAX_TILES), one block each.
struct Cnn3 {
  static size_t fwd_lds();
  static size_t bwd_lds();
  static void gather(const DevMesh& m, const double* U, const int* items, int count,
                     const CnnNorm& norm, unsigned short* X, hipStream_t s);
  static void forward(int count, const unsigned short* X, const unsigned short* Wb,
                      const float* params, unsigned short* A1, unsigned short* A2, float* Z,
                      hipStream_t s);
  static void backward(int count, const unsigned short* X, const unsigned short* A1,
                       const unsigned short* A2, const float* G, const unsigned short* Wb,
                       float* partials, float* grads, hipStream_t s);
  static void requests(int count, const float* Z, const int* items, float zt, uint8_t* flag,
                       hipStream_t s);
};

}  // namespace amr
