// Internal interface of the 2D refinement predictor kernels (cnn.hip).
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

struct CnnNorm {
  float mean[4];
  float istd[4];
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
  static void adam(float* params, const float* grads, float* m, float* v, float lr, int t,
                   unsigned short* Wb, hipStream_t s);
  static void to_bf16(const float* params, unsigned short* Wb, hipStream_t s);
  static void requests(int count, int n, const float* Z, const int* pids, float zt,
                       uint8_t* flag, hipStream_t s);
  static void mfma_selftest(const unsigned short* A, const unsigned short* B, float* D,
                            hipStream_t s);
};

}  // namespace amr
