// Scoring network shared by the simplify kernel (learned priority) and the
// training kernels: score(x) = w2 . relu(W1^T x + b1) + b2 with x, W1, w2 in
// bf16 and every sum in fp32.  The first layer is a dense 32 x 16 by 16 x 256
// contraction per wavefront and runs on the matrix cores
// (v_mfma_f32_32x32x16_bf16); the second layer is a 256-term dot product per
// row done on the VALU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "zx.h"

namespace zxmlp {

constexpr int IN = ZX_MLP_IN;     // 16 input features
constexpr int HID = ZX_MLP_HID;   // 256 hidden units
constexpr int TILES = HID / 32;   // 32-column tiles of the hidden layer

// parameter vector (fp32 master): W1[IN][HID] | b1[HID] | w2[HID] | b2
constexpr int P_W1 = 0;
constexpr int P_B1 = IN * HID;
constexpr int P_W2 = P_B1 + HID;
constexpr int P_B2 = P_W2 + HID;
constexpr int NPARAM = P_B2 + 1;
static_assert(NPARAM == ZX_MLP_NPARAM, "parameter count");
// bf16 copy: W1 transposed (hidden unit major, 16 inputs each) | w2
constexpr int Q_W1T = 0;
constexpr int Q_W2 = IN * HID;
constexpr int NBF16 = Q_W2 + HID;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// fp32 -> bf16, round to nearest even (finite inputs)
__host__ __device__ inline uint16_t to_bf16(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float from_bf16(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// Row of the 32 x 32 accumulator held in element i of a lane.
__device__ __forceinline__ int acc_row(int i, int lane) { return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3); }

// A operand of one lane: 8 bf16 features of row (lane & 31).
template <class P>
__device__ __forceinline__ bf16x8 load_a(P feats32 /* 32 rows x 16 bf16 */) {
  const int lane = threadIdx.x & 63;
  const uint4 q = *(const uint4*)(feats32 + (lane & 31) * IN + 8 * (lane >> 5));
  return __builtin_bit_cast(bf16x8, q);
}

// Scores of 32 rows; element i of s is the score of row acc_row(i, lane)
// (identical in the 32 lanes of a half-wave).  The weights of a tile are
// loaded inside the tile loop, which is kept rolled so that only one
// accumulator tile is live.
__device__ inline void score32(bf16x8 a, const uint16_t* wbf, const float* param, float s[16]) {
  const int lane = threadIdx.x & 63, g = lane >> 5;
#pragma unroll
  for (int i = 0; i < 16; ++i) s[i] = 0.f;
#pragma unroll 1
  for (int t = 0; t < TILES; ++t) {
    const int n = 32 * t + (lane & 31);
    const bf16x8 w = __builtin_bit_cast(bf16x8, *(const uint4*)(wbf + Q_W1T + n * IN + 8 * g));
    const float b1 = param[P_B1 + n];
    const float w2 = from_bf16(wbf[Q_W2 + n]);
    f32x16 z = {};
    const f32x16 acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, w, z, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i] += fmaxf(acc[i] + b1, 0.f) * w2;
  }
  // sum over the 32 hidden units a half-wave holds, fixed butterfly order
#pragma unroll
  for (int o = 1; o < 32; o <<= 1)
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i] += __shfl_xor(s[i], o, 64);
  const float b2 = param[P_B2];
#pragma unroll
  for (int i = 0; i < 16; ++i) s[i] += b2;
}

}  // namespace zxmlp
