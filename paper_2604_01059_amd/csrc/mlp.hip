// Training kernels of the scoring network (learned rewrite proposal):
// forward, per-state softmax cross-entropy, backward with a deterministic
// reduction, Adam.  Network and numerics: mlp_dev.h.
#include <algorithm>
#include "zx_internal.h"
#include "mlp_dev.h"

using namespace zxmlp;

namespace {

constexpr int FBS = 256;            // forward block: 4 wavefronts
constexpr int BBS = 128;            // backward block: 2 wavefronts (LDS partials)
constexpr int MAX_BWD_WAVES = 1024;  // partial gradients kept per backward call

__global__ void mlp_sync_kernel(const float* param, uint16_t* wbf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < IN * HID) {
    const int k = i / HID, n = i - k * HID;
    wbf[Q_W1T + n * IN + k] = to_bf16(param[P_W1 + i]);
  } else if (i < IN * HID + HID) {
    const int n = i - IN * HID;
    wbf[Q_W2 + n] = to_bf16(param[P_W2 + n]);
  }
}

// A operand for rows row0..row0+31 of x; rows >= rows read as zero.
__device__ inline bf16x8 load_a_global(const uint16_t* x, int64_t row0, int64_t rows) {
  const int lane = threadIdx.x & 63;
  const int64_t r = row0 + (lane & 31);
  uint4 q = {0, 0, 0, 0};
  if (r < rows) q = *(const uint4*)(x + r * IN + 8 * (lane >> 5));
  return __builtin_bit_cast(bf16x8, q);
}

__global__ __launch_bounds__(FBS) void mlp_forward_kernel(const uint16_t* wbf, const float* param,
                                                          const uint16_t* x, int64_t rows, float* score) {
  const int lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * (FBS / 64) + (threadIdx.x >> 6)) * 32;
  if (row0 >= rows) return;
  float s[16];
  score32(load_a_global(x, row0, rows), wbf, param, s);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t r = row0 + acc_row(i, lane);
    if ((lane & 31) == i && r < rows) score[r] = s[i];
  }
}

// One wavefront per segment.
__global__ void mlp_loss_kernel(const float* score, const int64_t* cost, const int32_t* seg_off,
                                int32_t n_seg, float* dscore, float* loss) {
  const int lane = threadIdx.x & 63;
  const int seg = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (seg >= n_seg) return;
  const int a = seg_off[seg], b = seg_off[seg + 1];
  // target: even over the present rows of least cost
  int64_t bc = INT64_MAX;
  float mx = -INFINITY;
  for (int r = a + lane; r < b; r += 64) {
    const int64_t cr = cost[r];
    if (cr < 0) continue;
    bc = cr < bc ? cr : bc;
    mx = fmaxf(mx, score[r]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t oc = __shfl_xor(bc, o);
    bc = oc < bc ? oc : bc;
    mx = fmaxf(mx, __shfl_xor(mx, o));
  }
  if (bc == INT64_MAX) {  // no present row
    for (int r = a + lane; r < b; r += 64) dscore[r] = 0.f;
    if (lane == 0) loss[seg] = 0.f;
    return;
  }
  float se = 0.f, st = 0.f;
  int nt = 0;
  for (int r = a + lane; r < b; r += 64) {
    if (cost[r] < 0) continue;
    se += expf(score[r] - mx);
    if (cost[r] == bc) {
      st += score[r];
      ++nt;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_xor(se, o);
    st += __shfl_xor(st, o);
    nt += __shfl_xor(nt, o);
  }
  const float inv = 1.0f / (float)n_seg, tw = 1.0f / (float)nt;
  for (int r = a + lane; r < b; r += 64) {
    float d = 0.f;
    if (cost[r] >= 0) d = (expf(score[r] - mx) / se - (cost[r] == bc ? tw : 0.f)) * inv;
    dscore[r] = d;
  }
  if (lane == 0) loss[seg] = logf(se) + mx - st * tw;
}

// Backward.  Wavefront w of nw handles the 32-row chunks w, w + nw, ... in
// order and accumulates its partial gradient in LDS (each entry owned by one
// lane); the partials are written to ws[w] and summed over w in order by
// mlp_reduce_kernel.
__global__ __launch_bounds__(BBS) void mlp_backward_kernel(const uint16_t* wbf, const float* param,
                                                           const uint16_t* x, const float* dscore,
                                                           int64_t rows, int nw, float* ws) {
  __shared__ float acc[BBS / 64][NPARAM];
  __shared__ __align__(16) uint16_t xs[BBS / 64][32 * IN];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 5;
  const int w = blockIdx.x * (BBS / 64) + wv;
  if (w >= nw) return;  // whole wavefronts only; no block barrier below
  float* A = acc[wv];
  for (int i = lane; i < NPARAM; i += 64) A[i] = 0.f;
  const int64_t nchunks = (rows + 31) / 32;
  for (int64_t ch = w; ch < nchunks; ch += nw) {
    const int64_t row0 = ch * 32;
    // stage the chunk's features (zero beyond rows)
    for (int i = lane; i < 32 * IN / 8; i += 64) {
      const int r = i / (IN / 8), part = i - r * (IN / 8);
      uint4 q = {0, 0, 0, 0};
      if (row0 + r < rows) q = *(const uint4*)(x + (row0 + r) * IN + 8 * part);
      *(uint4*)(&xs[wv][r * IN + 8 * part]) = q;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const bf16x8 a = __builtin_bit_cast(bf16x8, *(const uint4*)(&xs[wv][(lane & 31) * IN + 8 * g]));
    float ds[16];
    float dsum = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t r = row0 + acc_row(i, lane);
      ds[i] = r < rows ? dscore[r] : 0.f;
      dsum += ds[i];
    }
#pragma unroll 1
    for (int t = 0; t < TILES; ++t) {
      const int n = 32 * t + (lane & 31);
      const bf16x8 wv1 = __builtin_bit_cast(bf16x8, *(const uint4*)(wbf + Q_W1T + n * IN + 8 * g));
      const float b1 = param[P_B1 + n];
      const float w2 = from_bf16(wbf[Q_W2 + n]);
      f32x16 z = {};
      const f32x16 pre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, wv1, z, 0, 0, 0);
      float gw2 = 0.f, gb1 = 0.f, gw1[IN];
#pragma unroll
      for (int k = 0; k < IN; ++k) gw1[k] = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float p = pre[i] + b1;
        const float h = fmaxf(p, 0.f);
        gw2 += h * ds[i];
        const float dp = p > 0.f ? ds[i] * w2 : 0.f;
        gb1 += dp;
        const uint16_t* xr = &xs[wv][acc_row(i, lane) * IN];
        const uint4 q0 = *(const uint4*)xr, q1 = *(const uint4*)(xr + 8);
        const uint32_t qq[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int k = 0; k < IN; ++k) {
          const uint16_t hv = (uint16_t)(qq[k >> 1] >> (16 * (k & 1)));
          gw1[k] += from_bf16(hv) * dp;
        }
      }
      // the two half-waves hold the same column n for different rows
      gw2 += __shfl_xor(gw2, 32);
      gb1 += __shfl_xor(gb1, 32);
#pragma unroll
      for (int k = 0; k < IN; ++k) gw1[k] += __shfl_xor(gw1[k], 32);
      if (g == 0) {
        A[P_W2 + n] += gw2;
        A[P_B1 + n] += gb1;
#pragma unroll
        for (int k = 0; k < IN; ++k) A[P_W1 + k * HID + n] += gw1[k];
      }
    }
    // db2: sum of the chunk's dscore (each row counted once: elements of one
    // half-wave, any single lane of it)
    float d2 = dsum + __shfl_xor(dsum, 32);
    if (lane == 0) A[P_B2] += d2;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  float* out = ws + (int64_t)w * NPARAM;
  for (int i = lane; i < NPARAM; i += 64) out[i] = A[i];
}

__global__ void mlp_reduce_kernel(const float* ws, int nw, float* grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  float s = 0.f;
  for (int w = 0; w < nw; ++w) s += ws[(int64_t)w * NPARAM + i];
  grad[i] = s;
}

__global__ void mlp_adam_kernel(float* param, uint16_t* wbf, const float* grad, float* m, float* v,
                                float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float p = param[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  param[i] = p;
  if (i < IN * HID) {
    const int k = i / HID, n = i - k * HID;
    wbf[Q_W1T + n * IN + k] = to_bf16(p);
  } else if (i >= P_W2 && i < P_W2 + HID) {
    wbf[Q_W2 + (i - P_W2)] = to_bf16(p);
  }
}

int bwd_waves(int64_t rows) {
  const int64_t c = (rows + 31) / 32;
  return (int)std::min<int64_t>(std::max<int64_t>(c, 1), MAX_BWD_WAVES);
}

}  // namespace

extern "C" zx_status zx_mlp_sync(const zx_mlp* w, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(w && w->param && w->wbf16, "null network");
  hipLaunchKernelGGL(mlp_sync_kernel, dim3((NBF16 + 255) / 256), dim3(256), 0, s, w->param, w->wbf16);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" zx_status zx_mlp_forward(const zx_mlp* w, const uint16_t* x, int64_t rows, float* score,
                                    hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(w && w->param && w->wbf16, "null network");
  ZX_CHECK_ARG(rows >= 0, "negative rows");
  if (rows == 0) return ZX_OK;
  ZX_CHECK_ARG(x && score, "null buffer");
  const int64_t waves = (rows + 31) / 32;
  const int64_t blocks = (waves + FBS / 64 - 1) / (FBS / 64);
  ZX_CHECK_ARG(blocks <= INT32_MAX, "too many rows");
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((uint32_t)blocks), dim3(FBS), 0, s, w->wbf16, w->param, x,
                     rows, score);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" zx_status zx_mlp_loss(const float* score, const int64_t* cost, const int32_t* seg_off,
                                 int32_t n_seg, float* dscore, float* loss, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(n_seg >= 0, "negative segment count");
  if (n_seg == 0) return ZX_OK;
  ZX_CHECK_ARG(score && cost && seg_off && dscore && loss, "null buffer");
  const int per = 4;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3((n_seg + per - 1) / per), dim3(64 * per), 0, s, score, cost,
                     seg_off, n_seg, dscore, loss);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" size_t zx_mlp_workspace_bytes(int64_t rows) {
  if (rows < 0) return 0;
  return (size_t)bwd_waves(rows) * NPARAM * sizeof(float);
}

extern "C" zx_status zx_mlp_backward(const zx_mlp* w, const uint16_t* x, const float* dscore, int64_t rows,
                                     float* grad, void* ws, size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(w && w->param && w->wbf16, "null network");
  ZX_CHECK_ARG(rows >= 0 && grad && ws, "bad argument");
  ZX_CHECK_ARG(rows == 0 || (x && dscore), "null buffer");
  if (ws_bytes < zx_mlp_workspace_bytes(rows)) {
    zx_set_error("workspace too small");
    return ZX_ECAPACITY;
  }
  const int nw = bwd_waves(rows);
  const int blocks = (nw + BBS / 64 - 1) / (BBS / 64);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(blocks), dim3(BBS), 0, s, w->wbf16, w->param, x, dscore, rows,
                     nw, (float*)ws);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, (const float*)ws, nw,
                     grad);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" zx_status zx_mlp_adam(const zx_mlp* w, const float* grad, float* m, float* v, float lr,
                                 float beta1, float beta2, float eps, int32_t step, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(w && w->param && w->wbf16 && grad && m && v, "null buffer");
  ZX_CHECK_ARG(step >= 1, "step counts from 1");
  ZX_CHECK_ARG(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f, "bad Adam constants");
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, w->param, w->wbf16, grad,
                     m, v, lr, beta1, beta2, eps, bc1, bc2);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}
