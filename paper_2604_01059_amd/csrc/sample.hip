// Detector sampling f = T e (section on the repetition-code example,
// equation detector_sampling; the sampling paragraph after equation
// dets-only): per shot, the error mechanisms that fire are found by
// geometric gaps (drawn for the largest firing probability pmax, then
// thinned to each mechanism's own probability), and every firing
// mechanism's column of T is XORed into the shot's f bits.
//
// One lane per shot.  The shot's f row (fw <= 32 words) lives in LDS while
// the lane walks the mechanisms; the workgroup's rows are then written out
// as one contiguous block (rows of consecutive shots are adjacent when
// ld_out = fw).  Random numbers are counter-based SplitMix64 (Steele, Lea,
// Flood, OOPSLA 2014): draw t of shot s is mix64(seed + (s 2^32 + t + 1)
// GAMMA).  Per candidate: one draw for the gap, G = floor(ln U / ln(1 -
// pmax)), U = ((u >> 11) + 1) 2^-53 (no gap draw when pmax = 1), and one draw
// v for thinning: fire iff (v >> 11) < floor(p_j / pmax 2^53).  All in fp64.
#include "zx_internal.h"

namespace {

constexpr int DS_BS = 256;
constexpr int DS_MAX_FW = 32;

struct DetWs {
  ZxWsHeader hdr;      // status
  double pmax, log1m;  // largest probability, ln(1 - pmax)
  int32_t valid;
  int32_t pad[59];
  // followed by uint64_t thr[n_err]
};
static_assert(sizeof(DetWs) % 256 == 0, "workspace header size");

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// largest probability, its log, the thinning thresholds; one workgroup
// Also validates the model: col_ptr non-decreasing from 0 to nnz, every
// col_idx entry in [0, n_f), every probability in [0, 1]; otherwise the
// status becomes ZX_EINVAL and no shot is sampled (rows are written as zero).
__global__ __launch_bounds__(DS_BS) void det_prep_kernel(const int32_t* __restrict__ col_ptr,
                                                         const int32_t* __restrict__ col_idx, int64_t nnz,
                                                         const double* __restrict__ prob, int32_t n_err,
                                                         int32_t n_f, DetWs* ws, uint64_t* __restrict__ thr) {
  __shared__ double red[DS_BS];
  __shared__ int bad[DS_BS];
  double mx = 0.0;
  int b = 0;
  for (int j = threadIdx.x; j < n_err; j += DS_BS) {
    const double p = prob[j];
    if (!(p >= 0.0 && p <= 1.0)) b = 1;
    else mx = fmax(mx, p);
    if (col_ptr[j] > col_ptr[j + 1]) b = 1;
  }
  if (threadIdx.x == 0 && (col_ptr[0] != 0 || (int64_t)col_ptr[n_err] != nnz)) b = 1;
  for (int64_t q = threadIdx.x; q < nnz; q += DS_BS)
    if (col_idx[q] < 0 || col_idx[q] >= n_f) b = 1;
  red[threadIdx.x] = mx;
  bad[threadIdx.x] = b;
  __syncthreads();
  for (int o = DS_BS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
      bad[threadIdx.x] |= bad[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double pmax = red[0];
  const double two53 = 9007199254740992.0;
  if (bad[0]) {
    if (threadIdx.x == 0) {
      ws->hdr.status = ZX_EINVAL;
      ws->valid = 0;
    }
    return;
  }
  for (int j = threadIdx.x; j < n_err; j += DS_BS)
    thr[j] = pmax > 0.0 ? (uint64_t)(prob[j] / pmax * two53) : 0ull;
  if (threadIdx.x == 0) {
    ws->hdr.status = 0;
    ws->pmax = pmax;
    ws->log1m = log1p(-pmax);  // log(1 - pmax) would round to 0 below pmax = 2^-53
    ws->valid = 1;
  }
}

__global__ __launch_bounds__(DS_BS) void det_sample_kernel(const int32_t* __restrict__ col_ptr,
                                                           const int32_t* __restrict__ col_idx,
                                                           const DetWs* __restrict__ ws,
                                                           const uint64_t* __restrict__ thr, int32_t n_err,
                                                           int32_t fw, uint64_t seed, int64_t shot0,
                                                           int64_t n_shots, uint64_t* __restrict__ out,
                                                           int64_t ld_out) {
  extern __shared__ uint64_t rows[];  // [DS_BS][fw]
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * DS_BS + tid;
  uint64_t* row = rows + (size_t)tid * fw;
  for (int w = 0; w < fw; ++w) row[w] = 0;
  const double pmax = ws->pmax, log1m = ws->log1m;
  const bool run = ws->valid && pmax > 0.0 && i < n_shots;
  if (run) {
    const double two53 = 9007199254740992.0;
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    uint64_t state = seed + (((uint64_t)(shot0 + i)) << 32) * gamma;  // draw t: state + (t + 1) gamma
    int64_t pos = 0;
    for (;;) {
      if (pmax < 1.0) {
        state += gamma;
        const double U = (double)((sm_mix(state) >> 11) + 1) / two53;
        const double g = floor(log(U) / log1m);
        if (!(g < (double)(n_err - pos))) break;  // a NaN quotient ends the shot too
        pos += (int64_t)g;
      }
      if (pos >= n_err) break;
      state += gamma;
      if ((sm_mix(state) >> 11) < thr[pos]) {
        const int q1 = col_ptr[pos + 1];
        for (int q = col_ptr[pos]; q < q1; ++q) {
          const int bi = col_idx[q];
          row[bi >> 6] ^= 1ull << (bi & 63);
        }
      }
      pos += 1;
    }
  }
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * DS_BS;
  const int64_t nr = n_shots - r0 < DS_BS ? n_shots - r0 : DS_BS;
  for (int x = tid; x < nr * fw; x += DS_BS) {
    const int r = x / fw, w = x - r * fw;
    out[(r0 + r) * ld_out + w] = rows[(size_t)r * fw + w];
  }
}

}  // namespace

extern "C" size_t zx_detector_workspace_bytes(int32_t n_err) {
  if (n_err < 0) return 0;
  return sizeof(DetWs) + (((size_t)n_err * 8 + 255) & ~size_t(255));
}

extern "C" zx_status zx_detector_sample(const int32_t* col_ptr, const int32_t* col_idx, int64_t nnz,
                                        const double* prob, int32_t n_err, int32_t n_f, uint64_t seed,
                                        int64_t shot0, int64_t n_shots, uint64_t* out, int64_t ld_out, void* ws,
                                        size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(out && ws && col_ptr, "null argument");
  ZX_CHECK_ARG(n_err >= 0 && n_f > 0 && n_shots > 0 && shot0 >= 0 && nnz >= 0, "bad sizes");
  ZX_CHECK_ARG(n_err == 0 || prob, "null probabilities");
  ZX_CHECK_ARG(nnz == 0 || col_idx, "null col_idx");
  const int fw = (n_f + 63) / 64;
  ZX_CHECK_ARG(ld_out >= fw, "ld_out %lld < %d", (long long)ld_out, fw);
  ZX_CHECK_ARG(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  ZX_CHECK_ARG(shot0 + n_shots <= (1ll << 31), "shot index beyond 2^31");
  if (fw > DS_MAX_FW) {
    zx_set_error("n_f=%d beyond %d f bits per shot", n_f, 64 * DS_MAX_FW);
    return ZX_ECAPACITY;
  }
  if (ws_bytes < zx_detector_workspace_bytes(n_err)) {
    zx_set_error("workspace %zu < %zu bytes", ws_bytes, zx_detector_workspace_bytes(n_err));
    return ZX_ECAPACITY;
  }
  DetWs* W = (DetWs*)ws;
  uint64_t* thr = (uint64_t*)((uint8_t*)ws + sizeof(DetWs));
  hipLaunchKernelGGL(det_prep_kernel, dim3(1), dim3(DS_BS), 0, s, col_ptr, col_idx, nnz, prob, n_err, n_f, W, thr);
  ZX_HIP(hipGetLastError());
  const int64_t blocks = (n_shots + DS_BS - 1) / DS_BS;
  ZX_CHECK_ARG(blocks <= 0x7fffffff, "too many shots");
  const size_t lds = (size_t)DS_BS * fw * 8;
  ZX_HIP(hipFuncSetAttribute((const void*)det_sample_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(DS_BS * DS_MAX_FW * 8)));
  hipLaunchKernelGGL(det_sample_kernel, dim3((unsigned)blocks), dim3(DS_BS), lds, s, col_ptr, col_idx, W, thr,
                     n_err, fw, seed, shot0, n_shots, out, ld_out);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" zx_status zx_detector_status(const void* ws, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(ws, "null workspace");
  ZX_HIP(hipStreamSynchronize(s));
  int32_t st = 0;
  ZX_HIP(hipMemcpy(&st, ws, 4, hipMemcpyDeviceToHost));
  return st;
}
