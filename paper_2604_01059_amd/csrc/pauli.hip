// Symplectic commutation table of Pauli strings.
//
// A Pauli string is stored as two bit vectors x, z (the paper's per-qubit
// encoding (1,0) = X, (1,1) = Y, (0,1) = Z, (0,0) = I).  Strings i and j
// anticommute exactly when  sum_b x_i[b] z_j[b] + z_i[b] x_j[b]  is odd.
//
// Kernel: the table is symmetric, so only 64 x 64 tiles (i-tile it, j-word
// jw) with jw >= it are computed.  A workgroup of eight wavefronts covers
// eight consecutive j-words and IT consecutive i-tiles: wavefront w holds the
// 64 strings j of j-word jw = 8 bx + w in registers (loaded once when the
// qubits fit one chunk of 1024), and the i-tiles are staged in LDS one after
// another and read as broadcasts.  v_bitop3_b32 folds
// acc ^= (x_i & z_j) ^ (z_i & x_j) in two instructions per 32-bit half.
// Lane l accumulates the 64 parities of its string as a bit mask over i:
// that mask is word it of row j (the mirrored tile), and 64 ballots give
// word jw of the tile's rows i.  Keeping the j strings across IT tiles cuts
// their loads IT-fold (they were reloaded for every tile).
#include "zx_internal.h"

namespace {

constexpr int BS = 512;              // 8 wavefronts, one j-word each
constexpr int NJW = BS / 64;         // j-words per workgroup
constexpr int QCH = 16;              // 64-bit words of qubits per chunk
constexpr int IT = 8;                // i-tiles per workgroup

__device__ __forceinline__ uint32_t xor_and(uint32_t acc, uint32_t a, uint32_t b) {
  // acc ^ (a & b): truth table over (acc, a, b) = (0xF0, 0xCC, 0xAA) -> 0x78
  return __builtin_amdgcn_bitop3_b32(acc, a, b, 0x78);
}

// This lane's string j, qubit words [q0, q0 + nq) of the chunk, as halves.
__device__ __forceinline__ void load_j(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Z, int64_t j,
                                       int64_t n, int64_t ldq, int q0, int nq, int qw, uint64_t qmask,
                                       uint32_t* xj, uint32_t* zj) {
#pragma unroll
  for (int w = 0; w < QCH; ++w) {
    uint64_t xv = 0, zv = 0;
    if (w < nq && j < n) {
      const uint64_t mk = q0 + w == qw - 1 ? qmask : ~0ull;
      xv = X[j * ldq + q0 + w] & mk;
      zv = Z[j * ldq + q0 + w] & mk;
    }
    xj[2 * w] = (uint32_t)xv;
    xj[2 * w + 1] = (uint32_t)(xv >> 32);
    zj[2 * w] = (uint32_t)zv;
    zj[2 * w + 1] = (uint32_t)(zv >> 32);
  }
}

__global__ __launch_bounds__(BS) void pauli_kernel(const uint64_t* __restrict__ X,
                                                   const uint64_t* __restrict__ Z, int64_t n,
                                                   int qw, uint64_t qmask, int64_t ldq,
                                                   uint64_t* __restrict__ C, int64_t ldc) {
  __shared__ uint64_t xi_s[64][QCH];
  __shared__ uint64_t zi_s[64][QCH];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nwj = (n + 63) / 64;
  const int64_t jw0 = (int64_t)blockIdx.x * NJW, it0 = (int64_t)blockIdx.y * IT;
  if (jw0 + NJW - 1 < it0) return;  // every tile of the workgroup is below the diagonal
  const int64_t jw = jw0 + wv;
  const int64_t j = jw * 64 + lane;
  const bool one_chunk = qw <= QCH;
  uint32_t xj[2 * QCH], zj[2 * QCH];
  if (one_chunk) load_j(X, Z, j, n, ldq, 0, qw, qw, qmask, xj, zj);
  // every wave runs the same iterations (barriers inside); the bounds are
  // uniform over the workgroup
  for (int t = 0; t < IT && it0 + t < nwj; ++t) {
    const int64_t it = it0 + t, i0 = it * 64;
    const bool active = jw < nwj && jw >= it;
    uint64_t pbits = 0;  // bit i: parity of (i0 + i, j)
    for (int q0 = 0; q0 < qw; q0 += QCH) {
      const int nq = qw - q0 < QCH ? qw - q0 : QCH;
      __syncthreads();
      for (int x = threadIdx.x; x < 64 * QCH; x += BS) {
        const int r = x / QCH, w = x % QCH;
        const int64_t i = i0 + r;
        const bool in = i < n && w < nq;
        const uint64_t mk = q0 + w == qw - 1 ? qmask : ~0ull;
        xi_s[r][w] = in ? X[i * ldq + q0 + w] & mk : 0;
        zi_s[r][w] = in ? Z[i * ldq + q0 + w] & mk : 0;
      }
      if (!one_chunk && active) load_j(X, Z, j, n, ldq, q0, nq, qw, qmask, xj, zj);
      __syncthreads();
      if (!active) continue;
      // the 64 parities go into two 32-bit halves, one shift-or each
      uint32_t ph[2] = {0u, 0u};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        for (int rr = 0; rr < 32; ++rr) {
          const int r = 32 * h + rr;
          uint32_t acc = 0;
#pragma unroll
          for (int w = 0; w < QCH; ++w) {
            const uint64_t xi = xi_s[r][w], zi = zi_s[r][w];
            acc = xor_and(acc, (uint32_t)xi, zj[2 * w]);
            acc = xor_and(acc, (uint32_t)zi, xj[2 * w]);
            acc = xor_and(acc, (uint32_t)(xi >> 32), zj[2 * w + 1]);
            acc = xor_and(acc, (uint32_t)(zi >> 32), xj[2 * w + 1]);
          }
          ph[h] |= (__popc(acc) & 1u) << rr;
        }
      }
      pbits ^= ((uint64_t)ph[1] << 32) | ph[0];
    }
    if (!active) continue;
    // mirrored tile: row j, word it
    const uint64_t valid_i = (n - i0) >= 64 ? ~0ull : ((1ull << (n - i0)) - 1);
    if (j < n) C[j * ldc + it] = pbits & valid_i;
    // tile rows: row i0 + r, word jw
    uint64_t mine = 0;
    for (int r = 0; r < 64; ++r) {
      const uint64_t wrd = __ballot((pbits >> r) & 1);
      if (lane == r) mine = wrd;
    }
    const int64_t i = i0 + lane;
    if (i < n) C[i * ldc + jw] = mine;  // lanes j >= n contribute zeros
  }
}

}  // namespace

extern "C" zx_status zx_pauli_commute(const uint64_t* X, const uint64_t* Z, int64_t n_paulis,
                                      int32_t n_qubits, int64_t ld_q, uint64_t* C, int64_t ld_c,
                                      uint32_t flags, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(X && Z && C, "null argument");
  ZX_CHECK_ARG(n_paulis > 0 && n_qubits > 0, "empty input");
  const int qw = (n_qubits + 63) / 64;
  ZX_CHECK_ARG(ld_q >= qw, "ld_q too small");
  const int64_t nwj = (n_paulis + 63) / 64;
  ZX_CHECK_ARG(ld_c >= nwj, "ld_c too small");
  ZX_CHECK_ARG(nwj <= 65535 * (int64_t)NJW && (nwj + IT - 1) / IT <= 65535, "too many strings");
  ZX_CHECK_ARG((flags & (ZX_PAULI_FORCE_VALU | ZX_PAULI_FORCE_MFMA)) !=
                   (ZX_PAULI_FORCE_VALU | ZX_PAULI_FORCE_MFMA),
               "ZX_PAULI_FORCE_VALU and ZX_PAULI_FORCE_MFMA together");
  const bool mfma = (flags & ZX_PAULI_FORCE_MFMA) ||
                    (!(flags & ZX_PAULI_FORCE_VALU) && n_paulis >= ZX_PAULI_MFMA_MIN);
  if (mfma) {
    zx_status rc = zx_pauli_commute_mfma(X, Z, n_paulis, n_qubits, ld_q, C, ld_c, s);
    if (rc != ZX_OK) return rc;
  } else {
    const uint64_t qmask = (n_qubits % 64) ? ((1ull << (n_qubits % 64)) - 1) : ~0ull;
    dim3 grid((unsigned)((nwj + NJW - 1) / NJW), (unsigned)((nwj + IT - 1) / IT));
    hipLaunchKernelGGL(pauli_kernel, grid, dim3(BS), 0, s, X, Z, n_paulis, qw, qmask, ld_q, C, ld_c);
    ZX_HIP(hipGetLastError());
  }
  if (flags & ZX_SYNC) ZX_HIP(hipStreamSynchronize(s));
  return ZX_OK;
}
