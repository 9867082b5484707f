// GF(2) reduced row echelon form on one MI355X: one cooperative persistent
// launch, every 64-bit word column resident in a workgroup's LDS.
//
// Method.  Gauss-Jordan elimination over F2 (the paper keeps a linearly
// independent basis of a binary matrix this way; detectors/observables
// section, after equation detector_sampling), organised by 64-column word
// strips.  For strip s:
//   1. the workgroup that owns word column s picks up to 128 candidate rows
//      (not yet pivots, non-zero in the strip) and reduces them in one
//      wavefront: for each bit b, a ballot finds the first candidate with bit
//      b set, its word is broadcast and XORed into every other candidate
//      holding b.  This yields up to 64 pivot rows, their bit positions and,
//      per pivot, a 64-bit mask L saying which ORIGINAL pivot rows combine
//      into the reduced pivot row;
//   2. it publishes that "pass" (rows, bits, masks) plus a snapshot of its
//      column to the other workgroups through a small ring in the workspace
//      (release/acquire flags, cumulative acknowledgement counters);
//   3. every workgroup applies the pass to each of its columns c > s:
//      reduced pivot words P'_j = XOR of L_j-selected original pivot words,
//      then every other row r gets XOR of P' over the pivot bits set in its
//      strip word (Four-Russians: 16 tables of 16 nibble combinations, one
//      lookup per nibble, conflict-free in LDS), and pivot rows become P'.
// If a pass found fewer than 64 pivots while more non-zero rows existed
// than candidates, the owner runs further passes on the residual rows.  The
// pivot columns found are always leading bits of row-space vectors, and the
// passes only stop when every non-pivot row is zero in the strip, so the
// final rows are the unique RREF basis.  Rows stay in place; the output is
// written at the end, pivot rows in pivot-column order, then zero rows.
#include <string.h>

#include "zx_internal.h"

namespace {

constexpr int BS = 512;       // threads per workgroup
constexpr int RING = 8;       // pass records in flight
constexpr int NCAND = 128;    // candidate rows per pass
constexpr int MAX_M = 16384;  // rows that fit one column per workgroup in LDS
constexpr int MAX_CW = 4;     // word columns per workgroup

struct PassRec {
  int32_t strip;
  int32_t k;       // pivots in this pass (0 for an end-of-strip marker)
  int32_t last;    // strip finished with this record
  int32_t pad0;
  int32_t rows[64];
  int32_t bits[64];
  uint64_t L[64];
};

struct Ctl {
  uint32_t seq;        // records published
  uint32_t pad[63];
  uint32_t ack[RING];  // cumulative acknowledgements per slot
  uint32_t pad2[64 - RING];
};

struct WsLayout {
  size_t ctl, recs, snaps, piv_row, piv_col, bytes;
};

WsLayout ws_layout(int m) {
  WsLayout L;
  size_t o = 256;  // ZxWsHeader
  L.ctl = o;     o += (sizeof(Ctl) + 255) & ~size_t(255);
  L.recs = o;    o += ((sizeof(PassRec) * RING) + 255) & ~size_t(255);
  L.snaps = o;   o += (((size_t)m * 8 * RING) + 255) & ~size_t(255);
  L.piv_row = o; o += (((size_t)m * 4) + 255) & ~size_t(255);
  L.piv_col = o; o += (((size_t)m * 4) + 255) & ~size_t(255);
  L.bytes = o;
  return L;
}

struct Args {
  const uint64_t* A;
  uint64_t* R;
  int32_t m, n_cols, nw, cw;
  int64_t ld;
  int32_t* rank_dev;
  int32_t* piv_dev;
  int32_t* status;
  Ctl* ctl;
  PassRec* recs;
  uint64_t* snaps;
  int32_t* piv_row;
  int32_t* piv_col;
  uint64_t spin_ticks;  // time-out of one spin wait, in s_memrealtime ticks
};

__device__ __forceinline__ uint32_t ld_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin (thread 0 only) until *p >= target; false on time-out or abort.
__device__ bool spin_until(const uint32_t* p, uint32_t target, const Args& a) {
  uint64_t t0 = wall_clock64();
  for (;;) {
    if (ld_acquire(p) >= target) return true;
    if (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > a.spin_ticks) {
      zx_dev_fail(a.status, ZX_EDEVICE);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

__global__ void rref_init(Ctl* ctl, int32_t* status) {
  int t = threadIdx.x;
  uint32_t* c = (uint32_t*)ctl;
  for (int i = t; i < (int)(sizeof(Ctl) / 4); i += blockDim.x) c[i] = 0;
  if (t == 0) *status = 0;
}

struct Smem {
  // fixed part (after the columns)
  uint64_t tab[16 * 16];   // nibble tables of the column being updated
  uint64_t orig[64];       // original pivot words of the column
  uint64_t pp[64];         // reduced pivot words
  uint64_t Q[64];          // reduced pivot word by strip bit position (0 = no pivot)
  uint64_t L[64];
  int32_t rows[64];
  int32_t bits[64];
  int32_t cand[NCAND];
  int32_t scan[BS / 64 + 1];
  int32_t k, last, strip, ncand, total, flag, pad[2];
  uint64_t pivmask;
};

// Block-wide: first NCAND rows that are non-pivot and non-zero in column
// `col`; returns the total number of such rows.
__device__ int gather_candidates(const uint64_t* col, const uint64_t* pivflag, int m, Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (m + BS - 1) / BS;  // contiguous rows per thread (<= 32)
  const int r0 = tid * per;
  uint32_t mask = 0;
  for (int i = 0; i < per; ++i) {
    int r = r0 + i;
    if (r < m && !((pivflag[r >> 6] >> (r & 63)) & 1) && col[r] != 0) mask |= 1u << i;
  }
  int cnt = __popc(mask);
  // inclusive scan within the wave
  int x = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) S.scan[wv] = x;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int w = 0; w < BS / 64; ++w) {
      int v = S.scan[w];
      S.scan[w] = acc;
      acc += v;
    }
    S.scan[BS / 64] = acc;
  }
  __syncthreads();
  int pos = S.scan[wv] + x - cnt;
  while (mask && pos < NCAND) {
    int i = __ffs(mask) - 1;
    mask &= mask - 1;
    S.cand[pos++] = r0 + i;
  }
  int total = S.scan[BS / 64];
  __syncthreads();
  return total;
}

// Wave 0: reduce the candidates of strip `col`; fills S.k, rows, bits, L.
__device__ void factor_candidates(const uint64_t* col, int nc, Smem& S) {
  const int lane = threadIdx.x & 63;
  uint64_t w0 = lane < nc ? col[S.cand[lane]] : 0;
  uint64_t w1 = 64 + lane < nc ? col[S.cand[64 + lane]] : 0;
  uint64_t L0 = 0, L1 = 0;
  bool p0 = false, p1 = false;
  int j0 = -1, j1 = -1;
  int k = 0;
  for (int b = 0; b < 64 && k < 64; ++b) {
    const uint64_t bit = 1ull << b;
    uint64_t bal0 = __ballot(!p0 && (w0 & bit));
    uint64_t bal1 = __ballot(!p1 && (w1 & bit));
    if ((bal0 | bal1) == 0) continue;
    const bool hi = bal0 == 0;
    const int src = __ffsll((long long)(hi ? bal1 : bal0)) - 1;
    const uint64_t pw = __shfl(hi ? w1 : w0, src);
    const uint64_t pl = __shfl(hi ? L1 : L0, src) | (1ull << k);
    const bool me0 = !hi && lane == src, me1 = hi && lane == src;
    if (me0) { p0 = true; j0 = k; L0 |= 1ull << k; }
    if (me1) { p1 = true; j1 = k; L1 |= 1ull << k; }
    if ((w0 & bit) && !me0) { w0 ^= pw; L0 ^= pl; }
    if ((w1 & bit) && !me1) { w1 ^= pw; L1 ^= pl; }
    if (lane == 0) {
      S.rows[k] = S.cand[(hi ? 64 : 0) + src];
      S.bits[k] = b;
    }
    ++k;
  }
  if (j0 >= 0) S.L[j0] = L0;
  if (j1 >= 0) S.L[j1] = L1;
  if (lane == 0) S.k = k;
}

// Apply the pass held in S (k, rows, bits, L, pivmask) to one LDS column,
// with multipliers taken from snapshot `snap` (strip words before the pass).
__device__ void apply_pass(uint64_t* col, const uint64_t* snap, int m, Smem& S) {
  const int tid = threadIdx.x;
  const int k = S.k;
  if (tid < k) S.orig[tid] = col[S.rows[tid]];
  if (tid < 64) S.Q[tid] = 0;
  __syncthreads();
  if (tid < k) {
    uint64_t Lm = S.L[tid], x = 0;
    while (Lm) {
      int i = __ffsll((long long)Lm) - 1;
      Lm &= Lm - 1;
      x ^= S.orig[i];
    }
    S.pp[tid] = x;
    S.Q[S.bits[tid]] = x;
  }
  __syncthreads();
  if (tid < 256) {
    const int t = tid >> 4, e = tid & 15;
    uint64_t v = 0;
    for (int i = 0; i < 4; ++i)
      if ((e >> i) & 1) v ^= S.Q[4 * t + i];
    S.tab[tid] = v;
  }
  __syncthreads();
  const uint64_t pm = S.pivmask;
  for (int r = tid; r < m; r += BS) {
    uint64_t mr = snap[r] & pm;
    if (mr) {
      uint64_t acc = 0;
#pragma unroll
      for (int t = 0; t < 16; ++t) acc ^= S.tab[16 * t + ((mr >> (4 * t)) & 15)];
      col[r] ^= acc;
    }
  }
  __syncthreads();
  if (tid < k) col[S.rows[tid]] = S.pp[tid];
  __syncthreads();
}

__device__ void load_record(const PassRec* rec, Smem& S) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    S.k = rec->k;
    S.last = rec->last;
    S.strip = rec->strip;
  }
  __syncthreads();
  const int k = S.k;
  if (tid < k) {
    S.rows[tid] = rec->rows[tid];
    S.bits[tid] = rec->bits[tid];
    S.L[tid] = rec->L[tid];
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t pm = 0;
    for (int j = 0; j < k; ++j) pm |= 1ull << S.bits[j];
    S.pivmask = pm;
  }
  __syncthreads();
}

__device__ void mark_pivots(uint64_t* pivflag, Smem& S) {
  const int tid = threadIdx.x;
  if (tid < S.k) atomicOr((unsigned long long*)&pivflag[S.rows[tid] >> 6], 1ull << (S.rows[tid] & 63));
  __syncthreads();
}

__global__ __launch_bounds__(BS) void rref_kernel(Args a) {
  extern __shared__ __align__(16) uint64_t smem[];
  const int tid = threadIdx.x;
  const int g = blockIdx.x, G = gridDim.x;
  const int m = a.m;
  const int nown = (a.nw - g + G - 1) / G;  // columns owned: g, g+G, ...
  uint64_t* cols = smem;                                  // [cw][m]
  uint64_t* pivflag = cols + (size_t)a.cw * m;            // [ceil(m/64)]
  const int pw = (m + 63) / 64;
  Smem& S = *reinterpret_cast<Smem*>(pivflag + pw);

  // load owned columns (bits >= n_cols masked off)
  for (int j = 0; j < nown; ++j) {
    const int c = g + j * G;
    const int tail = a.n_cols - 64 * c;
    const uint64_t cm = tail >= 64 ? ~0ull : ((1ull << tail) - 1);
    for (int r = tid; r < m; r += BS) cols[(size_t)j * m + r] = a.A[(size_t)r * a.ld + c] & cm;
  }
  for (int i = tid; i < pw; i += BS) pivflag[i] = 0;
  __syncthreads();

  uint32_t seq = 0;  // next record index
  int rank = 0;
  bool ok = true;
  for (int s = 0; s < a.nw && rank < m && ok; ++s) {
    const int owner = s % G;
    if (owner == g) {
      // ---------------- produce strip s ----------------
      uint64_t* col = cols + (size_t)(s / G) * m;
      const int rank0 = rank;
      bool published_any = false;
      for (;;) {
        const int total = gather_candidates(col, pivflag, m, S);
        const int nc = total < NCAND ? total : NCAND;
        int k = 0, last = 1;
        if (total > 0) {
          if (tid < 64) factor_candidates(col, nc, S);
          __syncthreads();
          k = S.k;
          last = (k == 64 || total <= NCAND) ? 1 : 0;
        } else if (published_any) {
          // residual pass found nothing: strip ends with an empty marker
          k = 0;
          last = 1;
        } else {
          k = 0;
          last = 1;
        }
        // pivot list entries (global), sorted by column at the strip end
        if (tid < k) {
          a.piv_row[rank + tid] = S.rows[tid];
          a.piv_col[rank + tid] = 64 * s + S.bits[tid];
        }
        __syncthreads();
        if (last && published_any && tid == 0) {
          // multi-pass strip: sort this strip's pivots by column
          const int lo = rank0, hi = rank + k;
          for (int i = lo + 1; i < hi; ++i) {
            int kc = a.piv_col[i], kr = a.piv_row[i], j = i - 1;
            while (j >= lo && a.piv_col[j] > kc) {
              a.piv_col[j + 1] = a.piv_col[j];
              a.piv_row[j + 1] = a.piv_row[j];
              --j;
            }
            a.piv_col[j + 1] = kc;
            a.piv_row[j + 1] = kr;
          }
        }
        // wait until the ring slot is free
        const int slot = seq % RING;
        if (tid == 0) {
          const uint32_t need = (seq / RING) * (uint32_t)(G - 1);
          S.flag = spin_until(&a.ctl->ack[slot], need, a) ? 1 : 0;
        }
        __syncthreads();
        if (!S.flag) { ok = false; break; }
        PassRec* rec = a.recs + slot;
        uint64_t* snap = a.snaps + (size_t)slot * m;
        if (k > 0)
          for (int r = tid; r < m; r += BS) snap[r] = col[r];
        if (tid < k) {
          rec->rows[tid] = S.rows[tid];
          rec->bits[tid] = S.bits[tid];
          rec->L[tid] = S.L[tid];
        }
        if (tid == 0) {
          rec->strip = s;
          rec->k = k;
          rec->last = last;
          S.k = k;
          S.last = last;
          uint64_t pm = 0;
          for (int j = 0; j < k; ++j) pm |= 1ull << S.bits[j];
          S.pivmask = pm;
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) st_release(&a.ctl->seq, seq + 1);
        ++seq;
        published_any = true;
        if (k > 0) {
          // own columns c >= s (this strip first)
          for (int j = s / G; j < nown; ++j) apply_pass(cols + (size_t)j * m, snap, m, S);
          mark_pivots(pivflag, S);
          rank += k;
        }
        if (last) break;
      }
    } else {
      // ---------------- consume strip s ----------------
      for (;;) {
        const int slot = seq % RING;
        if (tid == 0) S.flag = spin_until(&a.ctl->seq, seq + 1, a) ? 1 : 0;
        __syncthreads();
        if (!S.flag) { ok = false; break; }
        const PassRec* rec = a.recs + slot;
        load_record(rec, S);
        const uint64_t* snap = a.snaps + (size_t)slot * m;
        const int k = S.k, last = S.last;
        if (k > 0) {
          // owned columns with index > s
          int j0 = (s - g) >= 0 ? (s - g) / G + 1 : 0;
          for (int j = j0; j < nown; ++j) apply_pass(cols + (size_t)j * m, snap, m, S);
          mark_pivots(pivflag, S);
          rank += k;
        }
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(&a.ctl->ack[slot], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        ++seq;
        if (last) break;
      }
    }
  }
  if (!ok) return;
  // ---------------- write the result ----------------
  __threadfence();
  __syncthreads();
  for (int j = 0; j < nown; ++j) {
    const int c = g + j * G;
    const uint64_t* col = cols + (size_t)j * m;
    for (int i = tid; i < m; i += BS) {
      uint64_t v = 0;
      if (i < rank) v = col[a.piv_row[i]];
      a.R[(size_t)i * a.ld + c] = v;
    }
  }
  if (g == 0) {
    for (int i = tid; i < m; i += BS) a.piv_dev[i] = i < rank ? a.piv_col[i] : -1;
    if (tid == 0) *a.rank_dev = rank;
  }
}

int co_resident_blocks(size_t lds) {
  static int cached_blocks = -1;
  static size_t cached_lds = 0;
  if (cached_blocks >= 0 && cached_lds == lds) return cached_blocks;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)rref_kernel, BS, lds) != hipSuccess)
    return 0;
  const ZxDevice* d = zx_device();
  cached_blocks = per_cu * (d ? d->n_cu : 0);
  cached_lds = lds;
  return cached_blocks;
}

size_t smem_bytes(int m, int cw) {
  return (size_t)cw * m * 8 + (size_t)((m + 63) / 64) * 8 + sizeof(Smem);
}

}  // namespace

extern "C" size_t zx_gf2_workspace_bytes(int32_t m, int32_t n_cols) {
  (void)n_cols;
  if (m <= 0) return 256;
  return ws_layout(m).bytes;
}

extern "C" zx_status zx_gf2_status(const void* ws, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(ws, "null workspace");
  ZX_HIP(hipStreamSynchronize(s));
  int32_t st = 0;
  ZX_HIP(hipMemcpy(&st, ws, 4, hipMemcpyDeviceToHost));
  return st;
}

extern "C" zx_status zx_gf2_eliminate(const uint64_t* A, uint64_t* R, int32_t m, int32_t n_cols,
                                      int64_t ld_words, int32_t* rank_dev, int32_t* pivot_cols_dev,
                                      void* ws, size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(A && R && rank_dev && pivot_cols_dev && ws, "null argument");
  ZX_CHECK_ARG(m > 0 && n_cols > 0, "empty matrix: m=%d n_cols=%d", m, n_cols);
  const int nw = (n_cols + 63) / 64;
  ZX_CHECK_ARG(ld_words >= nw, "ld_words %lld < %d", (long long)ld_words, nw);
  ZX_CHECK_ARG(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  if (A != R) {
    const char* a0 = (const char*)A;
    const char* a1 = a0 + (size_t)m * ld_words * 8;
    const char* r0 = (const char*)R;
    const char* r1 = r0 + (size_t)m * ld_words * 8;
    ZX_CHECK_ARG(a1 <= r0 || r1 <= a0, "A and R overlap without being equal");
  }
  if (m > MAX_M) {
    zx_set_error("m=%d exceeds %d rows per LDS column", m, MAX_M);
    return ZX_ECAPACITY;
  }
  WsLayout W = ws_layout(m);
  if (ws_bytes < W.bytes) {
    zx_set_error("workspace %zu < %zu bytes", ws_bytes, W.bytes);
    return ZX_ECAPACITY;
  }
  const ZxDevice* dev = zx_device();
  if (!dev) {
    zx_set_error("no HIP device");
    return ZX_EDEVICE;
  }
  // choose columns per workgroup so that the grid is co-resident
  int cw = 1, G = 0;
  size_t lds = 0;
  for (cw = 1; cw <= MAX_CW; ++cw) {
    lds = smem_bytes(m, cw);
    if (lds > dev->lds_per_block) break;
    G = (nw + cw - 1) / cw;
    ZX_HIP(hipFuncSetAttribute((const void*)rref_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (G <= co_resident_blocks(lds)) break;
    G = 0;
  }
  if (G == 0) {
    zx_set_error("matrix %d x %d does not fit the co-resident grid", m, n_cols);
    return ZX_ECAPACITY;
  }
  uint8_t* base = (uint8_t*)ws;
  Args a;
  a.A = A;
  a.R = R;
  a.m = m;
  a.n_cols = n_cols;
  a.nw = nw;
  a.cw = cw;
  a.ld = ld_words;
  a.rank_dev = rank_dev;
  a.piv_dev = pivot_cols_dev;
  a.status = (int32_t*)base;
  a.ctl = (Ctl*)(base + W.ctl);
  a.recs = (PassRec*)(base + W.recs);
  a.snaps = (uint64_t*)(base + W.snaps);
  a.piv_row = (int32_t*)(base + W.piv_row);
  a.piv_col = (int32_t*)(base + W.piv_col);
  a.spin_ticks = 100000000ull * 5;  // 5 s at the 100 MHz real-time counter
  hipLaunchKernelGGL(rref_init, dim3(1), dim3(256), 0, s, a.ctl, a.status);
  ZX_HIP(hipGetLastError());
  void* args[] = {&a};
  ZX_HIP(hipLaunchCooperativeKernel((const void*)rref_kernel, dim3(G), dim3(BS), args, (unsigned)lds, s));
  return ZX_OK;
}
