// Rewriting of graph-like ZX diagrams on the GPU: single local
// complementations and pivots, the batched fixed-point simplifier and the
// output-frontier elimination.
//
// Rules (appendix "Rewrite rules" of the paper):
//  * local complementation at an interior spider u of phase pi/2 + b pi:
//    complement the Hadamard edges among N(u), subtract pi/2 + b pi from
//    every neighbour's phase, delete u, scalar e^{-i b pi/2} e^{i pi/4}
//    times a power of sqrt(2);
//  * pivot on an edge u-v of interior Pauli spiders (phases a pi, b pi):
//    complement every edge between different classes of {N(u) only, N(v)
//    only, both}, add b pi / a pi / (a + b + 1) pi to their phases, delete u
//    and v, scalar e^{i a b pi} times a power of sqrt(2).
// For the sqrt(2) power both rules agree with the bookkeeping "every
// Hadamard edge carries 1/sqrt(2), every deleted Clifford spider sqrt(2)":
// a rewrite multiplies in sqrt(2)^(E_after - E_before + deleted).  This is
// the rules' printed scalar rewritten with the edge counts (the printed LC
// power (n-1)(n-2)/2 is the case with no edges among the neighbours).
//
// Data-parallel form.  A round applies a set S of rewrites whose spiders are
// pairwise non-adjacent (and distinct), so the rewrites commute and each
// neighbourhood is unaffected by the others.  The combined effect on a row
// w outside S is one GF(2) rank-|S| update
//     row_w ^= XOR over x in S with w ~ x of contrib(x),
// with contrib(u) = row_u for local complementation (the diagonal bit is
// cleared afterwards) and contrib(u) = row_v minus u, contrib(v) = row_u
// minus v for a pivot pair (u, v).  Rows are processed by "teams" of
// T = min(64, pow2(W)) lanes, lane t owning words t, t + T, ...
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "zx_internal.h"

namespace {

constexpr int MAXW = 128;   // words per row (n <= 8192)
constexpr int MAXS = 2;     // words per lane in a team of 64

__host__ __device__ inline int ldw_lds(int W) { return W | 1; }  // odd LDS row stride

__host__ __device__ inline int64_t aux_bytes(int n, int W) {
  int64_t k = (n + 7) & ~7;
  int64_t part = (2 * (int64_t)n + 7) & ~7;
  return k + k + part + 8 * 8 * (int64_t)W;
}
__host__ __device__ inline int64_t lds_adj_bytes(int n, int W) { return (int64_t)n * ldw_lds(W) * 8; }

struct Shared {
  int64_t E;           // Hadamard edges among present spiders
  int64_t pow_sqrt2;
  int64_t fill_in;
  int64_t acc64[4];    // per-round accumulators
  int32_t phase8;
  int32_t n_trace;
  int32_t round;
  int32_t any;
  int32_t any2;
  int32_t cnt;
  int32_t key;
  int32_t idx;
  int32_t status;
  int32_t rank;
  int64_t rowops;
};

struct Ctx {
  ZxHeader* h;
  uint8_t* base;
  int n, W, ldw, q_in, q_out;
  uint64_t* adj;     // work adjacency (LDS or global)
  int8_t* k;         // phases (LDS)
  int8_t* kc;        // per-selected contribution to neighbour phases (LDS)
  int16_t* partner;  // pivot partner (LDS)
  uint64_t* alive;
  uint64_t* bnd;
  uint64_t* cand;
  uint64_t* sel;
  uint64_t* inm;
  uint64_t* outm;
  uint64_t* blocked;
  uint64_t* omask;   // output-attached spiders
  int32_t* trace;    // global, 4 int32 per entry
  int T, nteams, team, tl;
};

__device__ __forceinline__ bool bit_of(const uint64_t* m, int v) { return (m[v >> 6] >> (v & 63)) & 1; }

__device__ __forceinline__ uint64_t wave_shfl64(uint64_t v, int src, int width) {
  return __shfl(v, src, width);
}

__device__ __forceinline__ int team_size(int W) {
  int T = 1;
  while (T < W && T < 64) T <<= 1;
  return T;
}

template <int BS>
__device__ void block_sync() { __syncthreads(); }

// --------------------------------------------------------------- setup --
template <int BS>
__device__ void setup_ctx(Ctx& c, uint8_t* arena, uint8_t* lds, bool lds_adj) {
  c.h = (ZxHeader*)arena;
  c.base = arena;
  c.n = c.h->n;
  c.W = c.h->W;
  c.q_in = c.h->n_in;
  c.q_out = c.h->n_out;
  const int n = c.n, W = c.W;
  uint8_t* p = lds;
  if (lds_adj) {
    c.adj = (uint64_t*)p;
    c.ldw = ldw_lds(W);
    p += lds_adj_bytes(n, W);
  } else {
    c.adj = (uint64_t*)(arena + c.h->off_adj);
    c.ldw = W;
  }
  const int64_t kb = (n + 7) & ~7;
  c.k = (int8_t*)p; p += kb;
  c.kc = (int8_t*)p; p += kb;
  c.partner = (int16_t*)p; p += (2 * (int64_t)n + 7) & ~7;
  c.alive = (uint64_t*)p; p += 8 * W;
  c.bnd = (uint64_t*)p; p += 8 * W;
  c.cand = (uint64_t*)p; p += 8 * W;
  c.sel = (uint64_t*)p; p += 8 * W;
  c.inm = (uint64_t*)p; p += 8 * W;
  c.outm = (uint64_t*)p; p += 8 * W;
  c.blocked = (uint64_t*)p; p += 8 * W;
  c.omask = (uint64_t*)p; p += 8 * W;
  c.trace = (int32_t*)(arena + c.h->off_trace);
  c.T = team_size(W);
  c.nteams = BS / c.T;
  c.team = threadIdx.x / c.T;
  c.tl = threadIdx.x % c.T;
}

__device__ __forceinline__ uint64_t* row_ptr(const Ctx& c, int r) { return c.adj + (size_t)r * c.ldw; }

// Sum over threads of v into an LDS 64-bit accumulator.
__device__ __forceinline__ void block_add(int64_t* acc, int64_t v) {
  if (v) atomicAdd((unsigned long long*)acc, (unsigned long long)v);
}

// Edge count of the work adjacency (rows are already masked to present spiders).
template <int BS>
__device__ int64_t count_edges(Ctx& c, Shared& sh) {
  if (threadIdx.x == 0) sh.acc64[3] = 0;
  __syncthreads();
  int64_t pc = 0;
  const int n = c.n, W = c.W;
  for (int64_t i = threadIdx.x; i < (int64_t)n * W; i += BS) {
    const int r = (int)(i / W), j = (int)(i % W);
    pc += __popcll(row_ptr(c, r)[j]);
  }
  block_add(&sh.acc64[3], pc);
  __syncthreads();
  const int64_t e = sh.acc64[3] / 2;
  __syncthreads();
  return e;
}

// Load a diagram's state.  from_source: SOURCE section, else CURRENT.
template <int BS>
__device__ void load_state(Ctx& c, Shared& sh, bool lds_adj, bool from_source) {
  const int n = c.n, W = c.W, tid = threadIdx.x;
  const uint64_t* src = (const uint64_t*)(c.base + (from_source ? c.h->off_src_adj : c.h->off_adj));
  const int8_t* srcph = (const int8_t*)(c.base + (from_source ? c.h->off_src_phase : c.h->off_phase));
  if (lds_adj || from_source) {
    for (int64_t i = tid; i < (int64_t)n * W; i += BS) {
      const int r = (int)(i / W), j = (int)(i % W);
      row_ptr(c, r)[j] = src[i];
    }
  }
  for (int v = tid; v < n; v += BS) {
    c.k[v] = srcph[v];
    c.kc[v] = 0;
    c.partner[v] = -1;
  }
  const uint64_t* bm = (const uint64_t*)(c.base + c.h->off_bndmask);
  const uint64_t* al = (const uint64_t*)(c.base + c.h->off_alive);
  for (int j = tid; j < W; j += BS) {
    uint64_t full = (j < W - 1 || (n & 63) == 0) ? ~0ull : ((1ull << (n & 63)) - 1);
    c.alive[j] = from_source ? full : al[j];
    c.bnd[j] = bm[j];
    c.cand[j] = c.sel[j] = c.inm[j] = c.outm[j] = c.blocked[j] = c.omask[j] = 0;
  }
  __syncthreads();
  const int32_t* outs = (const int32_t*)(c.base + c.h->off_out);
  for (int j = tid; j < c.q_out; j += BS) {
    const int v = outs[j];
    atomicOr((unsigned long long*)&c.omask[v >> 6], 1ull << (v & 63));
  }
  if (tid == 0) {
    if (from_source) {
      sh.pow_sqrt2 = 0;
      sh.phase8 = 0;
      sh.fill_in = 0;
    } else {
      sh.pow_sqrt2 = c.h->pow_sqrt2;
      sh.phase8 = c.h->phase8;
      sh.fill_in = c.h->fill_in;
    }
    sh.n_trace = 0;
    sh.round = 0;
    sh.status = 0;
  }
  __syncthreads();
  const int64_t e = count_edges<BS>(c, sh);
  if (tid == 0) sh.E = e;
  __syncthreads();
}

// Write the work state back to the CURRENT section and the header.
template <int BS>
__device__ void store_state(Ctx& c, Shared& sh, bool lds_adj) {
  const int n = c.n, W = c.W, tid = threadIdx.x;
  uint64_t* dst = (uint64_t*)(c.base + c.h->off_adj);
  if (lds_adj) {
    for (int64_t i = tid; i < (int64_t)n * W; i += BS) {
      const int r = (int)(i / W), j = (int)(i % W);
      dst[i] = row_ptr(c, r)[j];
    }
  }
  int8_t* ph = (int8_t*)(c.base + c.h->off_phase);
  for (int v = tid; v < n; v += BS) ph[v] = c.k[v];
  uint64_t* al = (uint64_t*)(c.base + c.h->off_alive);
  int cnt = 0;
  for (int j = tid; j < W; j += BS) {
    al[j] = c.alive[j];
    cnt += __popcll(c.alive[j]);
  }
  if (tid == 0) sh.cnt = 0;
  __syncthreads();
  if (cnt) atomicAdd(&sh.cnt, cnt);
  __syncthreads();
  if (tid == 0) {
    c.h->pow_sqrt2 = sh.pow_sqrt2;
    c.h->phase8 = sh.phase8 & 7;
    c.h->fill_in = sh.fill_in;
    c.h->n_edges = sh.E;
    c.h->n_alive = sh.cnt;
  }
  __syncthreads();
}

// ------------------------------------------------------- candidate masks --
// kind 0: local-complementation candidates (interior, k in {2, 6});
// kind 1: Pauli candidates (interior, k in {0, 4}).  Returns non-empty.
template <int BS>
__device__ bool build_candidates(Ctx& c, Shared& sh, int kind) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) sh.any = 0;
  __syncthreads();
  for (int j = wv; j < c.W; j += BS / 64) {
    const int v = 64 * j + lane;
    bool ok = false;
    if (v < c.n) {
      const int kk = c.k[v];
      ok = bit_of(c.alive, v) && !bit_of(c.bnd, v) && ((kk & 3) == (kind == 0 ? 2 : 0));
    }
    const uint64_t wrd = __ballot(ok);
    if (lane == 0) {
      c.cand[j] = wrd;
      if (wrd) sh.any = 1;
    }
  }
  __syncthreads();
  return sh.any != 0;
}

// Lexicographically-first maximal independent set of the candidates (in
// ascending spider id): a candidate joins when no lower candidate neighbour
// joined, is excluded when one did.  Sweeps until every candidate is decided.
template <int BS>
__device__ void lfmis(Ctx& c, Shared& sh) {
  const int tid = threadIdx.x, W = c.W;
  for (int j = tid; j < W; j += BS) {
    c.inm[j] = 0;
    c.outm[j] = 0;
  }
  __syncthreads();
  for (;;) {
    if (tid == 0) sh.any = 0;
    __syncthreads();
    for (int v = tid; v < c.n; v += BS) {
      if (!bit_of(c.cand, v) || bit_of(c.inm, v) || bit_of(c.outm, v)) continue;
      const uint64_t* row = row_ptr(c, v);
      const int vw = v >> 6;
      bool out = false, pending = false;
      for (int j = 0; j <= vw; ++j) {
        uint64_t low = row[j] & c.cand[j];
        if (j == vw) low &= (1ull << (v & 63)) - 1;
        if (low & c.inm[j]) { out = true; break; }
        if (low & ~c.outm[j]) pending = true;
      }
      if (out) atomicOr((unsigned long long*)&c.outm[vw], 1ull << (v & 63));
      else if (!pending) atomicOr((unsigned long long*)&c.inm[vw], 1ull << (v & 63));
      else sh.any = 1;
    }
    __syncthreads();
    if (!sh.any) break;
    __syncthreads();
  }
  for (int j = tid; j < W; j += BS) c.sel[j] = c.inm[j];
  __syncthreads();
}

// Wave 0: lexicographic pivot-pair selection among the Pauli candidates.
// Writes partner[], sel (both ends), blocked, the trace entries; returns
// the number of pairs through sh.cnt.
template <int BS>
__device__ void select_pivots(Ctx& c, Shared& sh) {
  const int tid = threadIdx.x, W = c.W;
  for (int j = tid; j < W; j += BS) {
    c.sel[j] = 0;
    c.blocked[j] = 0;
  }
  __syncthreads();
  if (tid < 64) {
    const int lane = tid;
    uint64_t blk[MAXS], Pm[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int j = lane + 64 * s;
      blk[s] = 0;
      Pm[s] = j < W ? c.cand[j] : 0;
    }
    int npairs = 0, nt = sh.n_trace;
    const int round = sh.round;
    for (int wi = 0; wi < W; ++wi) {
      uint64_t pw = c.cand[wi];
      while (pw) {
        const int b = __ffsll((long long)pw) - 1;
        pw &= pw - 1;
        const int u = 64 * wi + b;
        // blocked bit of u (owned by lane wi % 64, slot wi / 64)
        uint64_t bw = wave_shfl64(wi < 64 ? blk[0] : blk[1], wi & 63, 64);
        if ((bw >> b) & 1) continue;
        const uint64_t* ru = row_ptr(c, u);
        uint64_t t[MAXS];
#pragma unroll
        for (int s = 0; s < MAXS; ++s) {
          const int j = lane + 64 * s;
          uint64_t x = 0;
          if (j < W) {
            x = ru[j] & Pm[s] & ~blk[s];
            if (j < wi) x = 0;
            else if (j == wi) x &= ~((2ull << b) - 1);  // strictly above u
          }
          t[s] = x;
        }
        const uint64_t bal0 = __ballot(t[0] != 0);
        const uint64_t bal1 = MAXS > 1 ? __ballot(t[1] != 0) : 0;
        if ((bal0 | bal1) == 0) continue;
        int v;
        if (bal0) {
          const int src = __ffsll((long long)bal0) - 1;
          const uint64_t x = wave_shfl64(t[0], src, 64);
          v = 64 * src + __ffsll((long long)x) - 1;
        } else {
          const int src = __ffsll((long long)bal1) - 1;
          const uint64_t x = wave_shfl64(t[1], src, 64);
          v = 64 * (64 + src) + __ffsll((long long)x) - 1;
        }
        const uint64_t* rv = row_ptr(c, v);
#pragma unroll
        for (int s = 0; s < MAXS; ++s) {
          const int j = lane + 64 * s;
          if (j < W) {
            uint64_t add = ru[j] | rv[j];
            if (j == (u >> 6)) add |= 1ull << (u & 63);
            if (j == (v >> 6)) add |= 1ull << (v & 63);
            blk[s] |= add;
          }
        }
        if (lane == 0) {
          c.partner[u] = (int16_t)v;
          c.partner[v] = (int16_t)u;
          int32_t* e = c.trace + 4 * (int64_t)nt;
          e[0] = round;
          e[1] = 1;
          e[2] = u;
          e[3] = v;
          c.sel[u >> 6] |= 1ull << (u & 63);
          c.sel[v >> 6] |= 1ull << (v & 63);
        }
        ++npairs;
        ++nt;
      }
    }
    if (lane == 0) {
      sh.cnt = npairs;
      sh.n_trace = nt;
    }
  }
  __syncthreads();
}

// Per-round bookkeeping over the selected spiders (before the update).
// LC: acc64[0] = sum deg, acc64[1] = sum deg(deg-1)/2, acc64[2] = phase sum.
// Pivot: acc64[0] = sum (deg u + deg v - 1), acc64[1] = sum T_p, acc64[2] = phase.
// Also fills kc[] and, for pivots, swaps each pair's rows into contributions.
template <int BS>
__device__ void prepare_round(Ctx& c, Shared& sh, bool pivot, bool graph_only) {
  const int W = c.W;
  if (threadIdx.x == 0) sh.acc64[0] = sh.acc64[1] = sh.acc64[2] = 0;
  __syncthreads();
  for (int x = c.team; x < c.n; x += c.nteams) {
    if (!bit_of(c.sel, x)) continue;
    const int p = pivot ? c.partner[x] : -1;
    if (pivot && p < x) continue;  // one team per pair, at its lower end
    uint64_t* rx = row_ptr(c, x);
    int dx = 0, dp = 0, common = 0;
    for (int j = c.tl; j < W; j += c.T) {
      const uint64_t a = rx[j];
      dx += __popcll(a);
      if (pivot) {
        const uint64_t b = row_ptr(c, p)[j];
        dp += __popcll(b);
        common += __popcll(a & b);
      }
    }
    for (int o = c.T / 2; o > 0; o >>= 1) {
      dx += __shfl_xor(dx, o, c.T);
      dp += __shfl_xor(dp, o, c.T);
      common += __shfl_xor(common, o, c.T);
    }
    if (c.tl == 0) {
      if (!pivot) {
        block_add(&sh.acc64[0], dx);
        block_add(&sh.acc64[1], (int64_t)dx * (dx - 1) / 2);
        block_add(&sh.acc64[2], c.k[x] == 2 ? 1 : 7);  // e^{-i b pi/2} e^{i pi/4}
        c.kc[x] = (int8_t)((8 - c.k[x]) & 7);
      } else {
        // pair (x, p): |a| = dx - 1, |b| = dp - 1, common neighbours exclude x, p
        const int64_t A = dx - 1, B = dp - 1;
        block_add(&sh.acc64[0], dx + dp - 1);
        block_add(&sh.acc64[1], A * B - (int64_t)common * common);
        block_add(&sh.acc64[2], 4 * ((c.k[x] / 4) * (c.k[p] / 4)));
        c.kc[x] = c.k[p];
        c.kc[p] = c.k[x];
      }
    }
    if (pivot) {
      // contrib(x) = row_p minus x, contrib(p) = row_x minus p: swap rows
      uint64_t* rp = row_ptr(c, p);
      for (int j = c.tl; j < W; j += c.T) {
        uint64_t a = rx[j], b = rp[j];
        if (j == (x >> 6)) b &= ~(1ull << (x & 63));
        if (j == (p >> 6)) a &= ~(1ull << (p & 63));
        rx[j] = b;
        rp[j] = a;
      }
    }
  }
  __syncthreads();
  (void)graph_only;
}

// The rank-|S| update of every present row outside S.
template <int BS>
__device__ void apply_round(Ctx& c, Shared& sh, bool pivot, bool graph_only) {
  const int W = c.W, T = c.T, tl = c.tl;
  for (int w = c.team; w < c.n; w += c.nteams) {
    if (!bit_of(c.alive, w) || bit_of(c.sel, w)) continue;
    uint64_t* row = row_ptr(c, w);
    uint64_t mw[MAXS], acc[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int j = tl + s * T;
      mw[s] = j < W ? row[j] & c.sel[j] : 0;
      acc[s] = 0;
    }
    int dk = 0;
    bool any = false;
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      if (s * T >= W) break;
      for (int l = 0; l < T; ++l) {
        const int i = s * T + l;
        if (i >= W) break;
        uint64_t mi = wave_shfl64(mw[s], l, T);
        while (mi) {
          const int b = __ffsll((long long)mi) - 1;
          mi &= mi - 1;
          const int x = 64 * i + b;
          const uint64_t* rx = row_ptr(c, x);
#pragma unroll
          for (int s2 = 0; s2 < MAXS; ++s2) {
            const int j = tl + s2 * T;
            if (j < W) acc[s2] ^= rx[j];
          }
          if (!graph_only) {
            dk += c.kc[x];
            if (pivot) {
              const int p = c.partner[x];
              if ((row[p >> 6] >> (p & 63)) & 1) dk += 2;  // adjacent to both ends
            }
          }
          any = true;
        }
      }
    }
    if (!any) continue;
    // every lane of the team has read `row` above (mw, partner tests)
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int j = tl + s * T;
      if (j < W) {
        uint64_t v = row[j] ^ acc[s];
        if (!graph_only) v &= ~c.sel[j];
        if (j == (w >> 6)) v &= ~(1ull << (w & 63));
        row[j] = v;
      }
    }
    if (!graph_only && tl == 0) c.k[w] = (int8_t)((c.k[w] + dk) & 7);
  }
  __syncthreads();
}

// Delete the selected spiders (rows zeroed, alive cleared, phase 0).
template <int BS>
__device__ void delete_selected(Ctx& c) {
  const int W = c.W;
  for (int x = c.team; x < c.n; x += c.nteams) {
    if (!bit_of(c.sel, x)) continue;
    uint64_t* rx = row_ptr(c, x);
    for (int j = c.tl; j < W; j += c.T) rx[j] = 0;
    if (c.tl == 0) c.k[x] = 0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < W; j += BS) c.alive[j] &= ~c.sel[j];
  __syncthreads();
}

// Scalar and counters after a ZX round (not graph-only).
template <int BS>
__device__ void finish_round(Ctx& c, Shared& sh, bool pivot, int removed) {
  const int64_t e_before = sh.E;
  const int64_t e_after = count_edges<BS>(c, sh);
  if (threadIdx.x == 0) {
    sh.pow_sqrt2 += (e_after - e_before) + removed;
    sh.phase8 = (int32_t)((sh.phase8 + sh.acc64[2]) & 7);
    // edges toggled on = (pairs toggled + change among the other spiders) / 2
    const int64_t others_before = e_before - sh.acc64[0];
    sh.fill_in += (sh.acc64[1] + (e_after - others_before)) / 2;
    sh.E = e_after;
  }
  __syncthreads();
  (void)pivot;
}

// Trace entries of a local-complementation round (ascending spider id).
template <int BS>
__device__ void trace_lc_round(Ctx& c, Shared& sh) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int base = sh.n_trace;
    for (int j0 = 0; j0 < c.W; j0 += 64) {
      const int j = j0 + lane;
      const uint64_t wd = j < c.W ? c.sel[j] : 0;
      const int cnt = __popcll(wd);
      int x = cnt;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
      }
      int pos = base + x - cnt;
      uint64_t m = wd;
      while (m) {
        const int b = __ffsll((long long)m) - 1;
        m &= m - 1;
        int32_t* e = c.trace + 4 * (int64_t)pos;
        e[0] = sh.round;
        e[1] = 0;
        e[2] = 64 * j + b;
        e[3] = -1;
        ++pos;
      }
      base += __shfl(x, 63);
    }
    if (lane == 0) sh.n_trace = base;
  }
  __syncthreads();
}

// ----------------------------------------------------------- simplify --
template <int BS>
__device__ void simplify_rounds(Ctx& c, Shared& sh) {
  // local-complementation rounds
  for (;;) {
    if (!build_candidates<BS>(c, sh, 0)) break;
    lfmis<BS>(c, sh);
    if (threadIdx.x == 0) sh.cnt = 0;
    __syncthreads();
    int cnt = 0;
    for (int j = threadIdx.x; j < c.W; j += BS) cnt += __popcll(c.sel[j]);
    if (cnt) atomicAdd(&sh.cnt, cnt);
    __syncthreads();
    const int removed = sh.cnt;
    trace_lc_round<BS>(c, sh);
    prepare_round<BS>(c, sh, false, false);
    apply_round<BS>(c, sh, false, false);
    delete_selected<BS>(c);
    finish_round<BS>(c, sh, false, removed);
    if (threadIdx.x == 0) sh.round++;
    __syncthreads();
  }
  // pivot rounds
  for (;;) {
    if (!build_candidates<BS>(c, sh, 1)) break;
    select_pivots<BS>(c, sh);
    const int npairs = sh.cnt;
    if (npairs == 0) break;
    prepare_round<BS>(c, sh, true, false);
    apply_round<BS>(c, sh, true, false);
    delete_selected<BS>(c);
    finish_round<BS>(c, sh, true, 2 * npairs);
    for (int v = threadIdx.x; v < c.n; v += BS)
      if (bit_of(c.sel, v)) c.partner[v] = -1;
    if (threadIdx.x == 0) sh.round++;
    __syncthreads();
  }
}

// Output frontier: rows = spiders of outputs 0..q-1, columns = spider ids,
// bit c = edge to a present spider c not attached to an output; then
// Gauss-Jordan with the lowest-index pivot row, counting row additions.
// M: q x W words (LDS or global).
template <int BS>
__device__ void frontier(Ctx& c, Shared& sh, uint64_t* M) {
  const int q = c.q_out, W = c.W, tid = threadIdx.x;
  const int32_t* outs = (const int32_t*)(c.base + c.h->off_out);
  for (int64_t i = tid; i < (int64_t)q * W; i += BS) {
    const int r = (int)(i / W), j = (int)(i % W);
    M[i] = row_ptr(c, outs[r])[j] & c.alive[j] & ~c.omask[j];
  }
  if (tid == 0) {
    sh.rank = 0;
    sh.rowops = 0;
  }
  __syncthreads();
  int32_t* fpiv = (int32_t*)(c.base + c.h->off_fpiv);
  int cur = 0, cmin = 0;
  while (cur < q) {
    if (tid == 0) sh.key = 0x7fffffff;
    __syncthreads();
    // lowest (column, row) over rows >= cur
    for (int r = cur + tid; r < q; r += BS) {
      const uint64_t* mr = M + (size_t)r * W;
      for (int j = cmin >> 6; j < W; ++j) {
        if (mr[j]) {
          const int col = 64 * j + __ffsll((long long)mr[j]) - 1;
          atomicMin(&sh.key, (col << 15) | r);
          break;
        }
      }
    }
    __syncthreads();
    const int key = sh.key;
    if (key == 0x7fffffff) break;
    const int col = key >> 15, r = key & 0x7fff;
    if (r != cur) {
      for (int j = tid; j < W; j += BS) {
        const uint64_t a = M[(size_t)r * W + j];
        M[(size_t)r * W + j] = M[(size_t)cur * W + j];
        M[(size_t)cur * W + j] = a;
      }
    }
    __syncthreads();
    int ops = 0;
    const uint64_t* pr = M + (size_t)cur * W;
    for (int i = tid; i < q; i += BS) {
      if (i == cur) continue;
      uint64_t* mi = M + (size_t)i * W;
      if ((mi[col >> 6] >> (col & 63)) & 1) {
        for (int j = 0; j < W; ++j) mi[j] ^= pr[j];
        ++ops;
      }
    }
    if (ops) atomicAdd((unsigned long long*)&sh.rowops, (unsigned long long)ops);
    if (tid == 0) fpiv[cur] = col;
    ++cur;
    cmin = col + 1;
    __syncthreads();
  }
  uint64_t* front = (uint64_t*)(c.base + c.h->off_front);
  if (M != front)
    for (int64_t i = tid; i < (int64_t)q * W; i += BS) front[i] = M[i];
  for (int j = cur + tid; j < q; j += BS) fpiv[j] = -1;
  if (tid == 0) {
    c.h->rank = cur;
    c.h->rowops = sh.rowops;
  }
  __syncthreads();
}

// One diagram, start to finish.
template <int BS>
__device__ void process_diagram(uint8_t* arena, uint8_t* lds, int64_t lds_cap, int extract,
                                Shared& sh) {
  ZxHeader* h = (ZxHeader*)arena;
  const int n = h->n, W = h->W;
  const int64_t aux = aux_bytes(n, W);
  if (h->magic != ZX_MAGIC || W > MAXW || n > 32767 || aux > lds_cap) {
    if (threadIdx.x == 0) zx_dev_fail(&h->status, ZX_ECAPACITY);
    __syncthreads();
    return;
  }
  const bool lds_adj = lds_adj_bytes(n, W) + aux <= lds_cap;
  Ctx c;
  setup_ctx<BS>(c, arena, lds, lds_adj);
  load_state<BS>(c, sh, lds_adj, true);
  simplify_rounds<BS>(c, sh);
  store_state<BS>(c, sh, lds_adj);
  if (threadIdx.x == 0) {
    h->n_trace = sh.n_trace;
    h->rounds = sh.round;
  }
  if (extract && c.q_out > 0) {
    // LDS mode: the adjacency region is free once written back
    uint64_t* M = lds_adj ? (uint64_t*)lds : (uint64_t*)(arena + h->off_front);
    if (lds_adj) {
      // frontier rows must be built from the adjacency: copy them out first
      __syncthreads();
    }
    if (lds_adj) {
      // rebuild rows from the global copy just written
      c.adj = (uint64_t*)(arena + h->off_adj);
      c.ldw = W;
    }
    frontier<BS>(c, sh, M);
  } else if (threadIdx.x == 0) {
    h->rank = -1;
    h->rowops = 0;
  }
  __syncthreads();
}

struct Queue {
  uint32_t next;
  uint32_t pad[63];
};

template <int BS>
__global__ __launch_bounds__(BS) void simplify_kernel(uint8_t* const* table, int32_t n_graphs,
                                                      Queue* q, int64_t lds_cap, int extract) {
  extern __shared__ __align__(16) uint8_t smem_dyn[];
  __shared__ Shared sh;
  for (;;) {
    if (threadIdx.x == 0) sh.idx = (int32_t)atomicAdd(&q->next, 1u);
    __syncthreads();
    const int idx = sh.idx;
    __syncthreads();
    if (idx >= n_graphs) break;
    process_diagram<BS>(table[idx], smem_dyn, lds_cap, extract, sh);
  }
}

__global__ void queue_reset(Queue* q) {
  if (threadIdx.x == 0) q->next = 0;
}

// Single rewrite on the CURRENT diagram (global adjacency, masks in LDS).
template <int BS>
__global__ __launch_bounds__(BS) void single_rewrite_kernel(uint8_t* arena, int32_t u, int32_t v,
                                                            int32_t pivot, int32_t graph_only) {
  extern __shared__ __align__(16) uint8_t smem_dyn[];
  __shared__ Shared sh;
  ZxHeader* h = (ZxHeader*)arena;
  Ctx c;
  setup_ctx<BS>(c, arena, smem_dyn, false);
  load_state<BS>(c, sh, false, false);
  // precondition
  if (threadIdx.x == 0) {
    bool ok = u >= 0 && u < c.n && bit_of(c.alive, u);
    if (pivot) {
      ok = ok && v >= 0 && v < c.n && v != u && bit_of(c.alive, v) && ((row_ptr(c, u)[v >> 6] >> (v & 63)) & 1);
      if (!graph_only)
        ok = ok && !bit_of(c.bnd, u) && !bit_of(c.bnd, v) && (c.k[u] & 3) == 0 && (c.k[v] & 3) == 0;
    } else if (!graph_only) {
      ok = ok && !bit_of(c.bnd, u) && (c.k[u] & 3) == 2;
    }
    sh.any = ok ? 1 : 0;
    if (!ok) zx_dev_fail(&h->status, ZX_ENOMATCH);
  }
  __syncthreads();
  if (!sh.any) return;
  if (threadIdx.x == 0) {
    c.sel[u >> 6] |= 1ull << (u & 63);
    if (pivot) {
      c.sel[v >> 6] |= 1ull << (v & 63);
      c.partner[u] = (int16_t)v;
      c.partner[v] = (int16_t)u;
    }
  }
  __syncthreads();
  if (graph_only) {
    if (pivot) {
      // contributions without touching rows u, v: stage them in the blocked/inm masks
      // contrib(u) = row_v minus u (in inm), contrib(v) = row_u minus v (in outm)
      for (int j = threadIdx.x; j < c.W; j += BS) {
        uint64_t a = row_ptr(c, u)[j], b = row_ptr(c, v)[j];
        if (j == (u >> 6)) b &= ~(1ull << (u & 63));
        if (j == (v >> 6)) a &= ~(1ull << (v & 63));
        c.inm[j] = b;
        c.outm[j] = a;
      }
      __syncthreads();
      for (int w = c.team; w < c.n; w += c.nteams) {
        if (w == u || w == v || !bit_of(c.alive, w)) continue;
        uint64_t* row = row_ptr(c, w);
        const bool nu = (row[u >> 6] >> (u & 63)) & 1, nv = (row[v >> 6] >> (v & 63)) & 1;
        if (!nu && !nv) continue;
        __builtin_amdgcn_wave_barrier();
        for (int j = c.tl; j < c.W; j += c.T) {
          uint64_t x = row[j];
          if (nu) x ^= c.inm[j];
          if (nv) x ^= c.outm[j];
          if (j == (w >> 6)) x &= ~(1ull << (w & 63));
          row[j] = x;
        }
      }
      __syncthreads();
    } else {
      // tau_u: rows w in N(u) get row_u minus w
      for (int j = threadIdx.x; j < c.W; j += BS) c.inm[j] = row_ptr(c, u)[j];
      __syncthreads();
      for (int w = c.team; w < c.n; w += c.nteams) {
        if (!bit_of(c.inm, w)) continue;
        uint64_t* row = row_ptr(c, w);
        for (int j = c.tl; j < c.W; j += c.T) {
          uint64_t x = row[j] ^ c.inm[j];
          if (j == (w >> 6)) x &= ~(1ull << (w & 63));
          row[j] = x;
        }
      }
      __syncthreads();
    }
    const int64_t e = count_edges<BS>(c, sh);
    if (threadIdx.x == 0) sh.E = e;
    __syncthreads();
  } else {
    prepare_round<BS>(c, sh, pivot != 0, false);
    apply_round<BS>(c, sh, pivot != 0, false);
    delete_selected<BS>(c);
    finish_round<BS>(c, sh, pivot != 0, pivot ? 2 : 1);
  }
  store_state<BS>(c, sh, false);
}

__global__ void reset_kernel(uint8_t* arena) {
  ZxHeader* h = (ZxHeader*)arena;
  const int n = h->n, W = h->W;
  const uint64_t* src = (const uint64_t*)(arena + h->off_src_adj);
  uint64_t* dst = (uint64_t*)(arena + h->off_adj);
  const int8_t* sp = (const int8_t*)(arena + h->off_src_phase);
  int8_t* dp = (int8_t*)(arena + h->off_phase);
  uint64_t* al = (uint64_t*)(arena + h->off_alive);
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < (int64_t)n * W; i += nth) dst[i] = src[i];
  for (int64_t v = tid; v < n; v += nth) dp[v] = sp[v];
  for (int64_t j = tid; j < W; j += nth)
    al[j] = (j < W - 1 || (n & 63) == 0) ? ~0ull : ((1ull << (n & 63)) - 1);
  if (tid == 0) {
    int64_t e = 0;
    (void)e;
    h->pow_sqrt2 = 0;
    h->phase8 = 0;
    h->fill_in = 0;
    h->status = 0;
    h->n_trace = 0;
    h->rounds = 0;
    h->rank = -1;
    h->rowops = 0;
    h->n_alive = n;
  }
}

__global__ void reset_edges_kernel(uint8_t* arena) {
  // edge count of the source diagram (one block)
  ZxHeader* h = (ZxHeader*)arena;
  const int n = h->n, W = h->W;
  const uint64_t* src = (const uint64_t*)(arena + h->off_src_adj);
  __shared__ unsigned long long acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  unsigned long long pc = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)n * W; i += blockDim.x) pc += __popcll(src[i]);
  atomicAdd(&acc, pc);
  __syncthreads();
  if (threadIdx.x == 0) h->n_edges = (int64_t)(acc / 2);
}

// ------------------------------------------------------------ variants --
struct Variant {
  int bs;
  int64_t lds_cap;
  const char* name;
};
const Variant kVariants[] = {
    {256, 32 * 1024, "bs256-lds32k"},   {256, 64 * 1024, "bs256-lds64k"},
    {256, 96 * 1024, "bs256-lds96k"},   {256, 152 * 1024, "bs256-lds152k"},
    {512, 64 * 1024, "bs512-lds64k"},   {512, 152 * 1024, "bs512-lds152k"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kDefaultVariant = 1;

template <int BS>
zx_status launch_simplify_bs(uint8_t* const* table, int32_t n, Queue* q, int64_t lds_cap,
                             int extract, hipStream_t s) {
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  ZX_HIP(hipFuncSetAttribute((const void*)simplify_kernel<BS>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_cap));
  int per_cu = 0;
  ZX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)simplify_kernel<BS>, BS,
                                                      (size_t)lds_cap));
  if (per_cu < 1) {
    zx_set_error("simplify variant does not fit a CU");
    return ZX_ECAPACITY;
  }
  int grid = per_cu * d->n_cu;
  if (grid > n) grid = n;
  hipLaunchKernelGGL(queue_reset, dim3(1), dim3(64), 0, s, q);
  hipLaunchKernelGGL(simplify_kernel<BS>, dim3(grid), dim3(BS), (size_t)lds_cap, s, table, n, q,
                     lds_cap, extract);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

zx_status launch_simplify(int variant, uint8_t* const* table, int32_t n, Queue* q, int extract,
                          hipStream_t s) {
  const Variant& v = kVariants[variant];
  if (v.bs == 256) return launch_simplify_bs<256>(table, n, q, v.lds_cap, extract, s);
  return launch_simplify_bs<512>(table, n, q, v.lds_cap, extract, s);
}

// autotuner cache: (device name, size class) -> variant
std::map<std::string, int>& tune_cache() {
  static std::map<std::string, int> m;
  return m;
}

}  // namespace

// ===================================================================== ABI

struct zx_batch {
  uint8_t** table_dev;  // in the workspace
  Queue* queue;         // in the workspace
  int32_t n;
  std::vector<uint8_t*> arenas;  // scheduled order
  std::vector<int32_t> sizes;
  int32_t max_n;
  double mean_n;
  int32_t tuned;        // autotuned variant, -1 if none
};

extern "C" int32_t zx_simplify_variants(void) { return kNumVariants; }
extern "C" const char* zx_simplify_variant_name(int32_t id) {
  return (id >= 0 && id < kNumVariants) ? kVariants[id].name : "";
}

extern "C" size_t zx_simplify_workspace_bytes(int32_t n_graphs) {
  if (n_graphs < 0) return 0;
  return 256 + (size_t)sizeof(Queue) + (((size_t)n_graphs * 8 + 255) & ~size_t(255));
}

extern "C" zx_status zx_batch_prepare(zx_batch** b, zx_graph* const* graphs, int32_t n_graphs,
                                      void* ws, size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(b && graphs && ws && n_graphs > 0, "bad argument");
  ZX_CHECK_ARG(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  if (ws_bytes < zx_simplify_workspace_bytes(n_graphs)) {
    zx_set_error("workspace too small");
    return ZX_ECAPACITY;
  }
  std::vector<int32_t> order((size_t)n_graphs);
  for (int i = 0; i < n_graphs; ++i) {
    ZX_CHECK_ARG(graphs[i], "null graph %d", i);
    order[i] = i;
  }
  // longest first: work grows roughly with n^2 W
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return graphs[a]->n > graphs[c]->n; });
  zx_batch* B = new zx_batch();
  B->n = n_graphs;
  B->queue = (Queue*)((uint8_t*)ws + 256);
  B->table_dev = (uint8_t**)((uint8_t*)ws + 256 + sizeof(Queue));
  B->arenas.resize((size_t)n_graphs);
  B->sizes.resize((size_t)n_graphs);
  B->max_n = 0;
  double sum = 0;
  for (int i = 0; i < n_graphs; ++i) {
    B->arenas[i] = graphs[order[i]]->arena;
    B->sizes[i] = graphs[order[i]]->n;
    B->max_n = std::max(B->max_n, graphs[order[i]]->n);
    sum += graphs[order[i]]->n;
  }
  B->mean_n = sum / n_graphs;
  B->tuned = -1;
  hipError_t e = hipMemcpyAsync(B->table_dev, B->arenas.data(), (size_t)n_graphs * 8,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete B;
    zx_set_error("table upload failed: %s", hipGetErrorString(e));
    return ZX_EDEVICE;
  }
  *b = B;
  return ZX_OK;
}

extern "C" void zx_batch_destroy(zx_batch* b) { delete b; }

static std::string size_class(const zx_batch* b) {
  const ZxDevice* d = zx_device();
  char buf[256];
  int mb = 0;
  while ((1 << mb) < b->max_n) ++mb;
  int ab = 0;
  while ((1 << ab) < (int)b->mean_n) ++ab;
  int nb = 0;
  while ((1 << nb) < b->n) ++nb;
  snprintf(buf, sizeof(buf), "%s|max2^%d|mean2^%d|n2^%d", d ? d->name : "?", mb, ab, nb);
  return buf;
}

static bool variant_fits(const zx_batch* b, int v) {
  const ZxDevice* d = zx_device();
  if (!d || kVariants[v].lds_cap > (int64_t)d->lds_per_block) return false;
  const int W = (b->max_n + 63) / 64;
  return aux_bytes(b->max_n, W) <= kVariants[v].lds_cap;
}

static int pick_variant(const zx_batch* b, int tune_id) {
  if (tune_id >= 0 && tune_id < kNumVariants) return tune_id;
  if (b->tuned >= 0) return b->tuned;
  auto it = tune_cache().find(size_class(b));
  if (it != tune_cache().end()) return it->second;
  if (variant_fits(b, kDefaultVariant)) return kDefaultVariant;
  for (int v = 0; v < kNumVariants; ++v)
    if (variant_fits(b, v)) return v;
  return kDefaultVariant;
}

extern "C" zx_status zx_batch_simplify(zx_batch* b, const zx_simplify_opts* o, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(b, "null batch");
  zx_simplify_opts def = {ZX_POLICY_GREEDY, 1, -1, 0};
  if (!o) o = &def;
  ZX_CHECK_ARG(o->policy == ZX_POLICY_GREEDY, "unknown policy %d", o->policy);
  const int v = pick_variant(b, o->tune_id);
  zx_status st = launch_simplify(v, b->table_dev, b->n, b->queue, o->extract, s);
  if (st != ZX_OK) return st;
  if (o->flags & ZX_SYNC) ZX_HIP(hipStreamSynchronize(s));
  return ZX_OK;
}

extern "C" zx_status zx_batch_status(zx_batch* b, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(b, "null batch");
  ZX_HIP(hipStreamSynchronize(s));
  zx_status worst = ZX_OK;
  for (uint8_t* a : b->arenas) {
    int32_t st = 0;
    ZX_HIP(hipMemcpy(&st, a + offsetof(ZxHeader, status), 4, hipMemcpyDeviceToHost));
    if (st != 0 && worst == ZX_OK) worst = st;
  }
  return worst;
}

extern "C" zx_status zx_batch_autotune(zx_batch* b, int32_t extract, int32_t reps, int32_t* best_id,
                                       float* best_ms, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(b && reps > 0, "bad argument");
  hipEvent_t e0, e1;
  ZX_HIP(hipEventCreate(&e0));
  ZX_HIP(hipEventCreate(&e1));
  int best = -1;
  float bt = 1e30f;
  for (int v = 0; v < kNumVariants; ++v) {
    if (!variant_fits(b, v)) continue;
    if (launch_simplify(v, b->table_dev, b->n, b->queue, extract, s) != ZX_OK) continue;
    ZX_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch_simplify(v, b->table_dev, b->n, b->queue, extract, s);
    ZX_HIP(hipEventRecord(e1, s));
    ZX_HIP(hipEventSynchronize(e1));
    float ms = 0;
    ZX_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    if (ms < bt) {
      bt = ms;
      best = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (best < 0) {
    zx_set_error("no simplify variant could run");
    return ZX_ECAPACITY;
  }
  b->tuned = best;
  tune_cache()[size_class(b)] = best;
  if (best_id) *best_id = best;
  if (best_ms) *best_ms = bt;
  return ZX_OK;
}

extern "C" zx_status zx_simplify(zx_graph* const* graphs, int32_t n_graphs, const zx_simplify_opts* o,
                                 void* ws, size_t ws_bytes, hipStream_t s) {
  zx_batch* b = nullptr;
  zx_status st = zx_batch_prepare(&b, graphs, n_graphs, ws, ws_bytes, s);
  if (st != ZX_OK) return st;
  st = zx_batch_simplify(b, o, s);
  zx_batch_destroy(b);
  return st;
}

static zx_status single(zx_graph* g, int32_t u, int32_t v, int pivot, uint32_t flags, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g, "null graph");
  ZX_CHECK_ARG(u >= 0 && u < g->n, "spider %d out of range", u);
  if (pivot) ZX_CHECK_ARG(v >= 0 && v < g->n && v != u, "spider %d out of range", v);
  if (g->W > MAXW || g->n > 32767) {
    zx_set_error("diagram too large for the rewrite kernels");
    return ZX_ECAPACITY;
  }
  const size_t lds = (size_t)aux_bytes(g->n, g->W);
  ZX_HIP(hipFuncSetAttribute((const void*)single_rewrite_kernel<256>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(single_rewrite_kernel<256>, dim3(1), dim3(256), lds, s, g->arena, u, v, pivot,
                     (flags & ZX_GRAPH_ONLY) ? 1 : 0);
  ZX_HIP(hipGetLastError());
  if (flags & ZX_SYNC) ZX_HIP(hipStreamSynchronize(s));
  return ZX_OK;
}

extern "C" zx_status zx_local_comp(zx_graph* g, int32_t u, uint32_t flags, hipStream_t s) {
  return single(g, u, -1, 0, flags, s);
}
extern "C" zx_status zx_pivot(zx_graph* g, int32_t u, int32_t v, uint32_t flags, hipStream_t s) {
  return single(g, u, v, 1, flags, s);
}

extern "C" zx_status zx_graph_reset(zx_graph* g, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g, "null graph");
  hipLaunchKernelGGL(reset_kernel, dim3(32), dim3(256), 0, s, g->arena);
  hipLaunchKernelGGL(reset_edges_kernel, dim3(1), dim3(256), 0, s, g->arena);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}
