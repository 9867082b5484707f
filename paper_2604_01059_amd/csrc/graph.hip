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
// minus v for a pivot pair (u, v).  No contribution row holds a bit of a
// selected spider (they are pairwise non-adjacent), so the bits of a row at
// selected positions cannot change during the round: every (row, word)
// pair is updated by its own thread, which reads the row's selected bits
// straight from the row, and the selected columns are cleared afterwards.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "zx_internal.h"
#include "mlp_dev.h"

namespace {

constexpr int MAXW = 128;   // words per row (n <= 8192)
constexpr int MAXS = 2;     // words per lane in a team of 64

__host__ __device__ inline int ldw_lds(int W) { return W | 1; }  // odd LDS row stride

__host__ __device__ inline int64_t aux_bytes(int n, int W) {
  int64_t k = (n + 7) & ~7;
  int64_t part = (2 * (int64_t)n + 7) & ~7;
  return k + k + part + part + 8 * 8 * (int64_t)W;
}
__host__ __device__ inline int64_t lds_adj_bytes(int n, int W) { return (int64_t)n * ldw_lds(W) * 8; }

struct Shared {
  int64_t E;           // Hadamard edges among present spiders
  int64_t pow_sqrt2;
  int64_t fill_in;
  int64_t acc64[5];    // per-round accumulators ([4]: a team slice's edge count)
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
  int32_t nsw;         // words of the selected set (list in Ctx::blocked)
  int32_t ns;          // selected spiders (list in Ctx::slist)
  int64_t rowops;
  int32_t n_terms;     // phase-pair terms recorded (parameterized spiders)
  int32_t pad_terms;
};

// LDS pointers are typed as such so that the compiler emits ds_* accesses.
#define LDSP __attribute__((address_space(3)))
template <bool LA> struct AdjPtr { using type = uint64_t*; };
template <> struct AdjPtr<true> { using type = LDSP uint64_t*; };

// A team of workgroups shares the row update of an arena-mode round: the
// workgroup running the diagram publishes the round here (the selected
// spiders, their partners and phase contributions, the present and selected
// masks), and every member, itself included, claims 64-row slices of the
// update until none is left.  claim = (round sequence << 32) | next slice,
// taken by compare-and-swap, so a late member can never claim a slice of
// another round; the running workgroup waits only for slices already
// claimed, so it finishes alone if no helper comes.  Device-scope release
// and acquire order the round's data and results around claim and done.
constexpr int TEAM_SLICE = 64;     // rows per slice
constexpr int TEAM_MAXW = 128;     // words per row (n <= 8192)
constexpr int TEAM_MAXS = 64;      // selected spiders of a round
constexpr int TEAM_MIN_N = 1500;   // diagrams from this size get a team
constexpr int SERVE_BOARDS_PER_XCD = 4;  // serving: large requests with a team at once, per XCD
struct __attribute__((aligned(256))) TeamBoard {
  unsigned long long claim;
  uint32_t done;        // slices finished in the current round
  uint32_t exit;        // the team's diagrams are done
  uint32_t owner;       // serving: 1 while a workgroup runs a diagram with this board
  uint32_t pad0;
  unsigned long long pc;  // edges left on the updated rows (sum over slices)
  int32_t ns, pivot, n, W;
  int64_t ldw;
  uint64_t* adj;
  int8_t* dk;           // phase increment of each row in the round (n bytes)
  int16_t slist[TEAM_MAXS], partner[TEAM_MAXS];
  int8_t kc[TEAM_MAXS];
  uint64_t alive[TEAM_MAXW], sel[TEAM_MAXW];
};

template <bool LA>  // LA: the working adjacency is in LDS (else in the arena)
struct Ctx {
  ZxHeader* h;
  uint8_t* base;
  int n, W, ldw, q_in, q_out;
  typename AdjPtr<LA>::type adj;  // working adjacency
  LDSP int8_t* k;          // phases
  LDSP int8_t* kc;         // per-selected contribution to neighbour phases
  LDSP int16_t* partner;   // pivot partner
  LDSP int16_t* slist;     // selected spiders of the round, ascending
  LDSP uint64_t* alive;
  LDSP uint64_t* bnd;
  LDSP uint64_t* cand;
  LDSP uint64_t* sel;
  LDSP uint64_t* inm;
  LDSP uint64_t* outm;
  LDSP uint64_t* blocked;
  LDSP uint64_t* omask;    // output-attached spiders
  int32_t* trace;          // global, 4 int32 per entry
  int T, nteams, team, tl;
  LDSP uint64_t* scr;      // arena mode: free LDS for the round update
  int scr_words;
  int pw;                  // words per parameter row (0: no parameters)
  uint64_t* par;           // CURRENT parameter rows, n x pw (global)
  uint8_t* terms;          // recorded terms (global)
  TeamBoard* tb;           // arena mode with a team (else null)
};

template <class P>
__device__ __forceinline__ bool bit_of(P m, int v) { return (m[v >> 6] >> (v & 63)) & 1; }

__device__ __forceinline__ uint64_t wave_shfl64(uint64_t v, int src, int width) {
  return __shfl(v, src, width);
}

// A value that every lane holds alike (read from LDS after a barrier), made
// visibly uniform to the compiler: branches and loop bounds on it then
// compile to scalar control flow instead of exec-mask control flow.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane l's 64-bit value, to every lane.  The builtin returns a signed int:
// each half is taken as uint32 so that the low word is not sign-extended.
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int team_size(int W) {
  int T = 1;
  while (T < W && T < 64) T <<= 1;
  return T;
}

template <int BS>
__device__ void block_sync() { __syncthreads(); }

// --------------------------------------------------------------- setup --
template <int BS, bool LA>
__device__ void setup_ctx(Ctx<LA>& c, uint8_t* arena, uint8_t* lds) {
  c.h = (ZxHeader*)arena;
  c.base = arena;
  c.n = uni(c.h->n);
  c.W = uni(c.h->W);
  c.q_in = uni(c.h->n_in);
  c.q_out = uni(c.h->n_out);
  const int n = c.n, W = c.W;
  uint8_t* p = lds;
  if constexpr (LA) {
    c.adj = (LDSP uint64_t*)p;
    c.ldw = ldw_lds(W);
    p += lds_adj_bytes(n, W);
  } else {
    c.adj = (uint64_t*)(arena + c.h->off_adj);
    c.ldw = W;
  }
  const int64_t kb = (n + 7) & ~7;
  c.k = (LDSP int8_t*)p; p += kb;
  c.kc = (LDSP int8_t*)p; p += kb;
  c.partner = (LDSP int16_t*)p; p += (2 * (int64_t)n + 7) & ~7;
  c.slist = (LDSP int16_t*)p; p += (2 * (int64_t)n + 7) & ~7;
  c.alive = (LDSP uint64_t*)p; p += 8 * W;
  c.bnd = (LDSP uint64_t*)p; p += 8 * W;
  c.cand = (LDSP uint64_t*)p; p += 8 * W;
  c.sel = (LDSP uint64_t*)p; p += 8 * W;
  c.inm = (LDSP uint64_t*)p; p += 8 * W;
  c.outm = (LDSP uint64_t*)p; p += 8 * W;
  c.blocked = (LDSP uint64_t*)p; p += 8 * W;
  c.omask = (LDSP uint64_t*)p; p += 8 * W;
  c.scr = nullptr;
  c.scr_words = 0;
  c.tb = nullptr;
  c.trace = (int32_t*)(arena + c.h->off_trace);
  c.pw = uni(c.h->pw);
  c.par = c.pw ? (uint64_t*)(arena + c.h->off_par) : nullptr;
  c.terms = c.pw ? arena + c.h->off_terms : nullptr;
  c.T = team_size(W);
  c.nteams = BS / c.T;
  c.team = threadIdx.x / c.T;
  c.tl = threadIdx.x % c.T;
}

template <bool LA>
__device__ __forceinline__ typename AdjPtr<LA>::type row_ptr(const Ctx<LA>& c, int r) {
  return c.adj + (size_t)r * c.ldw;
}

// Sum over threads of v into an LDS 64-bit accumulator.
__device__ __forceinline__ void block_add(int64_t* acc, int64_t v) {
  if (v) atomicAdd((unsigned long long*)acc, (unsigned long long)v);
}

// Edge count of the work adjacency (rows are already masked to present spiders).
template <int BS, bool LA>
__device__ int64_t count_edges(Ctx<LA>& c, Shared& sh) {
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
template <int BS, bool LA>
__device__ void load_state(Ctx<LA>& c, Shared& sh, bool from_source) {
  const int n = c.n, W = c.W, tid = threadIdx.x;
  const uint64_t* src = (const uint64_t*)(c.base + (from_source ? c.h->off_src_adj : c.h->off_adj));
  const int8_t* srcph = (const int8_t*)(c.base + (from_source ? c.h->off_src_phase : c.h->off_phase));
  if (LA || from_source) {
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
  if (c.pw && from_source) {
    const uint64_t* sp = (const uint64_t*)(c.base + c.h->off_src_par);
    for (int64_t i = tid; i < (int64_t)n * c.pw; i += BS) c.par[i] = sp[i];
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
    sh.n_terms = (from_source || !c.pw) ? 0 : c.h->n_terms;
  }
  __syncthreads();
  const int64_t e = count_edges<BS, LA>(c, sh);
  if (tid == 0) sh.E = e;
  __syncthreads();
}

// Write the work state back to the CURRENT section and the header.
template <int BS, bool LA>
__device__ void store_state(Ctx<LA>& c, Shared& sh) {
  const int n = c.n, W = c.W, tid = threadIdx.x;
  uint64_t* dst = (uint64_t*)(c.base + c.h->off_adj);
  if (LA) {
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
    if (c.pw) c.h->n_terms = sh.n_terms;
  }
  __syncthreads();
}

// ------------------------------------------------------- candidate masks --
// kind 0: local-complementation candidates (interior, k in {2, 6});
// kind 1: Pauli candidates (interior, k in {0, 4}).  Returns non-empty.
template <int BS, bool LA>
__device__ bool build_candidates(Ctx<LA>& c, Shared& sh, int kind) {
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
  return uni(sh.any) != 0;
}

// One wavefront, after the round's selection (c.sel): the selected
// spiders' count (sh.cnt, with set_cnt), with lc_trace their trace entries in ascending
// order, the list of the selected set's words (sh.nsw entries in c.blocked)
// and of the selected spiders in ascending order (sh.ns entries in
// c.slist).  The caller's barrier publishes them.
template <bool LA>
__device__ void list_selected_wave(Ctx<LA>& c, Shared& sh, bool lc_trace, bool set_cnt = true) {
  const int lane = threadIdx.x & 63;
  LDSP int32_t* sw = (LDSP int32_t*)c.blocked;
  int cnt = 0, ns = 0;
  const int nt0 = sh.n_trace, round = sh.round;
  for (int j0 = 0; j0 < c.W; j0 += 64) {
    const int j = j0 + lane;
    const uint64_t wd = j < c.W ? c.sel[j] : 0;
    const bool nz = wd != 0;
    const uint64_t b = __ballot(nz);
    if (nz) sw[cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0))] = j;
    cnt += __popcll(b);
    // exclusive prefix of the per-word popcounts, by bit planes
    const int pc = __popcll(wd);
    int ex = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 7; ++bit) {
      const uint64_t bb = __ballot((pc >> bit) & 1);
      ex += __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0)) << bit;
      tot += __popcll(bb) << bit;
    }
    uint64_t m = wd;
    int pos = ns + ex;
    while (m) {
      const int bit = __ffsll((long long)m) - 1;
      m &= m - 1;
      c.slist[pos] = (int16_t)(64 * j + bit);
      if (lc_trace && c.trace) {
        int32_t* e = c.trace + 4 * (int64_t)(nt0 + pos);
        e[0] = round;
        e[1] = 0;
        e[2] = 64 * j + bit;
        e[3] = -1;
      }
      ++pos;
    }
    ns += tot;
  }
  if (lane == 0) {
    sh.nsw = cnt;
    sh.ns = ns;
    if (set_cnt) sh.cnt = ns;
    if (lc_trace && c.trace) sh.n_trace = nt0 + ns;
  }
}

// Lexicographically-first maximal independent set of the candidates (scan
// in ascending spider id, take a candidate unless adjacent to one taken).
// One wavefront, one 64-spider block at a time.  The wave keeps the union
// of the taken spiders' rows (lane l: words l and l + 64), so a block's
// candidates that are adjacent to a spider taken in an earlier block are
// one word of it; the rest are resolved in ascending order with scalar bit
// operations on their rows' word b, loaded one block ahead; then the rows
// of the block's taken spiders are OR-ed into the union, four at a time.
// Per block, the only wait on memory is for those rows and the next
// block's words, issued together.  The same wavefront then counts, traces
// and lists the set (list_selected_wave), before the one closing barrier.
// The wavefront runs at raised priority: it is the round's serial step, and
// another workgroup's waves may share its SIMD (batched: 4.60 -> 4.54 ms).
template <int BS, bool LA>
__device__ void lfmis(Ctx<LA>& c, Shared& sh) {
  const int W = c.W;
  for (int j = threadIdx.x; j < W; j += BS) c.sel[j] = 0;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    __builtin_amdgcn_s_setprio(2);
    // clamped word indices (W <= 128): a lane's words past W are loaded
    // from word W - 1 and never read
    const int j0 = lane < W ? lane : W - 1;
    const int j1 = lane + 64 < W ? lane + 64 : W - 1;
    uint64_t blk0 = 0, blk1 = 0;
    uint64_t nxt = ((c.cand[0] >> lane) & 1) ? row_ptr(c, lane)[0] : 0;
    for (int b = 0; b < W; ++b) {
      const uint64_t cw = uni64((int64_t)c.cand[b]);
      const uint64_t inblk = nxt;
      if (b + 1 < W) {
        const uint64_t cn = c.cand[b + 1];
        nxt = ((cn >> lane) & 1) ? row_ptr(c, 64 * (b + 1) + lane)[b + 1] : 0;
      }
      if (!cw) continue;
      const uint64_t bw = readlane64(b < 64 ? blk0 : blk1, b & 63);
      uint64_t R = cw & ~bw;  // candidates with no taken neighbour in earlier blocks
      uint64_t taken = 0;
      while (R) {
        const int l = __builtin_ctzll(R);
        taken |= 1ull << l;
        R &= ~(readlane64(inblk, l) | (1ull << l));
      }
      if (lane == 0) c.sel[b] = taken;
      uint64_t tk = taken;
      while (tk) {
        // four taken spiders (repeating the first when fewer are left), so
        // that the eight loads are issued before one wait
        int t[4];
        t[0] = __builtin_ctzll(tk);
        tk &= tk - 1;
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          t[q] = tk ? __builtin_ctzll(tk) : t[0];
          tk &= tk - 1;
        }
        uint64_t a0 = 0, a1 = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const auto rt = row_ptr(c, 64 * b + t[q]);
          a0 |= rt[j0];
          a1 |= rt[j1];
        }
        blk0 |= a0;
        blk1 |= a1;
      }
    }
    __builtin_amdgcn_wave_barrier();
    list_selected_wave(c, sh, true);
    __builtin_amdgcn_s_setprio(0);
  }
  __syncthreads();
}

// Wave 0: lexicographic pivot-pair selection among the Pauli candidates.
// Writes partner[], sel (both ends), the trace entries; returns the number
// of pairs through sh.cnt.  RESUME: complete a round begun by another
// order: start from its blocked set (c.blocked: taken ends and their
// neighbours), selection (c.sel) and pair count (sh.cnt).
template <int BS, bool LA, bool RESUME = false>
__device__ void select_pivots(Ctx<LA>& c, Shared& sh) {
  const int tid = threadIdx.x, W = c.W;
  if constexpr (!RESUME) {
    for (int j = tid; j < W; j += BS) {
      c.sel[j] = 0;
      c.blocked[j] = 0;
    }
    __syncthreads();
  }
  if (tid < 64) {
    const int lane = tid;
    __builtin_amdgcn_s_setprio(2);
    uint64_t blk[MAXS], Pm[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int j = lane + 64 * s;
      blk[s] = RESUME && j < W ? c.blocked[j] : 0;
      Pm[s] = j < W ? c.cand[j] : 0;
    }
    int npairs = RESUME ? sh.cnt : 0, nt = sh.n_trace;
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
        const auto ru = row_ptr(c, u);
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
        const auto rv = row_ptr(c, v);
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
          if (c.trace) {
            int32_t* e = c.trace + 4 * (int64_t)nt;
            e[0] = round;
            e[1] = 1;
            e[2] = u;
            e[3] = v;
          }
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
    __builtin_amdgcn_wave_barrier();
    list_selected_wave(c, sh, false, false);  // the lists prepare_round takes
    __builtin_amdgcn_s_setprio(0);
  }
  __syncthreads();
}

// List the words of the selected set (sh.nsw entries in c.blocked) and the
// selected spiders in ascending order (sh.ns entries in c.slist).
template <int BS, bool LA>
__device__ void collect_swords(Ctx<LA>& c, Shared& sh) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    LDSP int32_t* sw = (LDSP int32_t*)c.blocked;
    int cnt = 0, ns = 0;
    for (int j0 = 0; j0 < c.W; j0 += 64) {
      const int j = j0 + lane;
      const uint64_t wd = j < c.W ? c.sel[j] : 0;
      const bool nz = wd != 0;
      const uint64_t b = __ballot(nz);
      if (nz) sw[cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0))] = j;
      cnt += __popcll(b);
      // ascending spider list: exclusive prefix of the per-word popcounts
      const int pc = __popcll(wd);
      int ex = 0, tot = 0;
#pragma unroll
      for (int bit = 0; bit < 7; ++bit) {
        const uint64_t bb = __ballot((pc >> bit) & 1);
        ex += __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0)) << bit;
        tot += __popcll(bb) << bit;
      }
      uint64_t m = wd;
      int pos = ns + ex;
      while (m) {
        const int bit = __ffsll((long long)m) - 1;
        m &= m - 1;
        c.slist[pos++] = (int16_t)(64 * j + bit);
      }
      ns += tot;
    }
    if (lane == 0) {
      sh.nsw = cnt;
      sh.ns = ns;
    }
  }
  __syncthreads();
}

// Per-round bookkeeping over the selected spiders (before the update),
// after listing them (collect_swords, unless listed: done with the
// selection).
// LC: acc64[0] = sum deg, acc64[1] = sum deg(deg-1)/2, acc64[2] = phase sum.
// Pivot: acc64[0] = sum (deg u + deg v - 1), acc64[1] = sum T_p, acc64[2] = phase.
// Also fills kc[] and, for pivots, swaps each pair's rows into contributions.
template <int BS, bool LA>
__device__ void prepare_round(Ctx<LA>& c, Shared& sh, bool pivot, bool listed) {
  const int W = c.W;
  if (threadIdx.x == 0) sh.acc64[0] = sh.acc64[1] = sh.acc64[2] = sh.acc64[3] = 0;
  if (listed)
    __syncthreads();
  else
    collect_swords<BS, LA>(c, sh);
  const int ns = uni(sh.ns);
  for (int i = c.team; i < ns; i += c.nteams) {
    const int x = c.slist[i];
    const int p = pivot ? c.partner[x] : -1;
    if (pivot && p < x) continue;  // one team per pair, at its lower end
    auto rx = row_ptr(c, x);
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
      auto rp = row_ptr(c, p);
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
}

// The rank-|S| update of every present row outside S, by (row, word)
// threads.  Also sums into sh.acc64[3] the popcounts of every present
// non-selected row with the selected columns masked out (twice the edge
// count after the round); selected columns are cleared by delete_selected.
//
// Few selected spiders (the common case): spider-major.  A thread keeps the
// words of up to MAXI rows in registers for the whole round; for each
// selected x it tests "w ~ x" as bit x of row w (the adjacency is symmetric,
// so this is also "x ~ w") and XORs in x's contribution word.  Rows are
// only written at the end, and all loads are independent.
// Many selected spiders: row-major, walking the selected bits of each row.
constexpr int MAXI = 4;
constexpr int SPIDER_MAJOR_MAX = 64;

// A team round as a slice sees it; the selected list, partners, phase
// contributions and the present and selected masks are staged in LDS once
// per round and member (TEAM_SLICE_LDS words, layout below).
struct SliceRound {
  uint64_t* adj;
  int8_t* dk;
  int64_t ldw;
  int n, W, ns, pivot;
};
constexpr int TS_NB = 64, TS_PB = 128, TS_SEL = 192, TS_ALIVE = 320;  // words; hit masks at 0
constexpr int TS_SL = 448, TS_PP = 464, TS_KC = 480;                 // int16, int16, int8 arrays
constexpr int TEAM_SLICE_LDS = 488;

// A helper's copy of the round on the board (after the acquire that made
// it visible).  Ends with a barrier.
template <int BS>
__device__ SliceRound team_stage_board(TeamBoard* tb, LDSP uint64_t* ls) {
  SliceRound r;
  r.adj = tb->adj;
  r.dk = tb->dk;
  r.ldw = tb->ldw;
  r.n = tb->n;
  r.W = tb->W;
  r.ns = tb->ns;
  r.pivot = tb->pivot;
  const int tid = threadIdx.x;
  if (tid < r.ns) {
    ((LDSP int16_t*)(ls + TS_SL))[tid] = tb->slist[tid];
    ((LDSP int16_t*)(ls + TS_PP))[tid] = tb->partner[tid];
    ((LDSP int8_t*)(ls + TS_KC))[tid] = tb->kc[tid];
  } else if (tid >= 64 && tid < 64 + r.W) {
    ls[TS_SEL + tid - 64] = tb->sel[tid - 64];
    ls[TS_ALIVE + tid - 64] = tb->alive[tid - 64];
  }
  __syncthreads();
  return r;
}

// Slice s of a team round, whole workgroup: rows 64 s .. 64 s + 63, whose
// bits in any row are that row's word s.  The adjacency is symmetric and
// the selected spiders' rows do not change during the round, so the
// slice's rows adjacent to a selected spider are word s of its row (for a
// pivot pair (x, p), whose rows prepare_round swapped into contributions,
// x's neighbours are word s of p's current row and p's those of x's): one
// word per selected spider (two for pivots) gives every row's hit mask and
// phase increment.  Those words and the first U (row, word) items of each
// thread are loaded together, before the hit masks; then the items are
// XOR-ed with their hit contributions, the row's own bit and the selected
// columns cleared.  The slice's edge count goes to sh.acc64[4].
template <int BS, int U>
__device__ void team_slice(const SliceRound& r, int slice, LDSP uint64_t* ls, Shared& sh) {
  static_assert(BS >= 192, "a round's staging takes 192 threads");
  const int tid = threadIdx.x, W = r.W, ns = r.ns;
  const int64_t ldw = r.ldw;
  uint64_t* adj = r.adj;
  const int lo = slice * TEAM_SLICE;
  const int rn = r.n - lo < TEAM_SLICE ? r.n - lo : TEAM_SLICE;
  const int items = rn * W;
  LDSP uint64_t* hm = ls;
  const LDSP int16_t* sl = (const LDSP int16_t*)(ls + TS_SL);
  const LDSP int16_t* pp = (const LDSP int16_t*)(ls + TS_PP);
  const LDSP int8_t* kc = (const LDSP int8_t*)(ls + TS_KC);
  // the selected spiders' words of the slice (spider 0 stands in past ns)
  const int x = tid < ns ? sl[tid] : 0;
  const int src = tid < ns && r.pivot ? pp[tid] : x;
  const uint64_t wa = adj[(int64_t)src * ldw + slice];
  const uint64_t wb = r.pivot ? adj[(int64_t)x * ldw + slice] : 0;
  const uint64_t am = ls[TS_ALIVE + slice] & ~ls[TS_SEL + slice];  // present, non-selected rows
  int64_t pc = 0;
  for (int base = 0; base < items; base += U * BS) {
    uint64_t old[U];
    int tt[U], jj[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int it = base + q * BS + tid;
      const int itc = it < items ? it : 0;
      tt[q] = itc / W;
      jj[q] = itc - tt[q] * W;
      old[q] = adj[(int64_t)(lo + tt[q]) * ldw + jj[q]];  // row lo + tt < n: in bounds
    }
    if (base == 0) {
      if (tid < ns) {
        ls[TS_NB + tid] = wa;
        ls[TS_PB + tid] = wb;
      }
      if (tid == 0) sh.acc64[4] = 0;
      __syncthreads();
      if (tid < rn) {
        uint64_t m = 0;
        int dk = 0;
        if ((am >> tid) & 1) {
          for (int i = 0; i < ns; ++i) {
            if ((ls[TS_NB + i] >> tid) & 1) {
              m |= 1ull << i;
              dk += kc[i];
              if (r.pivot && ((ls[TS_PB + i] >> tid) & 1)) dk += 2;  // adjacent to both ends
            }
          }
        }
        hm[tid] = m;
        r.dk[lo + tid] = (int8_t)(dk & 7);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int t = tt[q], j = jj[q];
      if (base + q * BS + tid >= items || !((am >> t) & 1)) continue;
      uint64_t v = old[q];
      uint64_t m = hm[t];
      while (m) {
        const int i = __builtin_ctzll(m);
        m &= m - 1;
        v ^= adj[(int64_t)sl[i] * ldw + j];
      }
      if (j == slice) v &= ~(1ull << t);
      v &= ~ls[TS_SEL + j];
      if (v != old[q]) adj[(int64_t)(lo + t) * ldw + j] = v;
      pc += __popcll(v);
    }
  }
  block_add(&sh.acc64[4], pc);
  __syncthreads();
}

// After a member's last slice of a round: its row and dk stores are
// acknowledged in every wave, then one release publishes them with the
// member's edge count and slice count (one cache write-back per member and
// round, not per slice).
template <int BS>
__device__ void team_publish(TeamBoard* tb, Shared& sh, int64_t pc, uint32_t slices) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0 && slices) {
    __hip_atomic_fetch_add(&tb->pc, (unsigned long long)pc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&tb->done, slices, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Thread 0: claim the next slice of round seq (compare-and-swap); -1 when
// none is left or the board holds another round.
__device__ __forceinline__ int team_claim(TeamBoard* tb, uint32_t seq) {
  unsigned long long c0 = __hip_atomic_load(&tb->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    if ((uint32_t)(c0 >> 32) != seq) return -1;
    const uint32_t idx = (uint32_t)c0;
    const int S = (tb->n + TEAM_SLICE - 1) / TEAM_SLICE;
    if ((int)idx >= S) return -1;
    if (__hip_atomic_compare_exchange_strong(&tb->claim, &c0, c0 + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return (int)idx;
  }
}

constexpr uint64_t TEAM_WAIT_TICKS = 100000000ull * 10;  // 10 s of the 100 MHz clock

// The running workgroup's side of a team round (rounds of at most
// TEAM_MAXS rewrites): publish, claim slices like any member, wait for the
// slices others claimed, then take the phase increments and edge counts.
template <int BS>
__device__ __noinline__ void apply_round_team(Ctx<false>& c, Shared& sh, bool pivot) {
  TeamBoard* tb = c.tb;
  const int tid = threadIdx.x, W = c.W, n = c.n, ns = uni(sh.ns);
  LDSP uint64_t* ls = c.scr;  // TEAM_SLICE_LDS words of the free LDS
  for (int i = tid; i < ns; i += BS) {
    const int x = c.slist[i];
    const int16_t p = pivot ? c.partner[x] : (int16_t)-1;
    tb->slist[i] = (int16_t)x;
    tb->partner[i] = p;
    tb->kc[i] = c.kc[x];
    ((LDSP int16_t*)(ls + TS_SL))[i] = (int16_t)x;
    ((LDSP int16_t*)(ls + TS_PP))[i] = p;
    ((LDSP int8_t*)(ls + TS_KC))[i] = c.kc[x];
  }
  for (int j = tid; j < W; j += BS) {
    tb->alive[j] = c.alive[j];
    tb->sel[j] = c.sel[j];
    ls[TS_ALIVE + j] = c.alive[j];
    ls[TS_SEL + j] = c.sel[j];
  }
  SliceRound r;
  r.adj = c.adj;
  r.dk = tb->dk;
  r.ldw = c.ldw;
  r.n = n;
  r.W = W;
  r.ns = ns;
  r.pivot = pivot ? 1 : 0;
  if (tid == 0) {
    tb->ns = ns;
    tb->pivot = pivot ? 1 : 0;
    tb->n = n;
    tb->W = W;
    tb->ldw = c.ldw;
    tb->adj = c.adj;
    tb->pc = 0;
    tb->done = 0;
  }
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores (and earlier row writes) are acknowledged
  __syncthreads();                // ... and every other wave's
  if (tid == 0) {
    const unsigned long long c0 = __hip_atomic_load(&tb->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t seq = (uint32_t)(c0 >> 32) + 1;
    sh.key = (int32_t)seq;
    // published with slice 0 already taken, by this workgroup
    __hip_atomic_store(&tb->claim, ((unsigned long long)seq << 32) | 1u, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const uint32_t seq = (uint32_t)uni(sh.key);
  int64_t mypc = 0;
  uint32_t mine = 0;
  for (bool first = true;; first = false) {
    if (tid == 0) sh.idx = first ? 0 : team_claim(tb, seq);
    __syncthreads();
    const int sl = uni(sh.idx);
    __syncthreads();
    if (sl < 0) break;
    team_slice<BS, 2>(r, sl, ls, sh);
    if (tid == 0) mypc += sh.acc64[4];
    ++mine;
  }
  team_publish<BS>(tb, sh, mypc, mine);
  if (tid == 0) {
    // relaxed polls (an acquire per poll would invalidate the caches each
    // time), then one acquire for everything the members published
    const uint32_t S = (uint32_t)((n + TEAM_SLICE - 1) / TEAM_SLICE);
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(&tb->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < S) {
      if (wall_clock64() - t0 > TEAM_WAIT_TICKS) {
        sh.status = ZX_EDEVICE;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sh.acc64[4] = (int64_t)__hip_atomic_load(&tb->pc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  // phase increments, eight rows per load (bytes from n on are not this
  // diagram's)
  const uint64_t* dk8 = (const uint64_t*)tb->dk;
  for (int q = tid; 8 * q < n; q += BS) {
    uint64_t d = dk8[q];
    if (8 * q + 8 > n) d &= (1ull << (8 * (n - 8 * q))) - 1;
    while (d) {
      const int b = __builtin_ctzll(d) >> 3;
      const int w = 8 * q + b;
      c.k[w] = (int8_t)((c.k[w] + (int)((d >> (8 * b)) & 0xff)) & 7);
      d &= ~(0xffull << (8 * b));
    }
  }
  if (tid == 0) sh.acc64[3] += sh.acc64[4];
  __syncthreads();
}

// Arena mode (rows in global memory), rounds of at most 64 rewrites.  Rows
// go in chunks that fit the free LDS: a per-row pass records which selected
// spiders the row is adjacent to (hit mask) and updates the row's phase;
// then a (row, word) pass XORs the hit contributions, staged in LDS when
// they fit, and drops the selected columns in the same write.  Each row
// word is read and written once; each selected-column bit once per row.
// Not inlined: its unrolled update would otherwise set the register
// allocation of the LDS-resident path that shares the kernel.
template <int BS>
__device__ __noinline__ void apply_round_arena(Ctx<false>& c, Shared& sh, bool pivot) {
  const int W = c.W, n = c.n, ns = uni(sh.ns), tid = threadIdx.x;
  const bool staged = (int64_t)ns * W + 64 + 8 <= c.scr_words;
  LDSP uint64_t* cs = c.scr;
  // slist index of each selected spider's pivot partner (64 bytes after the
  // staged contributions)
  LDSP int8_t* pidx = (LDSP int8_t*)(c.scr + (staged ? (int64_t)ns * W : 0));
  LDSP uint64_t* hm = staged ? c.scr + (int64_t)ns * W + 8 : c.scr;
  const int room = c.scr_words - (staged ? ns * W + 8 : 0);
  const int CH = room < n ? room : n;
  if (staged) {
    for (int i = tid; i < ns * W; i += BS) {
      const int si = i / W, j = i - si * W;
      cs[i] = row_ptr(c, c.slist[si])[j];
    }
    if (pivot)
      for (int i = tid; i < ns; i += BS) {
        const int p = c.partner[c.slist[i]];
        int q = 0;
        while (q < ns - 1 && c.slist[q] != p) ++q;
        pidx[i] = (int8_t)q;
      }
  }
  int64_t pc = 0;
  for (int r0 = 0; r0 < n; r0 += CH) {
    const int rn = n - r0 < CH ? n - r0 : CH;
    __syncthreads();  // staging done; the previous chunk is through with hm
    if (staged) {
      // Hit masks from the staged rows: w ~ x is bit w of x's row (the
      // adjacency is symmetric).  The staged row of a local complementation
      // is x's own row; a pivot swapped each pair's rows into contributions,
      // so x's row is its partner's staged row (without the partner's bit,
      // which is no unselected w).  Rows of one 64-row block read the same
      // staged words (LDS broadcast).
      for (int t = tid; t < rn; t += BS) {
        const int w = r0 + t;
        uint64_t m = 0;
        if (bit_of(c.alive, w) && !bit_of(c.sel, w)) {
          const int jw = w >> 6, bw = w & 63;
          uint64_t R = 0;
          for (int i = 0; i < ns; ++i) R |= ((cs[(int64_t)i * W + jw] >> bw) & 1ull) << i;
          if (pivot) {
            for (int i = 0; i < ns; ++i) m |= ((R >> pidx[i]) & 1ull) << i;
          } else {
            m = R;
          }
          int dk = 0;
          uint64_t mm = m;
          while (mm) {
            const int i = __builtin_ctzll(mm);
            mm &= mm - 1;
            dk += c.kc[c.slist[i]];
            if (pivot && ((m >> pidx[i]) & 1)) dk += 2;  // adjacent to both ends
          }
          if (dk) c.k[w] = (int8_t)((c.k[w] + dk) & 7);
        }
        hm[t] = m;
      }
    } else {
    for (int t = tid; t < rn; t += BS) {
      const int w = r0 + t;
      uint64_t m = 0;
      if (bit_of(c.alive, w) && !bit_of(c.sel, w)) {
        const auto rw = row_ptr(c, w);
        int dk = 0;
        for (int i = 0; i < ns; ++i) {
          const int x = c.slist[i];
          if ((rw[x >> 6] >> (x & 63)) & 1) {
            m |= 1ull << i;
            dk += c.kc[x];
            if (pivot) {
              const int pp = c.partner[x];
              if ((rw[pp >> 6] >> (pp & 63)) & 1) dk += 2;  // adjacent to both ends
            }
          }
        }
        if (dk) c.k[w] = (int8_t)((c.k[w] + dk) & 7);
      }
      hm[t] = m;
    }
    }
    __syncthreads();
    for (int64_t it = tid; it < (int64_t)rn * W; it += BS) {
      const int t = (int)(it / W), j = (int)(it - (int64_t)t * W);
      const int w = r0 + t;
      if (!bit_of(c.alive, w) || bit_of(c.sel, w)) continue;
      auto rw = row_ptr(c, w);
      const uint64_t old = rw[j];
      uint64_t v = old;
      uint64_t m = hm[t];
      while (m) {
        const int i = __builtin_ctzll(m);
        m &= m - 1;
        v ^= staged ? cs[(int64_t)i * W + j] : row_ptr(c, c.slist[i])[j];
      }
      if (j == (w >> 6)) v &= ~(1ull << (w & 63));
      v &= ~c.sel[j];
      if (v != old) rw[j] = v;
      pc += __popcll(v);
    }
  }
  __syncthreads();
  block_add(&sh.acc64[3], pc);
  __syncthreads();
}

// Returns true when the selected columns were already dropped from the rows.
template <int BS, bool LA>
__device__ bool apply_round(Ctx<LA>& c, Shared& sh, bool pivot) {
  if constexpr (!LA) {
    if constexpr (BS >= 256) {
      if (c.tb && uni(sh.ns) <= TEAM_MAXS && c.scr_words >= TEAM_SLICE_LDS) {
        apply_round_team<BS>(c, sh, pivot);
        return true;
      }
    }
    if (uni(sh.ns) <= SPIDER_MAJOR_MAX && c.scr_words >= 64) {
      apply_round_arena<BS>(c, sh, pivot);
      return true;
    }
  }
  const int W = c.W, n = c.n, nsw = uni(sh.nsw), ns = uni(sh.ns);
  const int rows_per = BS / W;
  const int tw = threadIdx.x / W, j = threadIdx.x - tw * W;
  int64_t pc = 0;
  if (tw < rows_per && ns <= SPIDER_MAJOR_MAX) {
    for (int w0 = tw; w0 < n; w0 += rows_per * MAXI) {
      uint64_t v[MAXI];
      int dk[MAXI];
      uint32_t act = 0;
#pragma unroll
      for (int i = 0; i < MAXI; ++i) {
        const int w = w0 + i * rows_per;
        const bool a = w < n && bit_of(c.alive, w) && !bit_of(c.sel, w);
        act |= (a ? 1u : 0u) << i;
        v[i] = a ? row_ptr(c, w)[j] : 0;
        dk[i] = 0;
      }
      if (act) {
        for (int sidx = 0; sidx < ns; ++sidx) {
          const int x = c.slist[sidx];
          const uint64_t val = row_ptr(c, x)[j];
          const int kx = c.kc[x];
          const int px = pivot ? c.partner[x] : 0;
#pragma unroll
          for (int i = 0; i < MAXI; ++i) {
            if (!((act >> i) & 1)) continue;
            const auto rw = row_ptr(c, w0 + i * rows_per);
            if ((rw[x >> 6] >> (x & 63)) & 1) {
              v[i] ^= val;
              if (j == 0) {
                dk[i] += kx;
                if (pivot && ((rw[px >> 6] >> (px & 63)) & 1)) dk[i] += 2;  // adjacent to both ends
              }
            }
          }
        }
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
          if (!((act >> i) & 1)) continue;
          const int w = w0 + i * rows_per;
          auto rw = row_ptr(c, w);
          uint64_t x = v[i];
          if (j == (w >> 6)) x &= ~(1ull << (w & 63));
          if (x != rw[j]) rw[j] = x;
          pc += __popcll(x & ~c.sel[j]);
          if (j == 0 && dk[i]) c.k[w] = (int8_t)((c.k[w] + dk[i]) & 7);
        }
      }
    }
  } else if (tw < rows_per) {
    const LDSP int32_t* sw = (const LDSP int32_t*)c.blocked;
    for (int w = tw; w < n; w += rows_per) {
      if (!bit_of(c.alive, w) || bit_of(c.sel, w)) continue;
      auto row = row_ptr(c, w);
      uint64_t acc = 0;
      int dk = 0;
      for (int q = 0; q < nsw; ++q) {
        const int kw = sw[q];
        uint64_t msk = row[kw] & c.sel[kw];
        while (msk) {
          const int b = __ffsll((long long)msk) - 1;
          msk &= msk - 1;
          const int x = 64 * kw + b;
          acc ^= row_ptr(c, x)[j];
          if (j == 0) {
            dk += c.kc[x];
            if (pivot) {
              const int p = c.partner[x];
              if ((row[p >> 6] >> (p & 63)) & 1) dk += 2;  // adjacent to both ends
            }
          }
        }
      }
      const uint64_t old = row[j];
      uint64_t v = old ^ acc;
      if (j == (w >> 6)) v &= ~(1ull << (w & 63));
      if (v != old) row[j] = v;
      pc += __popcll(v & ~c.sel[j]);
      if (j == 0 && dk) c.k[w] = (int8_t)((c.k[w] + dk) & 7);
    }
  }
  __syncthreads();  // the spider-major path reads rows it does not own until here
  block_add(&sh.acc64[3], pc);
  __syncthreads();
  return false;
}

// Delete the selected spiders: clear their columns in every other row, zero
// their rows, clear alive, phase 0.
template <int BS, bool LA>
__device__ void delete_selected(Ctx<LA>& c, Shared& sh, bool cols_done) {
  const int W = c.W, n = c.n, nsw = uni(sh.nsw);
  const LDSP int32_t* sw = (const LDSP int32_t*)c.blocked;
  if (nsw > 0 && !cols_done) {
    for (int it = threadIdx.x; it < n * nsw; it += BS) {
      const int w = it / nsw, q = it - w * nsw;
      const int kw = sw[q];
      auto row = row_ptr(c, w);
      if (bit_of(c.sel, w)) continue;
      const uint64_t v = row[kw];
      if (v & c.sel[kw]) row[kw] = v & ~c.sel[kw];
    }
  }
  const int ns = uni(sh.ns);
  for (int i = c.team; i < ns; i += c.nteams) {
    const int x = c.slist[i];
    auto rx = row_ptr(c, x);
    for (int j = c.tl; j < W; j += c.T) rx[j] = 0;
    if (c.tl == 0) c.k[x] = 0;
    for (int q = c.tl; q < c.pw; q += c.T) c.par[(int64_t)x * c.pw + q] = 0;
  }
  // (the column pass above reads the selected set, not the present one)
  for (int j = threadIdx.x; j < W; j += BS) c.alive[j] &= ~c.sel[j];
  __syncthreads();
}

// Scalar and counters after a ZX round; the edge count after the round comes
// from apply_round (sh.acc64[3] = twice the count).
template <int BS, bool LA>
__device__ void finish_round(Ctx<LA>& c, Shared& sh, int removed) {
  if (threadIdx.x == 0) {
    const int64_t e_before = sh.E;
    const int64_t e_after = sh.acc64[3] / 2;
    sh.pow_sqrt2 += (e_after - e_before) + removed;
    sh.phase8 = (int32_t)((sh.phase8 + sh.acc64[2]) & 7);
    // edges toggled on = (pairs toggled + change among the other spiders) / 2
    const int64_t others_before = e_before - sh.acc64[0];
    sh.fill_in += (sh.acc64[1] + (e_after - others_before)) / 2;
    sh.E = e_after;
  }
  __syncthreads();
}

// Trace entries of a local-complementation round (ascending spider id).
template <int BS, bool LA>
__device__ void trace_lc_round(Ctx<LA>& c, Shared& sh) {
  if (c.trace && threadIdx.x < 64) {
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

// ------------------------------------------------ parameterized spiders --
// A spider's phase is k pi/4 + (p . f) pi, p its parameter row (the paper's
// parameterized Pauli vertices; the rules of appendix "Rewrite rules" take
// phases pi/2 + b pi and a pi with binary a, b).

__device__ __forceinline__ bool par_nonzero(const uint64_t* par, int pw, int v) {
  uint64_t o = 0;
  for (int q = 0; q < pw; ++q) o |= par[(int64_t)v * pw + q];
  return o != 0;
}

// The two parameter steps are kept out of line and called only for diagrams
// with parameters: inlined, their registers pushed the greedy kernel from 120
// to about 184 VGPRs (two waves per SIMD instead of four) for every diagram.
//
// Terms of the round's rewrites whose scalar depends on the parameters, in
// trace order (ascending spider for local complementation, ascending lower
// end for pivots; slist is ascending).  Local complementation at u with
// p_u != 0: the factor e^{-i b pi/2}, b = (k_u - 2)/4 XOR p_u.f, is
// h(pi, pi/2; p_u.f, 0)/(2i) for k_u = 2 and -i h(0, pi/2; p_u.f, 0)/2 for
// k_u = 6: term (k_alpha, k_beta) = (4 or 0, 2), constant omega^-2 / 2 in
// place of the rule's e^{-i b0 pi/2}.  Pivot (u, v) with p_u or p_v != 0:
// (-1)^{ab} = h(a0 pi, b0 pi; p_u.f, p_v.f)/2: term (k_u, k_v), constant 1/2
// in place of (-1)^{a0 b0}.  The constants go straight into the scalar.
// Reads only phases, partners and parameter rows of the selected spiders,
// none of which the round has changed yet.
template <int BS, bool LA>
__device__ __noinline__ void terms_round(Ctx<LA>& c, Shared& sh, bool pivot) {
  if (!c.pw) return;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, pw = c.pw, ns = uni(sh.ns);
    const int64_t tb = zx_term_bytes(pw);
    int nt = sh.n_terms, dphase = 0, cnt = 0;
    for (int i0 = 0; i0 < ns; i0 += 64) {
      const int i = i0 + lane;
      bool has = false;
      int x = -1, p = -1;
      if (i < ns) {
        x = c.slist[i];
        p = pivot ? c.partner[x] : -1;
        if (!pivot || p > x)
          has = par_nonzero(c.par, pw, x) || (pivot && par_nonzero(c.par, pw, p));
      }
      const uint64_t b = __ballot(has);
      const int pos = nt + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0));
      if (has && pos <= c.n) {
        uint8_t* e = c.terms + (int64_t)pos * tb;
        ZxTermHead* hd = (ZxTermHead*)e;
        uint64_t* u = (uint64_t*)(e + 16);
        uint64_t* v = u + pw;
        if (!pivot) {
          hd->k_alpha = c.k[x] == 2 ? 4 : 0;
          hd->k_beta = 2;
          for (int q = 0; q < pw; ++q) {
            u[q] = c.par[(int64_t)x * pw + q];
            v[q] = 0;
          }
          dphase += c.k[x] == 2 ? -2 : 0;  // -1 in place of 1 - 2 b0
        } else {
          hd->k_alpha = c.k[x];
          hd->k_beta = c.k[p];
          for (int q = 0; q < pw; ++q) {
            u[q] = c.par[(int64_t)x * pw + q];
            v[q] = c.par[(int64_t)p * pw + q];
          }
          dphase -= 4 * ((c.k[x] / 4) * (c.k[p] / 4));  // 0 in place of 4 a0 b0
        }
        hd->pad0 = hd->pad1 = 0;
      }
      nt += __popcll(b);
      cnt += __popcll(b);
    }
    for (int o = 32; o > 0; o >>= 1) dphase += __shfl_xor(dphase, o);
    if (lane == 0) {
      if (nt > c.n + 1) sh.status = ZX_ECAPACITY;
      sh.n_terms = nt;
      sh.phase8 = (sh.phase8 + dphase) & 7;
      sh.pow_sqrt2 -= 2 * (int64_t)cnt;
    }
  }
  __syncthreads();
}

// Parameter rows after the round: local complementation at u gives every
// neighbour p_u; a pivot (u, v) gives N(u) p_v and N(v) p_u (common
// neighbours both).  So p_w ^= XOR over selected x adjacent to w of
// p_src(x), src(x) = x (local complementation) or x's partner (pivot).  One
// thread per (present unselected row, parameter word); runs before the
// round changes any unselected row (selected columns are still set).
template <int BS, bool LA>
__device__ __noinline__ void param_round(Ctx<LA>& c, Shared& sh, bool pivot) {
  if (!c.pw) return;
  const int pw = c.pw, n = c.n, nsw = uni(sh.nsw);
  const LDSP int32_t* sw = (const LDSP int32_t*)c.blocked;
  for (int64_t it = threadIdx.x; it < (int64_t)n * pw; it += BS) {
    const int w = (int)(it / pw), q = (int)(it - (int64_t)w * pw);
    if (!bit_of(c.alive, w) || bit_of(c.sel, w)) continue;
    const auto row = row_ptr(c, w);
    uint64_t d = 0;
    for (int s = 0; s < nsw; ++s) {
      const int kw = sw[s];
      uint64_t msk = row[kw] & c.sel[kw];
      while (msk) {
        const int b = __ffsll((long long)msk) - 1;
        msk &= msk - 1;
        const int x = 64 * kw + b;
        const int src = pivot ? c.partner[x] : x;
        d ^= c.par[(int64_t)src * pw + q];
      }
    }
    if (d) c.par[it] ^= d;
  }
  __syncthreads();
}

#include "policy_dev.h"

// ----------------------------------------------------------- simplify --
// Diagrams of at most 64 spiders without parameters, greedy schedule: the
// same rounds as simplify_rounds, run by one wavefront with the adjacency
// in registers (lane v holds row v and phase k_v), so that a round costs a
// few dozen wave instructions instead of a chain of LDS round trips and
// barriers.  Candidate masks are ballots; the independent set and the
// pivot pairs are chosen in ascending spider order with scalar bit
// operations on rows read by v_readlane; every selected spider's update is
// a uniform loop step that the rows it touches apply under their own mask.
// Selected spiders are pairwise non-adjacent (pivot ends: not adjacent to
// another pair's ends), so the rows they touch are read before the round's
// updates change anything.
struct Tiny {
  uint64_t row;  // this lane's row
  int k;         // this lane's phase (units of pi/4)
  uint64_t alive, bnd;
  int64_t E, pw2, fill;
  int phase8, nt, round, status;
};

__device__ __forceinline__ void tiny_rounds(Tiny& st, int n, int32_t* trace, int max_rounds) {
  const int lane = threadIdx.x;
  const bool mine = lane < n;
  const uint64_t self = 1ull << lane;
  const int round_cap = st.round + n + 1;
  for (int kind = 0; kind < 2; ++kind) {  // local complementation, then pivots
    for (;;) {
      if (max_rounds > 0 && st.round >= max_rounds) break;
      if (st.round > round_cap) {
        st.status = ZX_EDEVICE;
        break;
      }
      const bool isc = mine && ((st.alive >> lane) & 1) && !((st.bnd >> lane) & 1) &&
                       ((st.k & 3) == (kind == 0 ? 2 : 0));
      const uint64_t cand = __ballot(isc);
      if (!cand) break;
      uint64_t sel = 0;
      int npairs = 0;
      int partner = -1;  // this lane's pivot partner
      if (kind == 0) {
        // lexicographically-first maximal independent set
        uint64_t R = cand;
        while (R) {
          const int u = __builtin_ctzll(R);
          sel |= 1ull << u;
          R &= ~(readlane64(st.row, u) | (1ull << u));
        }
      } else {
        // pivot pairs: ascending u, its lowest unblocked candidate neighbour
        // v above it; the pair blocks both neighbourhoods
        uint64_t blocked = 0, P = cand;
        while (P) {
          const int u = __builtin_ctzll(P);
          P &= P - 1;
          if ((blocked >> u) & 1) continue;
          const uint64_t ru = readlane64(st.row, u);
          const uint64_t t = ru & cand & ~blocked & ~((2ull << u) - 1);
          if (!t) continue;
          const int v = __builtin_ctzll(t);
          const uint64_t rv = readlane64(st.row, v);
          blocked |= ru | rv | (1ull << u) | (1ull << v);
          sel |= (1ull << u) | (1ull << v);
          if (lane == u) partner = v;
          if (lane == v) partner = u;
          if (lane == 0 && trace) {
            int32_t* e = trace + 4 * (int64_t)(st.nt + npairs);
            e[0] = st.round;
            e[1] = 1;
            e[2] = u;
            e[3] = v;
          }
          ++npairs;
        }
        if (npairs == 0) break;
      }
      const int removed = kind == 0 ? __popcll(sel) : 2 * npairs;
      const bool is_sel = (sel >> lane) & 1;
      if (kind == 0) {
        if (is_sel && trace) {
          int32_t* e = trace + 4 * (int64_t)(st.nt + __popcll(sel & (self - 1)));
          e[0] = st.round;
          e[1] = 0;
          e[2] = lane;
          e[3] = -1;
        }
        st.nt += removed;
      } else {
        st.nt += npairs;
      }
      // bookkeeping over the selected spiders (prepare_round's sums), and
      // each selected lane's contribution row and phase contribution; the
      // partner's row and phase come by shuffle (a per-lane source)
      int64_t s0 = 0, s1 = 0, s2 = 0;
      uint64_t contrib = 0;
      int kc = 0;
      const uint64_t prow = wave_shfl64(st.row, partner < 0 ? lane : partner, 64);
      const int pk = __shfl(st.k, partner < 0 ? lane : partner, 64);
      if (is_sel) {
        if (kind == 0) {
          const int dx = __popcll(st.row);
          s0 = dx;
          s1 = (int64_t)dx * (dx - 1) / 2;
          s2 = st.k == 2 ? 1 : 7;
          contrib = st.row;
          kc = (8 - st.k) & 7;
        } else {
          contrib = prow & ~self;  // contribution of x: its partner's row minus x
          kc = pk;
          if (lane < partner) {
            const int dx = __popcll(st.row), dp = __popcll(prow), common = __popcll(st.row & prow);
            const int64_t A = dx - 1, B = dp - 1;
            s0 = dx + dp - 1;
            s1 = A * B - (int64_t)common * common;
            s2 = 4 * ((st.k / 4) * (pk / 4));
          }
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
      }
      // the update: rows of present, non-selected spiders, by the selected
      // spiders they touch (tested on the rows before the round)
      const bool upd = mine && ((st.alive >> lane) & 1) && !is_sel;
      const uint64_t hit = upd ? (st.row & sel) : 0;
      int dk = 0;
      uint64_t S = sel;
      while (S) {
        const int x = __builtin_ctzll(S);
        S &= S - 1;
        const uint64_t cx = readlane64(contrib, x);
        const int kcx = __builtin_amdgcn_readlane(kc, x);
        const int px = __builtin_amdgcn_readlane(partner, x);
        if ((hit >> x) & 1) {
          st.row ^= cx;
          dk += kcx;
          if (kind == 1 && ((hit >> px) & 1)) dk += 2;  // adjacent to both ends
        }
      }
      if (upd) {
        st.row &= ~self & ~sel;
        st.k = (st.k + dk) & 7;
      }
      if (is_sel) {
        st.row = 0;
        st.k = 0;
      }
      st.alive &= ~sel;
      int pc = __popcll(st.row);
      for (int o = 32; o > 0; o >>= 1) pc += __shfl_xor(pc, o, 64);
      // finish_round
      const int64_t e_after = pc / 2;
      st.pw2 += (e_after - st.E) + removed;
      st.phase8 = (int)((st.phase8 + s2) & 7);
      const int64_t others_before = st.E - s0;
      st.fill += (s1 + (e_after - others_before)) / 2;
      st.E = e_after;
      ++st.round;
    }
    if (st.status) break;
  }
}

// The rounds only, from and back to the LDS state (for callers that keep
// the rest of the pipeline in LDS).
template <int BS>
__device__ __noinline__ void simplify_rounds_tiny(Ctx<true>& c, Shared& sh, int max_rounds) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, n = c.n;
    const bool mine = lane < n;
    Tiny st;
    st.row = mine ? c.adj[(int64_t)lane * c.ldw] : 0;
    st.k = mine ? c.k[lane] : 0;
    st.alive = c.alive[0];
    st.bnd = c.bnd[0];
    st.E = sh.E;
    st.pw2 = sh.pow_sqrt2;
    st.fill = sh.fill_in;
    st.phase8 = sh.phase8;
    st.nt = sh.n_trace;
    st.round = sh.round;
    st.status = 0;
    tiny_rounds(st, n, c.trace, max_rounds);
    if (mine) {
      c.adj[(int64_t)lane * c.ldw] = st.row;
      c.k[lane] = (int8_t)st.k;
    }
    if (lane == 0) {
      c.alive[0] = st.alive;
      sh.E = st.E;
      sh.pow_sqrt2 = st.pw2;
      sh.fill_in = st.fill;
      sh.phase8 = st.phase8;
      sh.n_trace = st.nt;
      sh.round = st.round;
      if (st.status) sh.status = st.status;
    }
  }
  __syncthreads();
}

// Rounds until the fixed point, or until sh.round reaches max_rounds (> 0).
// LEARN: candidates taken in the network's priority order (pol), else the
// canonical order.
template <int BS, bool LA, bool LEARN>
__device__ void simplify_rounds(Ctx<LA>& c, Shared& sh, Pol* pol, int max_rounds) {
  if constexpr (LA && !LEARN) {
    if (c.W == 1 && c.pw == 0) {
      simplify_rounds_tiny<BS>(c, sh, max_rounds);
      return;
    }
  }
  // every round deletes at least one spider: more than n + 1 rounds from
  // here would be a defect, reported instead of looping on
  const int round_cap = uni(sh.round) + c.n + 1;
  // local-complementation rounds
  for (;;) {
    if (max_rounds > 0 && uni(sh.round) >= max_rounds) return;
    if (uni(sh.round) > round_cap) {
      sh.status = ZX_EDEVICE;
      return;
    }
    if (!build_candidates<BS, LA>(c, sh, 0)) break;
    if constexpr (LEARN) {
      const int C = list_lc<BS, LA>(c, sh, *pol);
      const float invN = pauli_mask_and_scale<BS, LA>(c, sh);
      policy_score<BS, LA>(c, *pol, C, invN, false);
      __syncthreads();
      sort_keys_desc<BS>(*pol, C);
      select_lc_priority<BS, LA>(c, sh, *pol, C);
    } else {
      lfmis<BS, LA>(c, sh);  // also counts, traces and lists the set
    }
    if constexpr (LEARN) {
      if (threadIdx.x == 0) sh.cnt = 0;
      __syncthreads();
      int cnt = 0;
      for (int j = threadIdx.x; j < c.W; j += BS) cnt += __popcll(c.sel[j]);
      if (cnt) atomicAdd(&sh.cnt, cnt);
      __syncthreads();
      trace_lc_round<BS, LA>(c, sh);
    }
    const int removed = uni(sh.cnt);
    prepare_round<BS, LA>(c, sh, false, !LEARN);
    if (c.pw) {
      terms_round<BS, LA>(c, sh, false);
      param_round<BS, LA>(c, sh, false);
    }
    const bool cc = apply_round<BS, LA>(c, sh, false);
    delete_selected<BS, LA>(c, sh, cc);
    if (threadIdx.x == 0) sh.round++;  // published by finish_round's barrier
    finish_round<BS, LA>(c, sh, removed);
  }
  // pivot rounds
  for (;;) {
    if (max_rounds > 0 && uni(sh.round) >= max_rounds) return;
    if (uni(sh.round) > round_cap) {
      sh.status = ZX_EDEVICE;
      return;
    }
    if (!build_candidates<BS, LA>(c, sh, 1)) break;
    if constexpr (LEARN) {
      const int C = list_pivots<BS, LA>(c, sh, *pol);
      const float invN = pauli_mask_and_scale<BS, LA>(c, sh);
      policy_score<BS, LA>(c, *pol, C, invN, true);
      __syncthreads();
      sort_keys_desc<BS>(*pol, C);
      select_pivots_priority<BS, LA>(c, sh, *pol, C);
    } else {
      select_pivots<BS, LA>(c, sh);
    }
    const int npairs = uni(sh.cnt);
    if (npairs == 0) break;
    prepare_round<BS, LA>(c, sh, true, true);  // lists built with the selection
    if (c.pw) {
      terms_round<BS, LA>(c, sh, true);
      param_round<BS, LA>(c, sh, true);
    }
    const bool cc = apply_round<BS, LA>(c, sh, true);
    delete_selected<BS, LA>(c, sh, cc);
    for (int i = threadIdx.x; i < uni(sh.ns); i += BS) c.partner[c.slist[i]] = -1;
    if (threadIdx.x == 0) sh.round++;  // both published by finish_round's barrier
    finish_round<BS, LA>(c, sh, 2 * npairs);
  }
}

// Output frontier: rows = spiders of outputs 0..q-1, columns = spider ids,
// bit c = edge to a present spider c not attached to an output; then
// Gauss-Jordan with the lowest-index pivot row (swapped into place),
// counting row additions.  M: q x W words (LDS or global).  The whole
// workgroup works on each pivot: every row keeps a pointer to its leading
// nonzero word (columns only move right as rows are reduced), the next pivot
// is the minimum (column, row) key over the rows not yet placed (LDS
// atomicMin), the rows holding the pivot column are marked, then all
// (row, word) pairs are updated at once.
// from_work: rows come from the working adjacency (else from the arena's
// CURRENT section, written back by store_state); write_out: store the
// pivots, the reduced frontier and the header fields (else only sh.rank and
// sh.rowops are set).
template <int BS, bool LA>
__device__ void frontier(Ctx<LA>& c, Shared& sh, uint64_t* M, bool from_work, bool write_out) {
  const int q = c.q_out, W = c.W, tid = threadIdx.x;
  const int32_t* outs = (const int32_t*)(c.base + c.h->off_out);
  const uint64_t* adj = (const uint64_t*)(c.base + c.h->off_adj);
  for (int64_t i = tid; i < (int64_t)q * W; i += BS) {
    const int r = (int)(i / W), j = (int)(i % W);
    const uint64_t x = from_work ? row_ptr(c, outs[r])[j] : adj[(size_t)outs[r] * W + j];
    M[i] = x & c.alive[j] & ~c.omask[j];
  }
  LDSP int16_t* lw = c.partner;  // leading nonzero word of each row (free after the rounds)
  LDSP uint64_t* hit = c.inm;    // rows other than the pivot row holding the pivot column
  for (int p = tid; p < q; p += BS) lw[p] = 0;
  __syncthreads();
  int32_t* fpiv = (int32_t*)(c.base + c.h->off_fpiv);
  constexpr int NOKEY = 0x7fffffff;
  const int qw = (q + 63) / 64;
  int cur = 0, cmin = 0;
  int64_t ops = 0;  // thread 0
  while (cur < q) {
    if (tid == 0) sh.key = NOKEY;
    for (int j = tid; j < qw; j += BS) hit[j] = 0;
    __syncthreads();
    for (int p = cur + tid; p < q; p += BS) {
      int j = lw[p];
      if (j < (cmin >> 6)) j = cmin >> 6;
      const uint64_t* mr = M + (size_t)p * W;
      while (j < W && mr[j] == 0) ++j;
      lw[p] = (int16_t)j;
      if (j < W) atomicMin(&sh.key, ((64 * j + __ffsll((long long)mr[j]) - 1) << 15) | p);
    }
    __syncthreads();
    const int mn = uni(sh.key);
    if (mn == NOKEY) break;
    const int col = mn >> 15, r = mn & 0x7fff;
    if (r != cur) {
      for (int j = tid; j < W; j += BS) {
        const uint64_t a = M[(size_t)r * W + j];
        M[(size_t)r * W + j] = M[(size_t)cur * W + j];
        M[(size_t)cur * W + j] = a;
      }
      if (tid == 0) {
        const int16_t t = lw[r];
        lw[r] = lw[cur];
        lw[cur] = t;
      }
      __syncthreads();
    }
    for (int p = tid; p < q; p += BS)
      if (p != cur && ((M[(size_t)p * W + (col >> 6)] >> (col & 63)) & 1))
        atomicOr((unsigned long long*)&hit[p >> 6], 1ull << (p & 63));
    __syncthreads();
    if (tid == 0) {
      for (int j = 0; j < qw; ++j) ops += __popcll(hit[j]);
      if (write_out) fpiv[cur] = col;
    }
    const uint64_t* pr = M + (size_t)cur * W;
    for (int64_t it = tid; it < (int64_t)q * W; it += BS) {
      const int p = (int)(it / W), j = (int)(it - (int64_t)p * W);
      if ((hit[p >> 6] >> (p & 63)) & 1) M[it] ^= pr[j];
    }
    __syncthreads();
    ++cur;
    cmin = col + 1;
  }
  if (write_out)
    for (int j = cur + tid; j < q; j += BS) fpiv[j] = -1;
  if (tid == 0) {
    sh.rank = cur;
    sh.rowops = ops;
  }
  __syncthreads();
  if (!write_out) return;
  uint64_t* front = (uint64_t*)(c.base + c.h->off_front);
  if (M != front)
    for (int64_t i = tid; i < (int64_t)q * W; i += BS) front[i] = M[i];
  if (tid == 0) {
    c.h->rank = sh.rank;
    c.h->rowops = sh.rowops;
  }
  __syncthreads();
}

struct SimpArgs {
  int64_t lds_cap;
  int32_t extract;
  int32_t max_rounds;  // 0: to the fixed point
  int32_t resume;      // continue from the CURRENT diagram
  int32_t fallback;    // learned policy: keep the greedy result where its gate2q is lower
  const uint16_t* wbf;  // learned policy: network (bf16 copy)
  const float* param;   // learned policy: network (fp32 master)
  TeamBoard* tb;        // arena-mode rounds shared with a team (else null)
};

// A whole greedy run of such a diagram in one wavefront's registers: the
// state from the arena (SOURCE, or CURRENT to resume), the rounds, the
// write-back of the CURRENT section and header, and the output frontier's
// Gauss-Jordan elimination (rows = the outputs' spiders; pivot = the lowest
// (leading column, row) pair among the rows not yet placed, swapped into
// place; every other row holding the column is reduced and counted).  The
// arena ends as run_diagram leaves it.
template <int BS>
__device__ __noinline__ void run_tiny(uint8_t* arena, const SimpArgs& a, Shared& sh) {
  ZxHeader* h = (ZxHeader*)arena;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int n = h->n, q = h->n_out;
    const bool mine = lane < n;
    const bool src = !a.resume;
    const uint64_t* adj0 = (const uint64_t*)(arena + (src ? h->off_src_adj : h->off_adj));
    const int8_t* ph0 = (const int8_t*)(arena + (src ? h->off_src_phase : h->off_phase));
    const int32_t* outs = (const int32_t*)(arena + h->off_out);
    Tiny st;
    st.row = mine ? adj0[lane] : 0;
    st.k = mine ? ph0[lane] : 0;
    st.alive = src ? (n == 64 ? ~0ull : ((1ull << n) - 1)) : *(const uint64_t*)(arena + h->off_alive);
    st.bnd = *(const uint64_t*)(arena + h->off_bndmask);
    const int out_sp = lane < q ? outs[lane] : 0;
    st.pw2 = src ? 0 : h->pow_sqrt2;
    st.phase8 = src ? 0 : h->phase8;
    st.fill = src ? 0 : h->fill_in;
    st.nt = src ? 0 : h->n_trace;
    st.round = src ? 0 : h->rounds;
    st.status = 0;
    int pc = __popcll(st.row);
    for (int o = 32; o > 0; o >>= 1) pc += __shfl_xor(pc, o, 64);
    st.E = pc / 2;
    tiny_rounds(st, n, (int32_t*)(arena + h->off_trace), a.max_rounds);
    // CURRENT section and header
    if (mine) {
      ((uint64_t*)(arena + h->off_adj))[lane] = st.row;
      ((int8_t*)(arena + h->off_phase))[lane] = (int8_t)st.k;
    }
    if (lane == 0) {
      *(uint64_t*)(arena + h->off_alive) = st.alive;
      h->pow_sqrt2 = st.pw2;
      h->phase8 = st.phase8 & 7;
      h->fill_in = st.fill;
      h->n_edges = st.E;
      h->n_alive = __popcll(st.alive);
      h->n_trace = st.nt;
      h->rounds = st.round;
      if (st.status) zx_dev_fail(&h->status, st.status);
    }
    int rank = -1;
    int64_t ops = 0;
    if (a.extract && q > 0) {
      // output frontier: row r = the row of output r's spider, present
      // columns not attached to an output
      uint64_t om = 0;
      {
        uint64_t b = lane < q ? (1ull << out_sp) : 0;
        for (int o = 32; o > 0; o >>= 1) b |= wave_shfl64(b, lane ^ o, 64);
        om = b;
      }
      uint64_t m = wave_shfl64(st.row, out_sp, 64) & st.alive & ~om;
      if (lane >= q) m = 0;
      int piv = -1;  // pivot column of row `lane` once placed
      int cur = 0;
      constexpr int NOKEY = 0x7fffffff;
      while (cur < q) {
        int key = (lane >= cur && m) ? ((__builtin_ctzll(m) << 15) | lane) : NOKEY;
        for (int o = 32; o > 0; o >>= 1) key = min(key, __shfl_xor(key, o, 64));
        key = uni(key);
        if (key == NOKEY) break;
        const int col = key >> 15, r = key & 0x7fff;
        if (r != cur) {
          const uint64_t mr = readlane64(m, r), mc = readlane64(m, cur);
          if (lane == r) m = mc;
          if (lane == cur) m = mr;
        }
        const uint64_t pr = readlane64(m, cur);
        const bool hit = lane < q && lane != cur && ((m >> col) & 1);
        ops += __popcll(__ballot(hit));
        if (hit) m ^= pr;
        if (lane == cur) piv = col;
        ++cur;
      }
      rank = cur;
      if (lane < q) {
        ((uint64_t*)(arena + h->off_front))[lane] = m;
        ((int32_t*)(arena + h->off_fpiv))[lane] = lane < cur ? piv : -1;
      }
    }
    if (lane == 0) {
      h->rank = rank;
      h->rowops = ops;
      h->policy_used = ZX_POLICY_GREEDY;
      sh.E = st.E;
      sh.rowops = ops;
      sh.rank = rank;
      sh.status = st.status;
    }
  }
  __syncthreads();
}

// One diagram, start to finish, with the adjacency in LDS (LA) or the arena.
template <int BS, bool LA, bool LEARN>
__device__ void run_diagram(uint8_t* arena, uint8_t* lds, const SimpArgs& a, Shared& sh) {
  ZxHeader* h = (ZxHeader*)arena;
  if constexpr (LA && !LEARN) {
    if (uni(h->W) == 1 && uni(h->pw) == 0) {
      run_tiny<BS>(arena, a, sh);
      return;
    }
  }
  Ctx<LA> c;
  setup_ctx<BS, LA>(c, arena, lds);
  load_state<BS, LA>(c, sh, !a.resume);
  if (a.resume && threadIdx.x == 0) {
    sh.n_trace = h->n_trace;
    sh.round = h->rounds;
  }
  __syncthreads();
  Pol pol;
  if constexpr (LEARN)
    setup_pol<BS>(pol, lds + (LA ? lds_adj_bytes(c.n, c.W) : 0) + aux_bytes(c.n, c.W), c.n, a.wbf,
                  a.param);
  if constexpr (!LA) {
    // the LDS the auxiliary arrays (and the policy areas) leave free
    const int64_t used = aux_bytes(c.n, c.W) + (LEARN ? pol_bytes(c.n, BS) : 0);
    uint8_t* at = align16(lds + used);
    const int64_t free_bytes = a.lds_cap - (int64_t)(at - lds);
    c.scr = (LDSP uint64_t*)at;
    c.scr_words = free_bytes > 0 ? (int)(free_bytes / 8) : 0;
    c.tb = c.W <= TEAM_MAXW ? a.tb : nullptr;
  }
  simplify_rounds<BS, LA, LEARN>(c, sh, &pol, a.max_rounds);
  store_state<BS, LA>(c, sh);
  if (threadIdx.x == 0) {
    h->n_trace = sh.n_trace;
    h->rounds = sh.round;
    if (sh.status) zx_dev_fail(&h->status, sh.status);
  }
  if (a.extract && c.q_out > 0) {
    // LDS mode: the adjacency region is free once written back
    uint64_t* M = LA ? (uint64_t*)lds : (uint64_t*)(arena + h->off_front);
    __syncthreads();
    frontier<BS, LA>(c, sh, M, false, true);
  } else {
    if (threadIdx.x == 0) {
      h->rank = -1;
      h->rowops = 0;
      sh.rowops = 0;
    }
  }
  if (threadIdx.x == 0) h->policy_used = LEARN ? ZX_POLICY_LEARNED : ZX_POLICY_GREEDY;
  __syncthreads();
}

// gate2q of the greedy schedule without keeping its result: Hadamard edges
// left plus the row additions of the output frontier.  Reads SOURCE; writes
// nothing a later run from SOURCE does not overwrite (arena mode works in
// the CURRENT adjacency, the frontier goes to the arena's frontier section);
// no trace, no parameter rows, no header fields.
template <int BS, bool LA>
__device__ int64_t greedy_cost(uint8_t* arena, uint8_t* lds, const SimpArgs& a, Shared& sh) {
  ZxHeader* h = (ZxHeader*)arena;
  Ctx<LA> c;
  setup_ctx<BS, LA>(c, arena, lds);
  c.trace = nullptr;
  c.pw = 0;
  c.par = nullptr;
  c.terms = nullptr;
  load_state<BS, LA>(c, sh, true);
  if constexpr (!LA) {
    uint8_t* at = align16(lds + aux_bytes(c.n, c.W));
    const int64_t free_bytes = a.lds_cap - (int64_t)(at - lds);
    c.scr = (LDSP uint64_t*)at;
    c.scr_words = free_bytes > 0 ? (int)(free_bytes / 8) : 0;
  }
  simplify_rounds<BS, LA, false>(c, sh, nullptr, 0);
  int64_t rowops = 0;
  if (a.extract && c.q_out > 0) {
    __syncthreads();
    frontier<BS, LA>(c, sh, (uint64_t*)(arena + h->off_front), true, false);
    rowops = uni64(sh.rowops);
  }
  const bool ok = uni(sh.status) == 0;
  const int64_t cost = uni64(sh.E) + rowops;
  __syncthreads();
  return ok ? cost : INT64_MAX;
}

template <int BS, bool LEARN>
__device__ void process_diagram(uint8_t* arena, uint8_t* lds, const SimpArgs& a, Shared& sh) {
  ZxHeader* h = (ZxHeader*)arena;
  const int n = uni(h->n), W = uni(h->W);
  const int64_t aux_g = aux_bytes(n, W);
  const int64_t aux = aux_g + (LEARN ? pol_bytes(n, BS) : 0);
  const bool valid = uni(h->magic) == ZX_MAGIC && n >= 1 && W == (n + 63) / 64 && W <= MAXW && n <= 32767;
  if constexpr (LEARN) {
    // Greedy fallback: the learned schedule where it fits and its gate2q is
    // not above the greedy one's, else the greedy schedule.
    if (a.fallback && valid && aux_g <= a.lds_cap) {
      const bool la_g = lds_adj_bytes(n, W) + aux_g <= a.lds_cap;
      const int32_t st0 = uni(h->status);
      bool learned_kept = false;
      if (aux <= a.lds_cap) {
        const int64_t cg = la_g ? greedy_cost<BS, true>(arena, lds, a, sh) : greedy_cost<BS, false>(arena, lds, a, sh);
        if (lds_adj_bytes(n, W) + aux <= a.lds_cap) run_diagram<BS, true, true>(arena, lds, a, sh);
        else run_diagram<BS, false, true>(arena, lds, a, sh);
        const int64_t cl = uni(sh.status) == 0 ? uni64(sh.E) + uni64(sh.rowops) : INT64_MAX;
        learned_kept = cl <= cg && cl != INT64_MAX;
        __syncthreads();
      }
      if (!learned_kept) {
        if (threadIdx.x == 0) h->status = st0;  // a failed learned run does not stick to the greedy result
        __syncthreads();
        if (la_g) run_diagram<BS, true, false>(arena, lds, a, sh);
        else run_diagram<BS, false, false>(arena, lds, a, sh);
      }
      return;
    }
  }
  if (!valid || aux > a.lds_cap) {
    if (threadIdx.x == 0) zx_dev_fail(&h->status, ZX_ECAPACITY);
    __syncthreads();
    return;
  }
  if (lds_adj_bytes(n, W) + aux <= a.lds_cap) run_diagram<BS, true, LEARN>(arena, lds, a, sh);
  else run_diagram<BS, false, LEARN>(arena, lds, a, sh);
}

struct Queue {
  uint32_t next;
  uint32_t pad[63];
};

// The greedy kernel keeps four waves per SIMD (at most 128 VGPRs): the
// 512-thread, 64 KiB variant runs two workgroups per CU only then, and it is
// the fastest on the batched workload by a wide margin (5.4 against 9.6 ms
// at three waves).  The learned kernel's matrix-core scoring needs more.
template <int BS, bool LEARN>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(LEARN ? 1 : 4)))
void simplify_kernel(uint8_t* const* table, int32_t n_graphs, Queue* q, SimpArgs a) {
  extern __shared__ __align__(16) uint8_t smem_dyn[];
  __shared__ Shared sh;
  // q null: a grid of n_graphs workgroups, diagram blockIdx.x each
  for (int k = 0;; ++k) {
    if (threadIdx.x == 0)
      sh.idx = q ? (int32_t)atomicAdd(&q->next, 1u) : (k == 0 ? (int32_t)blockIdx.x : n_graphs);
    __syncthreads();
    const int idx = uni(sh.idx);
    __syncthreads();
    if (idx >= n_graphs) break;
    process_diagram<BS, LEARN>(table[idx], smem_dyn, a, sh);
  }
}

// ------------------------------------------------------------- teams --
struct TeamCtl {
  uint32_t next;  // diagram queue
  uint32_t pad[63];
  TeamBoard board[8];
};

constexpr int64_t TEAM_DK_BYTES = (int64_t)TEAM_MAXW * 64;  // phase increments of up to 8192 rows
constexpr int64_t TEAM_LDS = 152 * 1024;

__global__ void team_reset(TeamCtl* t, int8_t* dk) {
  if (threadIdx.x == 0) t->next = 0;
  if (threadIdx.x < 8) {
    t->board[threadIdx.x].claim = 0;
    t->board[threadIdx.x].done = 0;
    t->board[threadIdx.x].exit = 0;
    t->board[threadIdx.x].dk = dk + TEAM_DK_BYTES * threadIdx.x;
  }
}

// A helper: claim slices of its team's rounds until the team is done.  It
// waits for a round it has not exhausted yet; a long silence (no round, no
// exit) ends it too, and the running workgroup then does the slices alone.
template <int BS>
__device__ void team_helper(TeamBoard* tb, LDSP uint64_t* hm, Shared& sh) {
  const int tid = threadIdx.x;
  uint32_t last = 0;  // the last round this member exhausted
  for (;;) {
    // wait (thread 0, relaxed polls) for a round other than `last`, or the end
    if (tid == 0) {
      uint32_t seq = 0;
      const uint64_t t0 = wall_clock64();
      for (;;) {
        const unsigned long long c0 = __hip_atomic_load(&tb->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        seq = (uint32_t)(c0 >> 32);
        if (seq != 0 && seq != last) break;
        if (__hip_atomic_load(&tb->exit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            wall_clock64() - t0 > TEAM_WAIT_TICKS) {
          seq = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (seq) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the round's data
      sh.key = (int32_t)seq;
    }
    __syncthreads();
    const uint32_t seq = (uint32_t)uni(sh.key);
    __syncthreads();
    if (seq == 0) break;
    // claim slices of round seq until none is left, then publish them
    // (a round finished meanwhile leaves no slice to claim, so a copy of a
    // later round's data is never used)
    const SliceRound r = team_stage_board<BS>(tb, hm);
    int64_t mypc = 0;
    uint32_t mine = 0;
    for (;;) {
      if (tid == 0) sh.idx = team_claim(tb, seq);
      __syncthreads();
      const int sl = uni(sh.idx);
      __syncthreads();
      if (sl < 0) break;
      team_slice<BS, 8>(r, sl, hm, sh);
      if (tid == 0) mypc += sh.acc64[4];
      ++mine;
    }
    team_publish<BS>(tb, sh, mypc, mine);
    last = seq;
  }
}

// Diagrams from TEAM_MIN_N spiders: blocks 8 k + x form team x (k = 0 runs
// the diagrams the team takes from the queue, k > 0 help with their
// rounds), so a team's members share one XCD and its L2.
template <int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(1)))
void team_kernel(uint8_t* const* table, int32_t n_graphs, TeamCtl* ctl, SimpArgs a) {
  extern __shared__ __align__(16) uint8_t smem_dyn[];
  __shared__ Shared sh;
  __shared__ uint64_t hm[TEAM_SLICE_LDS];
  TeamBoard* tb = &ctl->board[blockIdx.x & 7];
  if ((blockIdx.x >> 3) != 0) {
    team_helper<BS>(tb, (LDSP uint64_t*)hm, sh);
    return;
  }
  a.tb = tb;
  for (;;) {
    if (threadIdx.x == 0) sh.idx = (int32_t)atomicAdd(&ctl->next, 1u);
    __syncthreads();
    const int idx = uni(sh.idx);
    __syncthreads();
    if (idx >= n_graphs) break;
    process_diagram<BS, false>(table[idx], smem_dyn, a, sh);
  }
  if (threadIdx.x == 0) __hip_atomic_store(&tb->exit, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Rollouts: item i = (state i / per_state, candidate slot i % per_state).
// The state (CURRENT section of its arena) is only read; the work copy is in
// LDS, the frontier matrix in this block's slice of mbuf.
struct RollArgs {
  uint8_t* const* states;
  int32_t n_items;
  int32_t per_state;
  int64_t lds_cap;
  uint64_t* mbuf;
  int64_t mbuf_words;  // per block
  int64_t* cost;
  int64_t* fill;
  int32_t* move;
  uint16_t* feats;
};

// adjacency + auxiliary arrays + candidate list + one wavefront's features
__host__ __device__ inline int64_t roll_lds_bytes(int n, int W) {
  return lds_adj_bytes(n, W) + aux_bytes(n, W) + 16 + (int64_t)pol_cap(n) * 4 + 32 * zxmlp::IN * 2;
}

template <int BS>
__global__ __launch_bounds__(BS) void rollout_kernel(Queue* q, RollArgs a) {
  extern __shared__ __align__(16) uint8_t smem_dyn[];
  __shared__ Shared sh;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sh.idx = (int32_t)atomicAdd(&q->next, 1u);
    __syncthreads();
    const int idx = uni(sh.idx);
    __syncthreads();
    if (idx >= a.n_items) break;
    const int si = idx / a.per_state, k = idx - si * a.per_state;
    uint8_t* arena = a.states[si];
    const ZxHeader* h = (const ZxHeader*)arena;
    const int n = uni(h->n), W = uni(h->W), q_out = uni(h->n_out);
    const bool fits = uni(h->magic) == ZX_MAGIC && n >= 1 && W == (n + 63) / 64 && W <= MAXW &&
                      n <= 32767 && roll_lds_bytes(n, W) <= a.lds_cap && (int64_t)q_out * W <= a.mbuf_words;
    // One structured branch per item, no early exit from the body: every
    // wave of the block takes the same path through the same barriers.
    Ctx<true> c;
    Pol pol;
    int C = 0;
    bool piv = false;
    if (fits) {
      setup_ctx<BS, true>(c, arena, smem_dyn);
      c.trace = nullptr;
      c.pw = 0;  // the state is only read: parameter rows play no part in a rollout's cost
      c.par = nullptr;
      c.terms = nullptr;
      pol.wbf = nullptr;
      pol.param = nullptr;
      pol.cap = pol_cap(n);
      pol.key = nullptr;
      uint8_t* pa = align16(smem_dyn + lds_adj_bytes(n, W) + aux_bytes(n, W));
      pol.list = (LDSP uint32_t*)pa;
      pol.fbuf = (LDSP uint16_t*)(pa + (int64_t)pol.cap * 4);
      load_state<BS, true>(c, sh, false);
      // candidates of the next round: the LC candidates while there are
      // any, then the pivot edges
      if (build_candidates<BS, true>(c, sh, 0)) {
        C = list_lc<BS, true>(c, sh, pol);
      } else if (build_candidates<BS, true>(c, sh, 1)) {
        C = list_pivots<BS, true>(c, sh, pol);
        piv = true;
      }
    }
    if (fits && k < C) {
      const int ci = C <= a.per_state ? k : (int)((int64_t)k * C / a.per_state);
      const uint32_t ent = (uint32_t)uni((int)pol.list[ci]);
      const int u = piv ? (int)(ent >> 16) : (int)ent, v = piv ? (int)(ent & 0xffffu) : -1;
      const float invN = pauli_mask_and_scale<BS, true>(c, sh);
      if (tid < 64) {
        if (piv)
          pivot_features(c, u, v, invN, pol.fbuf);
        else
          candidate_features(c, u, invN, pol.fbuf);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        if (tid < zxmlp::IN) a.feats[(int64_t)idx * zxmlp::IN + tid] = pol.fbuf[tid];
      }
      for (int j = tid; j < W; j += BS) c.sel[j] = 0;
      __syncthreads();
      const int64_t fill0 = sh.fill_in;
      if (tid == 0) {
        a.move[3 * (int64_t)idx] = piv ? 1 : 0;
        a.move[3 * (int64_t)idx + 1] = u;
        a.move[3 * (int64_t)idx + 2] = v;
        c.sel[u >> 6] |= 1ull << (u & 63);
        if (piv) {
          c.sel[v >> 6] |= 1ull << (v & 63);
          c.partner[u] = (int16_t)v;
          c.partner[v] = (int16_t)u;
        }
      }
      __syncthreads();
      // the candidate as a one-rewrite round, then the greedy schedule
      prepare_round<BS, true>(c, sh, piv, false);
      const bool cc = apply_round<BS, true>(c, sh, piv);
      delete_selected<BS, true>(c, sh, cc);
      finish_round<BS, true>(c, sh, piv ? 2 : 1);
      if (piv) {
        for (int i = tid; i < uni(sh.ns); i += BS) c.partner[c.slist[i]] = -1;
        __syncthreads();
      }
      simplify_rounds<BS, true, false>(c, sh, nullptr, 0);
      if (c.q_out > 0) {
        frontier<BS, true>(c, sh, a.mbuf + (int64_t)blockIdx.x * a.mbuf_words, true, false);
      } else if (tid == 0) {
        sh.rowops = 0;
      }
      __syncthreads();
      if (tid == 0) {
        a.cost[idx] = sh.status ? -4 : sh.E + sh.rowops;
        a.fill[idx] = sh.fill_in - fill0;
      }
    } else {
      if (tid < zxmlp::IN) a.feats[(int64_t)idx * zxmlp::IN + tid] = 0;
      if (tid == 0) {
        a.cost[idx] = fits ? -1 : -3;
        a.fill[idx] = 0;
        a.move[3 * (int64_t)idx] = -1;
        a.move[3 * (int64_t)idx + 1] = -1;
        a.move[3 * (int64_t)idx + 2] = -1;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ features --
struct FeatArgs {
  uint8_t* arena;
  int32_t* cand;
  uint16_t* feats;
  int32_t max_cand;
  int32_t* n_cand;
};

// One workgroup: the candidates of the next round of one diagram's CURRENT
// state as the learned schedule lists them (LC candidates ascending, else
// pivot edges lexicographic) and the learned proposal's features of each
// (one wavefront per candidate), as the learned simplification computes
// them before scoring.  The host checked that the
// diagram fits the LDS (roll_lds_bytes).
template <int BS>
__global__ __launch_bounds__(BS) void features_kernel(FeatArgs a) {
  extern __shared__ __align__(16) uint8_t smem_dyn[];
  __shared__ Shared sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const ZxHeader* h = (const ZxHeader*)a.arena;
  const int n = uni(h->n), W = uni(h->W);
  Ctx<true> c;
  setup_ctx<BS, true>(c, a.arena, smem_dyn);
  c.trace = nullptr;
  c.pw = 0;
  c.par = nullptr;
  c.terms = nullptr;
  Pol pol;
  pol.wbf = nullptr;
  pol.param = nullptr;
  pol.cap = pol_cap(n);
  pol.key = nullptr;
  uint8_t* pa = align16(smem_dyn + lds_adj_bytes(n, W) + aux_bytes(n, W));
  pol.list = (LDSP uint32_t*)pa;
  pol.fbuf = (LDSP uint16_t*)(pa + (int64_t)pol.cap * 4);  // one row of features per wavefront
  load_state<BS, true>(c, sh, false);
  int C = 0;
  bool piv = false;
  if (build_candidates<BS, true>(c, sh, 0)) {
    C = list_lc<BS, true>(c, sh, pol);
  } else if (build_candidates<BS, true>(c, sh, 1)) {
    C = list_pivots<BS, true>(c, sh, pol);
    piv = true;
  }
  const float invN = pauli_mask_and_scale<BS, true>(c, sh);
  const int out = C < a.max_cand ? C : a.max_cand;
  LDSP uint16_t* f = pol.fbuf + wv * zxmlp::IN;
  for (int i = wv; i < out; i += BS / 64) {
    const uint32_t ent = (uint32_t)uni((int)pol.list[i]);
    const int u = piv ? (int)(ent >> 16) : (int)ent, v = piv ? (int)(ent & 0xffffu) : -1;
    if (piv)
      pivot_features(c, u, v, invN, f);
    else
      candidate_features(c, u, invN, f);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (lane < zxmlp::IN) a.feats[(int64_t)i * zxmlp::IN + lane] = f[lane];
    if (lane == 0) {
      a.cand[2 * (int64_t)i] = u;
      a.cand[2 * (int64_t)i + 1] = v;
    }
  }
  if (tid == 0) *a.n_cand = C;
}

// ------------------------------------------------------------- serving --

// Resident serving kernel: each workgroup claims the next ring entry (in
// submission order), simplifies that diagram, publishes its summary and the
// completion flag to host memory, and goes on until stopped or idle.
template <int BS, bool LEARN>
__global__ __launch_bounds__(BS) void serve_kernel(ZxServeArgs a, SimpArgs sa) {
  extern __shared__ __align__(16) uint8_t smem_dyn[];
  __shared__ Shared sh;
  __shared__ int64_t claimed;
  __shared__ uint64_t hm[TEAM_SLICE_LDS];
  uint64_t last = wall_clock64();  // used by thread 0 only
  // Large greedy requests share their round updates with the idle
  // workgroups of their XCD (the board of blockIdx & 7): an idle workgroup
  // that sees a round it has not helped with yet takes slices of it.
  // (boards x, x + 8, x + 16, x + 24 belong to XCD x = blockIdx & 7)
  TeamBoard* boards = (!LEARN && a.team) ? (TeamBoard*)a.team : nullptr;
  const int xcd = blockIdx.x & 7;
  uint32_t helped[SERVE_BOARDS_PER_XCD] = {};  // thread 0: the last round looked at, per board
  TeamBoard* board = nullptr;                    // the board being helped, or held
  for (;;) {
    // Idle workgroups look for work in device memory: dtail, a copy of the
    // host's ring tail.  One of them at a time (the one holding the poller
    // flag) reads the tail itself across the bus and raises dtail; with every
    // idle workgroup reading host memory in a loop, those small reads filled
    // the link and claims waited behind them.
    if (threadIdx.x == 0) {
      int64_t* dtail = a.head + 1;
      int64_t* poller = a.head + 2;
      int64_t* active = a.head + 3;  // device clock of the latest claim by any workgroup
      int64_t got = -1;
      for (int spin = 0; spin < 64 && got == -1; ++spin) {
        const int64_t t = __hip_atomic_load(dtail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t h = __hip_atomic_load(a.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < t) {
          if (__hip_atomic_compare_exchange_strong(a.head, &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)) {
            got = h;
            __hip_atomic_store(active, (int64_t)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          continue;  // claimed, or lost the race: look again at once
        }
        int64_t free_ = 0;
        if (__hip_atomic_compare_exchange_strong(poller, &free_, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
          // an acquire: a relaxed read of host memory can return a stale
          // cached line (the acquire drops such lines first), and with a
          // stale tail no workgroup would see the requests waiting
          const int64_t ht = __hip_atomic_load(a.tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
          if (ht > t) __hip_atomic_fetch_max(dtail, ht, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(poller, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (ht > t) continue;  // new entries: claim at once
        }
        // leave on the stop flag, or when the whole server has been idle:
        // no claim by this or any other workgroup for idle_ticks.  (A
        // workgroup idle on its own is not enough: under a thin stream of
        // requests most workgroups go without one for a while, and those
        // that left would not come back while others stay busy.)
        if (boards) {
          int hb = -1;
          uint32_t hseq = 0;
          for (int bi = 0; bi < SERVE_BOARDS_PER_XCD && hb < 0; ++bi) {
            TeamBoard* bd = boards + xcd + 8 * bi;
            const unsigned long long c0 = __hip_atomic_load(&bd->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t seq = (uint32_t)(c0 >> 32);
            if (seq != 0 && seq != helped[bi]) {
              helped[bi] = seq;
              hb = bi;
              hseq = seq;
            }
          }
          if (hb >= 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the round's data
            sh.key = (int32_t)hseq;
            sh.cnt = hb;
            got = -3;
            break;
          }
        }
        const uint64_t now = wall_clock64();
        const uint64_t act = (uint64_t)__hip_atomic_load(active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_load(a.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) ||
            (now - last > a.idle_ticks && (int64_t)(now - act) > (int64_t)a.idle_ticks)) {
          got = -2;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      claimed = got;
    }
    __syncthreads();
    const int64_t idx = uni64(claimed);
    __syncthreads();
    if (idx == -2) break;
    if (idx == -3) {
      // help with one round of the board's diagram, then look for work again
      const uint32_t seq = (uint32_t)uni(sh.key);
      board = boards + xcd + 8 * uni(sh.cnt);
      const SliceRound r = team_stage_board<BS>(board, (LDSP uint64_t*)hm);
      int64_t mypc = 0;
      uint32_t mine = 0;
      for (;;) {
        if (threadIdx.x == 0) sh.idx = team_claim(board, seq);
        __syncthreads();
        const int sl = uni(sh.idx);
        __syncthreads();
        if (sl < 0) break;
        team_slice<BS, 8>(r, sl, (LDSP uint64_t*)hm, sh);
        if (threadIdx.x == 0) mypc += sh.acc64[4];
        ++mine;
      }
      team_publish<BS>(board, sh, mypc, mine);
      continue;
    }
    if (idx >= 0) {
      const int64_t slot = idx & (a.cap - 1);
      const uint64_t t_claim = wall_clock64();
      // Entry idx was written before the host's release of a tail above idx;
      // the poller's read of that tail orders nothing for this workgroup, so
      // it acquires the host tail itself before reading the entry and the
      // staged bytes (the tail it reads is above idx: tails only grow).
      if (threadIdx.x == 0) (void)__hip_atomic_load(a.tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
      uint8_t* arena =
          (uint8_t*)uni64((int64_t)__hip_atomic_load(&a.entries[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
      const uint4* stage =
          (const uint4*)uni64((int64_t)__hip_atomic_load(&a.stage[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
      const int64_t sbytes =
          uni64((int64_t)__hip_atomic_load(&a.stage_bytes[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
      // the staged header and SOURCE sections into the arena (16 bytes per
      // thread and step), then drop this CU's L1 lines: the arena's memory
      // served earlier requests, and its old contents may still be cached
      uint4* dst = (uint4*)arena;
      for (int64_t i = threadIdx.x; i < sbytes / 16; i += BS) dst[i] = stage[i];
      __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      // a large request takes its XCD's board if no other request holds it
      SimpArgs sr = sa;
      sr.tb = nullptr;
      if (boards) {
        const ZxHeader* hh = (const ZxHeader*)arena;
        if (threadIdx.x == 0) {
          const int nn = hh->n;
          int held = -1;
          if (nn >= TEAM_MIN_N && (nn + 63) / 64 <= TEAM_MAXW)
            for (int bi = 0; bi < SERVE_BOARDS_PER_XCD && held < 0; ++bi) {
              uint32_t zero = 0;
              if (__hip_atomic_compare_exchange_strong(&boards[xcd + 8 * bi].owner, &zero, 1u, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                held = bi;
            }
          sh.cnt = held;
        }
        __syncthreads();
        const int held = uni(sh.cnt);
        if (held >= 0) sr.tb = boards + xcd + 8 * held;
        __syncthreads();
      }
      process_diagram<BS, LEARN>(arena, smem_dyn, sr, sh);
      __syncthreads();
      if (sr.tb && threadIdx.x == 0)
        __hip_atomic_store(&sr.tb->owner, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (threadIdx.x == 0) {
        const ZxHeader* h = (const ZxHeader*)arena;
        ZxServeRes* r = &a.res[slot];
        r->status = h->status;
        r->n_alive = h->n_alive;
        r->rounds = h->rounds;
        r->n_trace = h->n_trace;
        r->rank = h->rank;
        r->phase8 = h->phase8;
        r->n_edges = h->n_edges;
        r->rowops = h->rowops;
        r->pow_sqrt2 = h->pow_sqrt2;
        r->fill_in = h->fill_in;
        r->policy = h->policy_used;
        r->pad = 0;
        r->t_claim = t_claim;
        r->t_end = wall_clock64();
        __threadfence_system();
        __hip_atomic_store(&a.done[slot], idx + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        last = wall_clock64();
      }
      __syncthreads();
    }
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
  constexpr bool LA = false;
  Ctx<LA> c;
  setup_ctx<BS, LA>(c, arena, smem_dyn);
  load_state<BS, LA>(c, sh, false);
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
        auto row = row_ptr(c, w);
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
        auto row = row_ptr(c, w);
        for (int j = c.tl; j < c.W; j += c.T) {
          uint64_t x = row[j] ^ c.inm[j];
          if (j == (w >> 6)) x &= ~(1ull << (w & 63));
          row[j] = x;
        }
      }
      __syncthreads();
    }
    const int64_t e = count_edges<BS, LA>(c, sh);
    if (threadIdx.x == 0) sh.E = e;
    __syncthreads();
  } else {
    prepare_round<BS, LA>(c, sh, pivot != 0, false);
    terms_round<BS, LA>(c, sh, pivot != 0);
    param_round<BS, LA>(c, sh, pivot != 0);
    const bool cc = apply_round<BS, LA>(c, sh, pivot != 0);
    delete_selected<BS, LA>(c, sh, cc);
    finish_round<BS, LA>(c, sh, pivot ? 2 : 1);
  }
  store_state<BS, LA>(c, sh);
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
  if (h->pw) {
    const uint64_t* spar = (const uint64_t*)(arena + h->off_src_par);
    uint64_t* dpar = (uint64_t*)(arena + h->off_par);
    for (int64_t i = tid; i < (int64_t)n * h->pw; i += nth) dpar[i] = spar[i];
  }
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
    h->n_terms = 0;
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
    {64, 32 * 1024, "bs64-lds32k"},  // one wavefront: greedy schedule, small diagrams
};
constexpr int kOneWaveVariant = 6;
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kDefaultVariant = 1;

template <int BS, bool LEARN>
zx_status launch_simplify_bs(uint8_t* const* table, int32_t n, Queue* q, const SimpArgs& a,
                             hipStream_t s) {
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  const void* fn = (const void*)simplify_kernel<BS, LEARN>;
  // the LDS attribute and the occupancy, once per device and LDS size (one
  // diagram per launch spends most of its time on the host otherwise)
  static std::map<std::pair<int, int64_t>, int> occ;
  static std::mutex occ_mu;
  std::lock_guard<std::mutex> lock(occ_mu);
  const std::pair<int, int64_t> key(d->id, a.lds_cap);
  auto it = occ.find(key);
  int per_cu = 0;
  if (it != occ.end()) {
    per_cu = it->second;
  } else {
    ZX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)a.lds_cap));
    ZX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BS, (size_t)a.lds_cap));
    occ[key] = per_cu;
  }
  if (per_cu < 1) {
    zx_set_error("simplify variant does not fit a CU");
    return ZX_ECAPACITY;
  }
  int grid = per_cu * d->n_cu;
  if (grid >= n) {
    // a workgroup per diagram: no queue
    hipLaunchKernelGGL((simplify_kernel<BS, LEARN>), dim3(n), dim3(BS), (size_t)a.lds_cap, s, table, n,
                       (Queue*)nullptr, a);
  } else {
    hipLaunchKernelGGL(queue_reset, dim3(1), dim3(64), 0, s, q);
    hipLaunchKernelGGL((simplify_kernel<BS, LEARN>), dim3(grid), dim3(BS), (size_t)a.lds_cap, s, table, n,
                       q, a);
  }
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

zx_status launch_simplify(int variant, uint8_t* const* table, int32_t n, Queue* q, SimpArgs a,
                          bool learned, hipStream_t s) {
  const Variant& v = kVariants[variant];
  a.lds_cap = v.lds_cap;
  if (v.bs == 64) {
    if (learned) {
      zx_set_error("variant %s runs the greedy schedule only", v.name);
      return ZX_EINVAL;
    }
    return launch_simplify_bs<64, false>(table, n, q, a, s);
  }
  if (v.bs == 256)
    return learned ? launch_simplify_bs<256, true>(table, n, q, a, s)
                   : launch_simplify_bs<256, false>(table, n, q, a, s);
  return learned ? launch_simplify_bs<512, true>(table, n, q, a, s)
                 : launch_simplify_bs<512, false>(table, n, q, a, s);
}

// autotuner cache: (device name, size class) -> variant
std::map<std::string, int>& tune_cache() {
  static std::map<std::string, int> m;
  return m;
}

}  // namespace

// ===================================================================== ABI

// Greedy diagrams of TEAM_MIN_N spiders and more: one team of workgroups
// per XCD, the team buffer allocated and freed in stream order.
static zx_status launch_teams(uint8_t* const* table, int32_t n, SimpArgs a, hipStream_t s) {
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  const size_t bytes = sizeof(TeamCtl) + 8 * (size_t)TEAM_DK_BYTES;
  void* mem = nullptr;
  ZX_HIP(hipMallocAsync(&mem, bytes, s));
  TeamCtl* tc = (TeamCtl*)mem;
  hipLaunchKernelGGL(team_reset, dim3(1), dim3(64), 0, s, tc, (int8_t*)mem + sizeof(TeamCtl));
  a.lds_cap = TEAM_LDS;
  ZX_HIP(hipFuncSetAttribute((const void*)team_kernel<512>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)TEAM_LDS));
  const int per_xcd = d->n_cu / 8 > 0 ? d->n_cu / 8 : 1;
  hipLaunchKernelGGL(team_kernel<512>, dim3(8 * per_xcd), dim3(512), (size_t)TEAM_LDS, s, table, n, tc, a);
  ZX_HIP(hipGetLastError());
  ZX_HIP(hipFreeAsync(mem, s));
  return ZX_OK;
}

// The serving pool's team area: eight boards and their phase-increment rows.
constexpr int SERVE_BOARDS = 8 * SERVE_BOARDS_PER_XCD;
size_t zx_team_area_bytes() { return sizeof(TeamBoard) * SERVE_BOARDS + SERVE_BOARDS * (size_t)TEAM_DK_BYTES; }

__global__ void team_area_init(TeamBoard* b, int8_t* dk) {
  if (threadIdx.x < SERVE_BOARDS) {
    b[threadIdx.x].claim = 0;
    b[threadIdx.x].done = 0;
    b[threadIdx.x].exit = 0;
    b[threadIdx.x].owner = 0;
    b[threadIdx.x].dk = dk + TEAM_DK_BYTES * threadIdx.x;
  }
}

zx_status zx_team_area_init(void* area, hipStream_t s) {
  hipLaunchKernelGGL(team_area_init, dim3(1), dim3(64), 0, s, (TeamBoard*)area,
                     (int8_t*)area + sizeof(TeamBoard) * SERVE_BOARDS);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

// How many of the largest diagrams (sizes descending) to give teams.  The
// team kernel runs before the one-workgroup kernel and takes the whole GPU,
// so the teamed diagrams are serialised over the eight teams: a prefix pays
// when the largest diagrams would otherwise set the batch's time on one
// workgroup each.  Times from measured fits on this hardware (one
// workgroup: about 16.7 ms x (n / 2012)^3; a team: about 10.2 ms x
// (n / 2012)^1.6); the prefix minimises the teams' makespan (largest first,
// each to the least loaded team) plus the largest remaining diagram's time
// on one workgroup.
static int32_t team_prefix(const int32_t* sizes, int32_t n_graphs) {
  int32_t eligible = 0;
  while (eligible < n_graphs) {
    const int nn = sizes[eligible], ww = (nn + 63) / 64;
    if (nn < TEAM_MIN_N || ww > TEAM_MAXW || aux_bytes(nn, ww) + 1024 > TEAM_LDS) break;
    ++eligible;
  }
  auto one_wg = [](int nn) { const double r = nn / 2012.0; return 16.7 * r * r * r; };
  auto team = [](int nn) { return 10.2 * pow(nn / 2012.0, 1.6); };
  double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int32_t best = 0;
  double best_t = n_graphs > 0 ? one_wg(sizes[0]) : 0.0;
  for (int32_t k = 1; k <= eligible; ++k) {
    double* m = std::min_element(load, load + 8);
    *m += team(sizes[k - 1]);
    const double rest = k < n_graphs ? one_wg(sizes[k]) : 0.0;
    const double t = *std::max_element(load, load + 8) + rest;
    if (t < best_t) {
      best_t = t;
      best = k;
    }
  }
  return best;
}

struct zx_batch {
  uint8_t** table_dev;  // in the workspace
  Queue* queue;         // in the workspace
  int32_t n;
  std::vector<uint8_t*> arenas;  // scheduled order
  std::vector<int32_t> sizes;
  int32_t max_n;
  double mean_n;
  int32_t tuned;        // autotuned variant, -1 if none
  int32_t n_big;        // the first n_big diagrams (largest first) run with teams
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
  // diagrams whose arena-mode rounds a team of workgroups shares
  B->n_big = team_prefix(B->sizes.data(), n_graphs);
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

static bool variant_fits_n(int max_n, int v, bool learned) {
  const ZxDevice* d = zx_device();
  if (!d || kVariants[v].lds_cap > (int64_t)d->lds_per_block) return false;
  if (learned && kVariants[v].bs < 256) return false;
  if (max_n > 32767 || (max_n + 63) / 64 > MAXW) return false;
  const int W = (max_n + 63) / 64;
  const int64_t need = aux_bytes(max_n, W) + (learned ? pol_bytes(max_n, kVariants[v].bs) : 0);
  return need <= kVariants[v].lds_cap;
}
static bool variant_fits(const zx_batch* b, int v, bool learned) { return variant_fits_n(b->max_n, v, learned); }

static int pick_variant_n(int32_t max_n, bool learned);

static int pick_variant(const zx_batch* b, int tune_id, bool learned) {
  if (tune_id >= 0 && tune_id < kNumVariants) return tune_id;
  if (!learned) {
    if (b->tuned >= 0) return b->tuned;
    auto it = tune_cache().find(size_class(b));
    if (it != tune_cache().end()) return it->second;
    // a few diagrams of at most 64 spiders run in one wavefront's registers:
    // one-wave workgroups, each on its own CU
    if (b->max_n <= 64 && b->n <= 256 && variant_fits(b, kOneWaveVariant, false)) return kOneWaveVariant;
  }
  const int v = pick_variant_n(b->max_n, learned);
  return v >= 0 ? v : kDefaultVariant;
}

static SimpArgs simp_args(const zx_simplify_opts* o) {
  SimpArgs a{};
  a.lds_cap = 0;
  a.tb = nullptr;
  a.extract = o->extract;
  a.max_rounds = o->max_rounds > 0 ? o->max_rounds : 0;
  a.resume = (o->flags & ZX_RESUME) ? 1 : 0;
  a.fallback = (o->policy == ZX_POLICY_LEARNED && (o->flags & ZX_FALLBACK)) ? 1 : 0;
  a.wbf = o->mlp ? o->mlp->wbf16 : nullptr;
  a.param = o->mlp ? o->mlp->param : nullptr;
  return a;
}

int32_t zx_max_spiders(int32_t policy) {
  int32_t best = 0;
  for (int v = 0; v < kNumVariants; ++v) {
    int lo = 1, hi = 32767;
    if (!variant_fits_n(lo, v, policy == ZX_POLICY_LEARNED)) continue;
    while (lo < hi) {
      const int mid = lo + (hi - lo + 1) / 2;
      if (variant_fits_n(mid, v, policy == ZX_POLICY_LEARNED)) lo = mid;
      else hi = mid - 1;
    }
    best = std::max(best, lo);
  }
  return best;
}

// Variant for a batch whose largest diagram has max_n spiders: 512-thread
// workgroups; the 152 KiB budget when that diagram's adjacency then fits in
// LDS, else 64 KiB (arena mode either way, and two workgroups per CU).
static int pick_variant_n(int32_t max_n, bool learned) {
  const int W = (max_n + 63) / 64;
  const int64_t aux = aux_bytes(max_n, W) + (learned ? pol_bytes(max_n, 512) : 0);
  const int big = 5, small = 4;  // bs512-lds152k, bs512-lds64k
  if (lds_adj_bytes(max_n, W) + aux <= kVariants[big].lds_cap && variant_fits_n(max_n, big, learned)) return big;
  if (variant_fits_n(max_n, small, learned)) return small;
  for (int i = 0; i < kNumVariants; ++i)
    if (variant_fits_n(max_n, i, learned)) return i;
  return -1;
}

zx_status zx_launch_serve(const ZxServeArgs& a, hipStream_t s) {
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  constexpr int BS = 512;
  const int v = 4;  // bs512-lds64k
  zx_simplify_opts o = {a.policy, a.extract, -1, a.fallback ? ZX_FALLBACK : 0u, 0, 0, a.mlp};
  SimpArgs sa = simp_args(&o);
  sa.lds_cap = kVariants[v].lds_cap;
  const bool learned = a.policy == ZX_POLICY_LEARNED;
  const void* fn = learned ? (const void*)serve_kernel<BS, true> : (const void*)serve_kernel<BS, false>;
  ZX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sa.lds_cap));
  int per_cu = 0;
  ZX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BS, (size_t)sa.lds_cap));
  if (per_cu < 1) {
    zx_set_error("serving kernel does not fit a CU");
    return ZX_ECAPACITY;
  }
  // One resident workgroup per CU.  The kernel stays resident between
  // requests, so it must leave each CU room for other work: two 512-thread
  // workgroups of 128 VGPRs fill a CU's whole register file, and then no
  // other kernel -- a copy kernel of the request uploads among them -- can
  // start anywhere until the server idles out.
  const int grid = d->n_cu;
  if (learned)
    hipLaunchKernelGGL((serve_kernel<BS, true>), dim3(grid), dim3(BS), (size_t)sa.lds_cap, s, a, sa);
  else
    hipLaunchKernelGGL((serve_kernel<BS, false>), dim3(grid), dim3(BS), (size_t)sa.lds_cap, s, a, sa);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" zx_status zx_batch_simplify(zx_batch* b, const zx_simplify_opts* o, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(b, "null batch");
  zx_simplify_opts def = {ZX_POLICY_GREEDY, 1, -1, 0, 0, 0, nullptr};
  if (!o) o = &def;
  ZX_CHECK_ARG(o->policy == ZX_POLICY_GREEDY || o->policy == ZX_POLICY_LEARNED, "unknown policy %d",
               o->policy);
  const bool learned = o->policy == ZX_POLICY_LEARNED;
  if (learned)
    ZX_CHECK_ARG(o->mlp && o->mlp->param && o->mlp->wbf16, "learned policy needs a network");
  ZX_CHECK_ARG(o->max_rounds >= 0, "negative max_rounds");
  const bool fb = learned && (o->flags & ZX_FALLBACK);
  ZX_CHECK_ARG(!fb || (o->max_rounds == 0 && !(o->flags & ZX_RESUME)),
               "ZX_FALLBACK compares whole schedules: no max_rounds, no ZX_RESUME");
  int v = pick_variant(b, o->tune_id, learned);
  // with the fallback, diagrams beyond the learned policy's LDS budget run greedy
  if (fb && !variant_fits(b, v, true) && o->tune_id < 0) {
    v = pick_variant(b, o->tune_id, false);
    if (kVariants[v].bs < 256) {  // the learned kernel does not come in one wavefront
      const int w = pick_variant_n(b->max_n, false);
      v = w >= 0 ? w : kDefaultVariant;
    }
  }
  if (!variant_fits(b, v, learned && !fb)) {
    zx_set_error("diagrams too large for simplify variant %d", v);
    return ZX_ECAPACITY;
  }
  const int32_t n_big = learned ? 0 : b->n_big;
  if (n_big > 0) {
    zx_status st = launch_teams(b->table_dev, n_big, simp_args(o), s);
    if (st != ZX_OK) return st;
  }
  if (b->n > n_big) {
    zx_status st = launch_simplify(v, b->table_dev + n_big, b->n - n_big, b->queue, simp_args(o), learned, s);
    if (st != ZX_OK) return st;
  }
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
  zx_simplify_opts o = {ZX_POLICY_GREEDY, extract, -1, 0, 0, 0, nullptr};
  const SimpArgs a = simp_args(&o);
  for (int v = 0; v < kNumVariants; ++v) {
    if (!variant_fits(b, v, false)) continue;
    if (launch_simplify(v, b->table_dev, b->n, b->queue, a, false, s) != ZX_OK) continue;
    ZX_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch_simplify(v, b->table_dev, b->n, b->queue, a, false, s);
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
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
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

// ------------------------------------------------------------ rollouts --
namespace {
constexpr int kRollBS = 512;
constexpr int64_t kRollLds = 152 * 1024;
constexpr int kRollBlocksPerCU = 2;  // bound used to size the workspace

int64_t roll_mbuf_words(zx_graph* const* states, int32_t n_states) {
  int64_t mw = 1;
  for (int i = 0; i < n_states; ++i)
    if (states[i]) mw = std::max(mw, (int64_t)states[i]->n_out * states[i]->W);
  return (mw + 31) & ~int64_t(31);
}
int roll_grid_max() {
  const ZxDevice* d = zx_device();
  return (d ? d->n_cu : 256) * kRollBlocksPerCU;
}
}  // namespace

extern "C" zx_status zx_policy_features(const zx_graph* g, int32_t* cand, uint16_t* feats, int32_t max_cand,
                                        int32_t* n_cand, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g && n_cand && max_cand >= 0, "bad argument");
  ZX_CHECK_ARG(max_cand == 0 || (cand && feats), "null buffer");
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  const int64_t lds = std::min<int64_t>(kRollLds, (int64_t)d->lds_per_block);
  if (g->W > MAXW || g->n > 32767 || roll_lds_bytes(g->n, g->W) > lds) {
    zx_set_error("diagram with %d spiders does not fit the features kernel's LDS", g->n);
    return ZX_ECAPACITY;
  }
  const void* fn = (const void*)features_kernel<kRollBS>;
  ZX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  FeatArgs a;
  a.arena = g->arena;
  a.cand = cand;
  a.feats = feats;
  a.max_cand = max_cand;
  a.n_cand = n_cand;
  hipLaunchKernelGGL(features_kernel<kRollBS>, dim3(1), dim3(kRollBS), (size_t)lds, s, a);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" size_t zx_rollout_workspace_bytes(zx_graph* const* states, int32_t n_states) {
  if (!states || n_states <= 0) return 0;
  const size_t table = ((size_t)n_states * 8 + 255) & ~size_t(255);
  return 256 + sizeof(Queue) + table + (size_t)roll_grid_max() * roll_mbuf_words(states, n_states) * 8;
}

extern "C" zx_status zx_rollout(zx_graph* const* states, int32_t n_states, int32_t per_state,
                                int64_t* cost, int64_t* fill, int32_t* move, uint16_t* feats, void* ws,
                                size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(states && n_states > 0 && per_state > 0, "bad argument");
  ZX_CHECK_ARG(cost && fill && move && feats && ws, "null buffer");
  ZX_CHECK_ARG(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  ZX_CHECK_ARG((int64_t)n_states * per_state <= INT32_MAX, "too many items");
  if (ws_bytes < zx_rollout_workspace_bytes(states, n_states)) {
    zx_set_error("workspace too small");
    return ZX_ECAPACITY;
  }
  std::vector<uint8_t*> tab((size_t)n_states);
  for (int i = 0; i < n_states; ++i) {
    ZX_CHECK_ARG(states[i], "null state %d", i);
    tab[i] = states[i]->arena;
  }
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  const int64_t lds = std::min<int64_t>(kRollLds, (int64_t)d->lds_per_block);
  Queue* q = (Queue*)((uint8_t*)ws + 256);
  uint8_t** table = (uint8_t**)((uint8_t*)ws + 256 + sizeof(Queue));
  uint64_t* mbuf = (uint64_t*)((uint8_t*)table + (((size_t)n_states * 8 + 255) & ~size_t(255)));
  ZX_HIP(hipMemcpyAsync(table, tab.data(), (size_t)n_states * 8, hipMemcpyHostToDevice, s));
  const void* fn = (const void*)rollout_kernel<kRollBS>;
  ZX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = 0;
  ZX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kRollBS, (size_t)lds));
  if (per_cu < 1) {
    zx_set_error("rollout kernel does not fit a CU");
    return ZX_ECAPACITY;
  }
  const int32_t items = n_states * per_state;
  int grid = std::min(per_cu, kRollBlocksPerCU) * d->n_cu;
  grid = std::min(grid, roll_grid_max());
  if (grid > items) grid = items;
  RollArgs a;
  a.states = table;
  a.n_items = items;
  a.per_state = per_state;
  a.lds_cap = lds;
  a.mbuf = mbuf;
  a.mbuf_words = roll_mbuf_words(states, n_states);
  a.cost = cost;
  a.fill = fill;
  a.move = move;
  a.feats = feats;
  hipLaunchKernelGGL(queue_reset, dim3(1), dim3(64), 0, s, q);
  hipLaunchKernelGGL(rollout_kernel<kRollBS>, dim3(grid), dim3(kRollBS), (size_t)lds, s, q, a);
  ZX_HIP(hipGetLastError());
  ZX_HIP(hipStreamSynchronize(s));
  return ZX_OK;
}
