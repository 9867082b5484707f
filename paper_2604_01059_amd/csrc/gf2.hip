// GF(2) reduced row echelon form on one MI355X: one cooperative persistent
// launch, every 64-bit word column resident in a workgroup's LDS.
//
// Method.  Gauss-Jordan elimination over F2 (the paper keeps a linearly
// independent basis of a binary matrix this way; detectors/observables
// section, after equation detector_sampling), organised by 32-column strips
// (half a word column; both halves of a word column belong to the same
// workgroup).  For strip t:
//   1. its owner picks up to 64 candidate rows (not yet pivots, non-zero in
//      the strip) and reduces their 32-bit strip words in one wavefront: for
//      each bit b a ballot finds the first candidate holding b, its word is
//      broadcast through scalar registers and XORed into every other
//      candidate holding b.  This gives up to 32 pivot rows, their bit
//      positions and, per pivot, a 32-bit mask L of the ORIGINAL pivot rows
//      that combine into the reduced pivot row.  64 random rows have rank 32
//      with probability 1 - 2^-32;
//   2. the owner publishes that "pass" (rows, bits, masks) and a snapshot of
//      the strip word of every row through a ring in the workspace;
//   3. every workgroup applies the pass to each of its word columns at or
//      after the strip: reduced pivot words P'_j = XOR of the L_j-selected
//      original pivot words; every other row r gets the XOR of P' over the
//      pivot bits set in its snapshot word (Four-Russians: 8 tables of 16
//      nibble combinations, conflict-free in LDS); pivot rows become P'.
// The owner of strip t + 1 writes that strip's snapshot and collects its
// candidates while it applies the last pass of strip t, so its reduction
// starts as soon as that pass is applied.
//
// If a pass found fewer than 32 pivots while more non-zero rows existed than
// candidates, the owner runs further passes on the residual rows.  Pivot
// columns found are always leading bits of row-space vectors and a strip ends
// only when every non-pivot row is zero in it, so the final rows are the
// unique RREF basis.  Rows stay in place; at the end the pivot rows are
// written in pivot-column order, then zero rows.
//
// Cross-workgroup hand-off.  The L2 caches of the eight XCDs are not coherent
// with each other, so everything another workgroup reads (flags, records,
// snapshots) is written and read with device-scope relaxed atomics: on
// gfx950 those are vector loads/stores with the sc1 cache policy, which go
// to the device coherence point without the whole-L2 write-back/invalidate
// of acquire/release fences.  A producer makes every wave wait for its
// stores (s_waitcnt 0) before the barrier that precedes its flag store; a
// consumer issues its payload loads only after it has seen the flag.
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "zx_internal.h"

namespace {

// LDS pointers carry their address space, so that every access compiles to a
// ds_* instruction: a flat access counts on vmcnt as well, and its wait would
// also wait for every global store still in flight.
#define LDS __attribute__((address_space(3)))

constexpr int BS = 512;           // threads per workgroup
constexpr int NWAVE = BS / 64;
constexpr int SW = 32;            // columns per strip
constexpr int RING = 8;           // pass records in flight
constexpr int NCAND = 64;         // candidate rows per pass (one per lane)
constexpr int MAX_M = 16384;      // rows that fit one column per workgroup in LDS
constexpr int MAX_SL = MAX_M / BS;  // row slices per thread
constexpr int MAX_CW = 4;         // word columns per workgroup
constexpr int MAX_STRIPS = 8192;  // strips with profile slots
constexpr int PROF_SLOTS = 8;     // timestamps per strip (profiling only)
constexpr int GROUP = 4;          // row slices updated together (loads in flight together)
constexpr int PRE = 2 * GROUP;    // row slices whose snapshot multipliers are loaded right after the record
constexpr int EARLY_MIN = 48;     // wave-0 candidates that allow reducing the next strip early

// A published pass: one 64-bit word per pivot slot t, each carrying the
// record's tag, so that the record itself is the publication:
//   bits 0-13 pivot row, 14-18 its strip bit, 19 last (the strip is finished
//   with this record), 20 valid (t < k), 21-31 tag (record index mod 2048),
//   32-63 L_t (the original pivots that combine into pivot t, by strip bit).
// A record with no valid slot ends a strip without pivots.
struct PassRec {
  uint64_t e[SW];
};
static_assert(MAX_M <= (1 << 14), "pivot rows fit 14 bits of a record word");

struct Ctl {
  uint32_t fin;        // workgroups done with every pass
  uint32_t pad[63];
  uint32_t ack[RING];  // cumulative acknowledgements per slot
  uint32_t pad2[64 - RING];
};

struct WsLayout {
  size_t ctl, recs, snaps, piv_row, piv_col, prof, bytes;
};

constexpr size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace sections; the profile slots come last, so the bytes before
// them (ws_core_bytes) serve an elimination without profiling.
WsLayout ws_layout(int m) {
  WsLayout L;
  size_t o = 256;  // ZxWsHeader
  L.ctl = o;     o += al256(sizeof(Ctl));
  L.recs = o;    o += al256(sizeof(PassRec) * RING);
  L.snaps = o;   o += al256((size_t)m * 4 * RING);
  L.piv_row = o; o += al256((size_t)m * 4);
  L.piv_col = o; o += al256((size_t)m * 4);
  L.prof = o;    o += al256((size_t)MAX_STRIPS * PROF_SLOTS * 8);
  L.bytes = o;
  return L;
}

constexpr size_t ws_core_bytes(int m) {
  return 256 + al256(sizeof(Ctl)) + al256(sizeof(PassRec) * RING) + al256((size_t)m * 4 * RING) +
         2 * al256((size_t)m * 4);
}

struct Args {
  const uint64_t* A;
  uint64_t* R;
  uint64_t* T;          // optional transform (NULL = none), m x ldt words
  int32_t m, n_cols, nw, nw_a, cw, nstrips;  // nw: word columns held (A's nw_a, then T's)
  int64_t ld, ldt;
  int32_t* rank_dev;
  int32_t* piv_dev;
  int32_t* status;
  Ctl* ctl;
  PassRec* recs;
  uint32_t* snaps;
  int32_t* piv_row;
  int32_t* piv_col;
  uint64_t spin_ticks;  // time-out of one spin wait, in s_memrealtime ticks
  uint64_t* prof;       // optional per-strip timestamps (NULL = off)
};

__device__ __forceinline__ uint32_t ld_dev(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_dev32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev32(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// every store this wave issued has been acknowledged
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0); }
// A wave-uniform value loaded by the whole wave, consumed here on every
// path: the compiler waits for its load at this point, and no later write to
// its register waits on it (a load consumed under a lane condition only would
// stay pending for the compiler on the other path, and every later write to
// that register would wait for all memory operations in flight).
__device__ __forceinline__ uint32_t settle(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Spin (one thread) until *p >= target; false on time-out or abort.
__device__ bool spin_until(const uint32_t* p, uint32_t target, const Args& a) {
  const uint64_t t0 = wall_clock64();
  for (;;) {
    if (ld_dev(p) >= target) return true;
    if (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > a.spin_ticks) {
      zx_dev_fail(a.status, ZX_EDEVICE);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Before every elimination: rank -1, control words zero, every ring slot filled
// with all-ones words (tag 2047), which no record matches before its slot is
// rewritten (slot s holds records s, s + RING, ...), so that records left in
// a reused workspace by an earlier launch are never taken for this one's.
__global__ void rref_init(Ctl* ctl, PassRec* recs, int32_t* status, uint64_t* prof, int32_t* rank_dev) {
  const int t = threadIdx.x;
  if (t == 0) *rank_dev = -1;  // stays -1 if the elimination fails on the device
  uint32_t* c = (uint32_t*)ctl;
  for (int i = t; i < (int)(sizeof(Ctl) / 4); i += blockDim.x) c[i] = 0;
  for (int i = t; i < RING * SW; i += blockDim.x) recs[i / SW].e[i % SW] = ~0ull;
  if (prof)
    for (int i = t; i < MAX_STRIPS * PROF_SLOTS; i += blockDim.x) prof[i] = 0;
  if (t == 0) *status = 0;
}

// One pass in LDS: its pivot rows, their strip bits and masks of original
// pivots (bit q of L[t]: the original word of the pivot of strip bit q takes
// part in pivot t).  Two are kept: the pass being applied and the pass a
// wavefront reduces meanwhile.
struct Pass {
  int32_t k, last;
  uint32_t pivmask;
  int32_t rows[SW];
  int32_t bits[SW];
  uint32_t L[SW];
};

struct Smem {
  uint64_t tab[MAX_CW][128];   // 8 nibble tables of reduced pivot words, per column
  uint64_t pp[MAX_CW][SW];     // reduced pivot word of each strip bit (zero off the pivot mask), per column
  Pass ps[2];
  int32_t wcnt[NWAVE];         // candidates per wave
  int32_t cand[NCAND];
  int32_t prow[SW];            // sorted pivot list of a multi-pass strip
  int32_t pcol[SW];
  uint32_t ackc[RING];         // acknowledgements known per ring slot (a lower bound)
  uint64_t emask[NWAVE];       // candidate lanes of the early slice, per wave
  int32_t total, used, early, flag, cnt;
};

// 64-bit words of LDS before the columns (the Smem block, 16-byte aligned)
__host__ __device__ constexpr int smem_head_words() { return (int)((sizeof(Smem) + 15) / 16 * 2); }

__device__ __forceinline__ void prof_mark(const Args& a, int s, int slot) {
  if (a.prof && s < MAX_STRIPS) st_dev64(&a.prof[(size_t)s * PROF_SLOTS + slot], wall_clock64());
}

__device__ __forceinline__ bool bit_of(const LDS uint64_t* m, int r) { return (m[r >> 6] >> (r & 63)) & 1; }

__device__ __forceinline__ uint64_t rec_word(const LDS Pass& P, int t, int k, int last, uint32_t seq) {
  const bool valid = t < k;
  const uint32_t lo = (valid ? ((uint32_t)P.rows[t] | ((uint32_t)P.bits[t] << 14) | (1u << 20)) : 0u) |
                      ((uint32_t)last << 19) | ((seq & 0x7FFu) << 21);
  return ((uint64_t)(valid ? P.L[t] : 0u) << 32) | lo;
}

// Wave 0: wait until ring slot `rec` holds record `seq` (every word carries
// its tag; words of the slot's previous record or of a partly landed one do
// not) and unpack it into P.  False on time-out or abort.
__device__ bool read_record(const PassRec* rec, uint32_t seq, const Args& a, LDS Pass& P) {
  const int lane = threadIdx.x & 63;
  const uint32_t tag = seq & 0x7FFu;
  const uint64_t t0 = wall_clock64();
  uint64_t e;
  for (;;) {
    e = lane < SW ? ld_dev64(&rec->e[lane]) : ((uint64_t)tag << 21);
    // the abort status, loaded with the record words and consumed on every
    // path (settle)
    const int32_t st = (int32_t)settle((uint32_t)__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (__ballot(((uint32_t)e >> 21) != tag) == 0) break;
    if (st != 0) return false;
    if (wall_clock64() - t0 > a.spin_ticks) {
      if (lane == 0) zx_dev_fail(a.status, ZX_EDEVICE);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);  // a short pause between polls (measured 0.4 % faster)
  }
  const uint32_t lo = (uint32_t)e;
  const bool valid = lane < SW && ((lo >> 20) & 1);
  if (valid) {
    P.rows[lane] = (int32_t)(lo & 0x3FFFu);
    P.bits[lane] = (int32_t)((lo >> 14) & 31u);
    P.L[lane] = (uint32_t)(e >> 32);
  }
  const uint64_t vmask = __ballot(valid);  // the valid slots are 0..k-1
  if (lane == 0) {
    P.k = __popcll(vmask);
    P.last = (int32_t)((lo >> 19) & 1u);
    P.pivmask = 0;
  }
  // LDS operations of one wave complete in order: the clear comes first
  if (valid) __hip_atomic_fetch_or(&P.pivmask, 1u << ((lo >> 14) & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return true;
}

// Candidates from per-thread flags (bit i = row tid + i*BS): up to NCAND of
// them go to S.cand, the count of all to S.total.  Any set of candidate rows
// gives the same basis (the reduced echelon form is unique), so each wave
// places its own candidates after those of lower waves: one count per wave,
// one barrier, then a lane-prefix (v_mbcnt) per slice.
__device__ void compact_candidates(uint32_t flags, int nsl, LDS Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int cnt = 0;
  for (int i = 0; i < nsl; ++i) cnt += __popcll(__ballot((flags >> i) & 1));
  if (lane == 0) S.wcnt[wv] = cnt;
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int v = 0; v < NWAVE; ++v) {
    const int c = S.wcnt[v];
    base += v < wv ? c : 0;
    total += c;
  }
  if (tid == 0) S.total = total;
  for (int i = 0; i < nsl && base < NCAND; ++i) {
    const bool f = (flags >> i) & 1;
    const uint64_t b = __ballot(f);
    const int idx = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0));
    if (f && idx < NCAND) S.cand[idx] = i * BS + tid;
    base += __popcll(b);
  }
  __syncthreads();
}

// Waves 1..7 (while wave 0 reduces the candidates): write the strip snapshot,
// bits [shift, shift+32) of LDS column `col` of every row, to `snap`.  They do
// not wait for these stores here, and wave 0 issues none, so the reduction
// never waits on them (vmcnt counts stores as well as loads on this
// architecture); the publishing barrier waits for them.
__device__ void store_snapshot(const LDS uint64_t* col, int shift, int m, uint32_t* snap) {
  constexpr int T = BS - 64, U = 4;
  for (int r0 = (int)threadIdx.x - 64; r0 < m; r0 += U * T) {
    uint32_t v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) v[q] = r0 + q * T < m ? (uint32_t)(col[r0 + q * T] >> shift) : 0u;
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (r0 + q * T < m) st_dev(&snap[r0 + q * T], v[q]);
  }
}

// One elimination step of the candidate reduction, for strip bit B, in
// wavefront registers: w = the lane's candidate strip word, L = its mask of
// original pivots, indexed by their strip bits; P = lanes already pivots.
//   h = lanes holding bit B; c = h & ~P; if c is empty the step is a no-op;
//   else src = first lane of c becomes the pivot of bit B: every other lane
//   of h gets w ^= w[src], L ^= L[src] | 1 << B.  Lane src keeps L[src]: its
//   mask lacks its own bit B, which only ever changes by XOR afterwards, so
//   the pivot's mask is its final L with bit B flipped, applied once at the
//   end.
// Written out by hand (thirteen instructions; a single wave issues about one
// instruction per four cycles, so the count sets the cost): the XORs run
// under an exec mask of h minus src, and exec is restored before the block
// ends.
template <int B>
__device__ __forceinline__ void factor_step(uint32_t& w, uint32_t& L, uint64_t& P) {
  uint64_t c, sv;
  uint32_t t, spw, spl;
  int src;
  asm volatile(
      "v_and_b32 %[t], %[bit], %[w]\n\t"
      "v_cmp_ne_u32 vcc, 0, %[t]\n\t"
      "s_andn2_b64 %[c], vcc, %[P]\n\t"  // SCC = (c != 0)
      "s_cbranch_scc0 .Lfactor_skip%=\n\t"
      "s_ff1_i32_b64 %[src], %[c]\n\t"
      "s_bitset1_b64 %[P], %[src]\n\t"
      "s_bitset0_b64 vcc, %[src]\n\t"
      "v_readlane_b32 %[spw], %[w], %[src]\n\t"
      "v_readlane_b32 %[spl], %[L], %[src]\n\t"
      "s_or_b32 %[spl], %[spl], %[bit]\n\t"
      "s_and_saveexec_b64 %[sv], vcc\n\t"
      "v_xor_b32 %[w], %[spw], %[w]\n\t"
      "v_xor_b32 %[L], %[spl], %[L]\n\t"
      "s_mov_b64 exec, %[sv]\n"
      ".Lfactor_skip%=:"
      : [w] "+v"(w), [L] "+v"(L), [P] "+s"(P), [t] "=&v"(t), [c] "=&s"(c), [sv] "=&s"(sv), [spw] "=&s"(spw),
        [spl] "=&s"(spl), [src] "=&s"(src)
      : [bit] "s"(1u << B)
      : "vcc", "scc");
}

template <int B>
__device__ __forceinline__ void factor_steps(uint32_t& w, uint32_t& L, uint64_t& P) {
  factor_step<B>(w, L, P);
  if constexpr (B + 1 < SW) factor_steps<B + 1>(w, L, P);
}

// Wave 0 (all 64 lanes active): reduce the first nc candidates of S.cand,
// using bits [shift, shift + 32) of the LDS column `col`: Gauss-Jordan over
// the strip bits in ascending order.  Fills N (k, rows, bits, L, pivmask).
// The reduction is the serial chain's own step while the other waves update
// rows, so it runs at raised wave priority (1.2 % on the whole elimination).
__device__ void factor_candidates(const LDS uint64_t* col, int shift, int nc, LDS Pass& N, LDS Smem& S) {
  const int lane = threadIdx.x & 63;
  __builtin_amdgcn_s_setprio(3);
  uint32_t w = lane < nc ? (uint32_t)(col[S.cand[lane]] >> shift) : 0;
  uint32_t L = 0;
  uint64_t P = 0;
  factor_steps<0>(w, L, P);
  const int k = __popcll(P);
  // A pivot lane's strip bit is the lowest set bit of its final word: bits
  // below it that hold pivots were cleared at their steps, bits below it
  // without a pivot are clear in every lane that was not yet a pivot at that
  // step, and the pivots XORed in later are clear at both.  Its pivot index
  // is the number of pivot bits below its own.
  const bool piv = (P >> lane) & 1;
  const int b = piv ? __builtin_ctz(w) : 0;
  if (lane == 0) {
    N.k = k;
    N.pivmask = 0;
  }
  // LDS operations of one wave complete in order: the clear, the ORs, then
  // the read of the mask
  if (piv) __hip_atomic_fetch_or(&N.pivmask, 1u << b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const uint32_t pm = __hip_atomic_load(&N.pivmask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (piv) {
    const int j = __popc(pm & ((1u << b) - 1u));
    N.L[j] = L ^ (1u << b);
    N.rows[j] = S.cand[lane];
    N.bits[j] = b;
  }
  __builtin_amdgcn_s_setprio(0);
}

// XOR scan over each 16-lane DPP row of the wavefront: lane 15 of a row ends
// with the XOR of the row's 16 values (row_shr by 1, 2, 4, 8; lanes shifted
// in from outside the row contribute zero).
__device__ __forceinline__ uint32_t row_xor16(uint32_t v) {
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  return v;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Tables of pass R for `nc` columns, and R's pivot rows: marks them in
// newpiv (this pass) and pivflag (all passes), and writes their reduced
// words into the columns.  The reduction takes strip bits in ascending
// order, so the pivot at strip bit b is pivot t(b) = popcount(pivmask below
// b), and its reduced word is P'_b = XOR of the original words of the pivots
// whose strip bits are in L_t(b).  Strip bit b = 4w + r is DPP row r of wave
// w: each of its 16 lanes XORs the original words of the pivots of two strip
// bits of L_t(b), a row XOR scan
// leaves P'_b in the row's last lane, and wave w, which then holds the four
// strip bits of nibble table w, writes that table (entry e = XOR of the P'_b
// selected by the bits of e) and keeps its P'_b in S.pp.  After a barrier
// (every original word has been read) the pivot rows take their P'; a second
// barrier ends the call.  The row update that follows leaves newpiv rows as
// they are.
__device__ void make_tables(LDS uint64_t* const* cols, int nc, LDS uint64_t* newpiv, LDS uint64_t* pivflag,
                            const LDS Pass& R, LDS Smem& S) {
  static_assert(NWAVE * 4 == SW, "one wave per nibble table");
  const int tid = threadIdx.x, lane = tid & 63, k = R.k;
  if (tid < k) {
    const int r = R.rows[tid];
    __hip_atomic_fetch_or(&newpiv[r >> 6], 1ull << (r & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_or(&pivflag[r >> 6], 1ull << (r & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  const uint32_t pm = R.pivmask;
  const int w = tid >> 6, b = 4 * w + (lane >> 4), sub = lane & 15;
  // L is indexed by strip bits: bit q names the pivot of strip bit q
  const uint32_t Lm = ((pm >> b) & 1) ? R.L[__popc(pm & ((1u << b) - 1u))] : 0u;
  const int q0 = 2 * sub, q1 = 2 * sub + 1;
  const bool u0 = (Lm >> q0) & 1, u1 = (Lm >> q1) & 1;
  const int r0 = u0 ? R.rows[__popc(pm & ((1u << q0) - 1u))] : 0;
  const int r1 = u1 ? R.rows[__popc(pm & ((1u << q1) - 1u))] : 0;
  for (int j = 0; j < nc; ++j) {
    const LDS uint64_t* c = cols[j];
    const uint64_t x0 = c[r0], x1 = c[r1];
    const uint64_t v = (u0 ? x0 : 0ull) ^ (u1 ? x1 : 0ull);
    const uint64_t p = ((uint64_t)row_xor16((uint32_t)(v >> 32)) << 32) | row_xor16((uint32_t)v);
    const uint64_t p0 = readlane64(p, 15), p1 = readlane64(p, 31), p2 = readlane64(p, 47), p3 = readlane64(p, 63);
    if (lane < 16)
      S.tab[j][16 * w + lane] = ((lane & 1) ? p0 : 0ull) ^ ((lane & 2) ? p1 : 0ull) ^ ((lane & 4) ? p2 : 0ull) ^
                                ((lane & 8) ? p3 : 0ull);
    if (sub == 15) S.pp[j][b] = p;
  }
  __syncthreads();
  for (int x = tid; x < nc * SW; x += BS) {
    const int j = x / SW, t = x % SW;
    if (t < k) cols[j][R.rows[t]] = S.pp[j][R.bits[t]];
  }
  __syncthreads();
}

// Clear R's rows from newpiv once the update is done (after a barrier).
__device__ __forceinline__ void clear_newpiv(LDS uint64_t* newpiv, const LDS Pass& R) {
  if ((int)threadIdx.x < R.k) {
    const int r = R.rows[threadIdx.x];
    __hip_atomic_fetch_and(&newpiv[r >> 6], ~(1ull << (r & 63)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // v_bitop3: a ^ b ^ c in one instruction
}

// v ^ (XOR of the 8 nibble-table entries selected by mr)
__device__ __forceinline__ uint64_t lookup8(const LDS uint64_t* tab, uint32_t mr, uint64_t v) {
  uint64_t t[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) t[q] = tab[16 * q + __builtin_amdgcn_ubfe(mr, 4 * q, 4)];
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int q = 0; q < 8; q += 2) {
    lo = xor3(lo, (uint32_t)t[q], (uint32_t)t[q + 1]);
    hi = xor3(hi, (uint32_t)(t[q] >> 32), (uint32_t)(t[q + 1] >> 32));
  }
  return ((uint64_t)hi << 32) | lo;
}

// One group of GROUP row slices of one column: v ^= T(mr) row by row, all
// loads of the group in flight together (no branch between rows).  FULL:
// every slice of the group exists.  With FUSE, returns the candidate flags
// of the group's rows (bits [fshift, fshift+32) non-zero, not done).
template <bool FULL, bool FUSE>
__device__ __forceinline__ uint32_t apply_group(LDS uint64_t* c, const LDS uint64_t* tab, const uint32_t* mr,
                                                const uint64_t* done, int i0, int nsl, int fshift) {
  const int tid = threadIdx.x, lane = tid & 63;
  uint64_t v[GROUP];
#pragma unroll
  for (int q = 0; q < GROUP; ++q)
    if (FULL || i0 + q < nsl) v[q] = c[(i0 + q) * BS + tid];
#pragma unroll
  for (int q = 0; q < GROUP; ++q)
    if (FULL || i0 + q < nsl) v[q] = lookup8(tab, mr[q], v[q]);
#pragma unroll
  for (int q = 0; q < GROUP; ++q)
    if (FULL || i0 + q < nsl) c[(i0 + q) * BS + tid] = v[q];
  uint32_t f = 0;
  if (FUSE) {
#pragma unroll
    for (int q = 0; q < GROUP; ++q)
      if (FULL || i0 + q < nsl)
        f |= (((uint32_t)(v[q] >> fshift) != 0u) && !((done[q] >> lane) & 1)) ? (1u << (i0 + q)) : 0u;
  }
  return f;
}

template <bool FULL>
__device__ __forceinline__ uint32_t apply_cols(LDS uint64_t* const* cols, int nc, const uint32_t* mr,
                                               const uint64_t* done, int i0, int nsl, int fuse, int fshift,
                                               LDS Smem& S) {
  if (nc == 1)  // the usual case: table at a fixed address
    return fuse == 0 ? apply_group<FULL, true>(cols[0], S.tab[0], mr, done, i0, nsl, fshift)
                     : apply_group<FULL, false>(cols[0], S.tab[0], mr, done, i0, nsl, fshift);
  uint32_t f = 0;
  for (int j = 0; j < nc; ++j)
    f |= j == fuse ? apply_group<FULL, true>(cols[j], S.tab[j], mr, done, i0, nsl, fshift)
                   : apply_group<FULL, false>(cols[j], S.tab[j], mr, done, i0, nsl, fshift);
  return f;
}

// This thread's rows of `nc` LDS word columns updated by the pass whose
// tables are in S (pivmask pm).  Multipliers (the strip word of every row
// before the pass) come from the global snapshot `snap` (consumers) or from
// bits [shift, shift+32) of the LDS column `strip` (the owner; that column
// may be one of `cols`: a group's multipliers are all read before its rows
// are updated).  Rows in newpiv keep their value (multiplier 0 looks up table
// entry 0, which is zero).  With fuse >= 0, the rows not yet pivots whose
// bits [fshift, fshift+32) of column cols[fuse] are non-zero after the update
// are returned as candidate flags (bit i = row tid + i*BS).  `pre` (optional)
// holds the first PRE multipliers, already loaded.  LDS work only; no
// barrier.
__device__ uint32_t apply_rows(LDS uint64_t* const* cols, int nc, const uint32_t* snap, const LDS uint64_t* strip,
                               int shift, int m, const LDS uint64_t* pivflag, const LDS uint64_t* newpiv,
                               uint32_t pm, int fuse, int fshift, const uint32_t* pre, LDS Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nsl = (m + BS - 1) / BS;
  uint32_t flags = 0;
  for (int i0 = 0; i0 < nsl; i0 += GROUP) {
    uint32_t mr[GROUP];
    uint64_t done[GROUP];
#pragma unroll
    for (int q = 0; q < GROUP; ++q) {
      const int i = i0 + q, r = i * BS + tid;
      uint32_t x = 0;
      if (pre && i0 == 0) x = pre[q];
      else if (pre && i0 == GROUP) x = pre[GROUP + q];
      else if (r < m) x = snap ? ld_dev(&snap[r]) : (uint32_t)(strip[r] >> shift);
      // the wave's 64 rows of slice i share one word of each flag array
      const uint64_t npw = i < nsl ? newpiv[i * NWAVE + wv] : ~0ull;
      done[q] = i < nsl ? (pivflag[i * NWAVE + wv] | npw) : ~0ull;
      mr[q] = ((npw >> lane) & 1) ? 0u : (x & pm);
    }
    flags |= i0 + GROUP <= nsl ? apply_cols<true>(cols, nc, mr, done, i0, nsl, fuse, fshift, S)
                               : apply_cols<false>(cols, nc, mr, done, i0, nsl, fuse, fshift, S);
  }
  return flags;
}

// Candidate count of this wave from its threads' flags.
__device__ __forceinline__ int wave_count(uint32_t flags, int nsl) {
  int c = 0;
  for (int i = 0; i < nsl; ++i) c += __popcll(__ballot((flags >> i) & 1));
  return c;
}

// This wave's candidates (rows of its own threads), up to NCAND of them,
// into S.cand; returns how many were placed.  Wavefront-local: no barrier.
__device__ int wave_candidates(uint32_t flags, int nsl, LDS Smem& S) {
  const int tid = threadIdx.x;
  int base = 0;
  for (int i = 0; i < nsl && base < NCAND; ++i) {
    const bool f = (flags >> i) & 1;
    const uint64_t b = __ballot(f);
    const int idx = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0));
    if (f && idx < NCAND) S.cand[idx] = i * BS + tid;
    base += __popcll(b);
  }
  return base < NCAND ? base : NCAND;
}

// Bits [shift, shift+32) of this thread's rows of LDS column `col` to `snap`.
__device__ __forceinline__ void store_own_snapshot(const LDS uint64_t* col, int shift, int m, uint32_t* snap) {
  const int nsl = (m + BS - 1) / BS;
  for (int i = 0; i < nsl; ++i) {
    const int r = i * BS + (int)threadIdx.x;
    if (r < m) st_dev(&snap[r], (uint32_t)(col[r] >> shift));
  }
}

// The update by pass R (tables already in S) of this workgroup's columns
// when column cols[fuse] holds its next strip (bits [fshift, fshift+32)).
// Every wave updates its own rows and writes their next-strip snapshot words
// to snap_out.  Wave fw then takes the next strip's candidates among its own
// rows and, if it has at least EARLY_MIN of them, reduces them into N while
// the other waves are still updating (and loads the acknowledgements of ring
// slot ack_slot meanwhile).  fw rotates with the strip, so that pivots are
// drawn from every wave's rows alike.  Ends with a barrier.  Returns the
// thread's candidate flags; S.wcnt holds every wave's count, S.early /
// S.used whether wave fw reduced and how many candidates it used.
__device__ uint32_t update_and_reduce(LDS uint64_t* const* cols, int nc, const uint32_t* snap,
                                      const LDS uint64_t* strip, int shift, int m, LDS uint64_t* pivflag,
                                      LDS uint64_t* newpiv, uint32_t pm, int fuse, int fshift, const uint32_t* pre,
                                      uint32_t* snap_out, LDS Pass& N, int fw, const Args& a,
                                      uint32_t ack_slot, LDS Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nsl = (m + BS - 1) / BS;
  const uint32_t flags = apply_rows(cols, nc, snap, strip, shift, m, pivflag, newpiv, pm, fuse, fshift, pre, S);
  store_own_snapshot(cols[fuse], fshift, m, snap_out);
  const int cnt = wave_count(flags, nsl);
  if (lane == 0) S.wcnt[wv] = cnt;
  if (wv == fw) {
    const bool early = cnt >= EARLY_MIN;
    if (early) {
      const uint32_t ackv = ld_dev(&a.ctl->ack[ack_slot]);
      const int used = wave_candidates(flags, nsl, S);
      factor_candidates(cols[fuse], fshift, used, N, S);
      const uint32_t av = settle(ackv);
      if (lane == 0) {
        S.used = used;
        if (av > S.ackc[ack_slot]) S.ackc[ack_slot] = av;
      }
    }
    if (lane == 0) S.early = early ? 1 : 0;
  }
  __syncthreads();
  return flags;
}

// One row r of `nc` columns updated by the pass whose tables are in S
// (multiplier mv before masking with pm); returns whether the row is a
// candidate of the next strip (bits [fshift, fshift+32) of column cols[fuse]
// non-zero, not a pivot).  r lies in a 64-row block that the whole wave
// handles, so the flag words are uniform loads.
__device__ __forceinline__ bool update_row(LDS uint64_t* const* cols, int nc, int r, uint32_t mv, uint32_t pm,
                                           const LDS uint64_t* pivflag, const LDS uint64_t* newpiv, int fuse,
                                           int fshift, LDS Smem& S) {
  const int lane = threadIdx.x & 63;
  const uint64_t npw = newpiv[r >> 6];
  const uint64_t done = pivflag[r >> 6] | npw;
  const uint32_t mr = ((npw >> lane) & 1) ? 0u : (mv & pm);
  bool f = false;
  if (nc == 1) {
    const uint64_t v = lookup8(S.tab[0], mr, cols[0][r]);
    cols[0][r] = v;
    f = ((uint32_t)(v >> fshift) != 0u) && !((done >> lane) & 1);
  } else {
    for (int j = 0; j < nc; ++j) {
      const uint64_t v = lookup8(S.tab[j], mr, cols[j][r]);
      cols[j][r] = v;
      if (j == fuse) f = ((uint32_t)(v >> fshift) != 0u) && !((done >> lane) & 1);
    }
  }
  return f;
}

// The early slice, the reducing wave and the extra slice a wave updates for
// it, for the strip that follows strip t (every workgroup derives the same).
__device__ __forceinline__ int early_slice(int t, int nsl) { return (t + 1) % nsl; }
__device__ __forceinline__ int early_wave(int t) { return (t + 1) % NWAVE; }
__device__ __forceinline__ int extra_slice(int wv, int fw, int e) {
  const int kx = (wv - fw + NWAVE - 1) % NWAVE;
  return kx < e ? kx : kx + 1;
}

// The fused update with the next strip's reduction split off, for at most
// PRE row slices.  First every wave updates its row of slice e (the early
// slice, rotating with the strip) and records which of them are candidates;
// after a barrier wave fw takes up to NCAND of the slice's candidates and
// reduces them into N, while the other seven waves update their remaining
// slices and, one slice each, the rows of wave fw.  Every updated row's
// next-strip word goes to snap_out.  Multipliers: pre[i] (consumers: the
// thread's row of slice i) and prex (its extra row of wave fw), or the strip
// bits of LDS column `strip` (the owner).  Ends with a barrier; S.wcnt holds
// the candidate counts (each row counted once), S.early / S.used whether wave
// fw reduced and how many candidates it used.
__device__ void split_update_and_reduce(LDS uint64_t* const* cols, int nc, const LDS uint64_t* strip, int shift,
                                        int m, LDS uint64_t* pivflag, LDS uint64_t* newpiv, uint32_t pm, int fuse,
                                        int fshift, const uint32_t* pre, uint32_t prex, uint32_t* snap_out,
                                        LDS Pass& N, int fw, int e, const Args& a, uint32_t ack_slot, LDS Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nsl = (m + BS - 1) / BS;
  const LDS uint64_t* fc = cols[fuse];
  // phase A: slice e
  {
    const int r = e * BS + tid;
    uint32_t mv = 0;
#pragma unroll
    for (int i = 0; i < PRE; ++i)
      if (i == e) mv = pre ? pre[i] : (r < m ? (uint32_t)(strip[r] >> shift) : 0u);
    const bool f = r < m && update_row(cols, nc, r, mv, pm, pivflag, newpiv, fuse, fshift, S);
    const uint64_t b = __ballot(f);
    if (lane == 0) S.emask[wv] = b;
    if (r < m) st_dev(&snap_out[r], (uint32_t)(fc[r] >> fshift));
  }
  __syncthreads();
  int cnt = 0;
  if (wv == fw) {
    int base = 0;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v) {
      const uint64_t msk = S.emask[v];
      const int idx = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(msk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)msk, 0));
      if (((msk >> lane) & 1) && idx < NCAND) S.cand[idx] = e * BS + v * 64 + lane;
      base += __popcll(msk);
    }
    cnt = base;
    const bool early = base >= EARLY_MIN;
    if (early) {
      const uint32_t ackv = ld_dev(&a.ctl->ack[ack_slot]);
      const int used = base < NCAND ? base : NCAND;
      factor_candidates(fc, fshift, used, N, S);
      const uint32_t av = settle(ackv);
      if (lane == 0) {
        S.used = used;
        if (av > S.ackc[ack_slot]) S.ackc[ack_slot] = av;
      }
    }
    if (lane == 0) S.early = early ? 1 : 0;
  } else {
    // own rows of the other slices
#pragma unroll
    for (int i = 0; i < PRE; ++i) {
      const int r = i * BS + tid;
      if (i != e && i < nsl && r < m) {
        const uint32_t mv = pre ? pre[i] : (uint32_t)(strip[r] >> shift);
        cnt += __popcll(__ballot(update_row(cols, nc, r, mv, pm, pivflag, newpiv, fuse, fshift, S)));
        st_dev(&snap_out[r], (uint32_t)(fc[r] >> fshift));
      }
    }
    // one slice of wave fw's rows: the k-th slice other than e, k = this
    // wave's rank among the waves other than fw
    const int xs = extra_slice(wv, fw, e);
    const int r = xs * BS + fw * 64 + lane;
    if (xs < nsl && r < m) {
      const uint32_t mv = pre ? prex : (uint32_t)(strip[r] >> shift);
      cnt += __popcll(__ballot(update_row(cols, nc, r, mv, pm, pivflag, newpiv, fuse, fshift, S)));
      st_dev(&snap_out[r], (uint32_t)(fc[r] >> fshift));
    }
  }
  if (lane == 0) S.wcnt[wv] = cnt;
  __syncthreads();
}

// Candidate flags (bit i = row tid + i*BS) of the strip at bits [shift,
// shift+32) of LDS column `col`: non-zero and not a pivot.
__device__ __forceinline__ uint32_t strip_flags(const LDS uint64_t* col, int shift, int m,
                                                const LDS uint64_t* pivflag) {
  const int nsl = (m + BS - 1) / BS;
  uint32_t flags = 0;
  for (int i = 0; i < nsl; ++i) {
    const int r = i * BS + (int)threadIdx.x;
    if (r < m && (uint32_t)(col[r] >> shift) != 0 && !bit_of(pivflag, r)) flags |= 1u << i;
  }
  return flags;
}

__device__ __forceinline__ int candidates_total(const LDS Smem& S) {
  int total = 0;
#pragma unroll
  for (int v = 0; v < NWAVE; ++v) total += S.wcnt[v];
  return total;
}

// Acknowledgements are monotonic: a count read earlier (S.ackc, prefetched
// off the critical path) that already suffices saves the device-scope load.
__device__ bool wait_slot(uint32_t idx, int G, const Args& a, LDS Smem& S) {
  const uint32_t need = (idx / RING) * (uint32_t)(G - 1);
  if ((uint32_t)__builtin_amdgcn_readfirstlane((int)S.ackc[idx % RING]) >= need) return true;
  __syncthreads();  // every wave has read S.ackc before thread 0 rewrites it
  if (threadIdx.x == 0) {
    const bool ok = spin_until(&a.ctl->ack[idx % RING], need, a);
    S.flag = ok ? 1 : 0;
    if (ok) S.ackc[idx % RING] = need;
  }
  __syncthreads();
  return S.flag != 0;
}

// The column residue workgroup g owns: it holds word columns res, res + G,
// ...  Workgroups are dispatched to the eight XCDs in turn (workgroup g on
// XCD g mod 8), so consecutive residues go to workgroups of one XCD, G / 8 at
// a time: the owner of the next word column, which takes over the strip
// chain, then mostly sits on the same XCD.
__device__ __forceinline__ int col_residue(int g, int G) {
  if (G % 8 != 0) return g;
  const int per = G / 8;
  return (g % 8) * per + g / 8;
}

__global__ __launch_bounds__(BS) void rref_kernel(Args a) {
  extern __shared__ __align__(16) uint64_t smem[];
  const int tid = threadIdx.x;
  const int g = blockIdx.x, G = gridDim.x, res = col_residue(g, G);
  const int m = a.m;
  const int nsl = (m + BS - 1) / BS;
  const int nown = (a.nw - res + G - 1) / G;  // word columns owned: res, res+G, ...
  const int ms = nsl * BS;                  // column stride: rows padded with zeros
  const int pw = ms / 64;
  // the pass tables first, at a fixed LDS address (immediate offsets)
  LDS uint64_t* base = (LDS uint64_t*)smem;
  LDS Smem& S = *reinterpret_cast<LDS Smem*>(base);
  LDS uint64_t* cols = base + smem_head_words();                 // [cw][ms]
  LDS uint64_t* pivflag = cols + (size_t)a.cw * ms;              // [pw]
  LDS uint64_t* newpiv = pivflag + pw;                           // [pw]

  for (int j = 0; j < nown; ++j) {
    const int c = res + j * G;
    if (c < a.nw_a) {
      const int tail = a.n_cols - 64 * c;
      const uint64_t cm = tail >= 64 ? ~0ull : ((1ull << tail) - 1);
      for (int r = tid; r < ms; r += BS) cols[(size_t)j * ms + r] = r < m ? a.A[(size_t)r * a.ld + c] & cm : 0;
    } else {
      // the transform's columns start as the identity; every pass updates
      // them like A's columns, no strip of theirs is ever reduced
      const int tc = c - a.nw_a;
      for (int r = tid; r < ms; r += BS)
        cols[(size_t)j * ms + r] = (r < m && (r >> 6) == tc) ? (1ull << (r & 63)) : 0ull;
    }
  }
  for (int i = tid; i < pw; i += BS) {
    pivflag[i] = 0;
    newpiv[i] = 0;
  }
  if (tid < RING) S.ackc[tid] = 0;
  __syncthreads();

  uint32_t seq = 0;       // next record index
  int rank = 0;
  bool ok = true;
  int cur = 0;            // S.ps[cur]: the pass being published or applied
  bool prepared = false;  // candidates of my next strip in S.cand (all rows), S.total set
  bool factored = false;  // my next strip already reduced into S.ps[cur] during an update
  int early_total = 0, early_used = 0;
  // snapshot to be written by waves 1..7 during the next reduction
  const LDS uint64_t* pend_col = nullptr;
  int pend_shift = 0;
  uint32_t* pend_snap = nullptr;
  // (thread 64) ring slot whose acknowledgement waits until my next record
  // is out, or -1: in flight at my publication it would hold up its wait
  int pend_ack = -1;
  for (int t = 0; t < a.nstrips && rank < m && ok; ++t) {
    const int wc = t >> 1, shift = SW * (t & 1);
    if (wc % G == res) {
      // ---------------- produce strip t ----------------
      const int js = wc / G;
      LDS uint64_t* col = cols + (size_t)js * ms;
      const int rank0 = rank;
      bool multi = false;
      if (tid == 0) prof_mark(a, t, 0);
      for (;;) {
        PassRec* rec = a.recs + seq % RING;
        uint32_t* snap = a.snaps + (size_t)(seq % RING) * m;
        int total, used;
        // an early reduction that found no pivot while other candidates
        // exist is redone as a full pass (the snapshot is already written)
        if (factored && S.ps[cur].k == 0 && early_total > 0) factored = false;
        if (factored) {
          factored = false;
          total = early_total;
          used = early_used;
          if (tid == 0) prof_mark(a, t, 1);
        } else {
          if (!prepared) {
            if (!wait_slot(seq, G, a, S)) { ok = false; break; }
            uint32_t flags = 0;
            for (int i = 0; i < nsl; ++i) {
              const int r = i * BS + tid;
              if (r < m && (uint32_t)(col[r] >> shift) != 0 && !bit_of(pivflag, r)) flags |= 1u << i;
            }
            compact_candidates(flags, nsl, S);
            pend_col = col;
            pend_shift = shift;
            pend_snap = snap;
          }
          prepared = false;
          if (tid == 0) prof_mark(a, t, 1);
          total = S.total;
          used = total < NCAND ? total : NCAND;
          if (tid < 64) {
            // the next slot's acknowledgements, loaded while the reduction runs
            const uint32_t nslot = (seq + 1) % RING;
            const uint32_t ackv = ld_dev(&a.ctl->ack[nslot]);
            factor_candidates(col, shift, used, S.ps[cur], S);
            const uint32_t av = settle(ackv);
            if (tid == 0 && av > S.ackc[nslot]) S.ackc[nslot] = av;
          } else if (pend_snap) {
            store_snapshot(pend_col, pend_shift, m, pend_snap);
          }
          pend_snap = nullptr;
          __syncthreads();
        }
        if (tid == 0) prof_mark(a, t, 6);
        LDS Pass& Pc = S.ps[cur];
        const int k = Pc.k;
        const int last = (total == 0 || k == SW || total <= used) ? 1 : 0;
        // this pass's snapshot and every earlier store of the workgroup have
        // landed; then the record words publish the pass
        wait_stores();
        __syncthreads();
        if (tid < SW) st_dev64(&rec->e[tid], rec_word(Pc, tid, k, last, seq));
        if (tid == 64 && pend_ack >= 0) {
          __hip_atomic_fetch_add(&a.ctl->ack[pend_ack], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          pend_ack = -1;
        }
        if (!(last && multi) && tid < k) {
          // pivot list entries: read only after every workgroup is done
          st_dev32(&a.piv_row[rank + tid], Pc.rows[tid]);
          st_dev32(&a.piv_col[rank + tid], SW * t + Pc.bits[tid]);
        }
        if (last && multi && tid == 64) {
          // multi-pass strip (rare): sort its pivot list by column.  A strip
          // holds at most 32 pivots; earlier passes' entries (landed, waited
          // for above) are read back, this pass's come from the reduction.
          int cnt = 0;
          for (int i = rank0; i < rank; ++i) {
            S.prow[cnt] = ld_dev32(&a.piv_row[i]);
            S.pcol[cnt] = ld_dev32(&a.piv_col[i]);
            ++cnt;
          }
          for (int j = 0; j < k; ++j) {
            S.prow[cnt] = Pc.rows[j];
            S.pcol[cnt] = SW * t + Pc.bits[j];
            ++cnt;
          }
          for (int i = 1; i < cnt; ++i) {
            const int kc = S.pcol[i], kr = S.prow[i];
            int j = i - 1;
            while (j >= 0 && S.pcol[j] > kc) {
              S.pcol[j + 1] = S.pcol[j];
              S.prow[j + 1] = S.prow[j];
              --j;
            }
            S.pcol[j + 1] = kc;
            S.prow[j + 1] = kr;
          }
          S.cnt = cnt;
        }
        if (last && multi) {
          __syncthreads();
          if (tid < S.cnt) {
            st_dev32(&a.piv_row[rank0 + tid], S.prow[tid]);
            st_dev32(&a.piv_col[rank0 + tid], S.pcol[tid]);
          }
        }
        if (tid == 0) prof_mark(a, t, 2);
        ++seq;
        if (k > 0) {
          // the high half of this word column is my next strip: reduce it
          // during this update
          const bool fused = last && (t & 1) == 0 && t + 1 < a.nstrips;
          if (fused && !wait_slot(seq, G, a, S)) { ok = false; break; }
          LDS uint64_t* list[MAX_CW];
          int nc = 0;
          for (int j = js; j < nown; ++j) list[nc++] = cols + (size_t)j * ms;
          make_tables(list, nc, newpiv, pivflag, Pc, S);
          if (fused) {
            uint32_t* snap_out = a.snaps + (size_t)(seq % RING) * m;
            uint32_t flags = 0;
            if (nsl <= PRE)
              split_update_and_reduce(list, nc, col, shift, m, pivflag, newpiv, Pc.pivmask, 0, SW, nullptr, 0u,
                                      snap_out, S.ps[cur ^ 1], early_wave(t), early_slice(t, nsl), a,
                                      (seq + 1) % RING, S);
            else
              flags = update_and_reduce(list, nc, nullptr, col, shift, m, pivflag, newpiv, Pc.pivmask, 0, SW,
                                        nullptr, snap_out, S.ps[cur ^ 1], early_wave(t), a, (seq + 1) % RING, S);
            clear_newpiv(newpiv, Pc);
            early_total = candidates_total(S);
            if (S.early) {
              factored = true;
              early_used = S.used;
              cur ^= 1;
            } else {
              if (nsl <= PRE) flags = strip_flags(col, SW, m, pivflag);
              compact_candidates(flags, nsl, S);
              prepared = true;
            }
          } else {
            apply_rows(list, nc, nullptr, col, shift, m, pivflag, newpiv, Pc.pivmask, -1, SW, nullptr, S);
            __syncthreads();
            clear_newpiv(newpiv, Pc);
          }
          rank += k;
        }
        if (tid == 0) prof_mark(a, t, 3);
        if (last) break;
        multi = true;
      }
    } else {
      // ---------------- consume strip t ----------------
      // my next strip follows directly when t is the high half of the word
      // column just before one of mine
      const bool own_next = (t + 1 < a.nstrips) && (((t + 1) >> 1) % G) == res && ((t + 1) & 1) == 0;
      for (;;) {
        const int slot = seq % RING;
        const PassRec* rec = a.recs + slot;
        const uint32_t* snap = a.snaps + (size_t)slot * m;
        LDS Pass& Pc = S.ps[cur];
        if (tid < 64) {
          const bool got = read_record(rec, seq, a, Pc);
          if (tid == 0) {
            S.flag = got ? 1 : 0;
            if (got && own_next) {
              const uint32_t nslot = (seq + 1) % RING, v = ld_dev(&a.ctl->ack[nslot]);
              if (v > S.ackc[nslot]) S.ackc[nslot] = v;
            }
          }
        }
        __syncthreads();
        if (!S.flag) { ok = false; break; }
        // the first multipliers, in flight during the tables
        uint32_t pre[PRE];
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
          const int r = q * BS + tid;
          pre[q] = r < m ? ld_dev(&snap[r]) : 0;
        }
        // the row of the reducing wave this thread updates in a split update
        uint32_t prex = 0;
        if (own_next && nsl <= PRE) {
          const int fw = early_wave(t), xs = extra_slice(tid >> 6, fw, early_slice(t, nsl));
          const int r = xs * BS + fw * 64 + (tid & 63);
          if ((tid >> 6) != fw && xs < nsl && r < m) prex = ld_dev(&snap[r]);
        }
        const int k = Pc.k, last = Pc.last;
        const bool fused = own_next && last && k > 0;
        if (tid == 0 && own_next && last) prof_mark(a, t, 4);
        if (fused && !wait_slot(seq + 1, G, a, S)) { ok = false; break; }
        if (k > 0) {
          rank += k;  // every workgroup tracks the rank (the loops end together)
          // owned word columns after wc
          LDS uint64_t* list[MAX_CW];
          int nc = 0, fuse = -1;
          for (int j = (wc - res) >= 0 ? (wc - res) / G + 1 : 0; j < nown; ++j) {
            if (fused && res + j * G == ((t + 1) >> 1)) fuse = nc;
            list[nc++] = cols + (size_t)j * ms;
          }
          if (nc > 0) {
            make_tables(list, nc, newpiv, pivflag, Pc, S);
            if (fused) {
              // wait for the multipliers here, before any snapshot store: a
              // wait for them inside the loops below would also wait for the
              // stores issued there (vmcnt counts both in issue order).  The
              // empty asm statements mark them as defined after this wait, so
              // the compiler places no further wait for their loads.
              wait_stores();
#pragma unroll
              for (int q = 0; q < PRE; ++q) asm volatile("" : "+v"(pre[q]));
              asm volatile("" : "+v"(prex));
              uint32_t* snap_out = a.snaps + (size_t)((seq + 1) % RING) * m;
              uint32_t flags = 0;
              if (nsl <= PRE)
                split_update_and_reduce(list, nc, nullptr, 0, m, pivflag, newpiv, Pc.pivmask, fuse, 0, pre, prex,
                                        snap_out, S.ps[cur ^ 1], early_wave(t), early_slice(t, nsl), a,
                                        (seq + 2) % RING, S);
              else
                flags = update_and_reduce(list, nc, snap, nullptr, 0, m, pivflag, newpiv, Pc.pivmask, fuse, 0, pre,
                                          snap_out, S.ps[cur ^ 1], early_wave(t), a, (seq + 2) % RING, S);
              clear_newpiv(newpiv, Pc);
              early_total = candidates_total(S);
              if (S.early) {
                factored = true;
                early_used = S.used;
                cur ^= 1;
              } else {
                if (nsl <= PRE) flags = strip_flags(list[fuse], 0, m, pivflag);
                compact_candidates(flags, nsl, S);
                prepared = true;
              }
            } else {
              apply_rows(list, nc, snap, nullptr, 0, m, pivflag, newpiv, Pc.pivmask, -1, 0, pre, S);
              __syncthreads();
              clear_newpiv(newpiv, Pc);
            }
          }
        }
        // the prefetched multipliers are consumed on every path (they have
        // landed long since): a load left unconsumed on some path stays
        // pending for the compiler, and every later write to its register
        // would wait for all memory operations in flight
#pragma unroll
        for (int q = 0; q < PRE; ++q) asm volatile("" ::"v"(pre[q]));
        asm volatile("" ::"v"(prex));
        __syncthreads();
        // done with the slot; when my own strip comes next, the
        // acknowledgement follows my record (the slot is rewritten only
        // RING - 1 records after that one)
        if (tid == 64) {
          if (own_next && last) pend_ack = slot;
          else __hip_atomic_fetch_add(&a.ctl->ack[slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid == 0 && own_next && last) prof_mark(a, t, 5);
        ++seq;
        if (last) break;
      }
    }
  }
  if (!ok) return;
  if (tid == 64 && pend_ack >= 0)
    __hip_atomic_fetch_add(&a.ctl->ack[pend_ack], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // every workgroup's pivot list entries have landed before any reads them
  wait_stores();
  __syncthreads();
  if (tid == 0) {
    __hip_atomic_fetch_add(&a.ctl->fin, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    S.flag = spin_until(&a.ctl->fin, (uint32_t)G, a) ? 1 : 0;
  }
  __syncthreads();
  if (!S.flag) return;
  // ---------------- write the result ----------------
  // T: rows in pivot order, then the rows that are no pivot, ascending (their
  // transform rows span the left null space); piv_base[w] = non-pivot rows in
  // flag words before w
  const bool has_t = a.T && nown > 0 && res + (nown - 1) * G >= a.nw_a;
  if (has_t) {
    if (tid == 0) {
      int acc = 0;
      for (int w = 0; w < pw; ++w) {
        newpiv[w] = (uint64_t)acc;  // free now: reused for the prefix counts
        const int lo = 64 * w;
        const uint64_t valid = lo + 64 <= m ? ~0ull : (lo >= m ? 0ull : ((1ull << (m - lo)) - 1));
        acc += __popcll(~pivflag[w] & valid);
      }
    }
    __syncthreads();
  }
  for (int j = 0; j < nown; ++j) {
    const int c = res + j * G;
    const LDS uint64_t* col = cols + (size_t)j * ms;
    if (c < a.nw_a) {
      for (int i = tid; i < m; i += BS) {
        uint64_t v = 0;
        if (i < rank) v = col[ld_dev32(&a.piv_row[i])];
        a.R[(size_t)i * a.ld + c] = v;
      }
    } else {
      const int tc = c - a.nw_a;
      for (int i = tid; i < rank; i += BS) a.T[(size_t)i * a.ldt + tc] = col[ld_dev32(&a.piv_row[i])];
      for (int r = tid; r < m; r += BS) {
        const uint64_t pf = pivflag[r >> 6];
        if ((pf >> (r & 63)) & 1) continue;
        const int idx = rank + (int)newpiv[r >> 6] + __popcll(~pf & ((1ull << (r & 63)) - 1));
        a.T[(size_t)idx * a.ldt + tc] = col[r];
      }
    }
  }
  if (g == 0) {
    for (int i = tid; i < m; i += BS) a.piv_dev[i] = i < rank ? ld_dev32(&a.piv_col[i]) : -1;
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
  const size_t ms = (size_t)(m + BS - 1) / BS * BS;
  return (size_t)smem_head_words() * 8 + (size_t)cw * ms * 8 + 2 * (ms / 64) * 8;
}

// Host-side argument checks shared by both elimination entry points.
zx_status check_rref_args(const uint64_t* A, uint64_t* R, int32_t m, int32_t n_cols, int64_t ld_words,
                          int32_t* rank_dev, int32_t* pivot_cols_dev, uint64_t* T, int64_t ld_t) {
  ZX_CHECK_ARG(A && R && rank_dev && pivot_cols_dev, "null argument");
  ZX_CHECK_ARG(m > 0 && n_cols > 0, "empty matrix: m=%d n_cols=%d", m, n_cols);
  const int nw_a = (n_cols + 63) / 64;
  ZX_CHECK_ARG(ld_words >= nw_a, "ld_words %lld < %d", (long long)ld_words, nw_a);
  const int mw = (m + 63) / 64;
  if (T) {
    ZX_CHECK_ARG(ld_t >= mw, "ld_t %lld < %d", (long long)ld_t, mw);
    const char* t0 = (const char*)T;
    const char* t1 = t0 + (size_t)m * ld_t * 8;
    const char* a0 = (const char*)A;
    const char* a1 = a0 + (size_t)m * ld_words * 8;
    const char* r0 = (const char*)R;
    const char* r1 = r0 + (size_t)m * ld_words * 8;
    ZX_CHECK_ARG((t1 <= a0 || a1 <= t0) && (t1 <= r0 || r1 <= t0), "T overlaps A or R");
  }
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
  return ZX_OK;
}

// Launch rref_init and rref_kernel with the workspace sections of an m-row
// elimination at base (prof: record per-strip timestamps in its profile
// section, which must then exist).
zx_status launch_rref(const uint64_t* A, uint64_t* R, int32_t m, int32_t n_cols, int64_t ld_words,
                      int32_t* rank_dev, int32_t* pivot_cols_dev, uint64_t* T, int64_t ld_t, uint8_t* base,
                      bool prof, hipStream_t s) {
  const ZxDevice* dev = zx_device();
  if (!dev) {
    zx_set_error("no HIP device");
    return ZX_EDEVICE;
  }
  const int nw_a = (n_cols + 63) / 64;
  const int mw = (m + 63) / 64;
  const int nw = nw_a + (T ? mw : 0);
  // word columns per workgroup: the smallest count whose grid is co-resident
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
  const WsLayout W = ws_layout(m);
  Args a;
  a.A = A;
  a.R = R;
  a.T = T;
  a.ldt = T ? ld_t : 0;
  a.m = m;
  a.n_cols = n_cols;
  a.nw = nw;
  a.nw_a = nw_a;
  a.cw = cw;
  a.nstrips = (n_cols + SW - 1) / SW;
  a.ld = ld_words;
  a.rank_dev = rank_dev;
  a.piv_dev = pivot_cols_dev;
  a.status = (int32_t*)base;
  a.ctl = (Ctl*)(base + W.ctl);
  a.recs = (PassRec*)(base + W.recs);
  a.snaps = (uint32_t*)(base + W.snaps);
  a.piv_row = (int32_t*)(base + W.piv_row);
  a.piv_col = (int32_t*)(base + W.piv_col);
  a.spin_ticks = 100000000ull * 5;  // 5 s at the 100 MHz real-time counter
  a.prof = prof ? (uint64_t*)(base + W.prof) : nullptr;
  hipLaunchKernelGGL(rref_init, dim3(1), dim3(256), 0, s, a.ctl, a.recs, a.status, a.prof, a.rank_dev);
  ZX_HIP(hipGetLastError());
  void* args[] = {&a};
  ZX_HIP(hipLaunchCooperativeKernel((const void*)rref_kernel, dim3(G), dim3(BS), args, (unsigned)lds, s));
  return ZX_OK;
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

extern "C" zx_status zx_gf2_profile_read(const void* ws, int32_t m, int64_t* ticks, int32_t max_strips,
                                         hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(ws && ticks && m > 0 && max_strips >= 0, "bad argument");
  const int n = max_strips < MAX_STRIPS ? max_strips : MAX_STRIPS;
  ZX_HIP(hipStreamSynchronize(s));
  const WsLayout W = ws_layout(m);
  ZX_HIP(hipMemcpy(ticks, (const uint8_t*)ws + W.prof, (size_t)n * PROF_SLOTS * 8, hipMemcpyDeviceToHost));
  return ZX_OK;
}

extern "C" zx_status zx_gf2_eliminate(const uint64_t* A, uint64_t* R, int32_t m, int32_t n_cols,
                                      int64_t ld_words, int32_t* rank_dev, int32_t* pivot_cols_dev,
                                      uint64_t* T, int64_t ld_t, void* ws, size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(ws, "null workspace");
  zx_status rc = check_rref_args(A, R, m, n_cols, ld_words, rank_dev, pivot_cols_dev, T, ld_t);
  if (rc != ZX_OK) return rc;
  ZX_CHECK_ARG(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  const WsLayout W = ws_layout(m);
  if (ws_bytes < W.bytes) {
    zx_set_error("workspace %zu < %zu bytes", ws_bytes, W.bytes);
    return ZX_ECAPACITY;
  }
  static const bool prof_on = getenv("ZX_RREF_PROFILE") && getenv("ZX_RREF_PROFILE")[0] == '1';
  return launch_rref(A, R, m, n_cols, ld_words, rank_dev, pivot_cols_dev, T, ld_t, (uint8_t*)ws, prof_on, s);
}

// ---------------------------------------------------------------------------
// Allocation-free elimination.  Its workspace is this static device array,
// sized for the largest m the kernel takes, without profile slots.  Each GPU
// holds its own copy at its own address.  In host code the array's name is
// only a stand-in for the device symbol: the device address comes from
// hipGetSymbolAddress, once per device, and only that address is ever passed
// to a kernel.
static __device__ __align__(256) uint8_t scratch[ws_core_bytes(MAX_M)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of scratch on the current device (nullptr and the error
// message set on failure).
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    zx_set_error("no current HIP device");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      zx_set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" zx_status zx_gf2_eliminate_noalloc(const uint64_t* A, uint64_t* R, int32_t m, int32_t n_cols,
                                              int64_t ld_words, int32_t* rank_dev, int32_t* pivot_cols_dev,
                                              uint64_t* T, int64_t ld_t, hipStream_t s) {
  zx_clear_error();
  zx_status rc = check_rref_args(A, R, m, n_cols, ld_words, rank_dev, pivot_cols_dev, T, ld_t);
  if (rc != ZX_OK) return rc;
  if (ws_core_bytes(m) > sizeof(scratch)) {
    zx_set_error("m=%d needs %zu scratch bytes > %zu", m, ws_core_bytes(m), sizeof(scratch));
    return ZX_ECAPACITY;
  }
  uint8_t* base = (uint8_t*)scratch_address();
  if (!base) return ZX_EDEVICE;
  return launch_rref(A, R, m, n_cols, ld_words, rank_dev, pivot_cols_dev, T, ld_t, base, false, s);
}
