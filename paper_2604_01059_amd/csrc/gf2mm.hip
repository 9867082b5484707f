// Dense products over GF(2) on the matrix cores, and the phase-pair product.
//
// 1. C[i][j] = (sum_k A[i][k] B[j][k]) mod 2 for bit-packed rows A_i, B_j.
//    This is the batched parity contraction a_k = XOR_i u_ki f_i of the
//    paper's parameterized evaluation (appendix "Parameterized evaluation of
//    Clifford ZX diagrams", equation parities), with A = U and B = the
//    parameter settings, and it is the symplectic commutation table of Pauli
//    strings with A_i = [x_i | z_i], B_j = [z_j | x_j] (appendix "Pauli
//    channels" for the encoding).  The paper contracts in floating point on
//    BLAS; here the bits enter v_mfma_scale_f32_32x32x64_f8f6f4 as FP4
//    (E2M1) values: a set bit is the code 0b0001 (0.5), the block scale 2^1
//    makes it 1.0, so every product is 0 or 1 and the fp32 sums (at most the
//    row length, far below 2^24) are exact counts; bit 0 of the count is the
//    parity.  Unpacking a 32-bit word of bits costs seven VALU operations:
//    nibble r of dword t of the operand holds bit 4r + t of the word, i.e.
//    operand dword t = (word >> t) & 0x11111111.  The order in which bits
//    reach the k positions of the instruction does not matter, since A and
//    B fragments are unpacked the same way and the sum runs over all k.
//
//    Two tilings.  The symmetric table (and K beyond 2048 bits): one
//    persistent workgroup of 512 threads per CU walking 256 x 256 output
//    tiles, each wavefront a 64 x 128 part (2 x 4 blocks of 32 x 32, 128
//    fp32 accumulators per lane, two wavefronts per SIMD).  The rows' bits go through LDS in chunks of
//    256 bits (4 words, double buffered): 16 KiB per chunk for the 512 rows
//    of the tile; the next chunk's rows are loaded while a chunk is
//    multiplied, across tile boundaries too.  For each 64-bit step of a
//    chunk, lane half h of a fragment takes dword 4h + s of its row's chunk.
//    General products with K up to 2048 bits: 128 x 128 tiles whose rows are
//    staged whole (below), two workgroups per CU.  Parities leave through
//    wave ballots (row words) and, for the symmetric table, through per-lane
//    packing (the mirrored tile's row words).  Tiles are dealt to the eight
//    XCDs in contiguous runs of the tile order, so one XCD's tiles share rows
//    in its L2.  Row loads are branch-free (the compiler otherwise waits for
//    each load before issuing the next).  65536-string table: 5.25 ms with
//    one wavefront per SIMD, per-tile workgroups and branching loads; 3.96
//    ms persistent with branch-free loads; 2.79 ms with two wavefronts per
//    SIMD.
//
// 2. Per setting l: omega^phase8 sqrt(2)^pow * prod_k h(alpha_k, beta_k;
//    a_kl, b_kl), h of equation phase_pair, phases multiples of pi/4.  One
//    lane per setting, fp32 complex products, renormalised to a power of two
//    every 8 factors.
#include "zx_internal.h"

namespace {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

#define LDS __attribute__((address_space(3)))

// Waves per workgroup of the 256 x 256 kernel: 8 (each a 64 x 128 part, 128
// accumulators, two waves per SIMD, so one wave's operand unpacking and
// loads overlap the other's products): 2.79 ms for the 65536-string table
// against 3.76 ms with 4 (each a 128 x 128 quarter, one wave per SIMD).
constexpr int MM_NW = 8;
constexpr int MM_T = 256;     // output tile edge
constexpr int MM_CW = 4;      // words per chunk
constexpr int SCALE_ONE = 128;  // E8M0 2^1: FP4 code 0b0001 (0.5) scaled to 1.0

struct MmArgs {
  const uint64_t* a0;  // row i of A = a0 row i (kw0 words) then a1 row i (kw1 words)
  const uint64_t* a1;
  const uint64_t* b0;  // row j of B = b0 row j (kw0 words) then b1 row j (kw1 words)
  const uint64_t* b1;
  int64_t lda, ldb;    // words per row of a0/a1 and of b0/b1
  int64_t m, n;        // rows of A, rows of B
  int32_t kw0, kw1;
  uint64_t mask0, mask1;  // valid bits of the last word of each part
  uint64_t* C;
  int64_t ldc;
  int64_t cw;          // words of C written per row: ceil(n / 64)
  int32_t tm, tn;      // tiles along m and n
  int32_t sym;         // symmetric table: tiles ti <= tj, mirror written too
  int64_t n_tiles;
  int64_t per_xcd;     // tiles per XCD run
};

// Word w of row r of a two-part operand (p0: kw0 words, then p1: kw1 words),
// with the last word of each part masked to its valid bits; 0 beyond the
// rows or the words.  Branch-free: w is the same in every lane, so the part,
// the offset and the mask are scalar; the row is clamped to a valid address
// and the lane's result selected.  (Branches here made the compiler wait
// for each load before issuing the next.)
__device__ __forceinline__ uint64_t row_word(const uint64_t* p0, const uint64_t* p1, int64_t ld, int64_t r,
                                             int64_t nrows, int w, int kw0, int kw1, uint64_t m0,
                                             uint64_t m1) {
  const bool first = w < kw0;
  const bool in_k = w < kw0 + kw1;
  const uint64_t* p = (first || !in_k) ? p0 : p1;
  const int ww = first ? w : (in_k ? w - kw0 : 0);
  uint64_t m = !in_k ? 0 : first ? (w == kw0 - 1 ? m0 : ~0ull) : (ww == kw1 - 1 ? m1 : ~0ull);
  const int64_t rr = r < nrows ? r : nrows - 1;
  const uint64_t v = p[rr * ld + ww];
  return r < nrows ? v & m : 0;
}

__device__ __forceinline__ v8i unpack_fp4(uint32_t d) {
  v8i o;
  o[0] = (int)(d & 0x11111111u);
  o[1] = (int)((d >> 1) & 0x11111111u);
  o[2] = (int)((d >> 2) & 0x11111111u);
  o[3] = (int)((d >> 3) & 0x11111111u);
  o[4] = 0;
  o[5] = 0;
  o[6] = 0;
  o[7] = 0;
  return o;
}

// Accumulators start at 2^23: a count below 2^23 added to it stays an exact
// fp32 integer in [2^23, 2^24), where one unit is the last mantissa bit, so
// bit 0 of the float's bits is the count's parity.
constexpr float ACC_BASE = 8388608.0f;

// s_waitcnt operand that waits for LDS (lgkmcnt 0) and nothing else
// (vmcnt and expcnt at their maximum).
constexpr int WAIT_LDS = 0xC07F;

// Parity bits of the 16 accumulator registers of each 32 x 32 block, as
// one 16-bit mask per block (bit r = register r).
template <int WI>
__device__ __forceinline__ void parity_masks(const v16f (&acc)[WI][4], uint32_t (&par)[WI][4]) {
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t m = 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) m |= (__float_as_uint(acc[i][j][r]) & 1u) << r;
      par[i][j] = m;
    }
}

// Parities out of a wave's 32 WI x 128 part of the 256 x 256 tile (waves
// laid out two across: rows (wv >> 1) 32 WI, columns (wv & 1) 128).
// Register r of block (i, j) in lane (h, l32) is row 32 i + 8 (r / 4) +
// 4 h + (r % 4), column 32 j + l32 of the part.  scratch: 32 WI x 4 dwords
// of LDS per wave.
template <int WI>
__device__ __forceinline__ void write_tile(const MmArgs& a, const uint32_t (&par)[WI][4], int ti, int tj,
                                           LDS uint32_t* scratch) {
  constexpr int PR = 32 * WI;  // rows of the part
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * PR, wc = (wv & 1) * 128;
  const int h = lane >> 5, l32 = lane & 31;
  const int64_t m0 = (int64_t)ti * MM_T, n0 = (int64_t)tj * MM_T;
  LDS uint32_t* rows = scratch + wv * (PR * 4);  // [PR rows][4 dwords]
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint64_t bal = __ballot((par[i][j] >> r) & 1u);
        const int row = 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
        if (l32 == 0) rows[row * 4 + j] = (uint32_t)(bal >> (32 * h));
      }
      // one block's ballots at a time (hoisting all of them runs out of registers)
      __builtin_amdgcn_sched_barrier(0);
    }
  __builtin_amdgcn_s_waitcnt(WAIT_LDS);  // LDS only: the next chunks' loads stay in flight
  __builtin_amdgcn_wave_barrier();
  // row words: lane -> rows lane (+ 64 p) of the part, two words each
  const int64_t cword = (n0 + wc) / 64;
#pragma unroll
  for (int p = 0; p < PR / 64; ++p) {
    const int row = lane + 64 * p;
    const int64_t gi = m0 + wr + row;
    if (gi < a.m) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int64_t wcol = cword + q;
        if (wcol < a.cw) {
          const uint64_t v = (uint64_t)rows[row * 4 + 2 * q] | ((uint64_t)rows[row * 4 + 2 * q + 1] << 32);
          a.C[gi * a.ldc + wcol] = v;
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (!a.sym || ti == tj) return;
  // mirrored tile: row (column 32 j + l32 of the part), words over the
  // part's rows; this lane holds rows 32 i + 8 q + 4 h + s (r = 4 q + s),
  // so block (i, j)'s mask spreads to bits 8 q + s of a 32-bit word, shifted
  // by 4 h, and the two lane halves OR together; lane half h writes word h
  // of the part's PR / 64 words
  const int64_t rword = (m0 + wr) / 64;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t d[WI];
#pragma unroll
    for (int i = 0; i < WI; ++i) {
      const uint32_t x = par[i][j];
      d[i] = ((x & 0xFu) | ((x & 0xF0u) << 4) | ((x & 0xF00u) << 8) | ((x & 0xF000u) << 12)) << (4 * h);
      d[i] |= (uint32_t)__shfl_xor((int)d[i], 32);
    }
    uint64_t w;
    if constexpr (WI == 4)
      w = h ? ((uint64_t)d[2] | ((uint64_t)d[3] << 32)) : ((uint64_t)d[0] | ((uint64_t)d[1] << 32));
    else
      w = (uint64_t)d[0] | ((uint64_t)d[1] << 32);
    const int64_t gj = n0 + wc + 32 * j + l32;
    const int64_t wcol = rword + h;
    if (h < PR / 64 && gj < a.n && wcol < a.cw) a.C[gj * a.ldc + wcol] = w;
  }
}

// Upper-triangle tile t -> (ti, tj): row i of the triangle starts at tile
// i tn - i (i - 1) / 2; i from the quadratic formula, then corrected by one
// step either way against rounding.
__device__ __forceinline__ int64_t tri_start(int64_t i, int64_t tn) { return i * tn - i * (i - 1) / 2; }

__device__ __forceinline__ void tile_coords(const MmArgs& a, int64_t t, int& ti, int& tj) {
  if (!a.sym) {
    ti = (int)(t / a.tn);
    tj = (int)(t % a.tn);
    return;
  }
  const int64_t tn = a.tn;
  const double b = 2.0 * (double)tn + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  if (i > tn - 1) i = tn - 1;
  while (i > 0 && tri_start(i, tn) > t) --i;
  while (i + 1 < tn && tri_start(i + 1, tn) <= t) ++i;
  ti = (int)i;
  tj = (int)(i + (t - tri_start(i, tn)));
}

// The tile G places further in the order (row by row; in the upper
// triangle row i starts at column i).  Past the last tile ti reaches the
// row count; such a tile is never multiplied (its loads read clamped rows).
__device__ __forceinline__ void tile_step(const MmArgs& a, int& ti, int& tj, int G) {
  tj += G;
  if (a.sym) {
    while (tj >= a.tn && ti < a.tn) {
      ++ti;
      tj = tj - a.tn + ti;
    }
  } else {
    while (tj >= a.tn) {
      tj -= a.tn;
      ++ti;
    }
  }
}

// Persistent: workgroup k of XCD x (blockIdx = 8 k + x) takes tiles
// x * per_xcd + k + j G (j = 0, 1, ...; G workgroups per XCD) of its XCD's
// run, so the tiles in flight on one XCD are a contiguous window of the
// tile order and share rows in its L2.  The chunks of all its tiles form one
// sequence s = j nch + c: chunk s + 1 waits in registers while chunk s is
// multiplied, goes to the other LDS buffer, and the loads of chunk s + 2
// start, so the next tile's first chunk is in flight during a tile's parity
// write-out (which has LDS of its own).
template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void gf2mm_kernel(MmArgs a) {
  constexpr int BS = 64 * NW;    // threads
  constexpr int WI = 16 / NW;    // 32-row blocks per wave (4 x 4 or 2 x 4 blocks)
  constexpr int RPT = 2 * MM_T / BS;  // staged rows per thread per chunk
  // two chunk buffers: [buf][row 0..255 A, 256..511 B][4 words]
  __shared__ __attribute__((aligned(16))) uint64_t sbuf[2][2 * MM_T][MM_CW];
  __shared__ __attribute__((aligned(16))) uint32_t wscr[NW * 32 * WI * 4];  // write-out rows, per wave
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int G = (int)(gridDim.x >> 3);
  const int64_t t_first = (int64_t)(blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
  int64_t t_last = (int64_t)((blockIdx.x & 7) + 1) * a.per_xcd;
  if (t_last > a.n_tiles) t_last = a.n_tiles;
  if (t_first >= t_last) return;
  const int kw = a.kw0 + a.kw1;
  const int nch = (kw + MM_CW - 1) / MM_CW;
  const int64_t n_seq = (t_last - t_first + G - 1) / G * nch;

  // The loads of chunk q are straight-line code (no branch may separate them
  // from the stash that uses them, or the compiler waits for each at once):
  // the tile of q is one of the next three, whose first rows are kept in
  // rm[0..2] / rn[0..2] (chunk q of a tile past the end loads clamped rows
  // and is never used); tiles advance by tile_step, without divisions.
  int64_t rm[3], rn[3];
  int sti, stj;  // tile j + 2
  tile_coords(a, t_first, sti, stj);
  rm[0] = (int64_t)sti * MM_T;
  rn[0] = (int64_t)stj * MM_T;
  tile_step(a, sti, stj, G);
  rm[1] = (int64_t)sti * MM_T;
  rn[1] = (int64_t)stj * MM_T;
  tile_step(a, sti, stj, G);
  rm[2] = (int64_t)sti * MM_T;
  rn[2] = (int64_t)stj * MM_T;
  // staged row q (0 .. 511: A rows, then B rows) of thread tid: q = tid + BS k
  uint64_t rr[RPT][MM_CW];
#define GF2MM_FETCH(JOFF, C)                                                                                    \
  do {                                                                                                          \
    const int64_t fm_ = (JOFF) == 0 ? rm[0] : ((JOFF) == 1 ? rm[1] : rm[2]);                                     \
    const int64_t fn_ = (JOFF) == 0 ? rn[0] : ((JOFF) == 1 ? rn[1] : rn[2]);                                     \
    _Pragma("unroll") for (int k = 0; k < RPT; ++k) {                                                           \
      const int q_ = tid + BS * k;                                                                              \
      const bool isb_ = q_ >= MM_T; /* the same in the whole wave */                                            \
      const uint64_t* o0_ = isb_ ? a.b0 : a.a0;                                                                 \
      const uint64_t* o1_ = isb_ ? a.b1 : a.a1;                                                                 \
      const int64_t ld_ = isb_ ? a.ldb : a.lda;                                                                 \
      const int64_t r_ = isb_ ? fn_ + q_ - MM_T : fm_ + q_;                                                     \
      const int64_t nr_ = isb_ ? a.n : a.m;                                                                     \
      _Pragma("unroll") for (int w = 0; w < MM_CW; ++w) rr[k][w] =                                              \
          row_word(o0_, o1_, ld_, r_, nr_, (C) * MM_CW + w, a.kw0, a.kw1, a.mask0, a.mask1);                    \
    }                                                                                                           \
  } while (0)
#define GF2MM_STASH(BUF)                                                              \
  do {                                                                                \
    _Pragma("unroll") for (int k = 0; k < RPT; ++k)                                   \
        _Pragma("unroll") for (int w = 0; w < MM_CW; ++w) sbuf[(BUF)][tid + BS * k][w] = rr[k][w]; \
  } while (0)

  const int wr = (wv >> 1) * (32 * WI), wc = (wv & 1) * 128;  // this wave's part
  const int h = lane >> 5, l32 = lane & 31;
  GF2MM_FETCH(0, 0);
  GF2MM_STASH(0);
  GF2MM_FETCH(nch > 1 ? 0 : 1, nch > 1 ? 1 : 0);
  __syncthreads();
  const int64_t n_my = n_seq / nch;
  for (int64_t j = 0; j < n_my; ++j) {
    if (j > 0) {
      rm[0] = rm[1];
      rn[0] = rn[1];
      rm[1] = rm[2];
      rn[1] = rn[2];
      tile_step(a, sti, stj, G);
      rm[2] = (int64_t)sti * MM_T;
      rn[2] = (int64_t)stj * MM_T;
    }
    const int ti = (int)(rm[0] / MM_T), tj = (int)(rn[0] / MM_T);
    v16f acc[WI][4];
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][jj][r] = ACC_BASE;
    for (int c = 0; c < nch; ++c) {
      const int64_t s = j * nch + c;
      const int buf = (int)(s & 1);
      // this lane's fragments: dword 4h + st of each row's chunk at step st,
      // read just before that step's products
      const uint32_t* pa0 = (const uint32_t*)&sbuf[buf][wr + l32][2 * h];
      const uint32_t* pb0 = (const uint32_t*)&sbuf[buf][MM_T + wc + l32][2 * h];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        v8i oa[WI], ob[4];
#pragma unroll
        for (int i = 0; i < WI; ++i) oa[i] = unpack_fp4(pa0[32 * i * 2 * MM_CW + st]);
#pragma unroll
        for (int i = 0; i < 4; ++i) ob[i] = unpack_fp4(pb0[32 * i * 2 * MM_CW + st]);
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            acc[i][jj] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(oa[i], ob[jj], acc[i][jj], 4, 4, 0,
                                                                          SCALE_ONE, 0, SCALE_ONE);
      }
      // chunk s + 1 into the other buffer (past the end: a buffer no one
      // reads), then the loads of chunk s + 2
      GF2MM_STASH(buf ^ 1);
      const int c2 = c + 2;
      const int joff = c2 < nch ? 0 : (c2 < 2 * nch ? 1 : 2);
      GF2MM_FETCH(joff, c2 - joff * nch);
      if (c + 1 < nch) __syncthreads();
    }
    uint32_t par[WI][4];
    parity_masks<WI>(acc, par);
    write_tile<WI>(a, par, ti, tj, (LDS uint32_t*)wscr);
    __syncthreads();
  }
#undef GF2MM_FETCH
#undef GF2MM_STASH
}

constexpr int MM_KMAX = 32;  // words of K (per row) the 128 x 128 kernel stages whole

// Whole-K kernel of 128 x 128 tiles (four waves of 64 x 64, 2 x 2 blocks):
// 67.5 KiB of LDS at K = 32 words, so two workgroups share a CU and one's
// row staging and parity write-out overlap the other's products.  Bits are
// unpacked by bit plane: plane t of four consecutive dwords (bits 4r + t)
// is an operand as it stands, d & (0x11111111 << t), whose FP4 nibbles are
// 0.5, 1, 2 for t = 0, 1, 2 (block scales 2^1, 2^0, 2^-1); plane 3 would be
// the sign bit, so it is shifted down to plane 2.  Which bit meets which k
// does not matter as long as A and B agree.
constexpr int M2_T = 128;
constexpr int M2_BS = 256;

__device__ __forceinline__ void write_tile2(const MmArgs& a, v16f (&acc)[2][2], int ti, int tj,
                                            LDS uint32_t* scratch) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;
  const int h = lane >> 5, l32 = lane & 31;
  const int64_t m0 = (int64_t)ti * M2_T, n0 = (int64_t)tj * M2_T;
  uint32_t par[2][2];  // bit r: parity of accumulator r of block (i, j)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      uint32_t m = 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) m |= ((uint32_t)acc[i][j][r] & 1u) << r;
      par[i][j] = m;
    }
  // row words: ballots over the lanes (columns), one 64-column word per row
  LDS uint32_t* rows = scratch + wv * (64 * 2);  // [64 rows][2 dwords]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint64_t bal = __ballot((par[i][j] >> r) & 1u);
        const int row = 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
        if (l32 == 0) rows[row * 2 + j] = (uint32_t)(bal >> (32 * h));
      }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  {
    const int64_t gi = m0 + wr + lane;
    const int64_t wcol = (n0 + wc) / 64;
    if (gi < a.m && wcol < a.cw)
      a.C[gi * a.ldc + wcol] = (uint64_t)rows[lane * 2] | ((uint64_t)rows[lane * 2 + 1] << 32);
  }
  if (!a.sym || ti == tj) return;
  // mirrored tile: the row of column 32 j + l32, one word over the quarter's
  // 64 rows; this lane holds rows 32 i + 8 q + 4 h + s (r = 4 q + s)
  const int64_t wcol = (m0 + wr) / 64;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    uint64_t w = 0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        w |= (uint64_t)((par[i][j] >> r) & 1u) << (32 * i + 8 * (r >> 2) + 4 * h + (r & 3));
    w |= (uint64_t)__shfl_xor((long long)w, 32);
    const int64_t gj = n0 + wc + 32 * j + l32;
    if (h == 0 && gj < a.n && wcol < a.cw) a.C[gj * a.ldc + wcol] = w;
  }
}

__global__ __launch_bounds__(M2_BS, 2) void gf2mm_tile2_kernel(MmArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint64_t sm[];  // [2 * M2_T][kwq + 1], kwq = kw rounded to 2
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t t = (int64_t)(blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
  if (t >= a.n_tiles) return;
  int ti, tj;
  tile_coords(a, t, ti, tj);
  const int64_t m0 = (int64_t)ti * M2_T, n0 = (int64_t)tj * M2_T;
  const int kw = a.kw0 + a.kw1;
  const int kwq = (kw + 1) & ~1;  // whole 128-bit groups; the pad word is zero
  const int ld = kwq + 1;
  LDS uint64_t* s64 = (LDS uint64_t*)sm;
  int kwp = 2;
  while (kwp < kwq) kwp <<= 1;
  const int per_row = kwp / 2, rows_per = M2_BS / per_row;
  const int wp = 2 * (tid % per_row), r_first = tid / per_row;
  for (int r0 = r_first; r0 < 2 * M2_T; r0 += 8 * rows_per) {
    uint64_t v0[8], v1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = r0 + u * rows_per;
      v0[u] = v1[u] = 0;
      if (r < 2 * M2_T && wp < kwq) {
        if (r < M2_T) {
          v0[u] = row_word(a.a0, a.a1, a.lda, m0 + r, a.m, wp, a.kw0, a.kw1, a.mask0, a.mask1);
          v1[u] = row_word(a.a0, a.a1, a.lda, m0 + r, a.m, wp + 1, a.kw0, a.kw1, a.mask0, a.mask1);
        } else {
          v0[u] = row_word(a.b0, a.b1, a.ldb, n0 + r - M2_T, a.n, wp, a.kw0, a.kw1, a.mask0, a.mask1);
          v1[u] = row_word(a.b0, a.b1, a.ldb, n0 + r - M2_T, a.n, wp + 1, a.kw0, a.kw1, a.mask0, a.mask1);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = r0 + u * rows_per;
      if (r < 2 * M2_T && wp < kwq) {
        s64[r * ld + wp] = v0[u];
        s64[r * ld + wp + 1] = v1[u];
      }
    }
  }
  __syncthreads();

  v16f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;
  const int h = lane >> 5, l32 = lane & 31;
  // a fragment is 128 bits of a row: lane half h takes word pair 2 g + h of
  // the row's pairs (g = 128-bit group pair), four dwords at once
  const LDS uint32_t* s32 = (const LDS uint32_t*)sm;
  const int ld32 = 2 * ld;
  const LDS uint32_t* pa = s32 + (wr + l32) * ld32 + 4 * h;
  const LDS uint32_t* pb = s32 + (M2_T + wc + l32) * ld32 + 4 * h;
  const int ngrp = kwq / 4 + ((kwq % 4) ? 1 : 0);  // 256-bit groups (two 128-bit halves)
  for (int g = 0; g < ngrp; ++g) {
    uint32_t da[2][4], db[2][4];
    const bool half2 = 4 * g + 2 * h < kwq;  // this lane half's words exist
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        da[i][d] = half2 ? pa[32 * i * ld32 + 8 * g + d] : 0u;
        db[i][d] = half2 ? pb[32 * i * ld32 + 8 * g + d] : 0u;
      }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      v8i oa[2], ob[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          oa[i][d] = (int)(t < 3 ? da[i][d] & (0x11111111u << t) : (da[i][d] >> 1) & 0x44444444u);
          ob[i][d] = (int)(t < 3 ? db[i][d] & (0x11111111u << t) : (db[i][d] >> 1) & 0x44444444u);
        }
        oa[i][4] = oa[i][5] = oa[i][6] = oa[i][7] = 0;
        ob[i][4] = ob[i][5] = ob[i][6] = ob[i][7] = 0;
      }
      // nibble value 0.5, 1, 2, 2 for planes 0..3: scales 2^1, 2^0, 2^-1, 2^-1
      const int sc = t == 0 ? 128 : (t == 1 ? 127 : 126);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(oa[i], ob[j], acc[i][j], 4, 4, 0, sc, 0, sc);
    }
  }
  __syncthreads();  // every wave is through with the rows before the epilogue reuses LDS
  write_tile2(a, acc, ti, tj, (LDS uint32_t*)sm);
}

// ------------------------------------------------------ phase-pair product --

constexpr int PP_BS = 256;
constexpr int PP_CHUNK = 256;   // terms whose h tables sit in LDS at a time
constexpr float RH = 0.70710678118654752440f;

// cos(k pi/4): exact 0 and +-1 where they occur
__device__ __forceinline__ float cos_q(int k) {
  k &= 7;
  const float mag = (k & 1) ? RH : ((k & 2) ? 0.0f : 1.0f);
  return (k >= 3 && k <= 5) ? -mag : mag;
}

// e^{i k pi/4} = (cos(k pi/4), sin(k pi/4)), sin(x) = cos(x - pi/2)
__device__ __forceinline__ float2 omega_pow(int k) { return make_float2(cos_q(k), cos_q(k + 6)); }

__device__ __forceinline__ float2 cmul(float2 x, float2 y) {
  return make_float2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

// scale z by a power of two so that max(|re|, |im|) is in [0.5, 1)
__device__ __forceinline__ void renorm(float2& z, int& e) {
  const float mx = fmaxf(fabsf(z.x), fabsf(z.y));
  if (mx == 0.0f) return;
  const int ex = __builtin_amdgcn_frexp_expf(mx);
  z.x = ldexpf(z.x, -ex);
  z.y = ldexpf(z.y, -ex);
  e += ex;
}

__global__ __launch_bounds__(PP_BS) void phase_pair_kernel(const uint64_t* __restrict__ A,
                                                           const uint64_t* __restrict__ B, int64_t ld,
                                                           int32_t m, int64_t n_set,
                                                           const int8_t* __restrict__ ka,
                                                           const int8_t* __restrict__ kb, int32_t phase8,
                                                           int64_t pow_sqrt2, float2* __restrict__ mant,
                                                           int32_t* __restrict__ expo) {
  __shared__ float2 tab[PP_CHUNK][4];  // h(k; a, b) at index a + 2 b
  const int64_t l = (int64_t)blockIdx.x * PP_BS + threadIdx.x;
  // uniform over the wave: the term words are scalar loads
  const int64_t wcol = __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * PP_BS + (threadIdx.x & ~63)) >> 6));
  const int bitpos = (int)(l & 63);
  // c = omega^phase8 sqrt(2)^pow
  const bool odd = (pow_sqrt2 & 1) != 0;
  int e = (int)((pow_sqrt2 - (odd ? 1 : 0)) / 2);
  float2 z = omega_pow(phase8);
  if (odd) {
    z.x *= 1.41421356237309504880f;
    z.y *= 1.41421356237309504880f;
  }
  renorm(z, e);
  for (int k0 = 0; k0 < m; k0 += PP_CHUNK) {
    const int nk = m - k0 < PP_CHUNK ? m - k0 : PP_CHUNK;
    __syncthreads();
    for (int x = threadIdx.x; x < nk * 4; x += PP_BS) {
      const int k = x >> 2, ab = x & 3, av = ab & 1, bv = ab >> 1;
      const int ak = ka[k0 + k], bk = kb[k0 + k];
      const float2 p = omega_pow(ak + 4 * av), q = omega_pow(bk + 4 * bv), r = omega_pow(ak + bk + 4 * av + 4 * bv);
      tab[k][ab] = make_float2(1.0f + p.x + q.x - r.x, p.y + q.y - r.y);
    }
    __syncthreads();
    if (l < n_set) {
      for (int k = 0; k < nk; ++k) {
        const uint64_t aw = A[(int64_t)(k0 + k) * ld + wcol];
        const uint64_t bw = B[(int64_t)(k0 + k) * ld + wcol];
        const int idx = (int)((aw >> bitpos) & 1) + 2 * (int)((bw >> bitpos) & 1);
        z = cmul(z, tab[k][idx]);
        if ((k & 7) == 7) renorm(z, e);
      }
      renorm(z, e);
    }
  }
  if (l < n_set) {
    if (z.x == 0.0f && z.y == 0.0f) e = 0;
    mant[l] = z;
    expo[l] = e;
  }
}

// coeff[i] bit j = D[i][piv[j]] for j < rank (zero beyond), words < cwords
__global__ void basis_coeff_kernel(const uint64_t* __restrict__ D, int32_t m, int64_t ld,
                                   const int32_t* __restrict__ rank_dev, const int32_t* __restrict__ piv,
                                   uint64_t* __restrict__ coeff, int64_t ldc, int32_t cwords) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= (int64_t)m * cwords) return;
  const int i = (int)(it / cwords), jw = (int)(it - (int64_t)i * cwords);
  const int rank = *rank_dev;
  uint64_t w = 0;
  for (int b = 0; b < 64; ++b) {
    const int j = 64 * jw + b;
    if (j >= rank) break;
    const int c = piv[j];
    w |= ((D[(int64_t)i * ld + (c >> 6)] >> (c & 63)) & 1ull) << b;
  }
  coeff[(int64_t)i * ldc + jw] = w;
}

zx_status launch_gf2mm(MmArgs a, hipStream_t s) {
  const int kw = a.kw0 + a.kw1;
  // General products with K up to 32 words: 128 x 128 tiles, whole K staged
  // (the parity products: 0.379 -> 0.234 ms for 4096 x 65536 x 1024 bits).
  // The symmetric table keeps 256 x 256 tiles with K in double-buffered
  // chunks: with 128 x 128 tiles it took 7.3 ms against 5.3 ms for the
  // chunked kernel as it then was (four times the tiles, each with its
  // mirrored write-out).
  const bool whole = kw <= MM_KMAX && !a.sym;
  const int T = whole ? M2_T : MM_T;
  a.tm = (int32_t)((a.m + T - 1) / T);
  a.tn = (int32_t)((a.n + T - 1) / T);
  a.n_tiles = a.sym ? (int64_t)a.tn * (a.tn + 1) / 2 : (int64_t)a.tm * a.tn;
  a.per_xcd = (a.n_tiles + 7) / 8;
  const int64_t blocks = 8 * a.per_xcd;
  if (blocks > 0x7fffffff) {
    zx_set_error("product of %lld x %lld rows has too many tiles", (long long)a.m, (long long)a.n);
    return ZX_ECAPACITY;
  }
  if (whole) {
    const int kwq = (kw + 1) & ~1;
    const size_t lds = (size_t)2 * M2_T * (kwq + 1) * 8;
    static bool attr_set = false;  // the attribute covers the largest staged K
    if (!attr_set) {
      ZX_HIP(hipFuncSetAttribute((const void*)gf2mm_tile2_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)((size_t)2 * M2_T * (MM_KMAX + 1) * 8)));
      attr_set = true;
    }
    hipLaunchKernelGGL(gf2mm_tile2_kernel, dim3((unsigned)blocks), dim3(M2_BS), lds, s, a);
  } else {
    // one persistent workgroup per CU, the same count on every XCD
    const ZxDevice* d = zx_device();
    if (!d) return ZX_EDEVICE;
    const int64_t per = (d->n_cu / 8) > 0 ? d->n_cu / 8 : 1;
    const int64_t g = per < a.per_xcd ? per : a.per_xcd;
    hipLaunchKernelGGL(gf2mm_kernel<MM_NW>, dim3((unsigned)(8 * g)), dim3(64 * MM_NW), 0, s, a);
  }
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

}  // namespace

// Symmetric commutation table on the matrix cores (called by zx_pauli_commute).
zx_status zx_pauli_commute_mfma(const uint64_t* X, const uint64_t* Z, int64_t n, int32_t n_qubits, int64_t ldq,
                                uint64_t* C, int64_t ldc, hipStream_t s) {
  MmArgs a{};
  const int qw = (n_qubits + 63) / 64;
  a.a0 = X;
  a.a1 = Z;
  a.b0 = Z;
  a.b1 = X;
  a.lda = a.ldb = ldq;
  a.m = a.n = n;
  a.kw0 = a.kw1 = qw;
  a.mask0 = a.mask1 = (n_qubits % 64) ? ((1ull << (n_qubits % 64)) - 1) : ~0ull;
  a.C = C;
  a.ldc = ldc;
  a.cw = (n + 63) / 64;
  a.sym = 1;
  return launch_gf2mm(a, s);
}

extern "C" zx_status zx_gf2_matmul(const uint64_t* A, int64_t m, int64_t lda, const uint64_t* B, int64_t n,
                                   int64_t ldb, int32_t k_bits, uint64_t* C, int64_t ldc, uint32_t flags,
                                   hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(A && B && C, "null argument");
  ZX_CHECK_ARG(m > 0 && n > 0 && k_bits > 0, "empty product: m=%lld n=%lld k_bits=%d", (long long)m,
               (long long)n, k_bits);
  const int kw = (k_bits + 63) / 64;
  ZX_CHECK_ARG(lda >= kw && ldb >= kw, "lda/ldb below %d words", kw);
  ZX_CHECK_ARG(ldc >= (n + 63) / 64, "ldc below %lld words", (long long)((n + 63) / 64));
  MmArgs a{};
  a.a0 = A;
  a.b0 = B;
  a.lda = lda;
  a.ldb = ldb;
  a.m = m;
  a.n = n;
  a.kw0 = kw;
  a.kw1 = 0;
  a.mask0 = (k_bits % 64) ? ((1ull << (k_bits % 64)) - 1) : ~0ull;
  a.mask1 = ~0ull;
  a.C = C;
  a.ldc = ldc;
  a.cw = (n + 63) / 64;
  a.sym = 0;
  zx_status rc = launch_gf2mm(a, s);
  if (rc == ZX_OK && (flags & ZX_SYNC)) ZX_HIP(hipStreamSynchronize(s));
  return rc;
}

extern "C" zx_status zx_phase_pair_product(const uint64_t* A, const uint64_t* B, int64_t ld, int32_t n_terms,
                                           int64_t n_settings, const int8_t* k_alpha, const int8_t* k_beta,
                                           int32_t phase8, int64_t pow_sqrt2, float* mant, int32_t* expo,
                                           hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(mant && expo, "null output");
  ZX_CHECK_ARG(n_terms >= 0 && n_settings > 0, "bad sizes: n_terms=%d n_settings=%lld", n_terms,
               (long long)n_settings);
  ZX_CHECK_ARG(n_terms == 0 || (A && B && k_alpha && k_beta), "null term input");
  ZX_CHECK_ARG(n_terms == 0 || ld >= (n_settings + 63) / 64, "ld below %lld words",
               (long long)((n_settings + 63) / 64));
  const int64_t blocks = (n_settings + PP_BS - 1) / PP_BS;
  ZX_CHECK_ARG(blocks <= 0x7fffffff, "too many settings");
  hipLaunchKernelGGL(phase_pair_kernel, dim3((unsigned)blocks), dim3(PP_BS), 0, s, A, B, ld, n_terms,
                     n_settings, k_alpha, k_beta, phase8 & 7, pow_sqrt2, (float2*)mant, expo);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}

extern "C" zx_status zx_gf2_basis(const uint64_t* D, int32_t m, int32_t n_cols, int64_t ld, uint64_t* R,
                                  int32_t* rank_dev, int32_t* pivot_cols_dev, uint64_t* coeff, int64_t ldc,
                                  void* ws, size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(D && R && coeff && D != R, "null argument or D == R");
  ZX_CHECK_ARG(m > 0 && n_cols > 0, "empty matrix");
  const int cwords = ((m < n_cols ? m : n_cols) + 63) / 64;
  ZX_CHECK_ARG(ldc >= cwords, "ldc %lld < %d", (long long)ldc, cwords);
  zx_status rc = zx_gf2_eliminate(D, R, m, n_cols, ld, rank_dev, pivot_cols_dev, nullptr, 0, ws, ws_bytes, s);
  if (rc != ZX_OK) return rc;
  const int64_t total = (int64_t)m * cwords;
  hipLaunchKernelGGL(basis_coeff_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, D, m, ld,
                     rank_dev, pivot_cols_dev, coeff, ldc, cwords);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}
