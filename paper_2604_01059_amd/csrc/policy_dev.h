// Learned selection priority: candidate list, candidate features, network
// scores, priority order and the selection of the round's rewrites in that
// order.  An LC round lists its candidate spiders; a pivot round lists the
// candidate edges u < v between Pauli candidates (lexicographic, at most the
// list capacity), visits them in priority order and then completes the
// round with the canonical pass, so it is maximal even when the list was
// cut short.  Included by graph.hip inside its namespace, after the round
// primitives.

// Policy work areas in LDS (after the auxiliary arrays).
struct Pol {
  const uint16_t* wbf;    // network, bf16 copy (global)
  const float* param;     // network, fp32 master (global; b1, b2 read)
  int cap;                // list capacity, power of two >= n (>= 64)
  LDSP uint32_t* list;    // candidates: spider u (LC round) or (u << 16) | v (pivot round)
  LDSP uint64_t* key;     // sort keys, descending = priority order
  LDSP uint16_t* fbuf;    // per wavefront 32 x ZX_MLP_IN bf16 features
  LDSP int32_t* thbuf;    // per wavefront 64 two-hop counts (32 first ends, 32 second ends)
  LDSP uint32_t* elist;   // per wavefront 64 endpoints (32 first ends, 32 second ends)
};

__host__ __device__ inline int pol_cap(int n) {
  int c = 64;
  while (c < n) c <<= 1;
  return c;
}
__host__ __device__ inline int64_t pol_bytes(int n, int bs) {
  const int cap = pol_cap(n);
  return 16 + (int64_t)cap * 4 + (int64_t)cap * 8 + (int64_t)(bs / 64) * 32 * zxmlp::IN * 2 +
         (int64_t)(bs / 64) * 64 * 4 * 2;
}

// The feature rows are read 16 bytes at a time: start the area on 16 bytes.
__device__ inline uint8_t* align16(uint8_t* p) { return (uint8_t*)(((uintptr_t)p + 15) & ~uintptr_t(15)); }

template <int BS>
__device__ void setup_pol(Pol& p, uint8_t* at, int n, const uint16_t* wbf, const float* param) {
  p.wbf = wbf;
  p.param = param;
  p.cap = pol_cap(n);
  at = align16(at);
  p.key = (LDSP uint64_t*)at;
  at += (int64_t)p.cap * 8;
  p.list = (LDSP uint32_t*)at;
  at += (int64_t)p.cap * 4;
  p.fbuf = (LDSP uint16_t*)at;
  at += (int64_t)(BS / 64) * 32 * zxmlp::IN * 2;
  p.thbuf = (LDSP int32_t*)at;
  at += (int64_t)(BS / 64) * 64 * 4;
  p.elist = (LDSP uint32_t*)at;
}

// Exclusive prefix over the wavefront of values in [0, 127], and the total.
__device__ __forceinline__ int wave_excl_scan7(int v, int& total) {
  int ex = 0, tot = 0;
#pragma unroll
  for (int bit = 0; bit < 7; ++bit) {
    const uint64_t bb = __ballot((v >> bit) & 1);
    ex += __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0)) << bit;
    tot += __popcll(bb) << bit;
  }
  total = tot;
  return ex;
}

// Sum over the wavefront of values in [0, 255].
__device__ __forceinline__ int wave_sum8(int v) {
  int tot = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) tot += __popcll(__ballot((v >> b) & 1)) << b;
  return tot;
}

// Candidate list of an LC round: the candidate spiders, ascending.
template <int BS, bool LA>
__device__ int list_lc(Ctx<LA>& c, Shared& sh, Pol& p) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int cnt = 0;
    for (int j0 = 0; j0 < c.W; j0 += 64) {
      const int j = j0 + lane;
      uint64_t m = j < c.W ? c.cand[j] : 0;
      int tot;
      int pos = cnt + wave_excl_scan7(__popcll(m), tot);
      while (m) {
        const int b = __ffsll((long long)m) - 1;
        m &= m - 1;
        p.list[pos++] = (uint32_t)(64 * j + b);
      }
      cnt += tot;
    }
    if (lane == 0) sh.cnt = cnt;
  }
  __syncthreads();
  const int cnt = uni(sh.cnt);
  __syncthreads();
  return cnt;
}

// Candidate list of a pivot round (c.cand = the Pauli candidates): the edges
// u < v between them, lexicographic, at most p.cap, as (u << 16) | v.  One
// wavefront: for each u, the words of u's row at or after u's word (lane j:
// word j) masked to candidates above u, placed by a prefix over the lanes.
template <int BS, bool LA>
__device__ int list_pivots(Ctx<LA>& c, Shared& sh, Pol& p) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, W = c.W;
    int cnt = 0;
    for (int wi = 0; wi < W && cnt < p.cap; ++wi) {
      uint64_t pw = (uint64_t)uni64((int64_t)c.cand[wi]);
      while (pw && cnt < p.cap) {
        const int b = __builtin_ctzll(pw);
        pw &= pw - 1;
        const int u = 64 * wi + b;
        const auto ru = row_ptr(c, u);
        for (int j0 = wi; j0 < W && cnt < p.cap; j0 += 64) {
          const int j = j0 + lane;
          uint64_t m = j < W ? ru[j] & c.cand[j] : 0;
          if (j == wi) m &= ~((2ull << b) - 1);  // v > u
          int tot;
          int pos = cnt + wave_excl_scan7(__popcll(m), tot);
          while (m && pos < p.cap) {
            const int v = 64 * j + __builtin_ctzll(m);
            m &= m - 1;
            p.list[pos++] = ((uint32_t)u << 16) | (uint32_t)v;
          }
          cnt += tot;
        }
      }
    }
    if (lane == 0) sh.cnt = cnt < p.cap ? cnt : p.cap;
  }
  __syncthreads();
  const int cnt = uni(sh.cnt);
  __syncthreads();
  return cnt;
}

// Present spiders with k = 0 mod 4 into c.inm (used by the features).
template <int BS, bool LA>
__device__ float pauli_mask_and_scale(Ctx<LA>& c, Shared& sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) sh.key = 0;
  __syncthreads();
  for (int j = wv; j < c.W; j += BS / 64) {
    const int v = 64 * j + lane;
    const bool ok = v < c.n && bit_of(c.alive, v) && (c.k[v] & 3) == 0;
    const uint64_t w = __ballot(ok);
    if (lane == 0) {
      c.inm[j] = w;
      atomicAdd(&sh.key, __popcll(c.alive[j]));
    }
  }
  __syncthreads();
  const int N = uni(sh.key) > 0 ? uni(sh.key) : 1;
  __syncthreads();
  return 1.0f / (float)N;
}

// The seven features of endpoint x into f[0..6] (one wavefront; lane 0
// writes).  Two-hop set: OR of the neighbours' rows minus N[x].
// Lanes form Q groups of Wp (Wp = W rounded up to a power of two, Q = 64 / Wp
// capped at 8; one group of 64 lanes with two words each beyond 64 words):
// lane (g, j) ORs word j of every neighbour whose place in the neighbour
// order is g mod Q.  Neighbours are taken eight at a time from the row's
// words, so each LDS load instruction reads Q neighbour rows and eight are
// in flight per pass; the groups' ORs are merged by lane shuffles.
template <bool LA>
__device__ void endpoint_features(Ctx<LA>& c, int x, float invN, LDSP uint16_t* f, int th_given = -1) {
  const int lane = threadIdx.x & 63, W = c.W;
  const auto rx = row_ptr(c, x);
  int Wp = 1;
  while (Wp < W && Wp < 64) Wp <<= 1;
  const int Q = W <= 64 ? (64 / Wp < 8 ? 64 / Wp : 8) : 1;
  const int g = lane / Wp, jl = lane - g * Wp;
  const bool act = g < Q && jl < W;
  const bool two = W > 64 && jl + 64 < W;
  uint64_t acc[MAXS] = {0, 0}, own[MAXS];
  own[0] = jl < W ? rx[jl] : 0;
  own[1] = two ? rx[jl + 64] : 0;
  for (int kw = 0; kw < (th_given < 0 ? W : 0); ++kw) {
    uint64_t m = (uint64_t)uni64((int64_t)rx[kw]);  // the same word in every lane
    while (m) {
      int nb[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        nb[t] = m ? 64 * kw + __builtin_ctzll(m) : -1;
        m &= m - 1;
      }
#pragma unroll
      for (int t0 = 0; t0 < 8; ++t0) {
        if (t0 % Q != 0 || nb[t0] < 0) continue;  // uniform
        int w = nb[t0];
#pragma unroll
        for (int q = 1; q < 8; ++q)
          if (t0 + q < 8 && q == g) w = nb[t0 + q];
        if (act && w >= 0) {
          const auto rw = row_ptr(c, w);
          acc[0] |= rw[jl];
          if (two) acc[1] |= rw[jl + 64];
        }
      }
    }
  }
  for (int o = Wp; o < 64; o <<= 1) {
    acc[0] |= (uint64_t)__shfl_xor((long long)acc[0], o);
    acc[1] |= (uint64_t)__shfl_xor((long long)acc[1], o);
  }
  int deg = 0, bn = 0, th = 0, pn = 0;
#pragma unroll
  for (int s = 0; s < MAXS; ++s) {
    const int j = jl + 64 * s;
    if (g == 0 && j < W) {
      uint64_t hop2 = acc[s] & ~own[s];
      if (j == (x >> 6)) hop2 &= ~(1ull << (x & 63));
      deg += __popcll(own[s]);
      bn += __popcll(own[s] & c.bnd[j]);
      th += __popcll(hop2);
      pn += __popcll(own[s] & c.inm[j]);
    }
  }
  deg = wave_sum8(deg);
  bn = wave_sum8(bn);
  th = th_given < 0 ? wave_sum8(th) : th_given;
  pn = wave_sum8(pn);
  if (lane == 0) {
    const int k = c.k[x];
    f[0] = zxmlp::to_bf16((float)deg * invN);
    f[1] = zxmlp::to_bf16((k & 3) == 0 ? 1.f : 0.f);
    f[2] = zxmlp::to_bf16((k & 3) == 2 ? 1.f : 0.f);
    f[3] = zxmlp::to_bf16((k & 1) ? 1.f : 0.f);
    f[4] = zxmlp::to_bf16((float)bn * invN);
    f[5] = zxmlp::to_bf16((float)th * invN);
    f[6] = zxmlp::to_bf16((float)pn * invN);
  }
}

// Features of LC candidate u into f[0..15] (one wavefront): its endpoint
// features, zeros for the second endpoint, rule bit 0, constant 1.
template <bool LA>
__device__ void candidate_features(Ctx<LA>& c, int u, float invN, LDSP uint16_t* f, int th_given = -1) {
  const int lane = threadIdx.x & 63;
  endpoint_features(c, u, invN, f, th_given);
  if (lane < 7) f[7 + lane] = 0;
  if (lane == 0) {
    f[14] = zxmlp::to_bf16(0.f);
    f[15] = zxmlp::to_bf16(1.f);
  }
}

// Features of pivot candidate (u, v) into f[0..15] (one wavefront): the
// endpoint features of u and of v, rule bit 1, constant 1.
template <bool LA>
__device__ void pivot_features(Ctx<LA>& c, int u, int v, float invN, LDSP uint16_t* f, int th_u = -1,
                               int th_v = -1) {
  const int lane = threadIdx.x & 63;
  endpoint_features(c, u, invN, f, th_u);
  endpoint_features(c, v, invN, f + 7, th_v);
  if (lane == 0) {
    f[14] = zxmlp::to_bf16(1.f);
    f[15] = zxmlp::to_bf16(1.f);
  }
}

typedef int pol_v8i __attribute__((ext_vector_type(8)));
typedef float pol_v16f __attribute__((ext_vector_type(16)));

// 32 bits as 32 FP4 (E2M1) operand values of a 64-deep matrix-core product:
// nibble r of dword t is bit 4r + t (code 1 = 0.5, or 0).
__device__ __forceinline__ pol_v8i bits_fp4(uint32_t d) {
  pol_v8i o;
  o[0] = (int)(d & 0x11111111u);
  o[1] = (int)((d >> 1) & 0x11111111u);
  o[2] = (int)((d >> 2) & 0x11111111u);
  o[3] = (int)((d >> 3) & 0x11111111u);
  o[4] = o[5] = o[6] = o[7] = 0;
  return o;
}

// Two-hop counts of candidates list[base + r], r < 32 (entries past C count
// nothing), into th[r] (one wavefront): the spiders v other than x and not
// adjacent to x that share a neighbour with x.  A x A counts the common
// neighbours of the 32 candidates and 32 spiders v at a time on the matrix
// cores (v_mfma_scale_f32_32x32x64_f8f6f4: a bit is the FP4 value 0.5 scaled
// by 2^1 to 1, every sum an exact fp32 count below 2^13).  Each block's
// accumulator first takes -12288 at v = x and at v adjacent to x (one more
// product: x's row with its own bit against a one-hot operand of value -6
// scaled by 2^11), so a positive sum marks exactly a two-hop spider; one
// ballot per accumulator register counts them per candidate.
template <bool LA>
__device__ void two_hop32(Ctx<LA>& c, const LDSP uint32_t* list, int base, int C, LDSP int32_t* th) {
  const int lane = threadIdx.x & 63, h = lane >> 5, l32 = lane & 31;
  const int n = c.n, W = c.W;
  const int xr = base + l32 < C ? (int)list[base + l32] : -1;
  const auto rx = row_ptr(c, xr < 0 ? 0 : xr);
  int cnt[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) cnt[r] = 0;
  for (int jb = 0; 32 * jb < n; ++jb) {
    const int v = 32 * jb + l32;
    const bool vin = v < n;
    const auto rv = row_ptr(c, vin ? v : 0);
    const int wj = jb >> 1;
    uint64_t ax = rx[wj] & (xr >= 0 ? ~0ull : 0ull);
    if (xr >= 0 && (xr >> 6) == wj) ax |= 1ull << (xr & 63);
    pol_v8i bo = bits_fp4(h == (jb & 1) && vin ? 1u << l32 : 0u);
    bo[0] *= 15;  // nibble 0xF: -6
    bo[1] *= 15;
    bo[2] *= 15;
    bo[3] *= 15;
    pol_v16f acc = {};
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bits_fp4((uint32_t)(ax >> (32 * h))), bo, acc, 4, 4, 0,
                                                          128, 0, 138);
    // rows rx and rv are always in range (row 0 stands in), so their words
    // are loaded without branches, four steps' worth before the first is used
    const uint32_t am = xr >= 0 ? 0xffffffffu : 0u, bm = vin ? 0xffffffffu : 0u;
    int ks = 0;
    for (; ks + 4 <= W; ks += 4) {
      uint64_t ra[4], rb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ra[q] = rx[ks + q];
        rb[q] = rv[ks + q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bits_fp4((uint32_t)(ra[q] >> (32 * h)) & am),
                                                              bits_fp4((uint32_t)(rb[q] >> (32 * h)) & bm), acc, 4,
                                                              4, 0, 128, 0, 128);
    }
    for (; ks < W; ++ks)
      acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bits_fp4((uint32_t)(rx[ks] >> (32 * h)) & am),
                                                            bits_fp4((uint32_t)(rv[ks] >> (32 * h)) & bm), acc, 4, 4,
                                                            0, 128, 0, 128);
    // register r of lane (h, l32): candidate 8 (r / 4) + 4 h + r % 4, spider 32 jb + l32
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint64_t b = __ballot(acc[r] > 0.0f);
      cnt[8 * (r >> 2) + (r & 3)] += __popcll(b & 0xffffffffull);
      cnt[8 * (r >> 2) + 4 + (r & 3)] += __popcll(b >> 32);
    }
  }
#pragma unroll
  for (int r = 0; r < 32; ++r)
    if (lane == r) th[r] = cnt[r];
}

// Features of a block of up to 32 candidates (list entries base..base+cnt)
// into fb (32 rows of IN), one endpoint per lane, the two-hop counts given
// (th; pivots: first ends th[0..32), second ends th[32..64), ends in el).
// Lane r (r < 32) takes candidate r's first endpoint, lane 32 + r a pivot's
// second endpoint: degree, boundary and input neighbours by popcounts over
// the endpoint's row, the phase bits, in the same arithmetic as
// endpoint_features.
template <bool LA>
__device__ void block_features(Ctx<LA>& c, const Pol& p, int base, int cnt, bool pivot, float invN,
                               LDSP uint16_t* fb, const LDSP int32_t* th, const LDSP uint32_t* el) {
  const int lane = threadIdx.x & 63, r = lane & 31, second = lane >> 5, W = c.W;
  int x = -1;
  if (r < cnt) {
    if (pivot)
      x = (int)el[32 * second + r];
    else if (second == 0)
      x = (int)p.list[base + r];
  }
  LDSP uint16_t* f = fb + r * zxmlp::IN;
  if (x >= 0) {
    const auto rx = row_ptr(c, x);
    int deg = 0, bn = 0, pn = 0;
#pragma unroll 4
    for (int j = 0; j < W; ++j) {
      const uint64_t w = rx[j];
      deg += __popcll(w);
      bn += __popcll(w & c.bnd[j]);
      pn += __popcll(w & c.inm[j]);
    }
    const int t = th[pivot ? 32 * second + r : r];
    const int k = c.k[x];
    LDSP uint16_t* fo = f + 7 * second;
    fo[0] = zxmlp::to_bf16((float)deg * invN);
    fo[1] = zxmlp::to_bf16((k & 3) == 0 ? 1.f : 0.f);
    fo[2] = zxmlp::to_bf16((k & 3) == 2 ? 1.f : 0.f);
    fo[3] = zxmlp::to_bf16((k & 1) ? 1.f : 0.f);
    fo[4] = zxmlp::to_bf16((float)bn * invN);
    fo[5] = zxmlp::to_bf16((float)t * invN);
    fo[6] = zxmlp::to_bf16((float)pn * invN);
  }
  if (second == 0) {
    if (r < cnt) {
      if (!pivot)
        for (int q = 7; q < 14; ++q) f[q] = 0;
      f[14] = zxmlp::to_bf16(pivot ? 1.f : 0.f);
      f[15] = zxmlp::to_bf16(1.f);
    } else {
      for (int q = 0; q < zxmlp::IN; ++q) f[q] = 0;
    }
  }
}

// Order-preserving map of a float onto uint32.
__device__ __forceinline__ uint32_t float_order(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Scores of list entries 0..C-1 into p.key as (order(score) << 32) |
// ~index, so that descending keys give descending scores, ties by index.
// pivot: the entries are edges; the two-hop counts of their first and
// second ends come from two matrix-core passes over the endpoint list.
template <int BS, bool LA>
__device__ void policy_score(Ctx<LA>& c, Pol& p, int C, float invN, bool pivot) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  LDSP uint16_t* fb = p.fbuf + wv * 32 * zxmlp::IN;
  LDSP int32_t* tb = p.thbuf + wv * 64;
  LDSP uint32_t* el = p.elist + wv * 64;
  for (int base = wv * 32; base < C; base += (BS / 64) * 32) {
    const int cnt = C - base < 32 ? C - base : 32;
    if (pivot) {
      const int r = lane & 31;
      const uint32_t e = r < cnt ? p.list[base + r] : 0u;
      el[lane] = lane < 32 ? e >> 16 : e & 0xffffu;
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      two_hop32(c, el, 0, cnt, tb);
      two_hop32(c, el, 32, 32 + cnt, tb + 32);
    } else {
      two_hop32(c, p.list, base, C, tb);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    block_features(c, p, base, cnt, pivot, invN, fb, tb, el);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    float s[16];
    zxmlp::score32(zxmlp::load_a(fb), p.wbf, p.param, s);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int idx = base + zxmlp::acc_row(i, lane);
      if ((lane & 31) == i && idx < C)
        p.key[idx] = ((uint64_t)float_order(s[i]) << 32) | (uint32_t)(0xffffffffu - (uint32_t)idx);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
}

// Bitonic sort of the C keys (padded with zeros to a power of two, which
// sort last), descending.  Element i is handled by thread i mod BS, so the partners of a
// step of distance below 64 are in the same wavefront.  Between two such
// steps only the wavefront's LDS accesses need ordering; a block barrier
// follows every step of distance 64 or more and every step that precedes
// one (the last step of a merge whose next merge starts at distance 64 or
// more).
template <int BS>
__device__ void sort_keys_desc(Pol& p, int C) {
  int P = 1;
  while (P < C) P <<= 1;
  for (int i = C + threadIdx.x; i < P; i += BS) p.key[i] = 0;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += BS) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = p.key[i], b = p.key[ixj];
          const bool desc = (i & k) == 0;
          if (desc ? (a < b) : (a > b)) {
            p.key[i] = b;
            p.key[ixj] = a;
          }
        }
      }
      const int next_j = j > 1 ? j >> 1 : k;  // the next step's distance (next merge: 2k, from k)
      if (j >= 64 || next_j >= 64) {
        __syncthreads();
      } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  __syncthreads();
}

__device__ __forceinline__ uint32_t key_index(uint64_t k) { return 0xffffffffu - (uint32_t)k; }

// LC round in priority order: take each candidate unless adjacent to one
// taken before it.  One wavefront, 64 candidates of the order at a time.
// The wavefront keeps the union of the taken spiders' rows (lane l: words l
// and l + 64), so a candidate adjacent to a spider taken in an earlier
// block is one bit of it.  The block's free candidates are then taken in
// order; each taken spider x drops the later ones adjacent to it (lane m
// reads bit u_m of x's row), and its row joins the union.
template <int BS, bool LA>
__device__ void select_lc_priority(Ctx<LA>& c, Shared& sh, Pol& p, int C) {
  const int W = c.W;
  for (int j = threadIdx.x; j < W; j += BS) c.sel[j] = 0;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    // clamped word indices (W <= 128): a lane's words past W are loaded
    // from word W - 1 and never read
    const int j0 = lane < W ? lane : W - 1;
    const int j1 = lane + 64 < W ? lane + 64 : W - 1;
    uint64_t blk0 = 0, blk1 = 0;
    for (int b = 0; b < C; b += 64) {
      const int e = b + lane;
      const int u = e < C ? (int)p.list[key_index(p.key[e])] : -1;
      const int wi = u >= 0 ? (u >> 6) : 0;  // u's word (word 0 stands in past C)
      const uint64_t b0 = wave_shfl64(blk0, wi & 63, 64), b1 = wave_shfl64(blk1, wi & 63, 64);
      const uint64_t bw = wi < 64 ? b0 : b1;
      uint64_t R = __ballot(u >= 0 && !((bw >> (u & 63)) & 1));
      uint64_t taken = 0;
      while (R) {
        const int l = __builtin_ctzll(R);
        taken |= 1ull << l;
        R &= ~(1ull << l);
        const int x = __builtin_amdgcn_readlane(u, l);
        const bool adj = u >= 0 && ((row_ptr(c, x)[wi] >> (u & 63)) & 1);
        R &= ~__ballot(adj);
      }
      if ((taken >> lane) & 1) atomicOr((unsigned long long*)&c.sel[u >> 6], 1ull << (u & 63));
      // the taken rows join the union, four at a time
      uint64_t tk = taken;
      while (tk) {
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
          const auto rt = row_ptr(c, __builtin_amdgcn_readlane(u, t[q]));
          a0 |= rt[j0];
          a1 |= rt[j1];
        }
        blk0 |= a0;
        blk1 |= a1;
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
}

// Pivot round in priority order: each listed edge is taken unless an end is
// taken or adjacent to a taken end (c.blocked holds the taken ends and their
// neighbours); then the canonical pass completes the round from that
// blocked set.  One wavefront for the ordered part: lane j keeps word j.
template <int BS, bool LA>
__device__ void select_pivots_priority(Ctx<LA>& c, Shared& sh, Pol& p, int C) {
  const int W = c.W;
  for (int j = threadIdx.x; j < W; j += BS) {
    c.sel[j] = 0;
    c.blocked[j] = 0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int npairs = 0, nt = sh.n_trace;
    const int round = sh.round;
    for (int e = 0; e < C; ++e) {
      const uint32_t ent = (uint32_t)uni((int)p.list[key_index(p.key[e])]);
      const int u = (int)(ent >> 16), v = (int)(ent & 0xffffu);
      if (uni(bit_of(c.blocked, u) || bit_of(c.blocked, v))) continue;
      const auto ru = row_ptr(c, u);
      const auto rv = row_ptr(c, v);
      for (int j = lane; j < W; j += 64) {
        uint64_t add = ru[j] | rv[j];
        if (j == (u >> 6)) add |= 1ull << (u & 63);
        if (j == (v >> 6)) add |= 1ull << (v & 63);
        c.blocked[j] |= add;
      }
      if (lane == 0) {
        c.partner[u] = (int16_t)v;
        c.partner[v] = (int16_t)u;
        if (c.trace) {
          int32_t* t = c.trace + 4 * (int64_t)nt;
          t[0] = round;
          t[1] = 1;
          t[2] = u;
          t[3] = v;
        }
        c.sel[u >> 6] |= 1ull << (u & 63);
        c.sel[v >> 6] |= 1ull << (v & 63);
      }
      ++npairs;
      ++nt;
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
      sh.cnt = npairs;
      sh.n_trace = nt;
    }
  }
  __syncthreads();
  select_pivots<BS, LA, true>(c, sh);
}
