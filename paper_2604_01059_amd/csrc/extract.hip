// Circuit extraction of graph-like diagrams on the GPU.
//
// The paper simplifies diagrams by local complementation and pivoting and
// eliminates binary matrices over F2, but leaves extraction to the standard
// procedure (Backens, Miller-Bakewell, de Felice, Lobski, van de Wetering,
// "There and back again: a circuit extraction tale", Quantum 2021), which
// this kernel runs on the CURRENT diagram of each arena:
//
//   * every input spider v is first unfused into input -- a -H- b -H- v
//     (b is a phase-free spider between two Hadamard edges, a plain wire),
//     so the input spiders a carry nothing but their wire;
//   * the frontier starts at the outputs (a Hadamard output wire is an H
//     gate); each round turns the frontier spiders' phases into Z rotations
//     and their mutual edges into CZ gates, then reduces the biadjacency
//     between the frontier spiders that are not input spiders and their
//     other neighbours N by Gauss-Jordan elimination over F2 (lowest pivot
//     column first, lowest row within it; a row swap is three row
//     additions); each row addition row_t += row_s is a CNOT (control t,
//     target s) and is applied to the graph;
//   * every frontier row left with a single neighbour w is an H gate: the
//     qubit's frontier moves to w;
//   * when no frontier spider has a neighbour outside the frontier, the
//     frontier is the input spiders: their order is the input permutation.
//
// Gates come out closest to the outputs first; the unitary of the diagram is
// G_1 G_2 ... G_m times the input permutation (and the Hadamards of Hadamard
// input wires), up to a scalar.
//
// One workgroup per diagram (a work queue over the batch) with the extended
// adjacency (n + 2 n_in spiders) in LDS.  Gate lists are ordered, so every
// emission is a ballot compaction in one wavefront, or a block count of the
// rows a pivot hits (rows in ascending order) followed by positions from
// popcounts.  The rows of the eliminated spiders change only in N's columns;
// the transposed bits in N's rows are written back once per round, before
// anything reads them.
#include "zx_internal.h"

namespace {

#define LDS __attribute__((address_space(3)))

constexpr int EX_BS = 256;
constexpr int EX_MAXN = 1024;  // n + 2 n_in spiders (the adjacency is N x N bits in LDS)
constexpr int EX_NOKEY = 0x7fffffff;

struct ExEntry {
  uint8_t* arena;
  int64_t gate_off;  // first gate of this diagram
  int64_t perm_off;  // first perm entry of this diagram
};

struct ExWs {
  ZxWsHeader hdr;
  uint32_t next;
  uint32_t pad[63];
  // followed by ExEntry[n_graphs]
};
static_assert(sizeof(ExWs) % 256 == 0, "workspace header size");

struct ExShared {
  int32_t idx, key, ng, cnt, na, any, err;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t gate(uint32_t type, int a, int b) {
  return (type << 30) | ((uint32_t)a << 15) | (uint32_t)b;
}

__device__ __forceinline__ bool bit(const LDS uint64_t* row, int j) { return (row[j >> 6] >> (j & 63)) & 1; }

__host__ __device__ inline int ex_hit_words(int n_ext, int q) {
  const int we = (n_ext + 63) / 64, hq = (q + 63) / 64;
  return we > hq ? we : hq;
}

struct Ex {
  LDS uint64_t* A;  // n_ext x We
  LDS uint64_t *fm, *alive, *inm, *nm, *hit;
  LDS int16_t *front, *act, *rows, *lw;
  LDS int8_t* k;
  int n, n_ext, We, Q, cap;
  uint32_t* out;
};

// Wave 0: gates g(i) for i in [0, cnt) where flag(i), in ascending i.
template <typename Flag, typename Make>
__device__ void emit_ordered(Ex& e, ExShared& sh, int cnt, Flag flag, Make make) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int base = sh.ng;
    for (int i0 = 0; i0 < cnt; i0 += 64) {
      const int i = i0 + lane;
      const bool f = i < cnt && flag(i);
      const uint64_t b = __ballot(f);
      if (f) {
        const int pos = base + __popcll(b & ((1ull << lane) - 1));
        if (pos < e.cap) e.out[pos] = make(i);
      }
      base += __popcll(b);
    }
    if (lane == 0) sh.ng = base;
  }
  __syncthreads();
}

__global__ __launch_bounds__(EX_BS) void extract_kernel(ExWs* ws, const ExEntry* table, int32_t n_graphs,
                                                         int32_t max_gates, uint32_t* gates, int32_t* n_gates,
                                                         int32_t* perm, int32_t* status) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ ExShared sh;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sh.idx = (int32_t)atomicAdd(&ws->next, 1u);
    __syncthreads();
    const int gi = uni(sh.idx);
    __syncthreads();
    if (gi >= n_graphs) break;
    const uint8_t* arena = table[gi].arena;
    const ZxHeader* h = (const ZxHeader*)arena;
    const int n = uni(h->n), W = uni(h->W), q_in = uni(h->n_in), q_out = uni(h->n_out);
    const int n_ext = n + 2 * q_in;
    if (uni(h->magic) != ZX_MAGIC || n < 1 || q_in < 0 || q_out < 0 || n_ext > EX_MAXN || q_out > EX_MAXN ||
        W != (n + 63) / 64 || uni(h->status) != 0) {
      if (tid == 0) {
        status[gi] = uni(h->status) != 0 ? uni(h->status) : ZX_ECAPACITY;
        n_gates[gi] = 0;
      }
      __syncthreads();
      continue;
    }
    const uint64_t* adj = (const uint64_t*)(arena + h->off_adj);
    const int8_t* phase = (const int8_t*)(arena + h->off_phase);
    const uint64_t* alive_g = (const uint64_t*)(arena + h->off_alive);
    const int32_t* ins = (const int32_t*)(arena + h->off_in);
    const int32_t* outs = (const int32_t*)(arena + h->off_out);
    const uint8_t* is_h = arena + h->off_is_h;

    Ex e;
    e.n = n;
    e.n_ext = n_ext;
    e.We = (n_ext + 63) / 64;
    e.Q = q_out;
    e.cap = max_gates;
    e.out = gates + table[gi].gate_off;
    const int We = e.We, Q = q_out;
    // LDS: A | fm | alive | inm | nm (We words each) | hit (one bit per frontier row) |
    //      front | act | rows | lw (Q int16 each) | k (n_ext)
    e.A = (LDS uint64_t*)smem;
    e.fm = e.A + (size_t)n_ext * We;
    e.alive = e.fm + We;
    e.inm = e.alive + We;
    e.nm = e.inm + We;
    e.hit = e.nm + We;
    e.front = (LDS int16_t*)(e.hit + ex_hit_words(n_ext, Q));
    e.act = e.front + Q;
    e.rows = e.act + Q;
    e.lw = e.rows + Q;
    e.k = (LDS int8_t*)(e.lw + Q);

    // extended adjacency: present spiders' rows, then the unfused inputs
    for (int it = tid; it < n_ext * We; it += EX_BS) {
      const int r = it / We, j = it - r * We;
      uint64_t v = 0;
      if (r < n && j < W && ((alive_g[r >> 6] >> (r & 63)) & 1)) v = adj[(size_t)r * W + j] & alive_g[j];
      e.A[it] = v;
    }
    for (int j = tid; j < We; j += EX_BS) {
      e.fm[j] = 0;
      e.inm[j] = 0;
      e.alive[j] = j < W ? alive_g[j] : 0;
    }
    for (int v = tid; v < n_ext; v += EX_BS) e.k[v] = v < n ? (int8_t)(phase[v] & 7) : 0;
    if (tid == 0) {
      sh.ng = 0;
      sh.err = 0;
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i < q_in; ++i) {
        const int a = n + 2 * i, b = a + 1, v = ins[i];
        e.A[(size_t)a * We + (b >> 6)] |= 1ull << (b & 63);
        e.A[(size_t)b * We + (a >> 6)] |= 1ull << (a & 63);
        e.A[(size_t)b * We + (v >> 6)] |= 1ull << (v & 63);
        e.A[(size_t)v * We + (b >> 6)] |= 1ull << (b & 63);
        e.alive[a >> 6] |= 1ull << (a & 63);
        e.alive[b >> 6] |= 1ull << (b & 63);
        e.inm[a >> 6] |= 1ull << (a & 63);
      }
      for (int q = 0; q < Q; ++q) {
        const int v = outs[q];
        e.front[q] = (int16_t)v;
        e.fm[v >> 6] |= 1ull << (v & 63);
      }
    }
    __syncthreads();
    // Hadamard output wires
    emit_ordered(e, sh, Q, [&](int q) { return is_h[q_in + q] != 0; },
                 [&](int q) { return gate(ZX_GATE_H, q, 0); });

    for (int round = 0; round <= n_ext; ++round) {
      // Z rotations of the frontier phases
      emit_ordered(e, sh, Q, [&](int q) { return e.k[e.front[q]] != 0; },
                   [&](int q) { return gate(ZX_GATE_RZ, q, e.k[e.front[q]]); });
      for (int q = tid; q < Q; q += EX_BS) e.k[e.front[q]] = 0;
      // CZ gates of the frontier's mutual edges, pairs (a, b) in order
      for (int a = 0; a < Q; ++a) {
        if (tid < 64) {
          const int lane = tid;
          const int fa = e.front[a];
          LDS uint64_t* ra = e.A + (size_t)fa * We;
          int base = sh.ng;
          for (int b0 = a + 1; b0 < Q; b0 += 64) {
            const int b = b0 + lane;
            const int fb = b < Q ? e.front[b] : 0;
            const bool f = b < Q && bit(ra, fb);
            const uint64_t bl = __ballot(f);
            if (f) {
              const int pos = base + __popcll(bl & ((1ull << lane) - 1));
              if (pos < e.cap) e.out[pos] = gate(ZX_GATE_CZ, a, b);
              e.A[(size_t)fb * We + (fa >> 6)] &= ~(1ull << (fa & 63));
              atomicAnd((unsigned long long*)&ra[fb >> 6], ~(1ull << (fb & 63)));
            }
            base += __popcll(bl);
          }
          if (lane == 0) sh.ng = base;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
      }
      __syncthreads();
      // N: neighbours of the frontier outside it
      if (tid == 0) sh.any = 0;
      __syncthreads();
      for (int j = tid; j < We; j += EX_BS) {
        uint64_t m = 0;
        for (int q = 0; q < Q; ++q) m |= e.A[(size_t)e.front[q] * We + j];
        m &= ~e.fm[j];
        e.nm[j] = m;
        if (m) sh.any = 1;
      }
      __syncthreads();
      if (!uni(sh.any)) break;
      // rows to eliminate: the qubits whose frontier spider is not an input spider
      if (tid < 64) {
        int base = 0;
        for (int q0 = 0; q0 < Q; q0 += 64) {
          const int q = q0 + tid;
          const bool f = q < Q && !bit(e.inm, e.front[q]);
          const uint64_t bl = __ballot(f);
          if (f) {
            const int t = base + __popcll(bl & ((1ull << tid) - 1));
            e.act[t] = (int16_t)q;
            e.rows[t] = e.front[q];
            e.lw[t] = 0;
          }
          base += __popcll(bl);
        }
        if (tid == 0) sh.na = base;
      }
      __syncthreads();
      const int na = uni(sh.na);
      const int hw = (na + 63) / 64;
      // Gauss-Jordan on the rows' N columns (the rows hold no other bits)
      int cur = 0;
      while (cur < na) {
        if (tid == 0) sh.key = EX_NOKEY;
        for (int j = tid; j < hw; j += EX_BS) e.hit[j] = 0;
        __syncthreads();
        for (int t = cur + tid; t < na; t += EX_BS) {
          const LDS uint64_t* rr = e.A + (size_t)e.rows[t] * We;
          int j = e.lw[t];
          while (j < We && rr[j] == 0) ++j;
          e.lw[t] = (int16_t)j;
          if (j < We) atomicMin(&sh.key, ((64 * j + __builtin_ctzll(rr[j])) << 15) | t);
        }
        __syncthreads();
        const int key = uni(sh.key);
        if (key == EX_NOKEY) break;
        const int col = key >> 15, r = key & 0x7fff;
        if (r != cur) {
          // rows cur and r trade places: three row additions
          LDS uint64_t* x = e.A + (size_t)e.rows[cur] * We;
          LDS uint64_t* y = e.A + (size_t)e.rows[r] * We;
          for (int j = tid; j < We; j += EX_BS) {
            const uint64_t t = x[j];
            x[j] = y[j];
            y[j] = t;
          }
          if (tid == 0) {
            const int qc = e.act[cur], qr = e.act[r];
            const int ng = sh.ng;
            if (ng < e.cap) e.out[ng] = gate(ZX_GATE_CNOT, qc, qr);
            if (ng + 1 < e.cap) e.out[ng + 1] = gate(ZX_GATE_CNOT, qr, qc);
            if (ng + 2 < e.cap) e.out[ng + 2] = gate(ZX_GATE_CNOT, qc, qr);
            sh.ng = ng + 3;
            const int16_t lt = e.lw[r];
            e.lw[r] = e.lw[cur];
            e.lw[cur] = lt;
          }
          __syncthreads();
        }
        // every other row with the pivot column takes the pivot row
        for (int t = tid; t < na; t += EX_BS)
          if (t != cur && bit(e.A + (size_t)e.rows[t] * We, col))
            atomicOr((unsigned long long*)&e.hit[t >> 6], 1ull << (t & 63));
        __syncthreads();
        {
          const int base = uni(sh.ng);
          for (int t = tid; t < na; t += EX_BS) {
            if (!((e.hit[t >> 6] >> (t & 63)) & 1)) continue;
            int pos = base + __popcll(e.hit[t >> 6] & ((1ull << (t & 63)) - 1));
            for (int j = 0; j < (t >> 6); ++j) pos += __popcll(e.hit[j]);
            if (pos < e.cap) e.out[pos] = gate(ZX_GATE_CNOT, e.act[t], e.act[cur]);
          }
          const LDS uint64_t* pr = e.A + (size_t)e.rows[cur] * We;
          for (int it = tid; it < na * We; it += EX_BS) {
            const int t = it / We, j = it - t * We;
            if ((e.hit[t >> 6] >> (t & 63)) & 1) e.A[(size_t)e.rows[t] * We + j] ^= pr[j];
          }
          __syncthreads();
          if (tid == 0) {
            int c = 0;
            for (int j = 0; j < hw; ++j) c += __popcll(e.hit[j]);
            sh.ng = base + c;
          }
        }
        __syncthreads();
        ++cur;
      }
      __syncthreads();
      // transposed bits: column rows[t] of every row w in N
      for (int w = tid; w < n_ext; w += EX_BS) {
        if (!bit(e.nm, w)) continue;
        LDS uint64_t* rw = e.A + (size_t)w * We;
        for (int t = 0; t < na; ++t) {
          const int v = e.rows[t];
          const uint64_t b = 1ull << (v & 63);
          if (bit(e.A + (size_t)v * We, w))
            rw[v >> 6] |= b;
          else
            rw[v >> 6] &= ~b;
        }
      }
      __syncthreads();
      // rows with a single neighbour: an H gate, and the frontier moves on
      if (tid < 64) {
        const int lane = tid;
        int base = sh.ng, moved = 0;
        for (int t0 = 0; t0 < na; t0 += 64) {
          const int t = t0 + lane;
          int pc = 0, at = -1, v = -1;
          if (t < na) {
            v = e.rows[t];
            const LDS uint64_t* rr = e.A + (size_t)v * We;
            for (int j = 0; j < We && pc < 2; ++j) {
              const uint64_t x = rr[j];
              if (x) {
                pc += __popcll(x);
                at = 64 * j + __builtin_ctzll(x);
              }
            }
          }
          const bool f = t < na && pc == 1;
          const uint64_t bl = __ballot(f);
          if (f) {
            const int pos = base + __popcll(bl & ((1ull << lane) - 1));
            const int q = e.act[t];
            if (pos < e.cap) e.out[pos] = gate(ZX_GATE_H, q, 0);
            e.A[(size_t)v * We + (at >> 6)] &= ~(1ull << (at & 63));
            e.A[(size_t)at * We + (v >> 6)] &= ~(1ull << (v & 63));
            e.front[q] = (int16_t)at;
          }
          base += __popcll(bl);
          moved += __popcll(bl);
        }
        if (lane == 0) {
          sh.ng = base;
          sh.cnt = moved;
        }
      }
      __syncthreads();
      if (uni(sh.cnt) == 0) {
        if (tid == 0) sh.err = ZX_ENOMATCH;  // no frontier row with a single neighbour
        __syncthreads();
        break;
      }
      // the moved spiders leave the diagram; the frontier mask follows
      for (int j = tid; j < We; j += EX_BS) e.fm[j] = 0;
      __syncthreads();
      if (tid == 0) {
        for (int q = 0; q < Q; ++q) {
          const int v = e.front[q];
          e.fm[v >> 6] |= 1ull << (v & 63);
        }
        for (int t = 0; t < na; ++t) {
          const int v = e.rows[t];
          if (!bit(e.fm, v)) e.alive[v >> 6] &= ~(1ull << (v & 63));
        }
      }
      __syncthreads();
    }
    // the frontier must be exactly the input spiders still present
    if (tid == 0) {
      int err = sh.err;
      for (int j = 0; j < We && !err; ++j)
        if (e.alive[j] != e.fm[j]) err = ZX_ENOMATCH;
      int32_t* pm = perm + table[gi].perm_off;
      for (int q = 0; q < Q; ++q) {
        const int v = e.front[q];
        const int i = (v - n) >> 1;
        if (v < n || ((v - n) & 1)) {
          if (!err) err = ZX_ENOMATCH;  // a frontier spider without an input
          pm[q] = -1;
        } else {
          pm[q] = i;
        }
      }
      if (!err && sh.ng > e.cap) err = ZX_ECAPACITY;
      status[gi] = err;
      n_gates[gi] = sh.ng;
    }
    __syncthreads();
  }
}

__host__ __device__ inline int64_t ex_lds_bytes(int n_ext, int q) {
  const int64_t We = (n_ext + 63) / 64;
  return (int64_t)n_ext * We * 8 + 4 * We * 8 + 8 * (int64_t)ex_hit_words(n_ext, q) + 8 * (int64_t)q + n_ext + 16;
}

}  // namespace

extern "C" size_t zx_extract_workspace_bytes(int32_t n_graphs) {
  if (n_graphs < 0) return 0;
  return sizeof(ExWs) + (((size_t)n_graphs * sizeof(ExEntry) + 255) & ~size_t(255));
}

extern "C" zx_status zx_extract(zx_graph* const* graphs, int32_t n_graphs, int32_t max_gates, uint32_t* gates,
                                int32_t* n_gates, int32_t* perm, int32_t* status, void* ws, size_t ws_bytes,
                                hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(graphs && n_graphs > 0 && gates && n_gates && perm && status && ws, "null argument");
  ZX_CHECK_ARG(max_gates > 0, "max_gates %d must be positive", max_gates);
  ZX_CHECK_ARG(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  if (ws_bytes < zx_extract_workspace_bytes(n_graphs)) {
    zx_set_error("workspace %zu < %zu bytes", ws_bytes, zx_extract_workspace_bytes(n_graphs));
    return ZX_ECAPACITY;
  }
  std::vector<ExEntry> tab((size_t)n_graphs);
  int64_t poff = 0;
  int64_t lds = 0;
  for (int i = 0; i < n_graphs; ++i) {
    ZX_CHECK_ARG(graphs[i], "null graph %d", i);
    const int n_ext = graphs[i]->n + 2 * graphs[i]->n_in;
    if (n_ext > EX_MAXN || graphs[i]->n_out > EX_MAXN) {
      zx_set_error("graph %d has %d spiders, %d inputs and %d outputs; extraction takes n + 2 n_in <= %d "
                   "and n_out <= %d", i, graphs[i]->n, graphs[i]->n_in, graphs[i]->n_out, EX_MAXN, EX_MAXN);
      return ZX_ECAPACITY;
    }
    tab[i].arena = graphs[i]->arena;
    tab[i].gate_off = (int64_t)i * max_gates;
    tab[i].perm_off = poff;
    poff += graphs[i]->n_out;
    const int64_t b = ex_lds_bytes(n_ext, graphs[i]->n_out);
    lds = b > lds ? b : lds;
  }
  std::vector<uint8_t> head(sizeof(ExWs), 0);
  ZX_HIP(hipMemcpyAsync(ws, head.data(), head.size(), hipMemcpyHostToDevice, s));
  ZX_HIP(hipMemcpyAsync((uint8_t*)ws + sizeof(ExWs), tab.data(), tab.size() * sizeof(ExEntry),
                        hipMemcpyHostToDevice, s));
  ZX_HIP(hipStreamSynchronize(s));  // the host table is freed on return
  lds = (lds + 15) & ~int64_t(15);
  ZX_HIP(hipFuncSetAttribute((const void*)extract_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  const int grid = n_graphs < 2 * d->n_cu ? n_graphs : 2 * d->n_cu;
  hipLaunchKernelGGL(extract_kernel, dim3(grid), dim3(EX_BS), (size_t)lds, s, (ExWs*)ws,
                     (const ExEntry*)((uint8_t*)ws + sizeof(ExWs)), n_graphs, max_gates, gates, n_gates, perm,
                     status);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}
