// Generalised flow of graph-like diagrams on the GPU (the flow check that
// circuit extraction needs; the paper reduces diagrams and eliminates binary
// matrices over F2 but leaves extraction to the standard procedures).
//
// Layers (Mhalla and Perdrix, ICALP 2008): the output spiders form layer 0
// and are processed; the correctors are the processed spiders that carry no
// input.  A spider u not yet processed joins the next layer when some set K
// of correctors has odd neighbourhood, restricted to the unprocessed
// spiders, equal to {u}.  Those odd neighbourhoods are the row space of the
// correctors' adjacency rows restricted to the unprocessed columns, and e_u
// lies in a row space exactly when its reduced row echelon form holds the
// row e_u: so each layer is one Gauss-Jordan elimination, and the layer is
// the set of single-bit rows of the result (unique, as the reduced echelon
// form is).  A flow exists when every present spider gets a layer.
//
// One workgroup per diagram (a work queue over the batch), the matrix of
// corrector rows in LDS; the adjacency, alive mask and boundary tables are
// the CURRENT diagram of the arena.
#include "zx_internal.h"

namespace {

#define LDS __attribute__((address_space(3)))

constexpr int FL_BS = 256;
constexpr int FL_MAXN = 1024;  // spiders per diagram (the matrix is N x N bits in LDS)
constexpr int FL_NOKEY = 0x7fffffff;

struct FlowEntry {
  uint8_t* arena;
  int64_t layer_off;  // first entry of this diagram in the layer output
};

struct FlowWs {
  ZxWsHeader hdr;
  uint32_t next;
  uint32_t pad[63];
  // followed by FlowEntry[n_graphs]
};
static_assert(sizeof(FlowWs) % 256 == 0, "workspace header size");

struct FlowShared {
  int32_t idx, key, nc, nnew, any;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Gauss-Jordan of rows 0..nr-1 of M (W words each) into reduced row echelon
// form, whole workgroup; lw: leading word per row.  Returns the rank.
__device__ int block_rref(LDS uint64_t* M, int nr, int W, LDS int16_t* lw, LDS uint64_t* hit, FlowShared& sh) {
  const int tid = threadIdx.x;
  const int hw = (nr + 63) / 64;
  for (int r = tid; r < nr; r += FL_BS) lw[r] = 0;
  int cur = 0, cmin = 0;
  for (;;) {
    if (tid == 0) sh.key = FL_NOKEY;
    for (int j = tid; j < hw; j += FL_BS) hit[j] = 0;
    __syncthreads();
    for (int r = cur + tid; r < nr; r += FL_BS) {
      int j = lw[r];
      if (j < (cmin >> 6)) j = cmin >> 6;
      const LDS uint64_t* mr = M + (size_t)r * W;
      while (j < W && mr[j] == 0) ++j;
      lw[r] = (int16_t)j;
      if (j < W) atomicMin(&sh.key, ((64 * j + __builtin_ctzll(mr[j])) << 15) | r);
    }
    __syncthreads();
    const int mn = uni(sh.key);
    if (mn == FL_NOKEY) break;
    const int col = mn >> 15, r = mn & 0x7fff;
    if (r != cur) {
      for (int j = tid; j < W; j += FL_BS) {
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
    for (int p = tid; p < nr; p += FL_BS)
      if (p != cur && ((M[(size_t)p * W + (col >> 6)] >> (col & 63)) & 1))
        atomicOr((unsigned long long*)&hit[p >> 6], 1ull << (p & 63));
    __syncthreads();
    const LDS uint64_t* pr = M + (size_t)cur * W;
    for (int it = tid; it < nr * W; it += FL_BS) {
      const int p = it / W, j = it - p * W;
      if ((hit[p >> 6] >> (p & 63)) & 1) M[it] ^= pr[j];
    }
    __syncthreads();
    ++cur;
    cmin = col + 1;
  }
  __syncthreads();
  return cur;
}

__global__ __launch_bounds__(FL_BS) void gflow_kernel(FlowWs* ws, const FlowEntry* table, int32_t n_graphs,
                                                       int32_t* layers, int32_t* exists) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ FlowShared sh;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sh.idx = (int32_t)atomicAdd(&ws->next, 1u);
    __syncthreads();
    const int gi = uni(sh.idx);
    __syncthreads();
    if (gi >= n_graphs) break;
    uint8_t* arena = table[gi].arena;
    int32_t* layer = layers + table[gi].layer_off;
    const ZxHeader* h = (const ZxHeader*)arena;
    const int n = uni(h->n), W = uni(h->W), q_in = uni(h->n_in), q_out = uni(h->n_out);
    if (uni(h->magic) != ZX_MAGIC || n < 1 || n > FL_MAXN || W != (n + 63) / 64) {
      if (tid == 0) exists[gi] = ZX_ECAPACITY;  // layers left unwritten
      __syncthreads();
      continue;
    }
    const uint64_t* adj = (const uint64_t*)(arena + h->off_adj);
    const uint64_t* alive_g = (const uint64_t*)(arena + h->off_alive);
    const int32_t* ins = (const int32_t*)(arena + h->off_in);
    const int32_t* outs = (const int32_t*)(arena + h->off_out);
    // LDS: M (n x W) | processed | unprocessed | inputs | new layer | hit (W each) | corr | lw (n int16 each)
    LDS uint64_t* M = (LDS uint64_t*)smem;
    LDS uint64_t* proc = M + (size_t)n * W;
    LDS uint64_t* U = proc + W;
    LDS uint64_t* inm = U + W;
    LDS uint64_t* nw = inm + W;
    LDS uint64_t* hit = nw + W;
    LDS int16_t* corr = (LDS int16_t*)(hit + W);
    LDS int16_t* lw = corr + n;
    for (int j = tid; j < W; j += FL_BS) proc[j] = inm[j] = 0;
    for (int v = tid; v < n; v += FL_BS) layer[v] = -1;
    __syncthreads();
    for (int i = tid; i < q_in; i += FL_BS) {
      const int v = ins[i];
      atomicOr((unsigned long long*)&inm[v >> 6], 1ull << (v & 63));
    }
    for (int i = tid; i < q_out; i += FL_BS) {
      const int v = outs[i];
      atomicOr((unsigned long long*)&proc[v >> 6], 1ull << (v & 63));
      layer[v] = 0;
    }
    __syncthreads();
    // correctors: the outputs that carry no input, in output order
    if (tid == 0) {
      int nc = 0;
      for (int i = 0; i < q_out; ++i) {
        const int v = outs[i];
        if (!((inm[v >> 6] >> (v & 63)) & 1)) corr[nc++] = (int16_t)v;
      }
      sh.nc = nc;
    }
    __syncthreads();
    int k = 1;
    for (;;) {
      // unprocessed present spiders
      if (tid == 0) sh.any = 0;
      __syncthreads();
      for (int j = tid; j < W; j += FL_BS) {
        const uint64_t u = alive_g[j] & ~proc[j];
        U[j] = u;
        nw[j] = 0;
        if (u) sh.any = 1;
      }
      __syncthreads();
      const int nc = uni(sh.nc);
      if (!uni(sh.any) || nc == 0) break;
      for (int it = tid; it < nc * W; it += FL_BS) {
        const int r = it / W, j = it - r * W;
        M[it] = adj[(size_t)corr[r] * W + j] & U[j];
      }
      __syncthreads();
      const int rank = block_rref(M, nc, W, lw, hit, sh);
      // single-bit rows of the reduced form: the new layer
      if (tid == 0) sh.nnew = 0;
      __syncthreads();
      for (int r = tid; r < rank; r += FL_BS) {
        int pc = 0, at = -1;
        for (int j = 0; j < W && pc < 2; ++j) {
          const uint64_t x = M[(size_t)r * W + j];
          if (x) {
            pc += __popcll(x);
            at = 64 * j + __builtin_ctzll(x);
          }
        }
        if (pc == 1) {
          atomicOr((unsigned long long*)&nw[at >> 6], 1ull << (at & 63));
          atomicAdd(&sh.nnew, 1);
        }
      }
      __syncthreads();
      if (uni(sh.nnew) == 0) break;
      for (int j = tid; j < W; j += FL_BS) {
        uint64_t m = nw[j];
        proc[j] |= m;
        while (m) {
          const int b = __builtin_ctzll(m);
          m &= m - 1;
          layer[64 * j + b] = k;
        }
      }
      __syncthreads();
      // new correctors (ascending), those without an input
      if (tid == 0) {
        int nc2 = sh.nc;
        for (int j = 0; j < W; ++j) {
          uint64_t m = nw[j] & ~inm[j];
          while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            corr[nc2++] = (int16_t)(64 * j + b);
          }
        }
        sh.nc = nc2;
      }
      __syncthreads();
      ++k;
    }
    // a flow exists when every present spider is processed
    if (tid == 0) sh.any = 0;
    __syncthreads();
    for (int j = tid; j < W; j += FL_BS)
      if (alive_g[j] & ~proc[j]) sh.any = 1;
    __syncthreads();
    if (tid == 0) exists[gi] = sh.any ? 0 : 1;
    __syncthreads();
  }
}

__host__ __device__ inline int64_t flow_lds_bytes(int n) {
  const int64_t W = (n + 63) / 64;
  return (int64_t)n * W * 8 + 5 * W * 8 + 2 * (int64_t)n * 2 + 16;
}

}  // namespace

extern "C" size_t zx_gflow_workspace_bytes(int32_t n_graphs) {
  if (n_graphs < 0) return 0;
  return sizeof(FlowWs) + (((size_t)n_graphs * sizeof(FlowEntry) + 255) & ~size_t(255));
}

extern "C" zx_status zx_gflow(zx_graph* const* graphs, int32_t n_graphs, int32_t* layers, int32_t* exists, void* ws,
                              size_t ws_bytes, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(graphs && n_graphs > 0 && layers && exists && ws, "null argument");
  ZX_CHECK_ARG(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  if (ws_bytes < zx_gflow_workspace_bytes(n_graphs)) {
    zx_set_error("workspace %zu < %zu bytes", ws_bytes, zx_gflow_workspace_bytes(n_graphs));
    return ZX_ECAPACITY;
  }
  std::vector<FlowEntry> tab((size_t)n_graphs);
  int64_t off = 0;
  int max_n = 0;
  for (int i = 0; i < n_graphs; ++i) {
    ZX_CHECK_ARG(graphs[i], "null graph %d", i);
    if (graphs[i]->n > FL_MAXN) {
      zx_set_error("graph %d has %d spiders; the flow kernel takes up to %d", i, graphs[i]->n, FL_MAXN);
      return ZX_ECAPACITY;
    }
    tab[i].arena = graphs[i]->arena;
    tab[i].layer_off = off;
    off += graphs[i]->n;
    max_n = graphs[i]->n > max_n ? graphs[i]->n : max_n;
  }
  std::vector<uint8_t> head(sizeof(FlowWs), 0);
  ZX_HIP(hipMemcpyAsync(ws, head.data(), head.size(), hipMemcpyHostToDevice, s));
  ZX_HIP(hipMemcpyAsync((uint8_t*)ws + sizeof(FlowWs), tab.data(), tab.size() * sizeof(FlowEntry),
                        hipMemcpyHostToDevice, s));
  ZX_HIP(hipStreamSynchronize(s));  // the host table is freed on return
  const size_t lds = (size_t)flow_lds_bytes(max_n);
  ZX_HIP(hipFuncSetAttribute((const void*)gflow_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const ZxDevice* d = zx_device();
  if (!d) return ZX_EDEVICE;
  const int grid = n_graphs < 2 * d->n_cu ? n_graphs : 2 * d->n_cu;
  hipLaunchKernelGGL(gflow_kernel, dim3(grid), dim3(FL_BS), lds, s, (FlowWs*)ws,
                     (const FlowEntry*)((uint8_t*)ws + sizeof(FlowWs)), n_graphs, layers, exists);
  ZX_HIP(hipGetLastError());
  return ZX_OK;
}
