// Host runtime of libzx: error reporting, device properties, diagram arenas.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "zx_internal.h"

static thread_local char g_err[512];

void zx_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void zx_clear_error() { g_err[0] = 0; }

extern "C" const char* zx_last_error(void) { return g_err; }
extern "C" int32_t zx_version(void) { return ZX_ABI_VERSION; }

const ZxDevice* zx_device() {
  static ZxDevice devs[16];
  static bool init[16] = {false};
  int id = 0;
  if (hipGetDevice(&id) != hipSuccess || id < 0 || id >= 16) return nullptr;
  if (!init[id]) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, id) != hipSuccess) return nullptr;
    devs[id].id = id;
    devs[id].n_cu = p.multiProcessorCount;
    devs[id].lds_per_block = p.sharedMemPerBlock;
    snprintf(devs[id].name, sizeof(devs[id].name), "%s", p.gcnArchName);
    init[id] = true;
  }
  return &devs[id];
}

extern "C" zx_status zx_device_info(char* name, int32_t name_len, int32_t* n_cu) {
  const ZxDevice* d = zx_device();
  if (!d) {
    zx_set_error("no HIP device");
    return ZX_EDEVICE;
  }
  if (name && name_len > 0) snprintf(name, (size_t)name_len, "%s", d->name);
  if (n_cu) *n_cu = d->n_cu;
  return ZX_OK;
}

// ------------------------------------------------------------- arenas --

extern "C" size_t zx_graph_bytes(int32_t n, int32_t n_in, int32_t n_out) {
  if (n <= 0 || n_in < 0 || n_out < 0) return 0;
  return (size_t)zx_layout(n, n_in, n_out).bytes;
}

// Validate a diagram on the host and assemble its arena image (header,
// SOURCE and CURRENT sections, boundary tables, masks).  Bits at or beyond n,
// self loops, phases outside 0..7 and bad boundary ids are always rejected:
// the kernels index by spider id.  The O(n^2) symmetry test is optional.
// Validate a diagram and write its arena image into dst: the whole arena
// (source_only false, dst of the layout's bytes) or only the header and the
// SOURCE sections, which come first (source_only true, dst of off_adj bytes;
// a run from SOURCE initialises the rest).  L receives the layout.
zx_status zx_write_image(int32_t n, const uint64_t* adj_host, const int8_t* phase_host, const int32_t* in_spider,
                         int32_t n_in, const int32_t* out_spider, int32_t n_out, const uint8_t* bnd_is_h,
                         bool check_symmetry, int32_t n_params, const uint64_t* param_rows, bool source_only,
                         uint8_t* dst, size_t dst_bytes, ZxLayout* Lout) {
  ZX_CHECK_ARG(adj_host && phase_host, "null argument");
  ZX_CHECK_ARG(n > 0 && n <= (1 << 20), "n out of range: %d", n);
  ZX_CHECK_ARG(n_in >= 0 && n_out >= 0 && n_in + n_out <= n, "bad boundary counts");
  ZX_CHECK_ARG((n_in == 0 || in_spider) && (n_out == 0 || out_spider), "null boundary list");
  ZX_CHECK_ARG(n_params >= 0 && n_params <= ZX_MAX_PARAMS, "n_params %d not in 0..%d", n_params, ZX_MAX_PARAMS);
  ZX_CHECK_ARG(n_params == 0 || param_rows, "null parameter rows");
  ZX_CHECK_ARG(!source_only || n_params == 0, "parameters need the whole image");
  ZxLayout L = zx_layout(n, n_in, n_out, n_params);
  if (Lout) *Lout = L;
  const size_t need = source_only ? (size_t)L.off_adj : (size_t)L.bytes;
  ZX_CHECK_ARG(dst && dst_bytes >= need, "image buffer of %zu bytes < %zu", dst_bytes, need);
  const int pw = (n_params + 63) / 64;
  if (n_params % 64)
    for (int r = 0; r < n; ++r)
      ZX_CHECK_ARG((param_rows[(size_t)r * pw + pw - 1] >> (n_params % 64)) == 0,
                   "parameter bits beyond n_params in row %d", r);
  const int W = (n + 63) / 64;
  // validate on the host: symmetric, zero diagonal, no bits >= n, phases
  for (int r = 0; r < n; ++r) {
    const uint64_t* row = adj_host + (size_t)r * W;
    ZX_CHECK_ARG(!((row[r / 64] >> (r % 64)) & 1), "self loop at spider %d", r);
    if (n % 64) ZX_CHECK_ARG((row[W - 1] >> (n % 64)) == 0, "bits beyond n in row %d", r);
    ZX_CHECK_ARG(phase_host[r] >= 0 && phase_host[r] < 8, "phase of spider %d not in 0..7", r);
  }
  if (check_symmetry)
    for (int r = 0; r < n; ++r)
      for (int c = r + 1; c < n; ++c) {
        int a = (adj_host[(size_t)r * W + c / 64] >> (c % 64)) & 1;
        int b = (adj_host[(size_t)c * W + r / 64] >> (r % 64)) & 1;
        ZX_CHECK_ARG(a == b, "adjacency not symmetric at (%d,%d)", r, c);
      }
  std::vector<uint8_t> seen((size_t)n, 0);
  for (int i = 0; i < n_in + n_out; ++i) {
    int v = i < n_in ? in_spider[i] : out_spider[i - n_in];
    ZX_CHECK_ARG(v >= 0 && v < n, "boundary spider id %d out of range", v);
    ZX_CHECK_ARG(!seen[v], "spider %d carries two boundary wires", v);
    seen[v] = 1;
  }
  ZxHeader h;
  memset(&h, 0, sizeof(h));
  h.magic = ZX_MAGIC;
  h.n = n;
  h.n_in = n_in;
  h.n_out = n_out;
  h.W = W;
  h.rank = -1;
  h.n_alive = n;
  h.off_src_adj = L.off_src_adj;
  h.off_src_phase = L.off_src_phase;
  h.off_in = L.off_in;
  h.off_out = L.off_out;
  h.off_is_h = L.off_is_h;
  h.off_bndmask = L.off_bndmask;
  h.off_adj = L.off_adj;
  h.off_phase = L.off_phase;
  h.off_alive = L.off_alive;
  h.off_trace = L.off_trace;
  h.off_front = L.off_front;
  h.off_fpiv = L.off_fpiv;
  h.n_params = n_params;
  h.pw = pw;
  h.off_src_par = L.off_src_par;
  h.off_par = L.off_par;
  h.off_terms = L.off_terms;
  h.n_terms = 0;
  h.bytes = L.bytes;
  int64_t edges = 0;
  for (size_t i = 0; i < (size_t)n * W; ++i) edges += __builtin_popcountll(adj_host[i]);
  h.n_edges = edges / 2;
  // header and SOURCE sections (the gaps between them zeroed)
  memset(dst, 0, 256);
  memcpy(dst, &h, sizeof(h));
  memcpy(dst + L.off_src_adj, adj_host, (size_t)n * W * 8);
  memset(dst + L.off_src_phase, 0, (size_t)(L.off_in - L.off_src_phase));
  memcpy(dst + L.off_src_phase, phase_host, (size_t)n);
  memset(dst + L.off_in, 0, (size_t)(L.off_adj - L.off_in));
  if (n_in) memcpy(dst + L.off_in, in_spider, 4 * (size_t)n_in);
  if (n_out) memcpy(dst + L.off_out, out_spider, 4 * (size_t)n_out);
  if (bnd_is_h) memcpy(dst + L.off_is_h, bnd_is_h, (size_t)(n_in + n_out));
  uint64_t* bm = (uint64_t*)(dst + L.off_bndmask);
  for (int v = 0; v < n; ++v)
    if (seen[v]) bm[v / 64] |= (uint64_t)1 << (v % 64);
  if (source_only) return ZX_OK;
  // CURRENT sections: the diagram as given
  memset(dst + L.off_adj, 0, (size_t)(L.bytes - L.off_adj));
  memcpy(dst + L.off_adj, adj_host, (size_t)n * W * 8);
  memcpy(dst + L.off_phase, phase_host, (size_t)n);
  if (pw) {
    memcpy(dst + L.off_src_par, param_rows, (size_t)n * pw * 8);
    memcpy(dst + L.off_par, param_rows, (size_t)n * pw * 8);
  }
  uint64_t* al = (uint64_t*)(dst + L.off_alive);
  for (int v = 0; v < n; ++v) al[v / 64] |= (uint64_t)1 << (v % 64);
  int32_t* fp = (int32_t*)(dst + L.off_fpiv);
  for (int j = 0; j < n_out; ++j) fp[j] = -1;
  return ZX_OK;
}

zx_status zx_build_image(int32_t n, const uint64_t* adj_host, const int8_t* phase_host,
                         const int32_t* in_spider, int32_t n_in, const int32_t* out_spider,
                         int32_t n_out, const uint8_t* bnd_is_h, bool check_symmetry,
                         std::vector<uint8_t>& img, int32_t n_params, const uint64_t* param_rows) {
  ZX_CHECK_ARG(n > 0 && n <= (1 << 20), "n out of range: %d", n);
  ZX_CHECK_ARG(n_in >= 0 && n_out >= 0 && n_params >= 0 && n_params <= ZX_MAX_PARAMS, "bad sizes");
  img.assign((size_t)zx_layout(n, n_in, n_out, n_params).bytes, 0);
  return zx_write_image(n, adj_host, phase_host, in_spider, n_in, out_spider, n_out, bnd_is_h, check_symmetry,
                        n_params, param_rows, false, img.data(), img.size(), nullptr);
}

extern "C" size_t zx_graph_bytes_ex(int32_t n, int32_t n_in, int32_t n_out, int32_t n_params) {
  if (n <= 0 || n_in < 0 || n_out < 0 || n_params < 0 || n_params > ZX_MAX_PARAMS) return 0;
  return (size_t)zx_layout(n, n_in, n_out, n_params).bytes;
}

extern "C" zx_status zx_graph_create_ex(zx_graph** g, void* dev_arena, size_t arena_bytes, int32_t n,
                                        const uint64_t* adj_host, const int8_t* phase_host,
                                        const int32_t* in_spider, int32_t n_in,
                                        const int32_t* out_spider, int32_t n_out,
                                        const uint8_t* bnd_is_h, int32_t n_params,
                                        const uint64_t* param_rows, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g && dev_arena && adj_host && phase_host, "null argument");
  ZX_CHECK_ARG(n > 0 && n <= (1 << 20), "n out of range: %d", n);
  ZX_CHECK_ARG(n_in >= 0 && n_out >= 0 && n_in + n_out <= n, "bad boundary counts");
  ZX_CHECK_ARG((n_in == 0 || in_spider) && (n_out == 0 || out_spider), "null boundary list");
  ZX_CHECK_ARG(((uintptr_t)dev_arena & 255) == 0, "arena must be 256-byte aligned");
  ZX_CHECK_ARG(n_params >= 0 && n_params <= ZX_MAX_PARAMS, "n_params %d not in 0..%d", n_params, ZX_MAX_PARAMS);
  ZxLayout L = zx_layout(n, n_in, n_out, n_params);
  ZX_CHECK_ARG(arena_bytes >= (size_t)L.bytes, "arena too small: %zu < %lld", arena_bytes,
               (long long)L.bytes);
  std::vector<uint8_t> img;
  zx_status st = zx_build_image(n, adj_host, phase_host, in_spider, n_in, out_spider, n_out, bnd_is_h,
                                true, img, n_params, param_rows);
  if (st != ZX_OK) return st;
  const int W = (n + 63) / 64;
  ZX_HIP(hipMemcpyAsync(dev_arena, img.data(), img.size(), hipMemcpyHostToDevice, s));
  ZX_HIP(hipStreamSynchronize(s));  // the staging image is freed on return
  zx_graph* G = (zx_graph*)calloc(1, sizeof(zx_graph));
  if (!G) {
    zx_set_error("out of host memory");
    return ZX_ECAPACITY;
  }
  G->arena = (uint8_t*)dev_arena;
  G->bytes = arena_bytes;
  G->n = n;
  G->n_in = n_in;
  G->n_out = n_out;
  G->W = W;
  G->n_params = n_params;
  G->pw = (n_params + 63) / 64;
  G->L = L;
  *g = G;
  return ZX_OK;
}

extern "C" zx_status zx_graph_create(zx_graph** g, void* dev_arena, size_t arena_bytes, int32_t n,
                                     const uint64_t* adj_host, const int8_t* phase_host,
                                     const int32_t* in_spider, int32_t n_in,
                                     const int32_t* out_spider, int32_t n_out,
                                     const uint8_t* bnd_is_h, hipStream_t s) {
  return zx_graph_create_ex(g, dev_arena, arena_bytes, n, adj_host, phase_host, in_spider, n_in, out_spider,
                            n_out, bnd_is_h, 0, nullptr, s);
}

extern "C" zx_status zx_graph_attach(zx_graph** g, void* dev_arena, size_t arena_bytes) {
  zx_clear_error();
  ZX_CHECK_ARG(g && dev_arena, "null argument");
  ZxHeader h;
  ZX_HIP(hipMemcpy(&h, dev_arena, sizeof(h), hipMemcpyDeviceToHost));
  ZX_CHECK_ARG(h.magic == ZX_MAGIC, "arena not initialised by zx_graph_create");
  ZxLayout L = zx_layout(h.n, h.n_in, h.n_out, h.n_params);
  ZX_CHECK_ARG(arena_bytes >= (size_t)L.bytes, "arena too small");
  zx_graph* G = (zx_graph*)calloc(1, sizeof(zx_graph));
  if (!G) return ZX_ECAPACITY;
  G->arena = (uint8_t*)dev_arena;
  G->bytes = arena_bytes;
  G->n = h.n;
  G->n_in = h.n_in;
  G->n_out = h.n_out;
  G->W = h.W;
  G->n_params = h.n_params;
  G->pw = h.pw;
  G->L = L;
  *g = G;
  return ZX_OK;
}

extern "C" void zx_graph_destroy(zx_graph* g) { free(g); }
extern "C" void* zx_graph_arena(const zx_graph* g) { return g ? g->arena : nullptr; }

extern "C" zx_status zx_graph_read(const zx_graph* g, uint64_t* adj, int8_t* phase, uint64_t* alive,
                                   zx_graph_info* info, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g, "null graph");
  ZX_HIP(hipStreamSynchronize(s));
  const size_t aw = (size_t)g->n * g->W * 8;
  if (adj) ZX_HIP(hipMemcpy(adj, g->arena + g->L.off_adj, aw, hipMemcpyDeviceToHost));
  if (phase) ZX_HIP(hipMemcpy(phase, g->arena + g->L.off_phase, (size_t)g->n, hipMemcpyDeviceToHost));
  if (alive) ZX_HIP(hipMemcpy(alive, g->arena + g->L.off_alive, (size_t)g->W * 8, hipMemcpyDeviceToHost));
  if (info) {
    ZxHeader h;
    ZX_HIP(hipMemcpy(&h, g->arena, sizeof(h), hipMemcpyDeviceToHost));
    info->pow_sqrt2 = h.pow_sqrt2;
    info->phase8 = h.phase8;
    info->status = h.status;
    info->n = h.n;
    info->n_alive = h.n_alive;
    info->n_edges = h.n_edges;
    info->n_trace = h.n_trace;
    info->rounds = h.rounds;
    info->fill_in = h.fill_in;
    info->rank = h.rank;
    info->policy = h.policy_used;
    info->rowops = h.rowops;
  }
  return ZX_OK;
}

extern "C" zx_status zx_graph_read_trace(const zx_graph* g, int32_t* trace, int32_t cap,
                                         int32_t* n_trace, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g && n_trace, "null argument");
  ZX_HIP(hipStreamSynchronize(s));
  ZxHeader h;
  ZX_HIP(hipMemcpy(&h, g->arena, sizeof(h), hipMemcpyDeviceToHost));
  *n_trace = h.n_trace;
  int32_t cnt = h.n_trace < cap ? h.n_trace : cap;
  if (trace && cnt > 0)
    ZX_HIP(hipMemcpy(trace, g->arena + g->L.off_trace, (size_t)cnt * 16, hipMemcpyDeviceToHost));
  return ZX_OK;
}

extern "C" zx_status zx_graph_read_frontier(const zx_graph* g, uint64_t* rows, int32_t* pivots,
                                            hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g, "null graph");
  ZX_HIP(hipStreamSynchronize(s));
  if (rows && g->n_out)
    ZX_HIP(hipMemcpy(rows, g->arena + g->L.off_front, (size_t)g->n_out * g->W * 8,
                     hipMemcpyDeviceToHost));
  if (pivots && g->n_out)
    ZX_HIP(hipMemcpy(pivots, g->arena + g->L.off_fpiv, (size_t)g->n_out * 4, hipMemcpyDeviceToHost));
  return ZX_OK;
}

extern "C" zx_status zx_graph_read_params(const zx_graph* g, uint64_t* rows, int32_t* n_terms, int32_t* k_ab,
                                          uint64_t* u, uint64_t* v, int32_t cap, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g, "null graph");
  ZX_HIP(hipStreamSynchronize(s));
  const int pw = g->pw;
  if (rows && pw)
    ZX_HIP(hipMemcpy(rows, g->arena + g->L.off_par, (size_t)g->n * pw * 8, hipMemcpyDeviceToHost));
  int32_t nt = 0;
  if (pw) ZX_HIP(hipMemcpy(&nt, g->arena + offsetof(ZxHeader, n_terms), 4, hipMemcpyDeviceToHost));
  if (n_terms) *n_terms = nt;
  const int cnt = nt < cap ? nt : cap;
  if (cnt > 0 && (k_ab || u || v)) {
    const int64_t tb = zx_term_bytes(pw);
    std::vector<uint8_t> buf((size_t)cnt * tb);
    ZX_HIP(hipMemcpy(buf.data(), g->arena + g->L.off_terms, buf.size(), hipMemcpyDeviceToHost));
    for (int t = 0; t < cnt; ++t) {
      const uint8_t* e = buf.data() + (size_t)t * tb;
      const ZxTermHead* hd = (const ZxTermHead*)e;
      if (k_ab) {
        k_ab[2 * t] = hd->k_alpha;
        k_ab[2 * t + 1] = hd->k_beta;
      }
      if (u) memcpy(u + (size_t)t * pw, e + 16, (size_t)pw * 8);
      if (v) memcpy(v + (size_t)t * pw, e + 16 + 8 * pw, (size_t)pw * 8);
    }
  }
  return ZX_OK;
}

extern "C" zx_status zx_graph_status(const zx_graph* g, hipStream_t s) {
  zx_clear_error();
  ZX_CHECK_ARG(g, "null graph");
  ZX_HIP(hipStreamSynchronize(s));
  int32_t st = 0;
  ZX_HIP(hipMemcpy(&st, g->arena + offsetof(ZxHeader, status), 4, hipMemcpyDeviceToHost));
  return st;
}
