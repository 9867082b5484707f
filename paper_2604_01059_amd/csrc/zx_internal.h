// Internal definitions shared by the libzx sources: arena layout, error
// plumbing, small device helpers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <vector>

#include "../../include/zx.h"

#define ZX_ABI_VERSION 100

// ---------------------------------------------------------------- arena --
// One diagram arena: a 256-byte header followed by 256-byte aligned sections.
// Offsets are relative to the arena base.
#define ZX_MAGIC 0x5A584731  // "ZXG1"

struct ZxHeader {
  int32_t magic;
  int32_t n, n_in, n_out;
  int32_t W;            // words per adjacency row
  int32_t status;       // sticky zx_status
  int32_t n_trace;
  int32_t rounds;
  int32_t rank;         // frontier rank, -1 before extraction
  int32_t n_alive;
  int64_t pow_sqrt2;
  int32_t phase8;
  int32_t pad0;
  int64_t fill_in;
  int64_t rowops;
  int64_t n_edges;
  // section offsets
  int64_t off_src_adj, off_src_phase, off_in, off_out, off_is_h, off_bndmask;
  int64_t off_adj, off_phase, off_alive, off_trace, off_front, off_fpiv;
  int64_t bytes;
  // parameterized Pauli spiders (0 parameters: sections of size 0)
  int32_t n_params, pw;  // parameters, 64-bit words per parameter row
  int64_t off_src_par, off_par, off_terms;
  int32_t n_terms;       // phase-pair terms recorded
  int32_t policy_used;   // schedule of the CURRENT diagram: ZX_POLICY_GREEDY or ZX_POLICY_LEARNED
  int64_t reserved[2];
};
static_assert(sizeof(ZxHeader) <= 256, "header fits 256 bytes");

// A recorded phase-pair term: head, then u[pw], v[pw] words.
struct ZxTermHead {
  int32_t k_alpha, k_beta, pad0, pad1;
};
static inline __host__ __device__ int64_t zx_term_bytes(int pw) { return 16 + 16 * (int64_t)pw; }
constexpr int32_t ZX_MAX_PARAMS = 4096;

static inline __host__ __device__ int64_t zx_align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct ZxLayout {
  int64_t off_src_adj, off_src_phase, off_in, off_out, off_is_h, off_bndmask;
  int64_t off_adj, off_phase, off_alive, off_trace, off_front, off_fpiv;
  int64_t off_src_par, off_par, off_terms, bytes;
};

static inline __host__ __device__ ZxLayout zx_layout(int32_t n, int32_t n_in, int32_t n_out,
                                                     int32_t n_params = 0) {
  ZxLayout L;
  int64_t W = (n + 63) / 64;
  int64_t o = 256;
  L.off_src_adj = o;   o = zx_align256(o + (int64_t)n * W * 8);
  L.off_src_phase = o; o = zx_align256(o + n);
  L.off_in = o;        o = zx_align256(o + 4 * (int64_t)n_in);
  L.off_out = o;       o = zx_align256(o + 4 * (int64_t)n_out);
  L.off_is_h = o;      o = zx_align256(o + n_in + n_out);
  L.off_bndmask = o;   o = zx_align256(o + W * 8);
  L.off_adj = o;       o = zx_align256(o + (int64_t)n * W * 8);
  L.off_phase = o;     o = zx_align256(o + n);
  L.off_alive = o;     o = zx_align256(o + W * 8);
  L.off_trace = o;     o = zx_align256(o + 16 * (int64_t)(n + 1));
  L.off_front = o;     o = zx_align256(o + (int64_t)n_out * W * 8);
  L.off_fpiv = o;      o = zx_align256(o + 4 * (int64_t)(n_out + 1));
  // parameter sections last, so that a diagram without parameters keeps the
  // layout (and size) it had before they existed
  const int64_t pw = (n_params + 63) / 64;
  L.off_src_par = o;   o = zx_align256(o + (int64_t)n * pw * 8);
  L.off_par = o;       o = zx_align256(o + (int64_t)n * pw * 8);
  L.off_terms = o;     o = zx_align256(o + (pw ? (int64_t)(n + 1) * zx_term_bytes((int)pw) : 0));
  L.bytes = o;
  return L;
}

// Host handle of a diagram arena.
struct zx_graph {
  uint8_t* arena;  // device
  size_t bytes;
  int32_t n, n_in, n_out, W;
  int32_t n_params, pw;
  ZxLayout L;
};

// ------------------------------------------------------------ errors --
void zx_set_error(const char* fmt, ...);

// Host validation + arena image of a diagram (runtime.hip).
zx_status zx_write_image(int32_t n, const uint64_t* adj_host, const int8_t* phase_host, const int32_t* in_spider,
                         int32_t n_in, const int32_t* out_spider, int32_t n_out, const uint8_t* bnd_is_h,
                         bool check_symmetry, int32_t n_params, const uint64_t* param_rows, bool source_only,
                         uint8_t* dst, size_t dst_bytes, ZxLayout* L);
zx_status zx_build_image(int32_t n, const uint64_t* adj_host, const int8_t* phase_host,
                         const int32_t* in_spider, int32_t n_in, const int32_t* out_spider,
                         int32_t n_out, const uint8_t* bnd_is_h, bool check_symmetry,
                         std::vector<uint8_t>& img, int32_t n_params = 0,
                         const uint64_t* param_rows = nullptr);

// Largest diagram the simplify kernels take with this policy (graph.hip).
int32_t zx_max_spiders(int32_t policy);

// Serving ring (graph.hip runs the kernel, serve.hip the host side).  The
// host appends arena pointers to `entries` and then advances `tail`; resident
// workgroups claim entries in order through `head`, simplify the diagram and
// write its summary to `res` and then `done` = sequence number + 1.  entries,
// tail, stop, done and res are in host memory that both sides see coherently;
// head is device memory.  Every workgroup exits when `stop` is set or after
// idle_ticks (100 MHz clock) without work.
struct ZxServeRes {
  int32_t status, n_alive, rounds, n_trace, rank, phase8;
  int64_t n_edges, rowops, pow_sqrt2, fill_in;
  int32_t policy, pad;
  uint64_t t_claim, t_end;  // device wall clock: request claimed, result written
};
struct ZxServeArgs {
  uint64_t* entries;
  int64_t* tail;
  int32_t* stop;
  int64_t* done;
  ZxServeRes* res;
  int64_t* head;
  int64_t cap;  // power of two
  uint64_t idle_ticks;
  int32_t extract;
  int32_t policy;
  const zx_mlp* mlp;
  int32_t fallback;  // learned policy: keep the greedy result where it is cheaper
  int32_t pad;
  const uint64_t* stage;        // per entry: staged header + SOURCE sections (host memory)
  const uint64_t* stage_bytes;  // per entry: bytes to copy into the arena
  void* team;                   // device: the pool's team area (boards of large requests), or null
};
// The serving pool's team area (large requests share their round updates
// with idle workgroups): its size, and its initialisation on s.
size_t zx_team_area_bytes();
zx_status zx_team_area_init(void* area, hipStream_t s);
// Launch the resident serving kernel on s (grid: one workgroup per CU).
zx_status zx_launch_serve(const ZxServeArgs& a, hipStream_t s);
void zx_clear_error();

#define ZX_CHECK_ARG(cond, ...)            \
  do {                                     \
    if (!(cond)) {                         \
      zx_set_error(__VA_ARGS__);           \
      return ZX_EINVAL;                    \
    }                                      \
  } while (0)

#define ZX_HIP(call)                                                       \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      zx_set_error("%s failed: %s", #call, hipGetErrorString(e_));         \
      return ZX_EDEVICE;                                                   \
    }                                                                      \
  } while (0)

// device properties cached per device
struct ZxDevice {
  int id;
  int n_cu;
  size_t lds_per_block;  // max dynamic LDS per workgroup
  char name[128];
};
const ZxDevice* zx_device();

// Commutation table on the matrix cores (gf2mm.hip); zx_pauli_commute picks
// it from this many strings up unless a flag forces a variant.
constexpr int64_t ZX_PAULI_MFMA_MIN = 1024;
zx_status zx_pauli_commute_mfma(const uint64_t* X, const uint64_t* Z, int64_t n, int32_t n_qubits, int64_t ldq,
                                uint64_t* C, int64_t ldc, hipStream_t s);

// ---------------------------------------------------- device helpers --
// Device-side status update: keep the first error.
__device__ static inline void zx_dev_fail(int32_t* status, int32_t code) {
  atomicCAS(status, 0, code);
}

// Sticky status word of a workspace (first 256 bytes of every workspace).
struct ZxWsHeader {
  int32_t status;
  int32_t pad[63];
};
