// Serving loop: admission into a device pool, continuous batching of
// simplification requests, result harvest.  Host code plus one small
// result-gather kernel; the simplification itself is the persistent batch
// kernel of graph.hip.
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include "zx_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Per-request summary gathered from the arena headers after a batch.
struct ResDev {
  int32_t status, n_alive, rounds, n_trace, rank, phase8;
  int64_t n_edges, rowops, pow_sqrt2, fill_in;
};

__global__ void gather_kernel(uint8_t* const* table, int32_t n, ResDev* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const ZxHeader* h = (const ZxHeader*)table[i];
  ResDev r;
  r.status = h->status;
  r.n_alive = h->n_alive;
  r.rounds = h->rounds;
  r.n_trace = h->n_trace;
  r.rank = h->rank;
  r.phase8 = h->phase8;
  r.n_edges = h->n_edges;
  r.rowops = h->rowops;
  r.pow_sqrt2 = h->pow_sqrt2;
  r.fill_in = h->fill_in;
  out[i] = r;
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class PoolAlloc {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Req {
  int64_t ticket, tag;
  uint8_t* arena;
  size_t off, bytes;
  int32_t n;
  double t_submit, t_launch;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

constexpr int kSlots = 4;          // batches in flight at once
constexpr int kLargeSlots = 2;     // of which at most this many hold large requests
constexpr int32_t kLargeN = 1024;  // requests above this many spiders batch apart

// One batch in flight: its control data (device, from the pool), staging
// (pinned host), stream and completion event.
struct Slot {
  void* queue;
  uint8_t** table_dev;
  ResDev* res_dev;
  uint8_t** table_host;
  ResDev* res_host;
  hipStream_t stream;
  hipEvent_t done;
  bool large;
  std::vector<Req> running;
};

struct zx_server {
  uint8_t* pool;
  size_t pool_bytes;
  int32_t max_batch;
  uint32_t flags;
  zx_simplify_opts opts;
  int32_t max_n;
  uint8_t* arenas;  // request slices start here
  PoolAlloc alloc;
  Slot slot[kSlots];
  hipStream_t upload;
  std::deque<Req> pending;
  std::deque<zx_result> finished;
  int64_t next_ticket, submitted, refused, completed, batches;
};

static size_t slot_head_bytes(int32_t max_batch) {
  return ZX_QUEUE_BYTES + align256((size_t)max_batch * 8) + align256((size_t)max_batch * sizeof(ResDev));
}

extern "C" zx_status zx_server_create(zx_server** out, void* pool, size_t pool_bytes, int32_t max_batch,
                                      const zx_simplify_opts* o, uint32_t flags) {
  zx_clear_error();
  ZX_CHECK_ARG(out && pool, "null argument");
  ZX_CHECK_ARG(((uintptr_t)pool & 255) == 0, "pool must be 256-byte aligned");
  ZX_CHECK_ARG(max_batch > 0 && max_batch <= (1 << 20), "max_batch out of range");
  zx_simplify_opts def = {ZX_POLICY_GREEDY, 1, -1, 0, 0, 0, nullptr};
  if (!o) o = &def;
  ZX_CHECK_ARG(o->policy == ZX_POLICY_GREEDY || o->policy == ZX_POLICY_LEARNED, "unknown policy");
  if (o->policy == ZX_POLICY_LEARNED)
    ZX_CHECK_ARG(o->mlp && o->mlp->param && o->mlp->wbf16, "learned policy needs a network");
  const size_t per_slot = slot_head_bytes(max_batch);
  const size_t head = kSlots * per_slot;
  if (pool_bytes < head + 4096) {
    zx_set_error("pool too small for max_batch %d", max_batch);
    return ZX_ECAPACITY;
  }
  zx_server* S = new zx_server();
  S->pool = (uint8_t*)pool;
  S->pool_bytes = pool_bytes;
  S->max_batch = max_batch;
  S->flags = flags;
  S->opts = *o;
  S->opts.tune_id = -1;
  S->opts.max_rounds = 0;
  S->opts.flags = 0;
  S->max_n = zx_max_spiders(o->policy);
  S->arenas = S->pool + head;
  S->alloc.init(pool_bytes - head);
  S->upload = nullptr;
  S->next_ticket = S->submitted = S->refused = S->completed = S->batches = 0;
  hipError_t e = hipStreamCreateWithFlags(&S->upload, hipStreamNonBlocking);
  for (int i = 0; i < kSlots; ++i) {
    Slot& L = S->slot[i];
    uint8_t* base = S->pool + i * per_slot;
    L.queue = base;
    L.table_dev = (uint8_t**)(base + ZX_QUEUE_BYTES);
    L.res_dev = (ResDev*)(base + ZX_QUEUE_BYTES + align256((size_t)max_batch * 8));
    L.table_host = nullptr;
    L.res_host = nullptr;
    L.stream = nullptr;
    L.done = nullptr;
    L.large = false;
    if (e == hipSuccess) e = hipHostMalloc((void**)&L.table_host, (size_t)max_batch * 8, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&L.res_host, (size_t)max_batch * sizeof(ResDev), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    zx_set_error("server set-up failed: %s", hipGetErrorString(e));
    zx_server_destroy(S);
    return ZX_EDEVICE;
  }
  *out = S;
  return ZX_OK;
}

extern "C" void zx_server_destroy(zx_server* S) {
  if (!S) return;
  for (int i = 0; i < kSlots; ++i) {
    Slot& L = S->slot[i];
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.table_host) (void)hipHostFree(L.table_host);
    if (L.res_host) (void)hipHostFree(L.res_host);
  }
  if (S->upload) {
    (void)hipStreamSynchronize(S->upload);
    (void)hipStreamDestroy(S->upload);
  }
  delete S;
}

extern "C" zx_status zx_server_submit(zx_server* S, const zx_request* r, int64_t* ticket) {
  zx_clear_error();
  ZX_CHECK_ARG(S && r, "null argument");
  if (r->n > S->max_n) {
    zx_set_error("request of %d spiders exceeds the kernels' limit %d", r->n, S->max_n);
    return ZX_ECAPACITY;
  }
  std::vector<uint8_t> img;
  zx_status st = zx_build_image(r->n, r->adj, r->phase, r->inputs, r->n_in, r->outputs, r->n_out, r->bnd_is_h,
                                !(S->flags & ZX_SERVE_TRUSTED), img);
  if (st != ZX_OK) return st;
  const size_t bytes = align256(img.size());
  size_t off = 0;
  if (!S->alloc.alloc(bytes, &off)) {
    S->refused++;
    zx_set_error("pool full (%zu of %zu bytes in use)", S->alloc.used(), S->pool_bytes);
    return ZX_EBUSY;
  }
  uint8_t* arena = S->arenas + off;
  hipError_t e = hipMemcpyAsync(arena, img.data(), img.size(), hipMemcpyHostToDevice, S->upload);
  if (e == hipSuccess) e = hipStreamSynchronize(S->upload);
  if (e != hipSuccess) {
    S->alloc.release(off, bytes);
    zx_set_error("upload failed: %s", hipGetErrorString(e));
    return ZX_EDEVICE;
  }
  Req q;
  q.ticket = S->next_ticket++;
  q.tag = r->tag;
  q.arena = arena;
  q.off = off;
  q.bytes = bytes;
  q.n = r->n;
  q.t_submit = now_s();
  q.t_launch = 0;
  S->pending.push_back(q);
  S->submitted++;
  if (ticket) *ticket = q.ticket;
  return ZX_OK;
}

static void harvest(zx_server* S, Slot& L) {
  const double t = now_s();
  for (size_t i = 0; i < L.running.size(); ++i) {
    const Req& q = L.running[i];
    const ResDev& d = L.res_host[i];
    zx_result r;
    r.ticket = q.ticket;
    r.tag = q.tag;
    r.status = d.status;
    r.n_alive = d.n_alive;
    r.rounds = d.rounds;
    r.n_trace = d.n_trace;
    r.rank = d.rank;
    r.phase8 = d.phase8;
    r.n_edges = d.n_edges;
    r.rowops = d.rowops;
    r.pow_sqrt2 = d.pow_sqrt2;
    r.fill_in = d.fill_in;
    r.t_submit = q.t_submit;
    r.t_launch = q.t_launch;
    r.t_done = t;
    S->finished.push_back(r);
    S->alloc.release(q.off, q.bytes);
    S->completed++;
  }
  L.running.clear();
}

// Launch the oldest pending request's size class (up to max_batch of them,
// oldest first) into slot L.
static zx_status launch(zx_server* S, Slot& L, bool large) {
  L.running.clear();
  for (auto it = S->pending.begin(); it != S->pending.end() && (int32_t)L.running.size() < S->max_batch;) {
    if ((it->n > kLargeN) == large) {
      L.running.push_back(*it);
      it = S->pending.erase(it);
    } else {
      ++it;
    }
  }
  const size_t k = L.running.size();
  if (k == 0) return ZX_OK;
  L.large = large;
  // longest first inside the batch
  std::stable_sort(L.running.begin(), L.running.end(), [](const Req& a, const Req& b) { return a.n > b.n; });
  const double t = now_s();
  int32_t max_n = 0;
  for (size_t i = 0; i < k; ++i) {
    L.running[i].t_launch = t;
    L.table_host[i] = L.running[i].arena;
    max_n = std::max(max_n, L.running[i].n);
  }
  ZX_HIP(hipMemcpyAsync(L.table_dev, L.table_host, k * 8, hipMemcpyHostToDevice, L.stream));
  zx_status st = zx_launch_batch(L.table_dev, (int32_t)k, L.queue, max_n, &S->opts, L.stream);
  if (st != ZX_OK) return st;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, L.stream, L.table_dev,
                     (int32_t)k, L.res_dev);
  ZX_HIP(hipGetLastError());
  ZX_HIP(hipMemcpyAsync(L.res_host, L.res_dev, k * sizeof(ResDev), hipMemcpyDeviceToHost, L.stream));
  ZX_HIP(hipEventRecord(L.done, L.stream));
  S->batches++;
  return ZX_OK;
}

extern "C" zx_status zx_server_poll(zx_server* S, zx_result* out, int32_t max, int32_t* n_out) {
  zx_clear_error();
  ZX_CHECK_ARG(S && max >= 0 && (max == 0 || out), "bad argument");
  int busy_large = 0;
  for (int i = 0; i < kSlots; ++i) {
    Slot& L = S->slot[i];
    if (L.running.empty()) continue;
    const hipError_t q = hipEventQuery(L.done);
    if (q == hipSuccess) {
      harvest(S, L);
    } else if (q != hipErrorNotReady) {
      zx_set_error("batch failed: %s", hipGetErrorString(q));
      return ZX_EDEVICE;
    } else if (L.large) {
      busy_large++;
    }
  }
  // fill free slots: the class of the oldest pending request first; large
  // requests never take more than kLargeSlots slots
  for (int i = 0; i < kSlots && !S->pending.empty(); ++i) {
    Slot& L = S->slot[i];
    if (!L.running.empty()) continue;
    bool want_large = S->pending.front().n > kLargeN;
    if (want_large && busy_large >= kLargeSlots) {
      want_large = false;
      bool any_small = false;
      for (const Req& q : S->pending)
        if (q.n <= kLargeN) {
          any_small = true;
          break;
        }
      if (!any_small) break;
    }
    zx_status st = launch(S, L, want_large);
    if (st != ZX_OK) return st;
    if (want_large) busy_large++;
  }
  int32_t m = 0;
  while (m < max && !S->finished.empty()) {
    out[m++] = S->finished.front();
    S->finished.pop_front();
  }
  if (n_out) *n_out = m;
  return ZX_OK;
}

extern "C" zx_status zx_server_stats_read(const zx_server* S, zx_server_stats* st) {
  zx_clear_error();
  ZX_CHECK_ARG(S && st, "null argument");
  int64_t running = 0;
  for (int i = 0; i < kSlots; ++i) running += (int64_t)S->slot[i].running.size();
  st->submitted = S->submitted;
  st->refused = S->refused;
  st->completed = S->completed;
  st->batches = S->batches;
  st->pending = (int64_t)S->pending.size();
  st->running = running;
  st->pool_bytes = S->pool_bytes;
  st->pool_used = S->alloc.used();
  st->pool_peak = S->alloc.peak();
  return ZX_OK;
}
