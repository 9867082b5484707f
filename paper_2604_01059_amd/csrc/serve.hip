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

struct zx_server {
  uint8_t* pool;
  size_t pool_bytes;
  int32_t max_batch;
  uint32_t flags;
  zx_simplify_opts opts;
  int32_t max_n;
  // control data at the head of the pool
  void* queue;
  uint8_t** table_dev;
  ResDev* res_dev;
  uint8_t* arenas;  // request slices start here
  PoolAlloc alloc;
  // pinned host staging
  uint8_t** table_host;
  ResDev* res_host;
  hipStream_t compute, upload;
  hipEvent_t done;
  std::deque<Req> pending;
  std::vector<Req> running;
  std::deque<zx_result> finished;
  int64_t next_ticket, submitted, refused, completed, batches;
};

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
  const size_t head = ZX_QUEUE_BYTES + align256((size_t)max_batch * 8) + align256((size_t)max_batch * sizeof(ResDev));
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
  S->queue = S->pool;
  S->table_dev = (uint8_t**)(S->pool + ZX_QUEUE_BYTES);
  S->res_dev = (ResDev*)(S->pool + ZX_QUEUE_BYTES + align256((size_t)max_batch * 8));
  S->arenas = S->pool + head;
  S->alloc.init(pool_bytes - head);
  S->table_host = nullptr;
  S->res_host = nullptr;
  S->compute = S->upload = nullptr;
  S->done = nullptr;
  S->next_ticket = S->submitted = S->refused = S->completed = S->batches = 0;
  hipError_t e = hipHostMalloc((void**)&S->table_host, (size_t)max_batch * 8, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->res_host, (size_t)max_batch * sizeof(ResDev), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->compute, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->upload, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->done, hipEventDisableTiming);
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
  if (S->compute) (void)hipStreamSynchronize(S->compute);
  if (S->upload) (void)hipStreamSynchronize(S->upload);
  if (S->done) (void)hipEventDestroy(S->done);
  if (S->compute) (void)hipStreamDestroy(S->compute);
  if (S->upload) (void)hipStreamDestroy(S->upload);
  if (S->table_host) (void)hipHostFree(S->table_host);
  if (S->res_host) (void)hipHostFree(S->res_host);
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

static zx_status harvest(zx_server* S) {
  const double t = now_s();
  for (size_t i = 0; i < S->running.size(); ++i) {
    const Req& q = S->running[i];
    const ResDev& d = S->res_host[i];
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
  S->running.clear();
  return ZX_OK;
}

static zx_status launch(zx_server* S) {
  const size_t k = std::min(S->pending.size(), (size_t)S->max_batch);
  S->running.assign(S->pending.begin(), S->pending.begin() + (long)k);
  S->pending.erase(S->pending.begin(), S->pending.begin() + (long)k);
  // longest first inside the batch
  std::stable_sort(S->running.begin(), S->running.end(), [](const Req& a, const Req& b) { return a.n > b.n; });
  const double t = now_s();
  int32_t max_n = 0;
  for (size_t i = 0; i < k; ++i) {
    S->running[i].t_launch = t;
    S->table_host[i] = S->running[i].arena;
    max_n = std::max(max_n, S->running[i].n);
  }
  ZX_HIP(hipMemcpyAsync(S->table_dev, S->table_host, k * 8, hipMemcpyHostToDevice, S->compute));
  zx_status st = zx_launch_batch(S->table_dev, (int32_t)k, S->queue, max_n, &S->opts, S->compute);
  if (st != ZX_OK) return st;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, S->compute, S->table_dev,
                     (int32_t)k, S->res_dev);
  ZX_HIP(hipGetLastError());
  ZX_HIP(hipMemcpyAsync(S->res_host, S->res_dev, k * sizeof(ResDev), hipMemcpyDeviceToHost, S->compute));
  ZX_HIP(hipEventRecord(S->done, S->compute));
  S->batches++;
  return ZX_OK;
}

extern "C" zx_status zx_server_poll(zx_server* S, zx_result* out, int32_t max, int32_t* n_out) {
  zx_clear_error();
  ZX_CHECK_ARG(S && max >= 0 && (max == 0 || out), "bad argument");
  if (!S->running.empty()) {
    const hipError_t q = hipEventQuery(S->done);
    if (q == hipSuccess) {
      zx_status st = harvest(S);
      if (st != ZX_OK) return st;
    } else if (q != hipErrorNotReady) {
      zx_set_error("batch failed: %s", hipGetErrorString(q));
      return ZX_EDEVICE;
    }
  }
  if (S->running.empty() && !S->pending.empty()) {
    zx_status st = launch(S);
    if (st != ZX_OK) return st;
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
  st->submitted = S->submitted;
  st->refused = S->refused;
  st->completed = S->completed;
  st->batches = S->batches;
  st->pending = (int64_t)S->pending.size();
  st->running = (int64_t)S->running.size();
  st->pool_bytes = S->pool_bytes;
  st->pool_used = S->alloc.used();
  st->pool_peak = S->alloc.peak();
  return ZX_OK;
}
