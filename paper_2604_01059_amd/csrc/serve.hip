// Serving loop (host side): admission into a device pool, a request ring in
// coherent host memory read by the resident serving kernel of graph.hip,
// completion by per-entry flags, result harvest.  A request's header and
// SOURCE sections are written into pinned, coherent staging memory; the
// workgroup that claims the request copies them into its device arena, so
// a submission issues no copy and no synchronisation.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>
#include "zx_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
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
  size_t off, bytes;    // device pool slice
  size_t soff, sbytes;  // staging slice
  int32_t n;
  double t_submit;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace {

constexpr int64_t kRing = 1 << 16;               // ring entries (power of two)
constexpr uint64_t kIdleTicks = 50ull * 100000;  // 50 ms at 100 MHz

// Coherent host memory shared with the serving kernel.
struct Shared_ {
  uint64_t entries[kRing];
  uint64_t stage[kRing];        // staged header + SOURCE sections of the entry
  uint64_t stage_bytes[kRing];  // bytes to copy (a multiple of 256)
  int64_t done[kRing];
  ZxServeRes res[kRing];
  int64_t tail;
  int32_t stop;
  int32_t pad;
};

}  // namespace

struct zx_server {
  uint8_t* pool;
  size_t pool_bytes;
  uint32_t flags;
  zx_simplify_opts opts;
  int32_t max_n;
  int64_t* head;    // device, at the head of the pool
  uint8_t* team;    // device, the team area after the control block (null in small pools)
  uint8_t* arenas;  // request slices start here
  PoolAlloc alloc;
  uint8_t* staging;  // pinned, coherent host memory
  size_t staging_bytes;
  PoolAlloc salloc;
  Shared_* sh;      // coherent host memory
  hipStream_t stream, upload;
  hipEvent_t ended;  // recorded after each launch of the serving kernel
  bool running;
  int64_t next_seq;  // = tail
  std::unordered_map<int64_t, Req> inflight;  // by sequence number
  int64_t oldest;  // smallest sequence number not yet harvested
  std::deque<zx_result> finished;
  int64_t submitted, refused, completed, launches;
  double wall_hz;  // device wall clock (s_memrealtime) frequency
};

static zx_status relaunch(zx_server* S) {
  ZxServeArgs a;
  a.entries = S->sh->entries;
  a.tail = &S->sh->tail;
  a.stop = &S->sh->stop;
  a.done = S->sh->done;
  a.res = S->sh->res;
  a.head = S->head;
  a.cap = kRing;
  a.idle_ticks = kIdleTicks;
  a.extract = S->opts.extract;
  a.policy = S->opts.policy;
  a.mlp = S->opts.mlp;
  a.fallback = (S->opts.policy == ZX_POLICY_LEARNED && (S->opts.flags & ZX_FALLBACK)) ? 1 : 0;
  a.stage = S->sh->stage;
  a.stage_bytes = S->sh->stage_bytes;
  a.pad = 0;
  a.team = S->team;
  zx_status st = zx_launch_serve(a, S->stream);
  if (st != ZX_OK) return st;
  ZX_HIP(hipEventRecord(S->ended, S->stream));
  S->running = true;
  S->launches++;
  return ZX_OK;
}

extern "C" zx_status zx_server_create(zx_server** out, void* pool, size_t pool_bytes, int32_t max_batch,
                                      const zx_simplify_opts* o, uint32_t flags) {
  zx_clear_error();
  ZX_CHECK_ARG(out && pool, "null argument");
  ZX_CHECK_ARG(((uintptr_t)pool & 255) == 0, "pool must be 256-byte aligned");
  ZX_CHECK_ARG(max_batch > 0, "max_batch must be positive");
  zx_simplify_opts def = {ZX_POLICY_GREEDY, 1, -1, 0, 0, 0, nullptr};
  if (!o) o = &def;
  ZX_CHECK_ARG(o->policy == ZX_POLICY_GREEDY || o->policy == ZX_POLICY_LEARNED, "unknown policy");
  if (o->policy == ZX_POLICY_LEARNED)
    ZX_CHECK_ARG(o->mlp && o->mlp->param && o->mlp->wbf16, "learned policy needs a network");
  // control block (256 bytes), then, in a pool that can hold large requests
  // (64 MiB and more), the team area through which they share their rounds
  const size_t team_bytes = pool_bytes >= ((size_t)64 << 20) ? align256(zx_team_area_bytes()) : 0;
  const size_t head = 256 + team_bytes;
  if (pool_bytes < head + 4096) {
    zx_set_error("pool too small");
    return ZX_ECAPACITY;
  }
  zx_server* S = new zx_server();
  S->pool = (uint8_t*)pool;
  S->pool_bytes = pool_bytes;
  S->flags = flags;
  S->opts = *o;
  S->opts.tune_id = -1;
  S->opts.max_rounds = 0;
  S->opts.flags = o->flags & ZX_FALLBACK;
  // the serving kernel runs 64 KiB workgroups; with the greedy fallback a
  // request beyond the learned policy's budget runs greedy
  const bool learned_only = o->policy == ZX_POLICY_LEARNED && !(o->flags & ZX_FALLBACK);
  S->max_n = std::min(zx_max_spiders(learned_only ? ZX_POLICY_LEARNED : ZX_POLICY_GREEDY), learned_only ? 4096 : 8192);
  S->wall_hz = 1e8;
  {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
        khz > 0)
      S->wall_hz = 1e3 * khz;
  }
  S->head = (int64_t*)S->pool;
  S->arenas = S->pool + head;
  S->alloc.init(pool_bytes - head);
  S->staging = nullptr;
  S->staging_bytes = std::min(pool_bytes, (size_t)1 << 30);
  S->salloc.init(S->staging_bytes);
  S->sh = nullptr;
  S->stream = S->upload = nullptr;
  S->ended = nullptr;
  S->running = false;
  S->next_seq = 0;
  S->oldest = 0;
  S->submitted = S->refused = S->completed = S->launches = 0;
  hipError_t e = hipHostMalloc((void**)&S->sh, sizeof(Shared_), hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&S->staging, S->staging_bytes, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->upload, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ended, hipEventDisableTiming);
  // control block: head, device copy of the tail, host-poller flag
  if (e == hipSuccess) e = hipMemsetAsync(S->head, 0, 256, S->stream);
  if (e == hipSuccess && team_bytes && zx_team_area_init(S->pool + 256, S->stream) != ZX_OK)
    e = hipErrorLaunchFailure;
  S->team = team_bytes ? S->pool + 256 : nullptr;
  if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) {
    zx_set_error("server set-up failed: %s", hipGetErrorString(e));
    zx_server_destroy(S);
    return ZX_EDEVICE;
  }
  memset(S->sh, 0, sizeof(Shared_));
  *out = S;
  return ZX_OK;
}

extern "C" void zx_server_destroy(zx_server* S) {
  if (!S) return;
  if (S->sh) __atomic_store_n(&S->sh->stop, 1, __ATOMIC_RELEASE);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  if (S->upload) (void)hipStreamSynchronize(S->upload);
  if (S->ended) (void)hipEventDestroy(S->ended);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  if (S->upload) (void)hipStreamDestroy(S->upload);
  if (S->sh) (void)hipHostFree(S->sh);
  if (S->staging) (void)hipHostFree(S->staging);
  delete S;
}

extern "C" zx_status zx_server_submit(zx_server* S, const zx_request* r, int64_t* ticket) {
  zx_clear_error();
  ZX_CHECK_ARG(S && r, "null argument");
  if (r->n > S->max_n) {
    zx_set_error("request of %d spiders exceeds the serving limit %d", r->n, S->max_n);
    return ZX_ECAPACITY;
  }
  if (S->next_seq - S->oldest >= kRing) {
    S->refused++;
    zx_set_error("request ring full");
    return ZX_EBUSY;
  }
  ZX_CHECK_ARG(r->n > 0 && r->n_in >= 0 && r->n_out >= 0 && r->n_in + r->n_out <= r->n, "bad request sizes");
  const ZxLayout L = zx_layout(r->n, r->n_in, r->n_out);
  const size_t bytes = align256((size_t)L.bytes);
  // the kernel loads its working state from the header and SOURCE sections,
  // which come first in the arena: only they are staged
  const size_t sbytes = align256((size_t)L.off_adj);
  if (sbytes > S->staging_bytes) {
    zx_set_error("request of %zu staged bytes exceeds the staging area of %zu", sbytes, S->staging_bytes);
    return ZX_ECAPACITY;
  }
  size_t off = 0, soff = 0;
  if (!S->alloc.alloc(bytes, &off)) {
    S->refused++;
    zx_set_error("pool full (%zu of %zu bytes in use)", S->alloc.used(), S->pool_bytes);
    return ZX_EBUSY;
  }
  if (!S->salloc.alloc(sbytes, &soff)) {
    S->alloc.release(off, bytes);
    S->refused++;
    zx_set_error("staging full (%zu of %zu bytes in use)", S->salloc.used(), S->staging_bytes);
    return ZX_EBUSY;
  }
  zx_status st = zx_write_image(r->n, r->adj, r->phase, r->inputs, r->n_in, r->outputs, r->n_out, r->bnd_is_h,
                                !(S->flags & ZX_SERVE_TRUSTED), 0, nullptr, true, S->staging + soff, sbytes,
                                nullptr);
  if (st != ZX_OK) {
    S->alloc.release(off, bytes);
    S->salloc.release(soff, sbytes);
    return st;
  }
  uint8_t* arena = S->arenas + off;
  const int64_t seq = S->next_seq++;
  Req q;
  q.ticket = seq;
  q.tag = r->tag;
  q.arena = arena;
  q.off = off;
  q.bytes = bytes;
  q.soff = soff;
  q.sbytes = sbytes;
  q.n = r->n;
  q.t_submit = now_s();
  S->inflight.emplace(seq, q);
  const int64_t slot = seq & (kRing - 1);
  __atomic_store_n(&S->sh->done[slot], (int64_t)0, __ATOMIC_RELAXED);
  __atomic_store_n(&S->sh->entries[slot], (uint64_t)(uintptr_t)arena, __ATOMIC_RELAXED);
  __atomic_store_n(&S->sh->stage[slot], (uint64_t)(uintptr_t)(S->staging + soff), __ATOMIC_RELAXED);
  __atomic_store_n(&S->sh->stage_bytes[slot], (uint64_t)sbytes, __ATOMIC_RELAXED);
  __atomic_store_n(&S->sh->tail, seq + 1, __ATOMIC_RELEASE);  // publishes the entry
  S->submitted++;
  if (ticket) *ticket = seq;
  if (!S->running) return relaunch(S);
  return ZX_OK;
}

extern "C" zx_status zx_server_poll(zx_server* S, zx_result* out, int32_t max, int32_t* n_out) {
  zx_clear_error();
  ZX_CHECK_ARG(S && max >= 0 && (max == 0 || out), "bad argument");
  // kernel ended (idle or stopped)?
  if (S->running) {
    const hipError_t q = hipEventQuery(S->ended);
    if (q == hipSuccess) {
      S->running = false;
    } else if (q != hipErrorNotReady) {
      zx_set_error("serving kernel failed: %s", hipGetErrorString(q));
      return ZX_EDEVICE;
    }
  }
  // harvest finished entries
  const double t = now_s();
  for (auto it = S->inflight.begin(); it != S->inflight.end();) {
    const int64_t seq = it->first;
    const int64_t slot = seq & (kRing - 1);
    if (__atomic_load_n(&S->sh->done[slot], __ATOMIC_ACQUIRE) != seq + 1) {
      ++it;
      continue;
    }
    const Req& q = it->second;
    const ZxServeRes& d = S->sh->res[slot];
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
    r.policy = d.policy;
    r.pad = 0;
    r.t_submit = q.t_submit;
    r.t_device = d.t_end > d.t_claim ? (double)(d.t_end - d.t_claim) / S->wall_hz : 0.0;
    r.t_claim_dev = (double)d.t_claim / S->wall_hz;
    r.t_end_dev = (double)d.t_end / S->wall_hz;
    r.t_done = t;
    // start on the device, on the host clock: the poll that saw the result
    // minus the device time (the lag between the result's write and this
    // poll counts as device time)
    r.t_launch = std::max(q.t_submit, t - r.t_device);
    S->finished.push_back(r);
    S->alloc.release(q.off, q.bytes);
    S->salloc.release(q.soff, q.sbytes);
    S->completed++;
    it = S->inflight.erase(it);
  }
  S->oldest = S->next_seq;
  for (const auto& kv : S->inflight) S->oldest = std::min(S->oldest, kv.first);
  // work left but no kernel resident: start one
  if (!S->running && !S->inflight.empty()) {
    zx_status st = relaunch(S);
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
  st->batches = S->launches;
  st->pending = (int64_t)S->inflight.size();
  st->running = S->running ? 1 : 0;
  st->pool_bytes = S->pool_bytes;
  st->pool_used = S->alloc.used();
  st->pool_peak = S->alloc.peak();
  return ZX_OK;
}
