// Continuous-batching server over the pxt C ABI (see include/pxt.h).
//
// Lanes: each lane is one pxt context with its own HIP stream, device input
// and output buffers and pinned host staging; lanes run their batches
// concurrently, so the copy-in, reconstruction and copy-out of one batch
// overlap with the others on the device.  A dispatcher thread owns every
// HIP call and every lane: it admits pending events into a batch whenever a
// lane is free (first come, first served, while the batch fits the lane's
// capacities).  A small batch (at most kDirectHits hits: the one or few
// events of a lightly loaded server) is one pass on the lane's stream:
// copy-in of its hits, the reconstruction, and one kernel that copies the
// counts and exactly the tracks found (it reads their number on the device)
// into pinned host memory -- no host round trip before the copy-back.  A
// larger batch takes two phases, as a kernel's writes to host memory are
// slower than the copy engines for many megabytes: the reconstruction with
// the copy-back of the counts, then the copy-back of exactly the tracks
// found.  A lane holds up to two batches on its stream, each with its own
// pinned staging and result set: a new one is queued behind a one-pass
// batch at once, behind a two-phase batch once its track copy-back is
// queued (stream order keeps the lane's shared device buffers safe: a
// batch's copy-in and kernels run after the previous batch's copy-back has
// read them).  The server lock guards only the queue, the tickets and the
// counters: staging, HIP calls and result hand-over run outside it.
//
// Results are not copied on the host by the server: a finished batch's
// events point into its result set, and pxt_poll copies an event's tracks
// straight from there into the caller's buffers; a set (with its staging)
// is reused once every event in it has been polled.  This is the serving form of the paper's two
// throughput levers for one GPU: several events in flight at once and
// device memory allocated once and reused (Sec. 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_copy.h"
#include "pxt.h"

namespace {

using Clock = std::chrono::steady_clock;

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

// Pinned host memory of one batch: its hits' staging, and its counts and
// tracks as copied back.
struct ResultSet {
  float *hx = nullptr, *hy = nullptr, *hz = nullptr;
  int16_t* hl = nullptr;
  pxt_counts* counts = nullptr;
  uint32_t* per_event = nullptr;
  uint32_t* hit_idx = nullptr;
  uint8_t* nh = nullptr;
  uint8_t* flags = nullptr;
  float* params = nullptr;
  float* cov = nullptr;
  float* chi2 = nullptr;
  std::atomic<uint32_t> refs{0};  // events of the set not yet polled
};

struct Request {
  uint64_t ticket = 0;
  std::vector<float> x, y, z;
  std::vector<int16_t> layer;
  // arrival (submit, or the scheduled arrival of a replay), admission into
  // a batch, launch issued, counts back, tracks back
  Clock::time_point t_arrival, t_start, t_launch, t_device, t_ready;
  bool solo = false;
  bool done = false;
  int status = PXT_OK;
  uint32_t batch_events = 0;
  uint32_t n_tracks = 0;
  ResultSet* rs = nullptr;  // where the tracks are (status PXT_OK)
  uint32_t base = 0;        // first track of the event in rs
};
using ReqPtr = std::shared_ptr<Request>;

template <typename T>
bool dev_alloc(T** p, size_t n) {
  return hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1)) == hipSuccess;
}
template <typename T>
bool host_alloc(T** p, size_t n) {
  return hipHostMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1), hipHostMallocDefault) ==
         hipSuccess;
}

constexpr size_t kDirectHits = 32768;  // batches copied back by one kernel

// One batch on a lane.
struct Flight {
  std::vector<ReqPtr> batch;
  int phase = 0;             // 1 reconstruction in flight, 2 track copy-back in flight
  bool direct = false;       // one pass (tracks copied back by a kernel)
  int set = 0;               // its staging and result set
  hipEvent_t ev = nullptr;   // end of its current phase on the lane's stream
};

struct Lane {
  pxt_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  uint32_t max_hits = 0, max_events = 0, max_tracks = 0;
  // device buffers
  float *dx = nullptr, *dy = nullptr, *dz = nullptr;
  int16_t* dl = nullptr;
  uint32_t *d_hit_idx = nullptr, *d_evt = nullptr, *d_per_event = nullptr;
  uint8_t *d_nh = nullptr, *d_flags = nullptr;
  float *d_params = nullptr, *d_cov = nullptr, *d_chi2 = nullptr;
  pxt_counts* d_counts = nullptr;
  ResultSet res[2];
  // state (dispatcher thread only): up to two batches, fl[head] the older
  Flight fl[2];
  int head = 0, nfl = 0;
  std::vector<uint32_t> offsets;

  Flight& oldest() { return fl[head]; }
  Flight& next_free() { return fl[(head + nfl) & 1]; }
  void pop_oldest() {
    head = (head + 1) & 1;
    --nfl;
  }
  // a new batch may start: the lane is idle, or its one batch is a one-pass
  // batch or in copy-back
  bool can_start() const {
    return nfl == 0 || (nfl == 1 && (fl[head].direct || fl[head].phase == 2));
  }

  bool init(const pxt_config& cfg, int dev) {
    max_hits = cfg.max_hits;
    max_events = cfg.max_events;
    max_tracks = cfg.max_tuples;
    if (pxt_create(&cfg, dev, &ctx) != PXT_OK) return false;
    bool ok = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    for (auto& f : fl)
      ok = ok && hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && dev_alloc(&dx, max_hits) && dev_alloc(&dy, max_hits) && dev_alloc(&dz, max_hits) &&
         dev_alloc(&dl, max_hits);
    ok = ok && dev_alloc(&d_hit_idx, 8ull * max_tracks) && dev_alloc(&d_evt, max_tracks) &&
         dev_alloc(&d_per_event, max_events) && dev_alloc(&d_nh, max_tracks) &&
         dev_alloc(&d_flags, max_tracks) && dev_alloc(&d_params, 5ull * max_tracks) &&
         dev_alloc(&d_cov, 15ull * max_tracks) && dev_alloc(&d_chi2, 2ull * max_tracks) &&
         dev_alloc(&d_counts, 1);
    for (auto& r : res)
      ok = ok && host_alloc(&r.hx, max_hits) && host_alloc(&r.hy, max_hits) &&
           host_alloc(&r.hz, max_hits) && host_alloc(&r.hl, max_hits) &&
           host_alloc(&r.counts, 1) && host_alloc(&r.per_event, max_events) &&
           host_alloc(&r.hit_idx, 8ull * max_tracks) && host_alloc(&r.nh, max_tracks) &&
           host_alloc(&r.flags, max_tracks) && host_alloc(&r.params, 5ull * max_tracks) &&
           host_alloc(&r.cov, 15ull * max_tracks) && host_alloc(&r.chi2, 2ull * max_tracks);
    return ok;
  }

  // a result set nobody reads any more and no batch in flight writes, or -1
  int free_set() const {
    for (int i = 0; i < 2; ++i) {
      bool used = false;
      for (int k = 0; k < nfl; ++k) used |= fl[(head + k) & 1].set == i;
      if (!used && res[i].refs.load(std::memory_order_acquire) == 0) return i;
    }
    return -1;
  }

  void release() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : {(void*)dx, (void*)dy, (void*)dz, (void*)dl, (void*)d_hit_idx, (void*)d_evt,
                    (void*)d_per_event, (void*)d_nh, (void*)d_flags, (void*)d_params,
                    (void*)d_cov, (void*)d_chi2, (void*)d_counts})
      if (p) (void)hipFree(p);
    for (auto& r : res)
      for (void* p : {(void*)r.hx, (void*)r.hy, (void*)r.hz, (void*)r.hl, (void*)r.counts,
                      (void*)r.per_event, (void*)r.hit_idx, (void*)r.nh, (void*)r.flags,
                      (void*)r.params, (void*)r.cov, (void*)r.chi2})
        if (p) (void)hipHostFree(p);
    for (auto& f : fl)
      if (f.ev) (void)hipEventDestroy(f.ev);
    if (stream) (void)hipStreamDestroy(stream);
    if (ctx) pxt_destroy(ctx);
  }
};

}  // namespace

struct pxt_server {
  pxt_config cfg{};
  pxt_server_config scfg{};
  int device = 0;
  std::vector<Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_work;   // dispatcher wake-up
  std::condition_variable cv_done;   // pollers
  std::deque<ReqPtr> pending;
  std::unordered_map<uint64_t, ReqPtr> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  pxt_server_stats stats{};
  std::thread worker;

  void run();
  void take_batch(Lane& L, Flight& F);            // lock held
  void start_batch(Lane& L, Flight& F);           // lock not held
  bool advance(Lane& L);                          // lock not held
  void finish(Lane& L, Flight& F, int status);    // lock not held
  int submit(const float* x, const float* y, const float* z, const int16_t* layer,
             uint32_t n_hits, Clock::time_point arrival, uint64_t* ticket);
  int poll(uint64_t ticket, pxt_event_tracks* out, int timeout_ms, bool release_only);
};

// Move pending events into a new batch F of lane L (first come, first
// served, while the batch fits the lane); the server lock is held.
void pxt_server::take_batch(Lane& L, Flight& F) {
  std::vector<ReqPtr>& batch = F.batch;
  batch.clear();
  uint64_t hits = 0, est_d = 0;
  const uint32_t max_ev = std::min(scfg.max_batch_events, L.max_events);
  while (!pending.empty() && batch.size() < max_ev) {
    const ReqPtr& r = pending.front();
    const uint64_t h = r->x.size();
    const uint64_t d = h * scfg.doublets_per_hit;
    if (!batch.empty() && (r->solo || batch.front()->solo)) break;
    if (!batch.empty() && (hits + h > L.max_hits || est_d + d > cfg.max_doublets)) break;
    hits += h;
    est_d += d;
    batch.push_back(r);
    pending.pop_front();
  }
  stats.batches++;
  stats.events_in_batches += batch.size();
}

// Stage batch F's hits and queue its pass on the lane's stream (behind the
// lane's other batch, if any).
void pxt_server::start_batch(Lane& L, Flight& F) {
  const auto now = Clock::now();
  ResultSet& R = L.res[F.set];
  L.offsets.assign(1, 0u);
  uint32_t off = 0;
  for (auto& r : F.batch) {
    r->t_start = now;
    const uint32_t n = (uint32_t)r->x.size();
    std::memcpy(R.hx + off, r->x.data(), 4ull * n);
    std::memcpy(R.hy + off, r->y.data(), 4ull * n);
    std::memcpy(R.hz + off, r->z.data(), 4ull * n);
    std::memcpy(R.hl + off, r->layer.data(), 2ull * n);
    off += n;
    L.offsets.push_back(off);
  }
  const size_t H = off;
  bool ok = true;
  if (H) {
    ok = hipMemcpyAsync(L.dx, R.hx, 4 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
         hipMemcpyAsync(L.dy, R.hy, 4 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
         hipMemcpyAsync(L.dz, R.hz, 4 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
         hipMemcpyAsync(L.dl, R.hl, 2 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess;
  }
  const uint32_t nb = (uint32_t)F.batch.size();
  pxt_hits in{nb, L.offsets.data(), L.dx, L.dy, L.dz, L.dl, nullptr};
  pxt_tracks out{L.max_tracks, L.d_hit_idx, L.d_nh, L.d_evt, L.d_params, L.d_cov,
                 L.d_chi2, L.d_flags, L.d_per_event, L.d_counts, nullptr};
  ok = ok && pxt_reconstruct(L.ctx, &in, &out, L.stream) == PXT_OK;
  F.direct = H <= kDirectHits;
  if (F.direct) {
    const pxt::HostTracks host{R.hit_idx, R.nh,    R.params,    R.cov,
                               R.chi2,    R.flags, R.per_event, R.counts};
    ok = ok && pxt::launch_copy_out(out, nb, host, L.stream) == hipSuccess;
  } else {
    ok = ok && hipMemcpyAsync(R.counts, L.d_counts, sizeof(pxt_counts), hipMemcpyDeviceToHost,
                              L.stream) == hipSuccess;
    ok = ok && hipMemcpyAsync(R.per_event, L.d_per_event, 4ull * nb, hipMemcpyDeviceToHost,
                              L.stream) == hipSuccess;
  }
  ok = ok && hipEventRecord(F.ev, L.stream) == hipSuccess;
  F.phase = 1;
  const auto t = Clock::now();
  for (auto& r : F.batch) r->t_launch = t;
  ++L.nfl;
  if (!ok) {
    // a failed launch leaves the stream's earlier work in place: wait for
    // it, so that the lane's batches still end in order
    (void)hipStreamSynchronize(L.stream);
    finish(L, F, PXT_ERR_HIP);
    --L.nfl;
  }
}

// Hand batch F's events over: status, track counts and where their tracks
// are (status PXT_OK); then the pollers are woken.  F leaves the lane.
void pxt_server::finish(Lane& L, Flight& F, int status) {
  const auto now = Clock::now();
  const uint32_t nb = (uint32_t)F.batch.size();
  ResultSet* rs = &L.res[F.set];
  if (status == PXT_OK) rs->refs.store(nb, std::memory_order_release);
  uint32_t base = 0;
  for (uint32_t e = 0; e < nb; ++e) {
    Request& r = *F.batch[e];
    r.status = status;
    r.batch_events = nb;
    r.t_ready = now;
    if (status == PXT_OK) {
      r.n_tracks = rs->per_event[e];
      r.rs = rs;
      r.base = base;
      base += r.n_tracks;
    } else {
      r.n_tracks = 0;
      r.t_device = r.t_device == Clock::time_point{} ? now : r.t_device;
    }
  }
  {
    std::lock_guard<std::mutex> g(mu);
    for (auto& rp : F.batch) {
      Request& r = *rp;
      r.done = true;
      stats.completed++;
      if (status != PXT_OK) stats.failed++;
      stats.sum_queue_us += us_between(r.t_arrival, r.t_start);
      stats.sum_launch_us += us_between(r.t_start, r.t_launch);
      stats.sum_device_us += us_between(r.t_launch, r.t_device);
      stats.sum_copyback_us += us_between(r.t_device, r.t_ready);
    }
  }
  F.batch.clear();
  F.phase = 0;
  cv_done.notify_all();
}

// Move lane L's batches on as their device work finishes (in stream order:
// the older batch first); true if anything moved.
bool pxt_server::advance(Lane& L) {
  bool moved = false;
  while (L.nfl > 0) {
    Flight& F = L.oldest();
    const hipError_t q = hipEventQuery(F.ev);
    if (q == hipErrorNotReady) return moved;
    moved = true;
    if (q != hipSuccess) {
      finish(L, F, PXT_ERR_HIP);
      L.pop_oldest();
      continue;
    }
    if (F.phase == 2) {
      finish(L, F, PXT_OK);
      L.pop_oldest();
      continue;
    }
    // the reconstruction has ended
    const auto now = Clock::now();
    for (auto& r : F.batch) r->t_device = now;
    ResultSet& R = L.res[F.set];
    const int st = R.counts->status;
    if (st != PXT_OK) {
      if (F.batch.size() > 1) {
        // re-run each event alone, ahead of the queue, in order
        std::lock_guard<std::mutex> g(mu);
        for (auto it = F.batch.rbegin(); it != F.batch.rend(); ++it) {
          (*it)->solo = true;
          (*it)->t_device = Clock::time_point{};
          pending.push_front(*it);
        }
        stats.solo_retries += F.batch.size();
        F.batch.clear();
      } else {
        finish(L, F, st);
      }
      L.pop_oldest();
      continue;
    }
    if (F.direct) {
      finish(L, F, PXT_OK);
      L.pop_oldest();
      continue;
    }
    // two phases: the tracks' copy-back, sized by the counts (no batch runs
    // behind this one yet)
    const size_t n = R.counts->n_tracks;
    bool ok = true;
    if (n) {
      ok = hipMemcpyAsync(R.hit_idx, L.d_hit_idx, 32 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess &&
           hipMemcpyAsync(R.nh, L.d_nh, n, hipMemcpyDeviceToHost, L.stream) == hipSuccess &&
           hipMemcpyAsync(R.flags, L.d_flags, n, hipMemcpyDeviceToHost, L.stream) == hipSuccess &&
           hipMemcpyAsync(R.params, L.d_params, 20 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess &&
           hipMemcpyAsync(R.cov, L.d_cov, 60 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess &&
           hipMemcpyAsync(R.chi2, L.d_chi2, 8 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess;
    }
    ok = ok && hipEventRecord(F.ev, L.stream) == hipSuccess;
    if (!ok) {
      (void)hipStreamSynchronize(L.stream);
      finish(L, F, PXT_ERR_HIP);
      L.pop_oldest();
      continue;
    }
    F.phase = 2;
    return moved;
  }
  return moved;
}

void pxt_server::run() {
  (void)hipSetDevice(device);
  uint32_t idle_rounds = 0;
  for (;;) {
    bool progress = false, busy = false;
    for (auto& L : lanes) {
      if (advance(L)) progress = true;
      if (!L.can_start()) continue;
      const int set = L.free_set();
      if (set < 0) continue;
      Flight& F = L.next_free();
      {
        std::lock_guard<std::mutex> g(mu);
        if (pending.empty() || stop) continue;
        take_batch(L, F);
      }
      F.set = set;
      start_batch(L, F);
      progress = true;
    }
    for (auto& L : lanes) busy |= L.nfl != 0;
    std::unique_lock<std::mutex> lk(mu);
    if (stop) {
      // queued events are dropped; the batches on the lanes finish
      for (auto& r : pending) {
        r->status = PXT_ERR_BUSY;
        r->done = true;
        stats.completed++;
        stats.failed++;
      }
      if (!pending.empty()) cv_done.notify_all();
      pending.clear();
      if (!busy) break;
    }
    if (progress) {
      idle_rounds = 0;
      continue;
    }
    if (busy && ++idle_rounds < 2000) {
      // device work in flight: query the lanes again at once (a wait on
      // the condition variable would add tens of microseconds per phase)
      lk.unlock();
      std::this_thread::yield();
      continue;
    }
    idle_rounds = 0;
    cv_work.wait_for(lk, std::chrono::microseconds(busy ? 50 : 1000),
                     [&] { return stop || !pending.empty(); });
  }
}

int pxt_server::submit(const float* x, const float* y, const float* z, const int16_t* layer,
                       uint32_t n_hits, Clock::time_point arrival, uint64_t* ticket) {
  auto r = std::make_shared<Request>();
  r->x.assign(x, x + n_hits);
  r->y.assign(y, y + n_hits);
  r->z.assign(z, z + n_hits);
  r->layer.assign(layer, layer + n_hits);
  r->t_arrival = arrival;
  {
    std::lock_guard<std::mutex> g(mu);
    if (stop) return PXT_ERR_BUSY;
    if (pending.size() >= scfg.queue_depth) {
      stats.rejected++;
      return PXT_ERR_BUSY;
    }
    r->ticket = next_ticket++;
    tickets[r->ticket] = r;
    pending.push_back(r);
    stats.submitted++;
    *ticket = r->ticket;
  }
  cv_work.notify_one();
  return PXT_OK;
}

int pxt_server::poll(uint64_t ticket, pxt_event_tracks* out, int timeout_ms, bool release_only) {
  ReqPtr r;
  {
    std::unique_lock<std::mutex> lk(mu);
    auto it = tickets.find(ticket);
    if (it == tickets.end()) return PXT_ERR_INVALID_ARG;
    r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_ms < 0) {
      cv_done.wait(lk, ready);
    } else if (!cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
      return PXT_ERR_NOT_READY;
    }
    const uint32_t n = r->n_tracks;
    out->n_tracks = n;
    out->status = r->status;
    out->queue_us = us_between(r->t_arrival, r->t_start);
    out->batch_events = r->batch_events;
    if (r->status == PXT_OK && !release_only) {
      // a buffer too small keeps the ticket: the caller polls again with room
      // for out->n_tracks tracks
      if (n > out->capacity) return PXT_ERR_CAPACITY;
      if (n && (!out->hit_idx || !out->n_hits || !out->params || !out->cov || !out->chi2 ||
                !out->flags))
        return PXT_ERR_INVALID_ARG;
    }
    tickets.erase(it);
  }
  // the event's tracks straight from the lane's pinned result set
  const uint32_t n = r->n_tracks;
  if (r->status == PXT_OK && n && !release_only) {
    const ResultSet& R = *r->rs;
    const size_t b = r->base;
    std::memcpy(out->hit_idx, R.hit_idx + 8 * b, 32ull * n);
    std::memcpy(out->n_hits, R.nh + b, n);
    std::memcpy(out->flags, R.flags + b, n);
    std::memcpy(out->params, R.params + 5 * b, 20ull * n);
    std::memcpy(out->cov, R.cov + 15 * b, 60ull * n);
    std::memcpy(out->chi2, R.chi2 + 2 * b, 8ull * n);
  }
  const auto now = Clock::now();
  out->latency_us = us_between(r->t_arrival, now);
  if (r->rs && r->rs->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) cv_work.notify_one();
  {
    std::lock_guard<std::mutex> g(mu);
    stats.sum_deliver_us += us_between(r->t_ready, now);
    stats.sum_latency_us += out->latency_us;
    stats.delivered++;
  }
  return PXT_OK;
}

extern "C" {

int pxt_server_create(const pxt_config* cfg, const pxt_server_config* scfg, int hip_device,
                      pxt_server** out) {
  if (!cfg || !scfg || !out) return PXT_ERR_INVALID_ARG;
  *out = nullptr;
  if (scfg->n_lanes < 1 || scfg->n_lanes > 16 || scfg->queue_depth < 1 ||
      scfg->max_batch_events < 1)
    return PXT_ERR_INVALID_ARG;
  pxt_server* s = new (std::nothrow) pxt_server();
  if (!s) return PXT_ERR_OOM;
  s->cfg = *cfg;
  s->scfg = *scfg;
  s->device = hip_device;
  s->lanes = std::vector<Lane>(scfg->n_lanes);
  for (auto& L : s->lanes) {
    if (!L.init(*cfg, hip_device)) {
      for (auto& M : s->lanes) M.release();
      delete s;
      return PXT_ERR_OOM;
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return PXT_OK;
}

int pxt_submit(pxt_server* s, const float* x, const float* y, const float* z,
               const int16_t* layer, uint32_t n_hits, uint64_t* ticket) {
  if (!s || !ticket || (n_hits && (!x || !y || !z || !layer))) return PXT_ERR_INVALID_ARG;
  if (n_hits > s->cfg.max_hits) return PXT_ERR_INVALID_ARG;
  return s->submit(x, y, z, layer, n_hits, Clock::now(), ticket);
}

int pxt_poll(pxt_server* s, uint64_t ticket, pxt_event_tracks* out, int timeout_ms) {
  if (!s || !out) return PXT_ERR_INVALID_ARG;
  const bool release_only = out->capacity == 0 && out->hit_idx == nullptr;
  return s->poll(ticket, out, timeout_ms, release_only);
}

int pxt_server_replay(pxt_server* s, uint32_t n, const uint32_t* event_of_arrival,
                      const double* arrival_us, uint32_t n_pool, const uint32_t* pool_offsets,
                      const float* x, const float* y, const float* z, const int16_t* layer,
                      pxt_event_tracks* results) {
  if (!s || (n && (!event_of_arrival || !arrival_us || !pool_offsets || !results)) ||
      (n_pool && (!x || !y || !z || !layer)))
    return PXT_ERR_INVALID_ARG;
  for (uint32_t i = 0; i < n; ++i) {
    if (event_of_arrival[i] >= n_pool) return PXT_ERR_INVALID_ARG;
    if (i && arrival_us[i] < arrival_us[i - 1]) return PXT_ERR_INVALID_ARG;
    const uint32_t e = event_of_arrival[i];
    if (pool_offsets[e + 1] < pool_offsets[e] ||
        pool_offsets[e + 1] - pool_offsets[e] > s->cfg.max_hits)
      return PXT_ERR_INVALID_ARG;
  }
  std::vector<uint64_t> tix(n, 0);
  std::atomic<uint32_t> submitted{0};
  std::atomic<int> failure{PXT_OK};
  // collector: releases the events in arrival order as they finish
  std::thread collector([&] {
    for (uint32_t i = 0; i < n; ++i) {
      while (submitted.load(std::memory_order_acquire) <= i) {
        if (failure.load() != PXT_OK) return;
        std::this_thread::yield();
      }
      pxt_event_tracks& o = results[i];
      o.capacity = 0;
      o.hit_idx = nullptr;
      const int st = s->poll(tix[i], &o, -1, true);
      if (st != PXT_OK) failure.store(st);
    }
  });
  const auto t0 = Clock::now();
  for (uint32_t i = 0; i < n; ++i) {
    const auto due = t0 + std::chrono::duration_cast<Clock::duration>(
                              std::chrono::duration<double, std::micro>(arrival_us[i]));
    while (Clock::now() < due) {
      const auto left = due - Clock::now();
      if (left > std::chrono::microseconds(200))
        std::this_thread::sleep_for(left - std::chrono::microseconds(100));
    }
    const uint32_t e = event_of_arrival[i], a = pool_offsets[e], h = pool_offsets[e + 1] - a;
    int st;
    while ((st = s->submit(x + a, y + a, z + a, layer + a, h, due, &tix[i])) == PXT_ERR_BUSY)
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    if (st != PXT_OK) {
      failure.store(st);
      break;
    }
    submitted.store(i + 1, std::memory_order_release);
  }
  collector.join();
  return failure.load();
}

int pxt_server_get_stats(pxt_server* s, pxt_server_stats* out) {
  if (!s || !out) return PXT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  return PXT_OK;
}

void pxt_server_destroy(pxt_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& L : s->lanes) L.release();
  delete s;
}

}  // extern "C"
