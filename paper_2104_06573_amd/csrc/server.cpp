// Continuous-batching server over the pxt C ABI (see include/pxt.h).
//
// Lanes: each lane is one pxt context with its own HIP stream, device input
// and output buffers and pinned host staging; lanes run their batches
// concurrently, so the copy-in, reconstruction and copy-out of one batch
// overlap with the others on the device.  A dispatcher thread owns every
// HIP call: it admits pending events into a batch whenever a lane is free
// (first come, first served, while the batch fits the lane's capacities),
// and advances each busy lane through two phases -- reconstruction with the
// copy-back of the counts, then the copy-back of exactly the tracks found.
// Results are split per event (tracks come out grouped by event, in event
// order) and handed to pxt_poll.  This is the serving form of the paper's
// two throughput levers for one GPU: several events in flight at once and
// device memory allocated once and reused (Sec. 5).
#include <hip/hip_runtime.h>

#include <algorithm>
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

#include "pxt.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  std::vector<float> x, y, z;
  std::vector<int16_t> layer;
  Clock::time_point t_submit, t_start;
  bool solo = false;
  bool done = false;
  int status = PXT_OK;
  uint32_t batch_events = 0;
  uint32_t n_tracks = 0;
  std::vector<uint32_t> hit_idx;
  std::vector<uint8_t> n_hits, flags;
  std::vector<float> params, cov, chi2;
  double latency_us = 0.0, queue_us = 0.0;
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

struct Lane {
  pxt_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  uint32_t max_hits = 0, max_events = 0, max_tracks = 0;
  // device buffers
  float *dx = nullptr, *dy = nullptr, *dz = nullptr;
  int16_t* dl = nullptr;
  uint32_t *d_hit_idx = nullptr, *d_evt = nullptr, *d_per_event = nullptr;
  uint8_t *d_nh = nullptr, *d_flags = nullptr;
  float *d_params = nullptr, *d_cov = nullptr, *d_chi2 = nullptr;
  pxt_counts* d_counts = nullptr;
  // pinned host staging
  float *hx = nullptr, *hy = nullptr, *hz = nullptr;
  int16_t* hl = nullptr;
  pxt_counts* h_counts = nullptr;
  uint32_t *h_per_event = nullptr, *h_hit_idx = nullptr;
  uint8_t *h_nh = nullptr, *h_flags = nullptr;
  float *h_params = nullptr, *h_cov = nullptr, *h_chi2 = nullptr;
  // state
  int phase = 0;  // 0 idle, 1 reconstruction in flight, 2 track copy-back in flight
  std::vector<ReqPtr> batch;
  std::vector<uint32_t> offsets;

  bool init(const pxt_config& cfg, int dev) {
    max_hits = cfg.max_hits;
    max_events = cfg.max_events;
    max_tracks = cfg.max_tuples;
    if (pxt_create(&cfg, dev, &ctx) != PXT_OK) return false;
    bool ok = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && dev_alloc(&dx, max_hits) && dev_alloc(&dy, max_hits) && dev_alloc(&dz, max_hits) &&
         dev_alloc(&dl, max_hits);
    ok = ok && dev_alloc(&d_hit_idx, 8ull * max_tracks) && dev_alloc(&d_evt, max_tracks) &&
         dev_alloc(&d_per_event, max_events) && dev_alloc(&d_nh, max_tracks) &&
         dev_alloc(&d_flags, max_tracks) && dev_alloc(&d_params, 5ull * max_tracks) &&
         dev_alloc(&d_cov, 15ull * max_tracks) && dev_alloc(&d_chi2, 2ull * max_tracks) &&
         dev_alloc(&d_counts, 1);
    ok = ok && host_alloc(&hx, max_hits) && host_alloc(&hy, max_hits) &&
         host_alloc(&hz, max_hits) && host_alloc(&hl, max_hits) && host_alloc(&h_counts, 1) &&
         host_alloc(&h_per_event, max_events) && host_alloc(&h_hit_idx, 8ull * max_tracks) &&
         host_alloc(&h_nh, max_tracks) && host_alloc(&h_flags, max_tracks) &&
         host_alloc(&h_params, 5ull * max_tracks) && host_alloc(&h_cov, 15ull * max_tracks) &&
         host_alloc(&h_chi2, 2ull * max_tracks);
    return ok;
  }

  void release() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : {(void*)dx, (void*)dy, (void*)dz, (void*)dl, (void*)d_hit_idx, (void*)d_evt,
                    (void*)d_per_event, (void*)d_nh, (void*)d_flags, (void*)d_params,
                    (void*)d_cov, (void*)d_chi2, (void*)d_counts})
      if (p) (void)hipFree(p);
    for (void* p : {(void*)hx, (void*)hy, (void*)hz, (void*)hl, (void*)h_counts,
                    (void*)h_per_event, (void*)h_hit_idx, (void*)h_nh, (void*)h_flags,
                    (void*)h_params, (void*)h_cov, (void*)h_chi2})
      if (p) (void)hipHostFree(p);
    if (ev) (void)hipEventDestroy(ev);
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
  bool launch(Lane& L);
  void advance(Lane& L);
  void fail_batch(Lane& L, int status);
  void deliver(Lane& L);
};

namespace {

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

}  // namespace

// Form a batch from the pending events (lock held by the caller) and start
// it on lane L.  Returns true if a batch was started.
bool pxt_server::launch(Lane& L) {
  if (pending.empty()) return false;
  L.batch.clear();
  L.offsets.assign(1, 0u);
  uint64_t hits = 0, est_d = 0;
  const uint32_t max_ev = std::min(scfg.max_batch_events, L.max_events);
  while (!pending.empty() && L.batch.size() < max_ev) {
    const ReqPtr& r = pending.front();
    const uint64_t h = r->x.size();
    const uint64_t d = h * scfg.doublets_per_hit;
    if (!L.batch.empty() && (r->solo || L.batch.front()->solo)) break;
    if (!L.batch.empty() && (hits + h > L.max_hits || est_d + d > cfg.max_doublets)) break;
    hits += h;
    est_d += d;
    L.batch.push_back(r);
    pending.pop_front();
  }
  const auto now = Clock::now();
  uint32_t off = 0;
  for (auto& r : L.batch) {
    r->t_start = now;
    const uint32_t n = (uint32_t)r->x.size();
    std::memcpy(L.hx + off, r->x.data(), 4ull * n);
    std::memcpy(L.hy + off, r->y.data(), 4ull * n);
    std::memcpy(L.hz + off, r->z.data(), 4ull * n);
    std::memcpy(L.hl + off, r->layer.data(), 2ull * n);
    off += n;
    L.offsets.push_back(off);
  }
  stats.batches++;
  stats.events_in_batches += L.batch.size();
  const size_t H = off;
  bool ok = true;
  if (H) {
    ok = hipMemcpyAsync(L.dx, L.hx, 4 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
         hipMemcpyAsync(L.dy, L.hy, 4 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
         hipMemcpyAsync(L.dz, L.hz, 4 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
         hipMemcpyAsync(L.dl, L.hl, 2 * H, hipMemcpyHostToDevice, L.stream) == hipSuccess;
  }
  pxt_hits in{(uint32_t)L.batch.size(), L.offsets.data(), L.dx, L.dy, L.dz, L.dl, nullptr};
  pxt_tracks out{L.max_tracks, L.d_hit_idx, L.d_nh, L.d_evt, L.d_params, L.d_cov,
                 L.d_chi2, L.d_flags, L.d_per_event, L.d_counts};
  ok = ok && pxt_reconstruct(L.ctx, &in, &out, L.stream) == PXT_OK;
  ok = ok && hipMemcpyAsync(L.h_counts, L.d_counts, sizeof(pxt_counts), hipMemcpyDeviceToHost,
                            L.stream) == hipSuccess;
  ok = ok && hipMemcpyAsync(L.h_per_event, L.d_per_event, 4ull * L.batch.size(),
                            hipMemcpyDeviceToHost, L.stream) == hipSuccess;
  ok = ok && hipEventRecord(L.ev, L.stream) == hipSuccess;
  L.phase = 1;
  if (!ok) fail_batch(L, PXT_ERR_HIP);
  return true;
}

void pxt_server::fail_batch(Lane& L, int status) {
  const auto now = Clock::now();
  for (auto& r : L.batch) {
    r->status = status;
    r->done = true;
    r->n_tracks = 0;
    r->latency_us = us_between(r->t_submit, now);
    r->queue_us = us_between(r->t_submit, r->t_start);
    r->batch_events = (uint32_t)L.batch.size();
    stats.completed++;
    stats.failed++;
  }
  L.batch.clear();
  L.phase = 0;
  cv_done.notify_all();
}

void pxt_server::deliver(Lane& L) {
  const auto now = Clock::now();
  uint32_t base = 0;
  const uint32_t nb = (uint32_t)L.batch.size();
  for (uint32_t e = 0; e < nb; ++e) {
    Request& r = *L.batch[e];
    const uint32_t n = L.h_per_event[e];
    r.n_tracks = n;
    r.hit_idx.assign(L.h_hit_idx + 8ull * base, L.h_hit_idx + 8ull * (base + n));
    r.n_hits.assign(L.h_nh + base, L.h_nh + base + n);
    r.flags.assign(L.h_flags + base, L.h_flags + base + n);
    r.params.assign(L.h_params + 5ull * base, L.h_params + 5ull * (base + n));
    r.cov.assign(L.h_cov + 15ull * base, L.h_cov + 15ull * (base + n));
    r.chi2.assign(L.h_chi2 + 2ull * base, L.h_chi2 + 2ull * (base + n));
    r.status = PXT_OK;
    r.batch_events = nb;
    r.latency_us = us_between(r.t_submit, now);
    r.queue_us = us_between(r.t_submit, r.t_start);
    r.done = true;
    base += n;
    stats.completed++;
  }
  L.batch.clear();
  L.phase = 0;
  cv_done.notify_all();
}

// Move lane L on if its device work has finished (lock held).
void pxt_server::advance(Lane& L) {
  if (L.phase == 0) return;
  const hipError_t q = hipEventQuery(L.ev);
  if (q == hipErrorNotReady) return;
  if (q != hipSuccess) {
    fail_batch(L, PXT_ERR_HIP);
    return;
  }
  if (L.phase == 1) {
    const int st = L.h_counts->status;
    if (st != PXT_OK) {
      if (L.batch.size() > 1) {
        // re-run each event alone, ahead of the queue, in order
        for (auto it = L.batch.rbegin(); it != L.batch.rend(); ++it) {
          (*it)->solo = true;
          pending.push_front(*it);
        }
        stats.solo_retries += L.batch.size();
        L.batch.clear();
        L.phase = 0;
      } else {
        fail_batch(L, st);
      }
      return;
    }
    const size_t n = L.h_counts->n_tracks;
    bool ok = true;
    if (n) {
      ok = hipMemcpyAsync(L.h_hit_idx, L.d_hit_idx, 32 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess &&
           hipMemcpyAsync(L.h_nh, L.d_nh, n, hipMemcpyDeviceToHost, L.stream) == hipSuccess &&
           hipMemcpyAsync(L.h_flags, L.d_flags, n, hipMemcpyDeviceToHost, L.stream) == hipSuccess &&
           hipMemcpyAsync(L.h_params, L.d_params, 20 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess &&
           hipMemcpyAsync(L.h_cov, L.d_cov, 60 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess &&
           hipMemcpyAsync(L.h_chi2, L.d_chi2, 8 * n, hipMemcpyDeviceToHost, L.stream) ==
               hipSuccess;
    }
    ok = ok && hipEventRecord(L.ev, L.stream) == hipSuccess;
    if (!ok) {
      fail_batch(L, PXT_ERR_HIP);
      return;
    }
    L.phase = 2;
    return;
  }
  deliver(L);
}

void pxt_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = false;
    bool busy = false;
    for (auto& L : lanes) {
      const int before = L.phase;
      advance(L);
      if (L.phase != before) progress = true;
      if (L.phase == 0 && !pending.empty()) progress |= launch(L);
      busy |= L.phase != 0;
    }
    if (stop && !busy && pending.empty()) break;
    if (!progress) {
      if (busy) {
        // device work in flight: short wait, woken early by a submission
        cv_work.wait_for(lk, std::chrono::microseconds(20));
      } else {
        cv_work.wait(lk, [&] { return stop || !pending.empty(); });
      }
    }
  }
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
  s->lanes.resize(scfg->n_lanes);
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
  auto r = std::make_shared<Request>();
  r->x.assign(x, x + n_hits);
  r->y.assign(y, y + n_hits);
  r->z.assign(z, z + n_hits);
  r->layer.assign(layer, layer + n_hits);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return PXT_ERR_BUSY;
    if (s->pending.size() >= s->scfg.queue_depth) {
      s->stats.rejected++;
      return PXT_ERR_BUSY;
    }
    r->ticket = s->next_ticket++;
    r->t_submit = Clock::now();
    s->tickets[r->ticket] = r;
    s->pending.push_back(r);
    s->stats.submitted++;
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return PXT_OK;
}

int pxt_poll(pxt_server* s, uint64_t ticket, pxt_event_tracks* out, int timeout_ms) {
  if (!s || !out) return PXT_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return PXT_ERR_INVALID_ARG;
  ReqPtr r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return PXT_ERR_NOT_READY;
  }
  const uint32_t n = r->n_tracks;
  out->n_tracks = n;
  out->status = r->status;
  out->latency_us = r->latency_us;
  out->queue_us = r->queue_us;
  out->batch_events = r->batch_events;
  if (r->status == PXT_OK) {
    // a buffer too small keeps the ticket: the caller polls again with room
    // for out->n_tracks tracks
    if (n > out->capacity) return PXT_ERR_CAPACITY;
    if (n) {
      if (!out->hit_idx || !out->n_hits || !out->params || !out->cov || !out->chi2 || !out->flags)
        return PXT_ERR_INVALID_ARG;
      std::memcpy(out->hit_idx, r->hit_idx.data(), 32ull * n);
      std::memcpy(out->n_hits, r->n_hits.data(), n);
      std::memcpy(out->flags, r->flags.data(), n);
      std::memcpy(out->params, r->params.data(), 20ull * n);
      std::memcpy(out->cov, r->cov.data(), 60ull * n);
      std::memcpy(out->chi2, r->chi2.data(), 8ull * n);
    }
  }
  s->tickets.erase(it);
  return PXT_OK;
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
