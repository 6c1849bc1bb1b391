// RecHits: pixel clusters to 3-D hits (the paper's RecHits module, Sec. 2:
// the 3-D position of each cluster; its Fig. 3 shows the per-module step
// that limits each module's cluster count and turns the counts into the
// modules' first-hit offsets).  The reading is stated with pxt_rechits in
// pxt.h.  Three steps over a ragged batch of events:
//   count    one thread per cluster adds one to its (event, module) counter;
//   offsets  one workgroup per event limits its modules' counters to
//            max_per_module and scans them into offsets from the event's
//            first hit; one workgroup scans the event totals into the
//            events' first hits; a last pass makes the module offsets
//            absolute: the hits of all events come out contiguous, in event
//            and module order;
//   hits     one thread per cluster finds its rank among its module's
//            clusters (clusters arrive grouped by module, so the rank is its
//            distance from the module's first cluster, found by binary
//            search), and if the rank is within the limit computes the
//            charge-weighted centroid of its pixels and the 3-D position.
#pragma once

#include "common.h"

namespace pxt {

constexpr int kRhScanThreads = 1024;

struct RhIn {
  uint32_t n_events;
  uint32_t n_clusters;
  const uint32_t* event_offsets;  // [E + 1] clusters of each event
  const uint16_t* module;         // [nc] grouped by module within an event
  const uint32_t* pixel_offsets;  // [nc + 1]
  const uint16_t* pix_u;
  const uint16_t* pix_v;
  const uint16_t* charge;
};

struct RhOut {
  uint32_t capacity;
  float* x;
  float* y;
  float* z;
  int16_t* layer;
  uint16_t* module;
  uint32_t* cluster;
  uint32_t* module_start;  // [E * NM + 1]
  uint32_t* hit_offsets;   // [E + 1]
  int32_t* status;         // [1]
};

// Event of cluster i: the last e with event_offsets[e] <= i.
__device__ __forceinline__ uint32_t rh_event(const RhIn& in, uint32_t i) {
  uint32_t lo = 0, hi = in.n_events;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (in.event_offsets[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_rh_zero(RhOut o, uint32_t n) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride)
    o.module_start[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) o.status[0] = 0;
}

__global__ __launch_bounds__(256) void k_rh_count(RhIn in, RhOut o, uint32_t n_modules) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < in.n_clusters; i += stride) {
    const uint32_t e = rh_event(in, i);
    const uint32_t m = in.module[i];
    const bool bad = m >= n_modules ||
                     (i > in.event_offsets[e] && in.module[i - 1] > in.module[i]);
    if (bad) {
      atomicCAS((unsigned int*)o.status, 0u, (unsigned int)PXT_ERR_INVALID_ARG);
      continue;
    }
    atomicAdd(&o.module_start[(size_t)e * n_modules + m], 1u);
  }
}

// One workgroup per event: its modules' counters, limited to
// max_per_module, become offsets from the event's first hit (in place),
// and the event's hit total goes to hit_offsets[e + 1].
constexpr int kRhEvThreads = 256;
constexpr int kRhEvPer = 8;  // counters per thread per round

__global__ __launch_bounds__(kRhEvThreads) void k_rh_event_offsets(RhOut o, uint32_t n_events,
                                                                   uint32_t n_modules,
                                                                   uint32_t max_per_module) {
  __shared__ uint32_t s_scan[kRhEvThreads / kWave + 1];
  const uint32_t e = blockIdx.x;
  if (e >= n_events) return;
  uint32_t* ms = o.module_start + (size_t)e * n_modules;
  uint32_t run = 0;
  for (uint32_t r0 = 0; r0 < n_modules; r0 += kRhEvThreads * kRhEvPer) {
    const uint32_t a = r0 + threadIdx.x * kRhEvPer;
    uint32_t v[kRhEvPer];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kRhEvPer; ++q) {
      v[q] = a + q < n_modules ? min(ms[a + q], max_per_module) : 0u;
      sum += v[q];
    }
    uint32_t tot = 0;
    uint32_t x = run + block_excl_scan(sum, s_scan, tot);
#pragma unroll
    for (int q = 0; q < kRhEvPer; ++q) {
      if (a + q < n_modules) ms[a + q] = x;
      x += v[q];
    }
    run += tot;
  }
  if (threadIdx.x == 0) o.hit_offsets[e + 1] = run;
}

// One workgroup: the events' totals become their first-hit offsets; the
// last offset (all hits) closes module_start; an overflow of the caller's
// hit buffers is reported.
__global__ __launch_bounds__(kRhScanThreads) void k_rh_events(RhOut o, uint32_t n_events,
                                                              uint32_t n_modules) {
  __shared__ uint32_t s_scan[kRhScanThreads / kWave + 1];
  uint32_t run = 0;
  for (uint32_t e0 = 0; e0 < n_events; e0 += kRhScanThreads) {
    const uint32_t e = e0 + threadIdx.x;
    const uint32_t v = e < n_events ? o.hit_offsets[e + 1] : 0u;
    uint32_t tot = 0;
    const uint32_t x = run + block_excl_scan(v, s_scan, tot);
    if (e < n_events) o.hit_offsets[e] = x;
    run += tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    o.hit_offsets[n_events] = run;
    o.module_start[(size_t)n_events * n_modules] = run;
    if (run > o.capacity) atomicCAS((unsigned int*)o.status, 0u, (unsigned int)PXT_ERR_CAPACITY);
  }
}

// Event-relative module offsets to absolute ones.
__global__ __launch_bounds__(256) void k_rh_absolute(RhOut o, uint32_t n_events,
                                                     uint32_t n_modules) {
  const uint32_t n = n_events * n_modules;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    o.module_start[i] += o.hit_offsets[i / n_modules];
}

__global__ __launch_bounds__(256) void k_rh_hits(RhIn in, RhOut o, const double* __restrict__ table,
                                                 uint32_t n_modules, uint32_t max_per_module) {
  if (o.status[0]) return;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < in.n_clusters; i += stride) {
    const uint32_t e = rh_event(in, i);
    const uint32_t m = in.module[i];
    // first cluster of module m in event e (modules non-decreasing)
    uint32_t lo = in.event_offsets[e], hi = i;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (in.module[mid] < m) lo = mid + 1; else hi = mid;
    }
    const uint32_t rank = i - lo;
    if (rank >= max_per_module) continue;
    const uint32_t h = o.module_start[(size_t)e * n_modules + m] + rank;
    double Q = 0.0, SU = 0.0, SV = 0.0;
    const uint32_t p1 = in.pixel_offsets[i + 1];
    for (uint32_t p = in.pixel_offsets[i]; p < p1; ++p) {
      const double q = (double)in.charge[p];
      Q += q;
      SU += q * ((double)in.pix_u[p] + 0.5);
      SV += q * ((double)in.pix_v[p] + 0.5);
    }
    o.module[h] = (uint16_t)m;
    o.cluster[h] = i;
    if (!(Q > 0.0)) {
      o.x[h] = 0.0f;
      o.y[h] = 0.0f;
      o.z[h] = 0.0f;
      o.layer[h] = -1;
      continue;
    }
    const double* T = table + 10 * (size_t)m;
    const double c = T[2], s = T[3], r = T[4], zc = T[5];
    const double u = T[6] + T[8] * (SU / Q);
    const double v = T[7] + T[9] * (SV / Q);
    double gx, gy, gz;
    if (T[1] == 0.0) {
      // tangent-plane point projected radially onto the layer cylinder
      const double f = r / sqrt(r * r + u * u);
      gx = (r * c - u * s) * f;
      gy = (r * s + u * c) * f;
      gz = zc + v;
    } else {
      gx = (r + u) * c - v * s;
      gy = (r + u) * s + v * c;
      gz = zc;
    }
    o.x[h] = (float)gx;
    o.y[h] = (float)gy;
    o.z[h] = (float)gz;
    o.layer[h] = (int16_t)T[0];
  }
}

}  // namespace pxt
