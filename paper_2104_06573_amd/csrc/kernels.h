// Pipeline kernels: binning, doublets, links, n-tuplets, cleaning, fit.
//
// Every kernel works on a ragged batch of events at once: hits of all
// events are flattened, and each per-item kernel recovers its event from
// the item (binary search of the event offsets for input hits, a stored id
// for binned hits).  One event is simply a batch of one.  Kernels whose work
// size is only known on the device (doublets, cells, tuples) take it from
// device memory and loop grid-stride, so a launch sequence never waits for
// the host and can be captured in a HIP graph.
#pragma once

#include "common.h"
#include "cuts.h"
#include "fit.h"
#include "vertex.h"

namespace pxt {

struct OutPtrs {
  uint32_t capacity;
  uint32_t* hit_idx;
  uint8_t* n_hits;
  uint32_t* event_id;
  float* params;
  float* cov;
  float* chi2;
  uint8_t* flags;
  uint32_t* per_event_tracks;
  pxt_counts* counts;
};

// Per-call values live in device memory (CallDesc, copied from a pinned
// host slot at the start of each call), so a launch sequence captured once
// in a HIP graph serves every later call: only the descriptor changes.
struct CallDesc {
  uint32_t n_events;
  uint32_t n_hits;
  uint32_t has_vtx;  // 1: find the vertices of the tracks into vtx
  uint32_t bin_lds;  // 1: binning by k_bin_events, 0: by k_prep .. k_rmax
  const float* x;
  const float* y;
  const float* z;
  const int16_t* layer;
  OutPtrs out;
  VtxOut vtx;
};

// ------------------------------------------------------------------ clear

__global__ void k_clear(Ws w, DevCfg c) {
  const CallDesc* cd = w.call;
  const uint32_t E = cd->n_events;
  const uint32_t nbins = E * (uint32_t)c.n_layers * (uint32_t)c.nphi;
  uint32_t* per_event_tracks = cd->out.per_event_tracks;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t stride = gridDim.x * blockDim.x;
  const bool glob = !cd->bin_lds;
  if (glob)
    for (uint32_t i = tid; i < nbins + 1; i += stride) w.bin_cnt[i] = 0;
  for (uint32_t i = tid; i < E; i += stride) per_event_tracks[i] = 0;
  if (tid < C_NCTR) w.ctr[tid] = tid == C_NBINS && glob ? nbins : 0u;
  if (tid == 0) w.epoch[0] += 1u;
}

// The cleaning's per-doublet election slots are tagged with the call (see
// order_key) instead of being cleared for every doublet of every call; they
// are reset in full on the first call and every 256th after it, when the
// tag byte wraps.
__global__ __launch_bounds__(256) void k_slots_clear(Ws w, DevCfg c) {
  if (((w.epoch[0] - 1u) & 0xffu) != 0u) return;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c.cap_doublets; i += stride) {
    w.bkey[i] = ~0ull;
    w.best[i] = 0ull;
  }
}

// Fills n 64-bit words with v (used where device memory must be reset
// without a memset node in a stream that may be captured).
__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ------------------------------------------------------- binning (prep) --

__device__ __forceinline__ uint32_t phi_bin(const DevCfg& c, float phi) {
  const int b = (int)((phi + kPiF) * c.phi_scale);
  return (uint32_t)(b < 0 ? 0 : (b >= c.nphi ? c.nphi - 1 : b));
}

__global__ __launch_bounds__(256) void k_prep(Ws w, DevCfg c) {
  const CallDesc* cd = w.call;
  if (cd->bin_lds) return;
  const uint32_t H = cd->n_hits, E = cd->n_events;
  const float* __restrict__ x = cd->x;
  const float* __restrict__ y = cd->y;
  const int16_t* __restrict__ layer = cd->layer;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < H; g += gridDim.x * blockDim.x) {
    const uint32_t e = upper_bound_u32(w.evt_off, E + 1, g) - 1;
    const int l = layer[g];
    if (l < 0 || l >= c.n_layers) {
      w.keys[g] = kPad;
      continue;
    }
    const float xf = x[g], yf = y[g];
    const uint32_t b = phi_bin(c, atan2f(yf, xf));
    const uint32_t key = (e * (uint32_t)c.n_layers + (uint32_t)l) * (uint32_t)c.nphi + b;
    w.keys[g] = key;
    atomicAdd(&w.bin_cnt[key], 1u);
  }
}

__global__ __launch_bounds__(256) void k_fill(Ws w) {
  const CallDesc* cd = w.call;
  if (cd->bin_lds) return;
  const uint32_t H = cd->n_hits, E = cd->n_events;
  const float* __restrict__ x = cd->x;
  const float* __restrict__ y = cd->y;
  const float* __restrict__ z = cd->z;
  const int16_t* __restrict__ layer = cd->layer;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < H; g += gridDim.x * blockDim.x) {
    const uint32_t key = w.keys[g];
    if (key == kPad) continue;
    const uint32_t e = upper_bound_u32(w.evt_off, E + 1, g) - 1;
    const uint32_t pos = w.bin_off[key] + atomicSub(&w.bin_cnt[key], 1u) - 1u;
    const float xf = x[g], yf = y[g];
    w.bh[pos] = make_float4(xf, yf, z[g], atan2f(yf, xf));
    w.br[pos] = hit_xyz(xf, yf, 0.0f).r;
    w.bidx[pos] = g - w.evt_off[e];
    w.bevt[pos] = e;
    w.blay[pos] = (uint8_t)layer[g];
  }
}

// Largest transverse radius of each (event, layer): one wavefront per
// segment of the binned array (hits of one layer of one event are
// contiguous), a max-reduction across lanes.  Also the turning angle
// asin(kmax r / 2) of a curvature-kmax circle through the origin out to
// that radius (slightly enlarged), the outer term of the doublet phi
// window; infinity where the window is the whole layer.
__device__ __forceinline__ void store_rmax(Ws& w, const DevCfg& c, uint32_t sg, float m) {
  w.rmax[sg] = __float_as_uint(m);
  const float ao = 0.5f * c.kmax_f * (m * 1.000001f);
  w.rasin[sg] = ao >= 0.70710678f ? __builtin_huge_valf() : asinf(ao);
}

__global__ __launch_bounds__(256) void k_rmax(Ws w, DevCfg c) {
  if (w.call->bin_lds) return;
  const uint32_t n_layers = (uint32_t)c.n_layers, nphi = (uint32_t)c.nphi;
  const uint32_t nseg = w.call->n_events * n_layers;
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nwaves = gridDim.x * blockDim.x / kWave;
  for (uint32_t sg = wid; sg < nseg; sg += nwaves) {
    const uint32_t b0 = w.bin_off[sg * nphi], b1 = w.bin_off[(sg + 1) * nphi];
    float m = 0.0f;
    for (uint32_t i = b0 + lane_id(); i < b1; i += kWave) m = fmaxf(m, (float)w.br[i]);
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, kWave));
    if (lane_id() == 0) store_rmax(w, c, sg, m);
  }
}

// ---------------------------------------------------- single-pass scan --
// Exclusive scan of n = *n_dev entries of `in` into out[0..n] (out[n] is
// the total, also stored in *total_dst when non-null), in one launch by
// decoupled look-back (Merrill & Garland,
// "Single-pass parallel prefix scan with decoupled look-back", 2016).  Tile
// ids are taken from an atomic ticket (zeroed per call by k_clear), so every
// tile a block waits for belongs to a block that is already running.  Each
// tile publishes a 64-bit status word [epoch:30 | flag:2 | value:32]
// (flag 1: tile aggregate, 2: inclusive prefix); the epoch is unique per
// call and per scan of the call, so words left by earlier scans never match
// and the status array needs no clearing.  A status word carries its whole
// message, so it is read and written with relaxed (coherent) atomics: no
// other memory is published through it, and acquire/release at device
// scope would write back or invalidate the L2 of the XCD on every access.
// The look-back spin is bounded: on exhaustion the call fails with
// PXT_ERR_HIP instead of hanging.

constexpr int kTileItems = 16;
constexpr int kScanThreads1 = 1024;  // threads per tile
constexpr int kTile = kScanThreads1 * kTileItems;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint64_t scan_word(uint32_t epoch, uint32_t flag, uint32_t v) {
  return ((uint64_t)(epoch & 0x3fffffffu) << 34) | ((uint64_t)flag << 32) | v;
}

// Publishes the aggregate of `tile` and returns the exclusive prefix of
// the tiles before it.  Called by the 64 lanes of the block's first
// wavefront: lane l inspects predecessor p - l, so one round trip covers 64
// predecessors; the walk stops at the nearest one holding an inclusive
// prefix, once every tile between has published its aggregate.
__device__ uint32_t tile_lookback(Ws& w, uint32_t tile, uint32_t epoch, uint32_t agg) {
  const uint32_t lane = lane_id();
  const uint32_t ep = epoch & 0x3fffffffu;
  if (tile == 0) {
    if (lane == 0)
      __hip_atomic_store(&w.scan_status[0], scan_word(epoch, 2, agg), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(&w.scan_status[tile], scan_word(epoch, 1, agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  uint32_t prefix = 0;
  int32_t p = (int32_t)tile - 1;
  uint32_t spins = 0;
  for (;;) {
    const int32_t q = p - (int32_t)lane;
    uint32_t flag = 2, val = 0;  // before tile 0: an inclusive zero
    if (q >= 0) {
      const uint64_t s =
          __hip_atomic_load(&w.scan_status[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      flag = (uint32_t)(s >> 34) == ep ? (uint32_t)(s >> 32) & 3u : 0u;
      val = (uint32_t)s;
    }
    const uint64_t incl = __ballot(flag == 2);
    const uint64_t waiting = __ballot(flag == 0);
    const uint32_t first = incl ? (uint32_t)__ffsll((unsigned long long)incl) - 1u : 64u;
    const uint64_t upto = first >= 63u ? ~0ull : (2ull << first) - 1ull;
    if (waiting & upto) {
      if (++spins > kSpinLimit) {
        if (lane == 0) set_status(w.ctr, PXT_ERR_HIP);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    prefix += wave_sum(lane <= first ? val : 0u);
    if (first < 64u) break;
    p -= 64;
  }
  if (lane == 0)
    __hip_atomic_store(&w.scan_status[tile], scan_word(epoch, 2, prefix + agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return prefix;
}

// Takes the block's tile from the scan's ticket; returns false for a
// block beyond the `ntiles` tiles.  The grid is sized for the capacity, so
// blocks past the tile count leave without touching the ticket: exactly
// the first ntiles blocks take tickets 0 .. ntiles-1.
__device__ __forceinline__ bool take_tile(Ws& w, uint32_t scan_id, uint32_t ntiles,
                                          uint32_t& tile) {
  if (blockIdx.x >= ntiles) return false;
  __shared__ uint32_t s_tile;
  if (threadIdx.x == 0) s_tile = atomicAdd(&w.ctr[C_TICKET0 + scan_id], 1u);
  __syncthreads();
  tile = s_tile;
  return tile < ntiles;
}

__global__ __launch_bounds__(kScanThreads1) void k_scan1(const uint32_t* __restrict__ in,
                                                uint32_t* __restrict__ out, const uint32_t* n_dev,
                                                uint32_t* total_dst, Ws w, uint32_t scan_id) {
  if (w.ctr[C_STATUS]) return;
  __shared__ uint32_t s_prefix;
  __shared__ uint32_t lds[kScanThreads1 / kWave + 1];
  const uint32_t n = *n_dev;
  const uint32_t ntiles = n ? (n + kTile - 1) / kTile : 1u;
  uint32_t tile;
  if (!take_tile(w, scan_id, ntiles, tile)) return;
  const uint32_t epoch = w.epoch[0] * 8u + scan_id;
  const uint32_t base = tile * kTile + threadIdx.x * kTileItems;
  // a thread's 16 consecutive items: four 16-byte loads in a full tile
  // (each load one cache line per lane instead of sixteen scalar loads)
  const bool full = base + kTileItems <= n;
  uint32_t v[kTileItems];
  if (full) {
#pragma unroll
    for (int q = 0; q < kTileItems / 4; ++q) {
      const uint4 t = reinterpret_cast<const uint4*>(in + base)[q];
      v[4 * q] = t.x;
      v[4 * q + 1] = t.y;
      v[4 * q + 2] = t.z;
      v[4 * q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kTileItems; ++i) v[i] = base + i < n ? in[base + i] : 0u;
  }
  uint32_t tsum = 0;
#pragma unroll
  for (int i = 0; i < kTileItems; ++i) tsum += v[i];
  uint32_t agg;
  const uint32_t texcl = block_excl_scan(tsum, lds, agg);
  if (threadIdx.x < kWave) {
    const uint32_t pf = tile_lookback(w, tile, epoch, agg);
    if (threadIdx.x == 0) s_prefix = pf;
  }
  __syncthreads();
  uint32_t run = s_prefix + texcl;
  if (full) {
#pragma unroll
    for (int q = 0; q < kTileItems / 4; ++q) {
      uint4 t;
      t.x = run;
      t.y = t.x + v[4 * q];
      t.z = t.y + v[4 * q + 1];
      t.w = t.z + v[4 * q + 2];
      run = t.w + v[4 * q + 3];
      reinterpret_cast<uint4*>(out + base)[q] = t;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kTileItems; ++i) {
      if (base + i < n) out[base + i] = run;
      run += v[i];
    }
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) {
    const uint32_t total = s_prefix + agg;
    out[n] = total;
    if (total_dst) *total_dst = total;
  }
}

// The root doublets of the n-tuplet search -- no inner neighbour, at least
// one outer neighbour -- listed in ascending order: a stream compaction of
// the doublets by the same single-pass scan over their root flags.
__global__ __launch_bounds__(kScanThreads1) void k_roots(Ws w, uint32_t scan_id) {
  if (w.ctr[C_STATUS]) return;
  __shared__ uint32_t s_prefix;
  __shared__ uint32_t lds[kScanThreads1 / kWave + 1];
  const uint32_t n = w.ctr[C_ND];
  const uint32_t ntiles = n ? (n + kTile - 1) / kTile : 1u;
  uint32_t tile;
  if (!take_tile(w, scan_id, ntiles, tile)) return;
  const uint32_t epoch = w.epoch[0] * 8u + scan_id;
  const uint32_t base = tile * kTile + threadIdx.x * kTileItems;
  uint32_t flags = 0;
  if (base + kTileItems <= n) {
    // 16 flags of each kind as one 16-byte load
    const uint4 hv = *reinterpret_cast<const uint4*>(w.has_inner + base);
    const uint4 ov = *reinterpret_cast<const uint4*>(w.has_out + base);
    const uint32_t hw[4] = {hv.x, hv.y, hv.z, hv.w};
    const uint32_t ow[4] = {ov.x, ov.y, ov.z, ov.w};
#pragma unroll
    for (int q = 0; q < kTileItems / 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (((hw[q] >> (8 * b)) & 0xffu) == 0u && ((ow[q] >> (8 * b)) & 0xffu) != 0u)
          flags |= 1u << (4 * q + b);
  } else {
#pragma unroll
    for (int i = 0; i < kTileItems; ++i)
      if (base + i < n && !w.has_inner[base + i] && w.has_out[base + i]) flags |= 1u << i;
  }
  uint32_t agg;
  const uint32_t texcl = block_excl_scan((uint32_t)__popc(flags), lds, agg);
  if (threadIdx.x < kWave) {
    const uint32_t pf = tile_lookback(w, tile, epoch, agg);
    if (threadIdx.x == 0) s_prefix = pf;
  }
  __syncthreads();
  uint32_t run = s_prefix + texcl;
  while (flags) {
    const int i = __ffs(flags) - 1;
    flags &= flags - 1u;
    w.roots[run++] = base + (uint32_t)i;
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) w.ctr[C_NROOT] = s_prefix + agg;
}

// Binning with one block per event (an event's hits are contiguous in the
// input, a few thousand to a few tens of thousands of them): the event's
// (layer, phi bin) histogram, its exclusive scan, the fill cursors and each
// layer's largest radius all live in LDS, so no global atomics are made;
// only the event's place in the binned array comes from a decoupled
// look-back over the events before it (one tile per event, tiles taken in
// order from the ticket).  Used when the histogram (n_layers x phi bins
// counters) fits kBinLdsBins and the call has many events or only small
// ones: one block of one CU cannot bin a single large event as fast as the
// whole device does.  The layout it writes is the one k_prep, the scan,
// k_fill and k_rmax write (the order within a bin is arbitrary in both).
// The call's descriptor names the set that runs (a graph holds one set);
// the kernels of the other leave at once.
constexpr int kBinThreads = 1024;
constexpr uint32_t kBinLdsBins = 12288;  // 48 KB of counters
constexpr uint32_t kBinScan = 2;         // scan id of the event offsets (the global
                                         // binning's scan is id 0)
constexpr int kBinUnroll = 8;
constexpr uint32_t kBinLdsEvents = 8;     // calls of at least this many events,
constexpr uint32_t kBinLdsHits = 8192;    // or whose events are all this small

__global__ __launch_bounds__(kBinThreads) void k_bin_events(Ws w, DevCfg c) {
  extern __shared__ uint32_t s_hist[];  // [n_layers * nphi]
  __shared__ uint32_t s_lds[kBinThreads / kWave + 1];
  __shared__ uint32_t s_rmax[kMaxLayers];
  __shared__ uint32_t s_base;
  const CallDesc* cd = w.call;
  const uint32_t E = cd->n_events;
  if (!cd->bin_lds) return;
  if (E == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) w.bin_off[0] = 0u;
    return;
  }
  uint32_t e;
  if (!take_tile(w, kBinScan, E, e)) return;
  const float* __restrict__ x = cd->x;
  const float* __restrict__ y = cd->y;
  const float* __restrict__ z = cd->z;
  const int16_t* __restrict__ layer = cd->layer;
  const uint32_t tid = threadIdx.x;
  const uint32_t L = (uint32_t)c.n_layers, nphi = (uint32_t)c.nphi, per_ev = L * nphi;
  const uint32_t h0 = w.evt_off[e], h1 = w.evt_off[e + 1];
  for (uint32_t k = tid; k < per_ev; k += kBinThreads) s_hist[k] = 0u;
  if (tid < L) s_rmax[tid] = 0u;
  __syncthreads();
  // (each thread loads kBinUnroll hits before using any: the loads of a
  // round are in flight together)
  for (uint32_t g0 = h0 + tid; g0 < h1; g0 += kBinUnroll * kBinThreads) {
    int l[kBinUnroll];
    float xf[kBinUnroll], yf[kBinUnroll];
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u) {
      const uint32_t g = g0 + (uint32_t)u * kBinThreads;
      l[u] = g < h1 ? layer[g] : -1;
      xf[u] = g < h1 ? x[g] : 0.0f;
      yf[u] = g < h1 ? y[g] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u)
      if (l[u] >= 0 && l[u] < (int)L)
        atomicAdd(&s_hist[(uint32_t)l[u] * nphi + phi_bin(c, atan2f(yf[u], xf[u]))], 1u);
  }
  __syncthreads();
  // exclusive scan of the histogram in place: thread t sums its run of
  // consecutive counters, the block scans the sums
  const uint32_t per = (per_ev + kBinThreads - 1) / kBinThreads;
  const uint32_t k0 = min(per_ev, tid * per), k1 = min(per_ev, k0 + per);
  uint32_t tsum = 0;
  for (uint32_t k = k0; k < k1; ++k) tsum += s_hist[k];
  uint32_t agg;
  uint32_t run = block_excl_scan(tsum, s_lds, agg);
  if (tid < kWave) {
    const uint32_t pf = tile_lookback(w, e, w.epoch[0] * 8u + kBinScan, agg);
    if (tid == 0) s_base = pf;
  }
  for (uint32_t k = k0; k < k1; ++k) {
    const uint32_t n = s_hist[k];
    s_hist[k] = run;
    run += n;
  }
  __syncthreads();
  const uint32_t base = s_base;
  for (uint32_t k = tid; k < per_ev; k += kBinThreads) w.bin_off[e * per_ev + k] = base + s_hist[k];
  if (e == E - 1 && tid == 0) {
    w.bin_off[E * per_ev] = base + agg;
    w.ctr[C_NBINNED] = base + agg;
  }
  for (uint32_t g0 = h0 + tid; g0 < h1; g0 += kBinUnroll * kBinThreads) {
    int l[kBinUnroll];
    float xf[kBinUnroll], yf[kBinUnroll], zf[kBinUnroll];
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u) {
      const uint32_t g = g0 + (uint32_t)u * kBinThreads;
      l[u] = g < h1 ? layer[g] : -1;
      xf[u] = g < h1 ? x[g] : 0.0f;
      yf[u] = g < h1 ? y[g] : 0.0f;
      zf[u] = g < h1 ? z[g] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u) {
      if (!(l[u] >= 0 && l[u] < (int)L)) continue;
      const float phi = atan2f(yf[u], xf[u]);
      const uint32_t pos =
          base + atomicAdd(&s_hist[(uint32_t)l[u] * nphi + phi_bin(c, phi)], 1u);
      const double r = hit_xyz(xf[u], yf[u], 0.0f).r;
      w.bh[pos] = make_float4(xf[u], yf[u], zf[u], phi);
      w.br[pos] = r;
      w.bidx[pos] = g0 + (uint32_t)u * kBinThreads - h0;
      w.bevt[pos] = e;
      w.blay[pos] = (uint8_t)l[u];
      atomicMax(&s_rmax[l[u]], __float_as_uint((float)r));
    }
  }
  __syncthreads();
  if (tid < L) store_rmax(w, c, e * L + tid, __uint_as_float(s_rmax[tid]));
}

// ------------------------------------------------------------- doublets --
// For every binned inner hit and every layer pair leaving its layer, the
// outer layer's hits are visited only inside a phi window that is a
// superset of every pair passing D3/D4: a circle through the origin with
// curvature <= kmax turns by asin(kmax r_o / 2) - asin(kmax r_i / 2) between
// radii r_i and r_o, which grows with r_o, so the window uses the largest
// outer radius of the event's layer, plus one guard bin per side.  The cut
// itself decides, so the window never changes the result.
//
// Work split: a group of G lanes handles one inner hit; its lanes take
// consecutive candidates of the window, so the candidate loads are
// coalesced, and a ballot over the group gives each accepted doublet its
// position among the hit's doublets, so the writes are coalesced too and
// keep the candidate order.  Doublets are stored grouped by inner hit
// (binned order), in candidate order within a hit.

// Candidate runs of one (inner hit, outer layer) pair: the binned hits of
// the phi window, two runs when it wraps around; none when the layer lies
// inside the inner radius.
struct PairWin {
  uint32_t s0b, s0n, s1b, s1n;
};

__device__ __forceinline__ PairWin pair_window(const Ws& w, const DevCfg& c, uint32_t e, int lo,
                                               float ri, float phi, float ai) {
  PairWin r{0u, 0u, 0u, 0u};
  const uint32_t el = e * (uint32_t)c.n_layers + (uint32_t)lo;
  const float rmo = __uint_as_float(w.rmax[el]) * 1.000001f;
  if (!(rmo > ri * 0.999999f)) return r;
  const uint32_t bb = el * (uint32_t)c.nphi;
  const float ao = w.rasin[el];
  int blo = 0, bhi = c.nphi - 1;
  bool full = !(ao < __builtin_huge_valf());
  if (!full) {
    const float W = ao - ai;
    if (!(W >= 0.0f && W < 4.0f && phi >= -4.0f && phi <= 4.0f)) {
      full = true;  // non-finite input: fall back to the whole layer
    } else {
      blo = (int)floorf((phi - W + kPiF) * c.phi_scale) - 1;
      bhi = (int)floorf((phi + W + kPiF) * c.phi_scale) + 1;
      full = bhi - blo + 1 >= c.nphi;
    }
  }
  if (full) {
    r.s0b = w.bin_off[bb];
    r.s0n = w.bin_off[bb + c.nphi] - r.s0b;
  } else if (blo < 0) {
    r.s0b = w.bin_off[bb + blo + c.nphi];
    r.s0n = w.bin_off[bb + c.nphi] - r.s0b;
    r.s1b = w.bin_off[bb];
    r.s1n = w.bin_off[bb + bhi + 1] - r.s1b;
  } else if (bhi >= c.nphi) {
    r.s0b = w.bin_off[bb + blo];
    r.s0n = w.bin_off[bb + c.nphi] - r.s0b;
    r.s1b = w.bin_off[bb];
    r.s1n = w.bin_off[bb + bhi - c.nphi + 1] - r.s1b;
  } else {
    r.s0b = w.bin_off[bb + blo];
    r.s0n = w.bin_off[bb + bhi + 1] - r.s0b;
  }
  return r;
}

template <int G>
__device__ __forceinline__ uint64_t group_mask() {
  const uint32_t grp = lane_id() / G;
  return G == 64 ? ~0ull : ((1ull << (G % 64)) - 1ull) << (grp * G);
}

// The tiles (one round of a block's lane groups: blockDim/G consecutive
// inner hits) a block visits: each XCD owns a contiguous eighth of the
// tiles (its events stay in its L2) and its blocks take them in turn, so
// every block meets hits of all layers (the inner layers have several
// times the doublets of the outer ones).
struct TileWalk {
  uint32_t t, end, step;
};

__device__ __forceinline__ TileWalk tile_walk(uint32_t ntiles) {
  if (gridDim.x % 8u) return TileWalk{blockIdx.x, ntiles, gridDim.x};
  const uint32_t x = blockIdx.x % 8u, per = (ntiles + 7u) / 8u;
  return TileWalk{x * per + blockIdx.x / 8u, min(ntiles, (x + 1u) * per), gridDim.x / 8u};
}

// Visits the candidates of inner hit g with its lane group (inactive groups
// visit none) and calls round(ok, j, hi, ho, bal, cnt) once per round of G
// candidates with the whole wavefront: ok = lane's candidate j passes the
// doublet cuts, bal = the wavefront's ballot of ok, cnt = the group's
// accepted doublets before this round.  Returns the group's total.  The
// cuts take early exits: fewer instructions than evaluating every cut on
// every lane, which is what counts with several batches sharing the GPU.
template <int G, typename F>
__device__ __forceinline__ uint32_t visit_doublets(const Ws& w, const DevCfg& c, bool active,
                                                   uint32_t g, F&& round) {
  const uint32_t sub = lane_id() % G;
  const uint64_t gmask = group_mask<G>();
  int li = 0, npairs = 0;
  uint32_t e = 0;
  HitD hi{0.0, 0.0, 0.0, 0.0};
  float ri = 0.0f, phi = 0.0f;
  if (active) {
    li = w.blay[g];
    e = w.bevt[g];
    const float4 v = w.bh[g];
    hi = HitD{(double)v.x, (double)v.y, (double)v.z, w.br[g]};
    ri = (float)hi.r;
    phi = v.w;
    npairs = c.n_outer[li];
  }
  const float ai = asinf(0.5f * c.kmax_f * ri);  // inner term of the phi window
  // the windows of all pairs at once, lane sub of the group computing pairs
  // sub, sub + G, ... (their loads in flight together); the pair loop takes
  // them from that lane
  constexpr int NP = (kMaxOuterPerLayer + G - 1) / G;
  PairWin pws[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int p = (int)sub + u * G;
    pws[u] = PairWin{0u, 0u, 0u, 0u};
    if (active && p < npairs) pws[u] = pair_window(w, c, e, c.outer[li][p], ri, phi, ai);
  }
  const int gl = (int)(lane_id() - sub);  // the group's first lane
  uint32_t cnt = 0;
  for (uint32_t p = 0; __any((int)p < npairs); ++p) {
    const uint32_t u = p / G;
    PairWin src = pws[0];
#pragma unroll
    for (int x = 1; x < NP; ++x)
      if (u == (uint32_t)x) src = pws[x];
    const int from = gl + (int)(p % G);
    PairWin pw{(uint32_t)__shfl((int)src.s0b, from), (uint32_t)__shfl((int)src.s0n, from),
               (uint32_t)__shfl((int)src.s1b, from), (uint32_t)__shfl((int)src.s1n, from)};
    if (!(active && (int)p < npairs)) pw = PairWin{0u, 0u, 0u, 0u};
    const uint32_t tot = pw.s0n + pw.s1n;
    // software-pipelined: the next round's candidate is loaded before the
    // current one is tested
    auto cand = [&](uint32_t k) { return k < pw.s0n ? pw.s0b + k : pw.s1b + (k - pw.s0n); };
    float4 nv = make_float4(0.f, 0.f, 0.f, 0.f);
    double nr = 0.0;
    if (sub < tot) {
      const uint32_t j0 = cand(sub);
      nv = w.bh[j0];
      nr = w.br[j0];
    }
    for (uint32_t it = 0; __any(it * G < tot); ++it) {
      const uint32_t k = it * G + sub;
      const bool valid = k < tot;
      const uint32_t j = valid ? cand(k) : 0u;
      const HitD ho{(double)nv.x, (double)nv.y, (double)nv.z, nr};
      const uint32_t k1 = k + G;
      if (k1 < tot) {
        const uint32_t j1 = cand(k1);
        nv = w.bh[j1];
        nr = w.br[j1];
      }
      const bool ok = valid && doublet_ok_fast(c, hi, ho);
      const uint64_t bal = __ballot(ok);
      round(ok, j, hi, ho, bal, cnt);
      cnt += (uint32_t)__popcll(bal & gmask);
    }
  }
  return cnt;
}

// The per-doublet arrays written when doublet q = (g, j) is stored.
__device__ __forceinline__ void store_doublet(Ws& w, const DevCfg& c, uint32_t q, uint32_t g,
                                              uint32_t j, const HitD& hi, const HitD& ho) {
  w.cio[q] = make_uint2(g, j);
  w.has_inner[q] = 0;
  if (c.link_kernel == 1) w.has_out[q] = 0;
  w.th[q] = angle_units(rz_angle(hi, ho));
}

// Link-mask words of the largest out-degree: C_WSTRIDE is raised only when
// a block needs more than it already holds (a coherent load first), so the
// blocks do not all contend for one address.
__device__ __forceinline__ void raise_stride(Ws& w, uint32_t words) {
  if (words > __hip_atomic_load(&w.ctr[C_WSTRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(&w.ctr[C_WSTRIDE], words);
}

// Two passes: count (dcnt, then a scan gives cell_off) and fill, each
// evaluating the cuts.
template <int G, bool FILL>
__global__ __launch_bounds__(256) void k_doublets(Ws w, DevCfg c) {
  const uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t nb = ctr[C_NBINNED];
  if (FILL && w.cell_off[nb] > c.cap_doublets) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      set_status(w.ctr, PXT_ERR_CAPACITY);
      w.ctr[C_REQ_D] = w.cell_off[nb];
    }
    return;
  }
  const uint32_t lane = lane_id(), sub = lane % G;
  const uint64_t below = group_mask<G>() & ((1ull << lane) - 1ull);
  const uint32_t gpb = blockDim.x / G, gib = threadIdx.x / G;
  uint32_t wneed = 0;  // count pass: link-mask words of the largest out-degree
  for (TileWalk tw = tile_walk((nb + gpb - 1) / gpb); tw.t < tw.end; tw.t += tw.step) {
    const uint32_t g = tw.t * gpb + gib;
    const bool active = g < nb;
    const uint32_t pos = (FILL && active) ? w.cell_off[g] : 0u;
    const uint32_t cnt = visit_doublets<G>(
        w, c, active, g,
        [&](bool ok, uint32_t j, const HitD& hi, const HitD& ho, uint64_t bal, uint32_t before) {
          if (FILL && ok)
            store_doublet(w, c, pos + before + (uint32_t)__popcll(bal & below), g, j, hi, ho);
        });
    if (!FILL) {
      if (active && sub == 0) w.dcnt[g] = cnt;
      wneed = max(wneed, (cnt + 63u) >> 6);
    }
  }
  if (!FILL) {
    __shared__ uint32_t s_w[256 / kWave];
    const uint32_t wm = wave_max(wneed);
    if (lane == 0) s_w[threadIdx.x / kWave] = wm;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t m = 0;
      for (uint32_t i = 0; i < blockDim.x / kWave; ++i) m = max(m, s_w[i]);
      if (m) raise_stride(w, m);
    }
  }
}

// One pass: the cuts are evaluated once.  A tile is one round of the
// block's lane groups (blockDim/G consecutive inner hits); tiles are taken
// from a ticket and chained by decoupled look-back, like the scan tiles.
// Accepted candidates are staged in an LDS pool of 32-bit records
// (hit of the tile: 6 bits, index among that hit's doublets: 9 bits, outer
// hit relative to the first binned hit of its event: 17 bits); once the
// first wavefront has scanned the tile's per-hit counts and taken the
// tile's offset, every record is written to offset + the hit's exclusive
// count + its index, the same layout as the two-pass kernels.  A tile whose
// records do not fit (pool full, a hit with 512 doublets or more, an event
// of 2^17 binned hits or more) evaluates its cuts again and writes in place.
constexpr uint32_t kPoolKBits = 9, kPoolJBits = 17;
constexpr uint32_t kPoolRecords = 4096;  // LDS pool of the one-pass kernel (16 KB)
constexpr uint32_t kDoubletScan = 1;     // scan id of the doublet offsets

__device__ __forceinline__ uint32_t pool_record(uint32_t h, uint32_t k, uint32_t jr) {
  return (h << (kPoolKBits + kPoolJBits)) | (k << kPoolJBits) | jr;
}

template <int G>
__global__ __launch_bounds__(256) void k_doublets1(Ws w, DevCfg c) {
  constexpr uint32_t pool_cap = kPoolRecords;
  __shared__ uint32_t s_pool[kPoolRecords];
  __shared__ uint32_t s_cnt[kWave], s_excl[kWave], s_ebase[kWave];
  __shared__ uint32_t s_n, s_over, s_prefix, s_agg;
  const uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t nb = ctr[C_NBINNED];
  const uint32_t gpb = blockDim.x / G, gib = threadIdx.x / G;
  const uint32_t ntiles = nb ? (nb + gpb - 1) / gpb : 1u;
  uint32_t tile;
  if (!take_tile(w, kDoubletScan, ntiles, tile)) return;
  const uint32_t epoch = w.epoch[0] * 8u + kDoubletScan;
  const uint32_t lane = lane_id(), sub = lane % G;
  const uint64_t lbelow = (1ull << lane) - 1ull;
  const uint64_t below = group_mask<G>() & lbelow;
  const uint32_t t0 = tile * gpb, g = t0 + gib;
  const bool active = g < nb;
  const uint32_t per_ev = (uint32_t)c.n_layers * (uint32_t)c.nphi;
  if (threadIdx.x == 0) {
    s_n = 0;
    s_over = 0;
  }
  if (sub == 0) s_ebase[gib] = active ? w.bin_off[w.bevt[g] * per_ev] : 0u;
  __syncthreads();
  const uint32_t ebase = s_ebase[gib];
  const uint32_t cnt = visit_doublets<G>(
      w, c, active, g,
      [&](bool ok, uint32_t j, const HitD&, const HitD&, uint64_t bal, uint32_t before) {
        if (!bal) return;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&s_n, (uint32_t)__popcll(bal));
        base = __shfl(base, 0);
        if (ok) {
          const uint32_t k = before + (uint32_t)__popcll(bal & below);
          const uint32_t jr = j - ebase;
          const uint32_t slot = base + (uint32_t)__popcll(bal & lbelow);
          if (slot < pool_cap && k < (1u << kPoolKBits) && jr < (1u << kPoolJBits))
            s_pool[slot] = pool_record(gib, k, jr);
          else
            s_over = 1;
        }
      });
  if (sub == 0) s_cnt[gib] = active ? cnt : 0u;
  __syncthreads();
  if (threadIdx.x < kWave) {
    const uint32_t v = lane < gpb ? s_cnt[lane] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    const uint32_t agg = __shfl(inc, kWave - 1);
    s_excl[lane] = inc - v;
    const uint32_t wm = wave_max((v + 63u) >> 6);
    const uint32_t pf = tile_lookback(w, tile, epoch, agg);
    if (lane == 0) {
      s_prefix = pf;
      s_agg = agg;
      if (wm) raise_stride(w, wm);
      if (tile == ntiles - 1) {
        const uint32_t total = pf + agg;
        w.cell_off[nb] = total;
        w.ctr[C_ND] = total;
        if (total > c.cap_doublets) {
          set_status(w.ctr, PXT_ERR_CAPACITY);
          w.ctr[C_REQ_D] = total;
        }
      }
    }
  }
  __syncthreads();
  const uint32_t prefix = s_prefix;
  if (active && sub == 0) w.cell_off[g] = prefix + s_excl[gib];
  if (prefix + s_agg > c.cap_doublets) return;  // the call fails with the capacity status
  if (!s_over) {
    const uint32_t n = s_n;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t r = s_pool[i];
      const uint32_t h = r >> (kPoolKBits + kPoolJBits);
      const uint32_t k = (r >> kPoolJBits) & ((1u << kPoolKBits) - 1u);
      const uint32_t gi = t0 + h, j = s_ebase[h] + (r & ((1u << kPoolJBits) - 1u));
      store_doublet(w, c, prefix + s_excl[h] + k, gi, j, load_hit(w, gi), load_hit(w, j));
    }
  } else {
    const uint32_t pos = prefix + s_excl[gib];
    visit_doublets<G>(
        w, c, active, g,
        [&](bool ok, uint32_t j, const HitD& hi, const HitD& ho, uint64_t bal, uint32_t before) {
          if (ok) store_doublet(w, c, pos + before + (uint32_t)__popcll(bal & below), g, j, hi, ho);
        });
  }
}

// Staged doublets, for large batches: the cuts are evaluated once, without
// the one-pass kernel's tile-to-tile wait (a tile's count is known only
// once its cuts are done, so with very uneven tiles resident blocks queue
// behind a slow one).  k_dstage is the count pass, which also appends every
// accepted pair, as an 8-byte record (inner hit << 9 | index among its
// doublets, outer hit), to its wavefront's region of the staging buffer;
// the scan turns the per-hit counts into offsets; in k_dscatter (same
// grid) each wavefront writes its region's records to their hit's offset +
// index.  Wavefronts work alone (a cursor in registers, no block barrier),
// and the scatter issues the loads of four records per lane before any
// store.  A wavefront whose records do not fit (region full, an index of
// 512 or more, an inner hit beyond 2^23) evaluates the cuts of its hits
// again in the scatter instead.
constexpr uint32_t kRecKBits = 9, kRecGMax = 1u << 23;
constexpr uint32_t kRecOver = 0xffffffffu;  // region count of an overflowed wavefront

__device__ __forceinline__ uint2* stage_region(const Ws& w, uint32_t& cap, uint32_t& id) {
  const uint32_t nw = blockDim.x / kWave;
  id = blockIdx.x * nw + threadIdx.x / kWave;
  cap = (w.stage_words / 2u) / (gridDim.x * nw);
  return reinterpret_cast<uint2*>(w.stage) + (size_t)id * cap;
}

template <int G>
__global__ __launch_bounds__(256) void k_dstage(Ws w, DevCfg c) {
  __shared__ uint32_t s_w[256 / kWave];
  if (w.ctr[C_STATUS]) return;
  const uint32_t nb = w.ctr[C_NBINNED];
  const uint32_t lane = lane_id(), sub = lane % G, wib = threadIdx.x / kWave;
  const uint64_t lbelow = (1ull << lane) - 1ull;
  const uint64_t below = group_mask<G>() & lbelow;
  const uint32_t gpb = blockDim.x / G, gib = threadIdx.x / G;
  uint32_t cap, id;
  uint2* reg = stage_region(w, cap, id);
  uint32_t run = 0, wneed = 0;
  bool over = false;
  for (TileWalk tw = tile_walk((nb + gpb - 1) / gpb); tw.t < tw.end; tw.t += tw.step) {
    const uint32_t g = tw.t * gpb + gib;
    const bool active = g < nb;
    const uint32_t cnt = visit_doublets<G>(
        w, c, active, g,
        [&](bool ok, uint32_t j, const HitD&, const HitD&, uint64_t bal, uint32_t before) {
          if (ok) {
            const uint32_t k = before + (uint32_t)__popcll(bal & below);
            const uint32_t slot = run + (uint32_t)__popcll(bal & lbelow);
            if (slot < cap && k < (1u << kRecKBits) && g < kRecGMax)
              reg[slot] = make_uint2((g << kRecKBits) | k, j);
            else
              over = true;
          }
          run += (uint32_t)__popcll(bal);
        });
    if (active && sub == 0) w.dcnt[g] = cnt;
    wneed = max(wneed, (cnt + 63u) >> 6);
  }
  const bool wover = __any(over);
  if (lane == 0) w.dwn[id] = wover ? kRecOver : run;
  const uint32_t wm = wave_max(wneed);
  if (lane == 0) s_w[wib] = wm;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (uint32_t i = 0; i < blockDim.x / kWave; ++i) m = max(m, s_w[i]);
    if (m) raise_stride(w, m);
  }
}

template <int G>
__global__ __launch_bounds__(256) void k_dscatter(Ws w, DevCfg c) {
  if (w.ctr[C_STATUS]) return;
  const uint32_t nb = w.ctr[C_NBINNED];
  if (w.cell_off[nb] > c.cap_doublets) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      set_status(w.ctr, PXT_ERR_CAPACITY);
      w.ctr[C_REQ_D] = w.cell_off[nb];
    }
    return;
  }
  const uint32_t lane = lane_id();
  uint32_t cap, id;
  const uint2* reg = stage_region(w, cap, id);
  const uint32_t n = w.dwn[id];
  if (n == kRecOver) {
    // records incomplete: this wavefront's hits evaluate the cuts again
    const uint64_t below = group_mask<G>() & ((1ull << lane) - 1ull);
    const uint32_t gpb = blockDim.x / G, gib = threadIdx.x / G;
    for (TileWalk tw = tile_walk((nb + gpb - 1) / gpb); tw.t < tw.end; tw.t += tw.step) {
      const uint32_t g = tw.t * gpb + gib;
      const bool active = g < nb;
      const uint32_t pos = active ? w.cell_off[g] : 0u;
      visit_doublets<G>(
          w, c, active, g,
          [&](bool ok, uint32_t j, const HitD& hi, const HitD& ho, uint64_t bal,
              uint32_t before) {
            if (ok)
              store_doublet(w, c, pos + before + (uint32_t)__popcll(bal & below), g, j, hi, ho);
          });
    }
    return;
  }
  constexpr int U = 4;
  for (uint32_t i0 = 0; i0 < n; i0 += U * kWave) {
    uint2 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = i0 + (uint32_t)u * kWave + lane;
      r[u] = i < n ? reg[i] : make_uint2(0u, 0u);
    }
    // every load of the four records before any store (the stores could
    // alias the loaded arrays as far as the compiler knows)
    uint32_t q[U];
    float iz[U];
    double ir[U];
    HitD ho[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t g = r[u].x >> kRecKBits;
      q[u] = w.cell_off[g] + (r[u].x & ((1u << kRecKBits) - 1u));
      iz[u] = w.bh[g].z;
      ir[u] = w.br[g];
      ho[u] = load_hit(w, r[u].y);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + (uint32_t)u * kWave + lane < n) {
        const HitD hi{0.0, 0.0, (double)iz[u], ir[u]};
        store_doublet(w, c, q[u], r[u].x >> kRecKBits, r[u].y, hi, ho[u]);
      }
    }
  }
}

// ---------------------------------------------------------------- links --
// The candidate outer neighbours of doublet (a,b) are the doublets leaving
// hit b: the contiguous range cell_off[b] .. cell_off[b+1] (doublets are
// stored grouped by inner hit).  The angle prefilter, which passes only a
// few percent, streams the doublets' r-z angles (th, 16-bit units),
// and the survivors go on to the exact FP64 cuts with their three hits
// loaded from the binned-hit array (hit-indexed, a few MB per batch), not
// from per-doublet copies.  The accepted candidates form a bit mask over
// the range, one 64-bit word per 64.

// The link masks take C_WSTRIDE words per doublet (one word per 64
// candidates of the largest out-degree of the batch), stored word-major:
// word k of doublet d is masks[k * nd + d], so the words that consecutive
// doublets write are contiguous; only the words a doublet needs are
// touched.
__device__ __forceinline__ bool links_capacity(Ws& w, const DevCfg& c) {
  const uint64_t nwords = (uint64_t)w.ctr[C_ND] * w.ctr[C_WSTRIDE];
  const bool ok = nwords <= c.cap_words;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    w.ctr[C_NWORDS] = (uint32_t)min(nwords, 0xffffffffull);
    if (!ok) {
      set_status(w.ctr, PXT_ERR_CAPACITY);
      w.ctr[C_REQ_W] = (uint32_t)min(nwords, 0xffffffffull);
    }
  }
  return ok;
}

// Candidate range of a doublet with outer hit j: the doublets leaving j,
// from the per-hit offsets (the n-tuplet search finds it the same way).
__device__ __forceinline__ void outer_range(const Ws& w, uint32_t j, uint32_t& kb,
                                            uint32_t& deg) {
  kb = w.cell_off[j];
  deg = w.cell_off[j + 1] - kb;
}

// One thread per doublet (a,b) for its set-up (mask words and has-outer
// flag cleared, hit indices fetched); the angle prefilter over the candidates is spread
// evenly over the wavefront's lanes (below).  The few survivors are not tested
// in place -- their exact FP64 tests would run with most lanes idle -- but
// appended to a per-wavefront queue in LDS (ballot compaction) together
// with the doublet's hits, so that whenever 64 are queued they are tested
// with all lanes busy.  A doublet's mask words and has-outer flag are
// cleared by its own thread before any of its candidates is queued;
// accepted links set their bit with atomicOr.

// Queue entry: qa = (doublet, candidate doublet, inner hit, outer hit),
// qb = (candidate index, the doublet's number of candidates).  The flush
// loads the candidate's outer hit index and the three hits.
__device__ __forceinline__ void links_thread_flush(Ws& w, const DevCfg& c, const uint4* qa,
                                                   const uint2* qb, uint32_t n, uint32_t nd,
                                                   uint32_t& links) {
  const uint32_t lane = lane_id();
  if (lane < n) {
    const uint4 ea = qa[lane];
    const uint2 eb = qb[lane];
    const uint32_t d = ea.x, d2 = ea.y, k = eb.x;
    // the FP64 radii are loaded with the coordinates (an FP64 square root
    // per hit costs more than the load)
    const HitD ha = load_hit(w, ea.z), hb = load_hit(w, ea.w);
    const HitD hc = load_hit(w, w.cio[d2].y);
    if (link_rz_pass(c, ha, hb, hc.r, hc.z) && link_xy_pass(c, ha, hb, hc)) {
      atomicOr((unsigned long long*)&w.masks[(size_t)(k >> 6) * nd + d], 1ull << (k & 63u));
      w.has_out[d] = 1;
      w.has_inner[d2] = 1;
      ++links;
    }
  }
}

__global__ __launch_bounds__(256) void k_links_thread(Ws w, DevCfg c) {
  __shared__ uint4 s_qa[256 / kWave][kQueue];
  __shared__ uint2 s_qb[256 / kWave][kQueue];
  uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t nd = ctr[C_ND];
  if (!links_capacity(w, c)) return;
  const uint32_t lane = lane_id(), wib = threadIdx.x / kWave;
  const uint64_t below = (1ull << lane) - 1ull;
  uint4* qa = s_qa[wib];
  uint2* qb = s_qb[wib];
  uint32_t links = 0, qn = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  // every lane of the wavefront runs the same number of rounds, so the
  // queue's ballots see all lanes
  const uint32_t d0 = xcd_block() * blockDim.x + (threadIdx.x & ~(uint32_t)(kWave - 1));
  for (uint32_t dw = d0; dw < nd; dw += stride) {
    const uint32_t d = dw + lane;
    uint32_t k0 = 0, deg = 0, ha = 0, hb = 0;
    int tho = 0;  // the doublet's r-z angle (units)
    if (d < nd) {
      const uint2 io = w.cio[d];
      ha = io.x;
      hb = io.y;
      outer_range(w, hb, k0, deg);
      tho = w.th[d];
      const uint32_t nwd = (deg + 63u) >> 6;
      for (uint32_t j = 0; j < nwd; ++j) w.masks[(size_t)j * nd + d] = 0;
      w.has_out[d] = 0;
    }
    __threadfence_block();
    // the prefilter in chunks of 16 candidates spread evenly over the lanes:
    // a doublet's candidates (absolute indices k0 .. k0+deg-1) form the
    // 8-aligned chunks starting at (k0 & ~7) + 16 i; the wavefront's chunks
    // are numbered by a prefix sum over its doublets, and in each round
    // every lane takes the next chunk, finds its doublet by a binary search
    // of the prefix (shuffles) and reads the 16 16-bit angles as two aligned
    // 16-byte vectors
    const uint32_t nch = deg ? (k0 + deg - (k0 & ~7u) + 15u) >> 4 : 0u;
    const uint32_t cinc = wave_incl_scan(nch), cex = cinc - nch;
    const uint32_t C = __shfl(cinc, kWave - 1);
    for (uint32_t r0 = 0; r0 < C; r0 += kWave) {
      const uint32_t q = r0 + lane;
      // owner: the last lane whose chunks start at or before q
      uint32_t own = 0;
#pragma unroll
      for (uint32_t step = kWave / 2; step >= 1; step >>= 1)
        if (__shfl(cex, (int)(own + step)) <= q) own += step;
      const uint32_t ok0 = __shfl(k0, (int)own), odeg = __shfl(deg, (int)own);
      const int ta = __shfl(tho, (int)own);
      const uint32_t lo = ok0, hi = ok0 + odeg;
      const uint32_t a0 = (ok0 & ~7u) + 16u * (q - __shfl(cex, (int)own));
      uint32_t pm = 0;  // bit u: candidate a0 + u passes
      if (q < C) {
        int tc[16];
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          uint4 f = make_uint4(0u, 0u, 0u, 0u);
          if (a0 + 8u * v < hi) f = reinterpret_cast<const uint4*>(w.th)[a0 / 8u + v];
          const uint32_t fw[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            tc[8 * v + 2 * i] = (int)(int16_t)(fw[i] & 0xffffu);
            tc[8 * v + 2 * i + 1] = (int)(int16_t)(fw[i] >> 16);
          }
        }
        // the angle window first (one compare per candidate), the
        // anti-parallel window only where it can hold: angles lie within
        // +-32767 units, so two of them differ by q_far or more only if
        // |ta| >= q_far - 32767
        // (|tc - ta| <= W as one unsigned compare: tc + (W - ta) in [0, 2W])
        const int wa = c.q_win - ta;
        const uint32_t w2 = 2u * (uint32_t)c.q_win;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if ((uint32_t)(tc[u] + wa) <= w2) pm |= 1u << u;
        if (__any(q < C && abs(ta) >= c.q_far_min)) {
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (abs(tc[u] - ta) >= c.q_far) pm |= 1u << u;
        }
        // the owner's candidates within the chunk: a0 + u in [lo, hi)
        const uint32_t ub = lo > a0 ? lo - a0 : 0u, ue = min(16u, hi - a0);
        pm &= (ue >= 16u ? 0xffffu : (1u << ue) - 1u) & ~((1u << ub) - 1u);
      }
      // the owner's hits travel with its survivors
      const uint32_t od = dw + own;
      const uint32_t oha = __shfl(ha, (int)own), ohb = __shfl(hb, (int)own);
      // append the survivors, one per lane and round
      while (__any(pm != 0u)) {
        const bool has = pm != 0u;
        const uint32_t u = has ? (uint32_t)__ffs(pm) - 1u : 0u;
        pm &= pm - 1u;
        const uint64_t bal = __ballot(has);
        if (has) {
          const uint32_t slot = qn + (uint32_t)__popcll(bal & below);
          const uint32_t idx = a0 + u;
          qa[slot] = make_uint4(od, idx, oha, ohb);
          qb[slot] = make_uint2(idx - lo, odeg);
        }
        qn += (uint32_t)__popcll(bal);
        if (qn >= (uint32_t)kWave) {
          __threadfence_block();
          links_thread_flush(w, c, qa, qb, kWave, nd, links);
          __threadfence_block();
          const uint32_t rest = qn - kWave;
          uint4 ma = make_uint4(0, 0, 0, 0);
          uint2 mb = make_uint2(0, 0);
          if (lane < rest) {
            ma = qa[kWave + lane];
            mb = qb[kWave + lane];
          }
          __threadfence_block();
          if (lane < rest) {
            qa[lane] = ma;
            qb[lane] = mb;
          }
          __threadfence_block();
          qn = rest;
        }
      }
    }
  }
  __threadfence_block();
  links_thread_flush(w, c, qa, qb, qn, nd, links);
  links = wave_sum(links);
  if (lane_id() == 0 && links) atomicAdd(&ctr[C_NLINKS], links);
}

// A group of G lanes per doublet (a,b).  Each step covers 64 consecutive
// candidates: lane l of the group takes candidates l, l + G, ..., issuing
// the U = 64 / G angle loads back to back before the prefilter.  The few
// candidates that pass it are not tested further in place -- the exact
// tests (divisions, square roots) would run with almost all lanes idle --
// but pushed to a per-wavefront queue in LDS; whenever 64 are queued they
// are tested with all lanes busy.  Accepted links set their bit in the
// (pre-cleared) mask word with atomicOr and flag has_out.


__device__ __forceinline__ void links_flush(Ws& w, const DevCfg& c, const uint3* q, uint32_t n,
                                            uint32_t& links) {
  const uint32_t lane = lane_id();
  if (lane < n) {
    const uint3 it = q[lane];
    const uint32_t d = it.x, k = it.y;
    const uint2 io = w.cio[d];
    const HitD ha = load_hit(w, io.x);
    const HitD hb = load_hit(w, io.y);
    const uint32_t d2 = it.z;
    const HitD hc = load_hit(w, w.cio[d2].y);
    if (link_rz_pass(c, ha, hb, hc.r, hc.z) && link_xy_pass(c, ha, hb, hc)) {
      atomicOr((unsigned long long*)&w.masks[(size_t)(k >> 6) * w.ctr[C_ND] + d],
               1ull << (k & 63u));
      w.has_out[d] = 1;
      w.has_inner[d2] = 1;
      ++links;
    }
  }
}

template <int G>
__global__ __launch_bounds__(256) void k_links(Ws w, DevCfg c) {
  constexpr int U = kWave / G;
  __shared__ uint3 queue[256 / kWave][kQueue];  // (doublet, candidate index, candidate)
  uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t nd = ctr[C_ND];
  if (!links_capacity(w, c)) return;
  const uint32_t lane = lane_id(), sub = lane % G;
  uint3* q = queue[threadIdx.x / kWave];
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t gpb = blockDim.x / G, gib = threadIdx.x / G;
  uint32_t links = 0, qn = 0;
  for (TileWalk tw = tile_walk((nd + gpb - 1) / gpb); tw.t < tw.end; tw.t += tw.step) {
    const uint32_t d = tw.t * gpb + gib;
    uint32_t kb = 0, deg = 0;
    int ta = 0;
    if (d < nd) {
      ta = w.th[d];
      outer_range(w, w.cio[d].y, kb, deg);
    }
    const uint32_t maxw = wave_max((deg + 63u) / 64u);
    for (uint32_t wd = 0; wd < maxw; ++wd) {
      int tc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t k = wd * 64u + (uint32_t)(u * G) + sub;
        tc[u] = k < deg ? (int)w.th[kb + k] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t k = wd * 64u + (uint32_t)(u * G) + sub;
        const bool ok = k < deg && rz_prefilter(c, ta, tc[u]);
        const uint64_t bal = __ballot(ok);
        if (ok) q[qn + (uint32_t)__popcll(bal & below)] = make_uint3(d, k, kb + k);
        qn += (uint32_t)__popcll(bal);
        if (qn >= (uint32_t)kWave) {
          __threadfence_block();
          links_flush(w, c, q, kWave, links);
          __threadfence_block();
          const uint32_t rest = qn - kWave;
          const uint3 mv = lane < rest ? q[kWave + lane] : make_uint3(0, 0, 0);
          __threadfence_block();
          if (lane < rest) q[lane] = mv;
          __threadfence_block();
          qn = rest;
        }
      }
    }
  }
  __threadfence_block();
  links_flush(w, c, q, qn, links);
  links = wave_sum(links);
  if (lane_id() == 0 && links) atomicAdd(&ctr[C_NLINKS], links);
}

// Wave-cooperative link kernel.  A wavefront takes 64 consecutive doublets
// and flattens their candidate ranges (an exclusive prefix sum of the
// candidate counts over the lanes): in each round every lane takes the next
// candidate of the flattened list, finds the doublet it belongs to by a
// binary search over the prefix (lane shuffles) and applies the angle
// prefilter, so no lane idles on a doublet with few candidates.  Survivors
// go to a per-wavefront queue in LDS and are tested exactly 64 at a time.
// The doublets' mask words are staged in LDS (bits set with LDS atomics)
// and written out once, coalesced; a wavefront whose words exceed the
// staging area sets them in device memory instead.

constexpr int kWaveWords = 256;  // LDS mask words per wavefront

struct WaveLinks {
  uint64_t* sm;   // staged mask words of the wavefront
  uint32_t* cnt;  // accepted links per lane's doublet
  uint2* q;       // queue: (owner lane, candidate index)
};

__device__ __forceinline__ void wave_links_flush(Ws& w, const DevCfg& c, const WaveLinks& L,
                                                 uint32_t n, bool staged, uint32_t a,
                                                 float4 ob, uint32_t kb, uint32_t wex,
                                                 uint32_t mo, uint32_t& links) {
  const uint32_t lane = lane_id();
  const uint2 it = lane < n ? L.q[lane] : make_uint2(0, 0);
  const int own = (int)it.x;
  const uint32_t kk = it.y;
  // the owner's set-up, fetched from its lane (all lanes take part)
  const uint32_t ao = __shfl(a, own), kbo = __shfl(kb, own);
  const uint32_t wo = __shfl(wex, own), moo = __shfl(mo, own);
  const float bx = __shfl(ob.x, own), by = __shfl(ob.y, own), bz = __shfl(ob.z, own);
  if (lane < n) {
    const HitD ha = load_hit(w, ao);
    const HitD hb = hit_xyz(bx, by, bz);
    const uint32_t d2 = kbo + kk;
    const HitD hc = load_hit(w, w.cio[d2].y);
    if (link_rz_pass(c, ha, hb, hc.r, hc.z) && link_xy_pass(c, ha, hb, hc)) {
      const unsigned long long bit = 1ull << (kk & 63u);
      // LDS at workgroup scope, device memory at agent scope: two distinct
      // atomics (merged into one on a generic pointer they would need an
      // aperture check, which the gfx950 backend mis-encodes)
      if (staged)
        __hip_atomic_fetch_or((unsigned long long*)&L.sm[wo + (kk >> 6)], bit, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        __hip_atomic_fetch_or((unsigned long long*)&w.masks[(size_t)(kk >> 6) * w.ctr[C_ND] + moo],
                              bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      atomicAdd(&L.cnt[own], 1u);
      w.has_inner[d2] = 1;
      ++links;
    }
  }
}

__global__ __launch_bounds__(256) void k_links_wave(Ws w, DevCfg c) {
  __shared__ uint64_t s_mask[256 / kWave][kWaveWords];
  __shared__ uint2 s_q[256 / kWave][kQueue];
  __shared__ uint32_t s_cnt[256 / kWave][kWave];
  uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t nd = ctr[C_ND];
  if (!links_capacity(w, c)) return;
  const uint32_t lane = lane_id(), wib = threadIdx.x / kWave;
  const WaveLinks L{s_mask[wib], s_cnt[wib], s_q[wib]};
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t wpb = blockDim.x / kWave;
  const uint32_t nwaves = gridDim.x * wpb;
  uint32_t links = 0;
  for (uint32_t base = (xcd_block() * wpb + wib) * kWave; base < nd; base += nwaves * kWave) {
    const uint32_t d = base + lane;
    uint32_t a = 0, kb = 0, deg = 0, mo = 0;
    float4 ob = make_float4(0.f, 0.f, 0.f, 0.f);
    if (d < nd) {
      const uint2 io = w.cio[d];
      a = io.x;
      outer_range(w, io.y, kb, deg);
      ob = w.bh[io.y];  // the outer hit, with the doublet's r-z angle (units) in .w
      ob.w = __int_as_float((int)w.th[d]);
      mo = d;
    }
    const uint32_t nwd = (deg + 63u) >> 6;
    const uint32_t cinc = wave_incl_scan(deg), cex = cinc - deg;
    const uint32_t C = __shfl(cinc, kWave - 1);
    const uint32_t winc = wave_incl_scan(nwd), wex = winc - nwd;
    const uint32_t NW = __shfl(winc, kWave - 1);
    const bool staged = NW <= (uint32_t)kWaveWords;
    if (staged) {
      for (uint32_t i = lane; i < NW; i += kWave) L.sm[i] = 0;
    } else {
      for (uint32_t j = 0; j < nwd; ++j) w.masks[(size_t)j * nd + mo] = 0;
    }
    L.cnt[lane] = 0;
    __threadfence_block();
    uint32_t qn = 0;
    for (uint32_t r = 0; r * kWave < C; ++r) {
      const uint32_t k = r * kWave + lane;
      // owner: the last lane whose range starts at or before k
      uint32_t own = 0;
#pragma unroll
      for (uint32_t step = kWave / 2; step >= 1; step >>= 1)
        if (__shfl(cex, (int)(own + step)) <= k) own += step;
      const uint32_t kk = k - __shfl(cex, (int)own);
      const uint32_t kbo = __shfl(kb, (int)own);
      const int tao = __float_as_int(__shfl(ob.w, (int)own));
      const bool pass = k < C && rz_prefilter(c, tao, (int)w.th[kbo + kk]);
      const uint64_t bal = __ballot(pass);
      if (pass) L.q[qn + (uint32_t)__popcll(bal & below)] = make_uint2(own, kk);
      qn += (uint32_t)__popcll(bal);
      if (qn >= (uint32_t)kWave) {
        __threadfence_block();
        wave_links_flush(w, c, L, kWave, staged, a, ob, kb, wex, mo, links);
        __threadfence_block();
        const uint32_t rest = qn - kWave;
        const uint2 mv = lane < rest ? L.q[kWave + lane] : make_uint2(0, 0);
        __threadfence_block();
        if (lane < rest) L.q[lane] = mv;
        __threadfence_block();
        qn = rest;
      }
    }
    __threadfence_block();
    if (qn) wave_links_flush(w, c, L, qn, staged, a, ob, kb, wex, mo, links);
    __threadfence_block();
    if (d < nd) {
      if (staged)
        for (uint32_t j = 0; j < nwd; ++j) w.masks[(size_t)j * nd + mo] = L.sm[wex + j];
      w.has_out[d] = L.cnt[lane] != 0u;
    }
    __threadfence_block();
  }
  links = wave_sum(links);
  if (lane_id() == 0 && links) atomicAdd(&ctr[C_NLINKS], links);
}

// Clears the link-mask words ahead of the queued link kernel.
__global__ __launch_bounds__(256) void k_zero_words(Ws w, DevCfg c) {
  if (w.ctr[C_STATUS]) return;
  const uint64_t n = (uint64_t)w.ctr[C_ND] * w.ctr[C_WSTRIDE];
  if (n > c.cap_words) return;  // reported by the link kernel
  for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    w.masks[i] = 0;
}

// ------------------------------------------------------------ n-tuplets --
// One thread per root doublet (no inner neighbour, at least one outer;
// listed by k_roots, so no lane idles on the other doublets):
// iterative depth-first search over the outer-neighbour masks; every path
// that ends at a doublet without outer neighbours is an n-tuplet.  One
// walk: k_tuples<false> counts each root's paths and writes every path's
// row to its wavefront's region of a staging array, with the path's root
// and its index among the root's paths (slots from an LDS cursor per
// wavefront); an exclusive scan turns the counts into offsets; k_tuples<true>
// (same grid) moves each staged row to its root's offset + index.  A
// wavefront whose rows did not fit its region walks its roots again in
// k_tuples<true> and writes the rows in place.  No global atomics, and the
// n-tuplets come out ordered by root doublet (hence by event) and, within a
// root, in the walk's order.

constexpr uint32_t kRowIdxBits = 28;  // staged row: index among the root's paths

__device__ __forceinline__ uint32_t tuple_wave(uint32_t& nwaves) {
  nwaves = gridDim.x * (blockDim.x / kWave);
  return blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
}

// The walk of the roots of this thread; STAGE: count and stage (sets
// *over when the wavefront's region is full), else write the rows in place.
template <bool STAGE>
__device__ __forceinline__ void tuple_walk(Ws& w, uint32_t nr, uint32_t nd, uint32_t* s_cur,
                                           uint32_t cap, size_t rbase, bool& over) {
  uint32_t* ctr = w.ctr;
  for (uint32_t ri = blockIdx.x * blockDim.x + threadIdx.x; ri < nr;
       ri += gridDim.x * blockDim.x) {
    const uint32_t r = w.roots[ri];
    uint32_t path[kMaxCells];
    uint32_t word[kMaxCells];   // current mask word per depth
    uint64_t bits[kMaxCells];   // its remaining bits
    uint32_t nwd[kMaxCells];    // mask words per depth
    uint32_t kbase[kMaxCells];  // first candidate doublet per depth
    uint32_t phit[kMaxHits];    // the path's hits (doublet d spans d, d + 1)
    uint32_t cnt = 0;
    const uint32_t base = STAGE ? 0u : w.roff[ri];
    const uint2 rio = w.cio[r];
    int depth = 0;
    path[0] = r;
    phit[0] = rio.x;
    phit[1] = rio.y;
    {
      uint32_t deg;
      outer_range(w, rio.y, kbase[0], deg);
      nwd[0] = (deg + 63u) >> 6;
      word[0] = 0;
      bits[0] = nwd[0] ? w.masks[r] : 0ull;
    }
    bool overflow = false;
    while (depth >= 0) {
      if (bits[depth] == 0) {
        if (++word[depth] < nwd[depth]) {
          bits[depth] = w.masks[(size_t)word[depth] * nd + path[depth]];
          continue;
        }
        --depth;
        continue;
      }
      const int k = __ffsll((unsigned long long)bits[depth]) - 1;
      bits[depth] &= bits[depth] - 1;
      const uint32_t child = kbase[depth] + word[depth] * 64u + (uint32_t)k;
      if (depth + 1 >= kMaxCells) {
        overflow = true;
        break;
      }
      path[depth + 1] = child;
      // the child's outer hit is loaded with its link flag (no extra round
      // trip at a leaf); its candidate range follows from that hit
      const uint8_t nchild = w.has_out[child];
      const uint32_t hchild = w.cio[child].y;
      if (nchild == 0) {
        const int last = depth + 1;
        uint32_t hh[kMaxHits], cc[kMaxHits];
#pragma unroll
        for (int j = 0; j < kMaxHits; ++j)
          hh[j] = j <= last ? phit[j] : (j == last + 1 ? hchild : kPad);
#pragma unroll
        for (int j = 0; j < kMaxCells; ++j) cc[j] = j <= last ? path[j] : kPad;
        cc[kMaxCells] = kPad;
        uint4* row = nullptr;
        if (STAGE) {
          const uint32_t slot = atomicAdd(s_cur, 1u);
          if (slot < cap && cnt < (1u << kRowIdxBits)) {
            row = w.trow + (rbase + slot) * 4u;
            w.tmeta[rbase + slot] = make_uint2(ri, cnt | ((uint32_t)(last + 2) << kRowIdxBits));
          } else {
            over = true;
          }
          if (row) {
            row[0] = make_uint4(hh[0], hh[1], hh[2], hh[3]);
            row[1] = make_uint4(hh[4], hh[5], hh[6], hh[7]);
            row[2] = make_uint4(cc[0], cc[1], cc[2], cc[3]);
            row[3] = make_uint4(cc[4], cc[5], cc[6], cc[7]);
          }
        } else {
          const uint32_t t = base + cnt;
          // one n-tuplet row: two 16-byte stores per array
          uint4* th4 = reinterpret_cast<uint4*>(w.thit + (size_t)t * kMaxHits);
          uint4* tc4 = reinterpret_cast<uint4*>(w.tcell + (size_t)t * kMaxHits);
          th4[0] = make_uint4(hh[0], hh[1], hh[2], hh[3]);
          th4[1] = make_uint4(hh[4], hh[5], hh[6], hh[7]);
          tc4[0] = make_uint4(cc[0], cc[1], cc[2], cc[3]);
          tc4[1] = make_uint4(cc[4], cc[5], cc[6], cc[7]);
          w.tn[t] = (uint8_t)(last + 2);
        }
        ++cnt;
        continue;
      }
      ++depth;
      phit[depth + 1] = hchild;
      uint32_t deg;
      outer_range(w, hchild, kbase[depth], deg);
      nwd[depth] = (deg + 63u) >> 6;
      word[depth] = 0;
      bits[depth] = nwd[depth] ? w.masks[child] : 0ull;
    }
    if (overflow) set_status(ctr, PXT_ERR_PATH);
    if (STAGE) w.rcnt[ri] = cnt;
  }
}

// staged rows per wavefront region: the whole staging array split evenly
__device__ __forceinline__ uint32_t tuple_region(const DevCfg& c, uint32_t nwaves) {
  return c.cap_tuples / nwaves;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_tuples(Ws w, DevCfg c) {
  __shared__ uint32_t s_cur[256 / kWave];
  uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t nr = ctr[C_NROOT];
  const uint32_t T = c.cap_tuples;
  const uint32_t nd = ctr[C_ND];
  const uint32_t lane = lane_id(), wib = threadIdx.x / kWave;
  uint32_t nwaves;
  const uint32_t wid = tuple_wave(nwaves);
  const uint32_t cap = tuple_region(c, nwaves);
  const size_t rbase = (size_t)wid * cap;
  bool over = false;
  if (!FILL) {
    if (lane == 0) s_cur[wib] = 0u;
    __threadfence_block();
    tuple_walk<true>(w, nr, nd, &s_cur[wib], cap, rbase, over);
    __threadfence_block();
    const bool wover = __any(over);
    if (lane == 0) w.dwn[wid] = wover ? kRecOver : s_cur[wib];
    return;
  }
  if (w.roff[nr] > T) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      set_status(ctr, PXT_ERR_CAPACITY);
      ctr[C_REQ_T] = w.roff[nr];
    }
    return;
  }
  const uint32_t n = w.dwn[wid];
  if (n == kRecOver) {
    // rows incomplete: this wavefront's roots are walked again
    tuple_walk<false>(w, nr, nd, nullptr, 0u, 0u, over);
    return;
  }
  for (uint32_t i = lane; i < n; i += kWave) {
    const uint2 m = w.tmeta[rbase + i];
    const uint4* row = w.trow + (rbase + i) * 4u;
    const uint4 a = row[0], b = row[1], e = row[2], f = row[3];
    const uint32_t t = w.roff[m.x] + (m.y & ((1u << kRowIdxBits) - 1u));
    uint4* th4 = reinterpret_cast<uint4*>(w.thit + (size_t)t * kMaxHits);
    uint4* tc4 = reinterpret_cast<uint4*>(w.tcell + (size_t)t * kMaxHits);
    th4[0] = a;
    th4[1] = b;
    tc4[0] = e;
    tc4[1] = f;
    w.tn[t] = (uint8_t)(m.y >> kRowIdxBits);
  }
}

// ------------------------------------------------------------- cleaning --
// Each doublet keeps only its best n-tuplet under the total order: more
// hits, then lower score (a NaN score after every number, NaN scores
// equal), then the lexicographically smaller event-local hit tuple; a tuple
// survives iff it is the best at every one of its doublets.
//
// The per-doublet election runs in two rounds of atomics instead of a
// per-doublet list.  The order key packs (8 - hits) above the score's bits
// with their lowest eleven dropped: it never decreases along the order, so
// the best tuple of a doublet holds the smallest key there (k_score takes
// the atomicMin).  The tuples holding that key -- almost always just one --
// then settle the exact order by compare-and-swap on the doublet's best
// tuple (k_best): a swap only ever installs a better tuple, so the loop
// ends, and the result does not depend on the order the threads run in.
//
// The slots are not cleared per call.  The key's top byte is a call tag
// that falls by one per call (255 on the first call after a full reset,
// k_slots_clear), so a key left by an earlier call is larger than any key
// of this call; the best slot carries the call's epoch in its upper half,
// and a slot with another epoch counts as empty.

__device__ __forceinline__ uint64_t order_key(int n, double s, uint32_t epoch) {
  const uint64_t m = s != s ? 0x7fffffffffffffffull : (uint64_t)__double_as_longlong(s);
  const uint64_t tag = 0xffu - ((epoch - 1u) & 0xffu);
  return (tag << 56) | ((uint64_t)(kMaxHits - n) << 52) | (m >> 11);
}

// Best slot of a doublet on which two tuples of the call tied for the key
// (no tuple index: tuples are below the capacity, under 2^32 - 1).
__device__ __forceinline__ uint64_t tie_mark(uint32_t epoch) {
  return ((uint64_t)epoch << 32) | 0xffffffffull;
}

// The eight slots of an n-tuplet row (rows are 32 bytes, 32-byte aligned)
// as two 16-byte loads, and a slot picked by a run-time index without
// spilling the row to scratch.
static_assert(kMaxHits == 8, "n-tuplet rows are two 16-byte vectors");
__device__ __forceinline__ void load_row(const uint32_t* rows, uint32_t t, uint32_t r[kMaxHits]) {
  const uint4* p = reinterpret_cast<const uint4*>(rows + (size_t)t * kMaxHits);
  const uint4 a = p[0], b = p[1];
  r[0] = a.x;
  r[1] = a.y;
  r[2] = a.z;
  r[3] = a.w;
  r[4] = b.x;
  r[5] = b.y;
  r[6] = b.z;
  r[7] = b.w;
}

__device__ __forceinline__ uint32_t pick_slot(const uint32_t r[kMaxHits], int i) {
  uint32_t v = r[0];
#pragma unroll
  for (int j = 1; j < kMaxHits; ++j) v = i == j ? r[j] : v;
  return v;
}

__global__ __launch_bounds__(256) void k_score(Ws w, DevCfg c) {
  uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t ntup = ctr[C_NTUP];
  const uint32_t epoch = w.epoch[0];
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntup; t += gridDim.x * blockDim.x) {
    const int n = w.tn[t];
    uint32_t th[kMaxHits], tc[kMaxHits];
    load_row(w.thit, t, th);
    load_row(w.tcell, t, tc);
    HitD h0 = load_hit(w, th[0]);
    HitD h1 = load_hit(w, th[1]);
    double s = 0.0;
    for (int j = 1; j + 1 < n; ++j) {
      const HitD h2 = load_hit(w, pick_slot(th, j + 1));
      s += triple_score(c, h0, h1, h2);
      h0 = h1;
      h1 = h2;
    }
    w.tscore[t] = s;
    const uint64_t key = order_key(n, s, epoch);
    // a tuple that finds its own key already there ties with another one:
    // the doublet's best slot is marked, so that k_best settles it by
    // compare-and-swap (a tie at the minimum is always seen this way: the
    // second of two equal keys finds the first one still in place)
#pragma unroll
    for (int j = 0; j < kMaxCells; ++j)
      if (j + 1 < n &&
          atomicMin((unsigned long long*)&w.bkey[tc[j]], (unsigned long long)key) == key)
        w.best[tc[j]] = tie_mark(epoch);
  }
}

// true if tuple a ranks before tuple b
__device__ __forceinline__ bool ranks_before(const Ws& w, uint32_t T, uint32_t a, uint32_t b) {
  const int na = w.tn[a], nbh = w.tn[b];
  if (na != nbh) return na > nbh;
  const double sa = w.tscore[a], sb = w.tscore[b];
  const bool an = sa != sa, bn = sb != sb;
  if (an != bn) return bn;
  if (!an && sa != sb) return sa < sb;
  for (int j = 0; j < kMaxHits; ++j) {
    const uint32_t ha = w.thit[(size_t)a * kMaxHits + j], hb = w.thit[(size_t)b * kMaxHits + j];
    const uint32_t ia = ha == kPad ? kPad : w.bidx[ha];
    const uint32_t ib = hb == kPad ? kPad : w.bidx[hb];
    if (ia != ib) return ia < ib;
  }
  return false;
}

__global__ __launch_bounds__(256) void k_best(Ws w, DevCfg c) {
  if (w.ctr[C_STATUS]) return;
  const uint32_t ntup = w.ctr[C_NTUP];
  const uint32_t T = c.cap_tuples;
  const uint32_t epoch = w.epoch[0];
  const uint64_t tag = (uint64_t)epoch << 32;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntup; t += gridDim.x * blockDim.x) {
    const int n = w.tn[t];
    const uint64_t key = order_key(n, w.tscore[t], epoch);
    uint32_t tc[kMaxHits];
    load_row(w.tcell, t, tc);
#pragma unroll
    for (int j = 0; j < kMaxCells; ++j) {
      if (j + 1 >= n) continue;
      const uint32_t d = tc[j];
      if (w.bkey[d] != key) continue;
      unsigned long long cur = w.best[d];
      // a slot untouched by this call (another call's tag): no tie was
      // marked, so this tuple alone holds the doublet's minimum key
      if ((cur >> 32) != epoch) {
        w.best[d] = tag | t;
        continue;
      }
      // a tie (the slot holds the mark, or a tied tuple put there by the
      // loop): the exact order decides; the mark holds no tuple
      while (cur == tie_mark(epoch) || (cur >> 32) != epoch ||
             ranks_before(w, T, t, (uint32_t)cur)) {
        const unsigned long long prev =
            atomicCAS((unsigned long long*)&w.best[d], cur, (unsigned long long)(tag | t));
        if (prev == cur) break;
        cur = prev;
      }
    }
  }
}

// Survivors of the cleaning, in n-tuplet order, in one pass: a 1024-tuple
// tile per block (tiles taken by ticket), a tuple surviving when it is the
// elected best of every one of its doublets (and long enough for output);
// the block scans its survivor flags and takes its tile's offset by
// decoupled look-back, like the scans.  Each survivor's index goes to the
// survivor list.
//
// Also the fitting order.  The fit is compiled once per tuple length class
// (3 hits, 4 hits, 5 to 8 hits), and one kernel per class keeps each body's
// register budget its own and its wavefronts uniform; for that each class
// gets a list of its survivors (region c of sfit, c = class): the block
// takes a range of each class's list with one atomic per class and writes
// its survivors there (ballot ranks within a wavefront, the wavefronts'
// counts in LDS).  The order within a list depends on the order the blocks
// take their ranges; every result still goes to its survivor's slot, so
// only the work assignment changes.
//
// And the first survivor of each event: n-tuplets follow the events in
// order (as the binned hits, doublets and roots do), so a tuple whose event
// differs from its predecessor's records its survivor offset for the events
// from the predecessor's (exclusive) to its own; k_finish turns these into
// per-event track counts.
constexpr int kSurvThreads = 1024;
constexpr uint32_t kSurvScan = 5;  // scan id of the survivor offsets

__device__ __forceinline__ uint32_t fit_class(uint32_t n) { return n >= 5u ? 2u : n - 3u; }

__device__ __forceinline__ uint32_t tuple_event(const Ws& w, uint32_t t) {
  return w.bevt[w.thit[(size_t)t * kMaxHits]];
}

__global__ __launch_bounds__(kSurvThreads) void k_survive(Ws w, DevCfg c) {
  constexpr uint32_t NW = kSurvThreads / kWave;
  __shared__ uint32_t s_lds[NW + 1];
  __shared__ uint32_t s_cnt[NW][3];  // per wavefront and class
  __shared__ uint32_t s_base[3];     // the block's range of each class list
  __shared__ uint32_t s_prefix;
  uint32_t* ctr = w.ctr;
  if (ctr[C_STATUS]) return;
  const uint32_t ntup = ctr[C_NTUP];
  const uint32_t E = w.call->n_events;
  const uint32_t ntiles = ntup ? (ntup + kSurvThreads - 1u) / kSurvThreads : 1u;
  uint32_t tile;
  if (!take_tile(w, kSurvScan, ntiles, tile)) return;
  const uint32_t T = c.cap_tuples;
  const uint32_t lane = lane_id(), wib = threadIdx.x / kWave;
  const uint64_t tag = (uint64_t)w.epoch[0] << 32;
  const uint32_t t = tile * kSurvThreads + threadIdx.x;
  bool alive = false;
  uint32_t n = 0;
  if (t < ntup) {
    n = w.tn[t];
    // shorter n-tuplets than min_hits are not output (they never outrank a
    // longer one, so the others' fate does not depend on them)
    alive = n >= (uint32_t)c.min_hits;
    uint32_t tc[kMaxHits];
    load_row(w.tcell, t, tc);
#pragma unroll
    for (int j = 0; j < kMaxCells; ++j)
      if (j + 1 < (int)n && w.best[tc[j]] != (tag | t)) alive = false;
  }
  uint32_t agg;
  const uint32_t excl = block_excl_scan(alive ? 1u : 0u, s_lds, agg);
  if (threadIdx.x < kWave) {
    const uint32_t pf = tile_lookback(w, tile, w.epoch[0] * 8u + kSurvScan, agg);
    if (threadIdx.x == 0) s_prefix = pf;
  }
  const uint32_t cls = alive ? fit_class(n) : 3u;
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t rank = 0;
#pragma unroll
  for (uint32_t k = 0; k < 3; ++k) {
    const uint64_t m = __ballot(cls == k);
    if (cls == k) rank = (uint32_t)__popcll(m & below);
    if (lane == 0) s_cnt[wib][k] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const uint32_t k = threadIdx.x;
    uint32_t tot = 0;
    for (uint32_t i = 0; i < NW; ++i) tot += s_cnt[i][k];
    s_base[k] = tot ? atomicAdd(&ctr[C_FITN0 + 3 + k], tot) : 0u;
  }
  __syncthreads();
  const uint32_t s = s_prefix + excl;  // survivors before tuple t
  if (alive) {
    uint32_t base = s_base[cls];
    for (uint32_t i = 0; i < wib; ++i) base += s_cnt[i][cls];
    w.surv[s] = t;
    w.sfit[(size_t)cls * T + base + rank] = s;
  }
  // first survivor of each event
  if (t < ntup) {
    const uint32_t ev = tuple_event(w, t);
    const uint32_t from = t == 0 ? 0u : tuple_event(w, t - 1u) + 1u;
    for (uint32_t e = from; e <= ev; ++e) w.evt_surv[e] = s;
    if (t == ntup - 1u)
      for (uint32_t e = ev + 1u; e <= E; ++e) w.evt_surv[e] = s + (alive ? 1u : 0u);
  } else if (ntup == 0 && threadIdx.x == 0) {
    for (uint32_t e = 0; e <= E; ++e) w.evt_surv[e] = 0u;
  }
  if (tile == ntiles - 1u && threadIdx.x == 0) ctr[C_NSURV] = s_prefix + agg;
}

// ------------------------------------------------------------------ fit --

// Quality bits of a fitted track from its single-precision outputs:
// LOOSE = finite parameters and chi2 per degree of freedom within q_chi2 in
// both planes (transverse ndf n-3, at least 1; longitudinal n-2); STRICT =
// LOOSE and pT, |d0|, |z0| within their limits.
__device__ __forceinline__ uint32_t quality_flags(const DevCfg& c, int n, const float* p,
                                                  const float* chi2) {
  bool fin = true;
#pragma unroll
  for (int i = 0; i < 5; ++i) fin = fin && isfinite(p[i]);
  const float ndf_c = (float)(n - 3 > 1 ? n - 3 : 1), ndf_z = (float)(n - 2);
  const bool loose = fin && chi2[0] <= c.q_chi2 * ndf_c && chi2[1] <= c.q_chi2 * ndf_z;
  const bool strict = loose && fabsf(p[2]) <= c.q_qopt_max && fabsf(p[1]) <= c.q_d0_max &&
                      fabsf(p[4]) <= c.q_z0_max;
  return (loose ? PXT_FLAG_LOOSE : 0u) | (strict ? PXT_FLAG_STRICT : 0u);
}

// Fit survivor s; NFIX > 0: the tuple is known to have NFIX hits.
template <typename T, int NFIX = 0>
__device__ inline void fit_one(Ws& w, const DevCfg& c, const OutPtrs& o, uint32_t s,
                               bool fp64) {
  constexpr int NH = NFIX > 0 ? NFIX : kMaxHits;  // hit slots that can be used
  const uint32_t t = w.surv[s];
  const int n = NFIX > 0 ? NFIX : (int)w.tn[t];
  float X[kMaxHits], Y[kMaxHits], Z[kMaxHits];
  int kind[kMaxHits];
  uint32_t row[kMaxHits];
  load_row(w.thit, t, row);
  // the track's hit ids and event go out first, so that the ids are not
  // held through the fit
  if (!fp64) {
#pragma unroll
    for (int j = 0; j < kMaxHits; ++j) {
      const uint32_t h = j < NH ? row[j] : kPad;
      o.hit_idx[(size_t)s * 8 + j] = h == kPad ? kPad : w.bidx[h];
    }
    o.n_hits[s] = (uint8_t)n;
    o.event_id[s] = w.bevt[row[0]];
  }
#pragma unroll
  for (int j = 0; j < kMaxHits; ++j) {
    if (j < NH && j < n) {
      const uint32_t h = row[j];
      const float4 v = w.bh[h];
      X[j] = v.x;
      Y[j] = v.y;
      Z[j] = v.z;
      kind[j] = c.layer_kind[w.blay[h]];
    } else {
      X[j] = Y[j] = Z[j] = 0.0f;
      kind[j] = 0;
    }
  }
  FitOut f;
  f.cov = o.cov + (size_t)s * 15;
  if constexpr (NFIX > 0)
    fit_n<NFIX, T>(c, X, Y, Z, kind, f);
  else
    fit_tuple<T>(c, n, X, Y, Z, kind, f);
  if (!fp64 && f.need64) {
    const uint32_t k = atomicAdd(&w.ctr[C_NFP64], 1u);
    w.fp64_list[k] = s;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) o.params[(size_t)s * 5 + i] = f.params[i];
  o.chi2[(size_t)s * 2 + 0] = f.chi2[0];
  o.chi2[(size_t)s * 2 + 1] = f.chi2[1];
  o.flags[s] = (uint8_t)((fp64 ? PXT_FLAG_FP64 : 0u) | quality_flags(c, n, f.params, f.chi2));
}

// One kernel per tuple length N over that length's range of the fitting
// order (N = 0: all lengths from 5 up, rarer, in one kernel); the N = 3
// instance also reports an output overflow.  The grid has a thread for
// every tuple the context can hold.  The triplet fit, the most frequent,
// is held to 128 registers (four wavefronts per SIMD) and the 4-hit fit to
// 168 (three), which they meet without spilling.
template <int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(N == 3 ? 4 : (N == 4 ? 3 : 1))))
void k_fit32(Ws w, DevCfg c) {
  if (w.ctr[C_STATUS]) return;
  const OutPtrs o = w.call->out;
  const uint32_t ns = w.ctr[C_NSURV];
  if (ns > o.capacity) {
    if (N == 3 && blockIdx.x == 0 && threadIdx.x == 0) {
      set_status(w.ctr, PXT_ERR_CAPACITY);
      w.ctr[C_REQ_K] = ns;
    }
    return;
  }
  if (N > 0 && ns <= kSmallFit) return;  // k_fit_small fits them
  constexpr uint32_t CLS = N > 0 ? (uint32_t)N - 3u : 2u;  // the length class
  const size_t off = (size_t)CLS * c.cap_tuples;
  const uint32_t cnt = w.ctr[C_FITN0 + 3 + CLS];
  // one tuple per thread, no grid-stride loop: a loop would keep the values
  // derived from the configuration live across iterations and double the
  // register footprint (the grid covers the tuple capacity)
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) fit_one<float, N>(w, c, o, w.sfit[off + i], false);
}

// Calls with few tracks (one or two events: the plain and served paths)
// fit the 3-hit and 4-hit classes in one launch instead of two: block b
// takes the 3-hit list for b < ceil(n3 / 256), then the 4-hit list.  With
// so few wavefronts each kernel's time is the latency of one fit, so one
// kernel at the larger class's register budget beats two at their own; the
// per-class kernels of those classes leave at once (the 5-to-8-hit kernel
// always runs: together with it this kernel would spill).
__global__ __launch_bounds__(256) void k_fit_small(Ws w, DevCfg c) {
  if (w.ctr[C_STATUS]) return;
  const OutPtrs o = w.call->out;
  const uint32_t ns = w.ctr[C_NSURV];
  if (ns > kSmallFit || ns > o.capacity) return;  // the per-class kernels run (or report)
  const uint32_t n3 = w.ctr[C_FITN0 + 3], n4 = w.ctr[C_FITN0 + 4];
  const uint32_t b3 = (n3 + 255u) / 256u;
  if (blockIdx.x < b3) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n3) fit_one<float, 3>(w, c, o, w.sfit[i], false);
  } else {
    const uint32_t i = (blockIdx.x - b3) * 256u + threadIdx.x;
    if (i < n4) fit_one<float, 4>(w, c, o, w.sfit[(size_t)c.cap_tuples + i], false);
  }
}

__global__ __launch_bounds__(64) void k_fit64(Ws w, DevCfg c) {
  if (w.ctr[C_STATUS]) return;
  const OutPtrs o = w.call->out;
  const uint32_t n64 = w.ctr[C_NFP64];
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n64; k += gridDim.x * blockDim.x)
    fit_one<double>(w, c, o, w.fp64_list[k], true);
}

// --------------------------------------------------------------- finish --

__global__ void k_finish(Ws w) {
  const uint32_t* ctr = w.ctr;
  const int st = (int)ctr[C_STATUS];
  // per-event track counts from the events' first survivors (left at zero
  // when the call failed)
  const CallDesc* cd = w.call;
  if (st == 0 && ctr[C_NTUP] > 0)
    for (uint32_t e = threadIdx.x; e < cd->n_events; e += blockDim.x)
      cd->out.per_event_tracks[e] = w.evt_surv[e + 1] - w.evt_surv[e];
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  pxt_counts* k = cd->out.counts;
  k->status = st;
  k->n_tracks = st ? 0u : ctr[C_NSURV];
  k->n_doublets = ctr[C_ND];
  k->n_links = ctr[C_NLINKS];
  k->n_raw_tuples = ctr[C_NTUP];
  k->n_fp64 = ctr[C_NFP64];
  k->n_hits_binned = ctr[C_NBINNED];
  k->n_link_words = ctr[C_NWORDS];
  k->required[0] = ctr[C_REQ_D];
  k->required[1] = ctr[C_REQ_W];
  k->required[2] = ctr[C_REQ_T];
  k->required[3] = ctr[C_REQ_K];
  // the vertex step's summary starts empty (the vertex kernel follows)
  if (w.call->has_vtx) k_vtx_begin_body(w.call->vtx);
}

// --------------------------------------------------------------- vertices --
// The vertex step of a pxt_reconstruct call (after k_finish, which resets
// its summary), on the call's own outputs; nothing when the call has no
// vertex buffers.

__global__ __launch_bounds__(kVtxThreads) void k_vertices_call(Ws w, DevCfg c) {
  const CallDesc* cd = w.call;
  if (!cd->has_vtx) return;
  const VtxIn in{cd->n_events, cd->out.per_event_tracks, cd->out.n_hits, cd->out.params,
                 cd->out.cov, cd->out.counts};
  vertices_block(in, cd->vtx, c);
}

}  // namespace pxt
