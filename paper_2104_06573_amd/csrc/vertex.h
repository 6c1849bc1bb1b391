// Vertices of the fitted tracks: one-dimensional density-based clustering
// (DBSCAN, Ester et al. 1996) of the tracks' longitudinal impact parameter
// z0, then an inverse-variance weighted mean per cluster.  This is the
// reading of the paper's Vertices module (Sec. 2, Fig. 1: vertices are
// formed from the pixel tracks) stated with pxt_vertices in pxt.h.
//
// One workgroup of 1024 threads per event, everything in LDS (144 KB of
// gfx950's 160 KB):
//   select   tracks passing the selection append (z0, track) keys;
//   sort     bitonic sort of the keys by (z0, track index), four keys per
//            thread in registers, wavefront shuffles for the short
//            distances;
//   cores    each track counts its neighbours within eps by two binary
//            searches of the sorted z0 (the difference of two single-
//            precision values taken in double precision is monotone in
//            each, so the neighbours of a track are a contiguous range);
//   clusters in sorted order every core between two connected cores is
//            connected to both, so clusters are runs of consecutive cores
//            closer than eps: a scan over the cores numbers them;
//   borders  the nearest core below a non-core track is the previous core,
//            above it the next one: it takes the nearer (ties: the previous)
//            if within eps; the members of a cluster then form a contiguous
//            range of the sorted tracks;
//   vertex   one thread per cluster sums its range in sorted order (the
//            order the definition fixes), in double precision.
#pragma once

#include "common.h"

namespace pxt {

constexpr int kVtxThreads = 1024;
constexpr int kVtxMax = PXT_VTX_MAX_TRACKS;
constexpr int kVtxPer = kVtxMax / kVtxThreads;  // sorted entries per thread
static_assert(kVtxMax % kVtxThreads == 0, "vertex chunking");
static_assert(kVtxMax <= 4096, "selection slot takes 12 bits of the key");

// Outputs of the vertex step (the caller's pxt_vertices).
struct VtxOut {
  uint32_t max_per_event;
  float* z;
  float* z_err;
  float* chi2;
  uint32_t* n_tracks;
  uint32_t* n_vertices;
  int32_t* track_vertex;
  pxt_vertex_summary* summary;
};

// Inputs: tracks grouped by event in event order.
struct VtxIn {
  uint32_t n_events;
  const uint32_t* per_event_tracks;
  const uint8_t* n_hits;
  const float* params;
  const float* cov;
  const pxt_counts* counts;  // may be null
};

// z0 as an unsigned key that orders like the float (-0 taken as +0, so
// that equal values tie and fall back to the track index).
__device__ __forceinline__ uint32_t z_key(float z) {
  const uint32_t u = __float_as_uint(z + 0.0f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float z_of_key(uint64_t k) {
  const uint32_t u = (uint32_t)(k >> 32);
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Exclusive block-wide prefix sum over kVtxThreads threads; `tot` receives
// the total.  lds holds kVtxThreads / 64 + 1 words.
__device__ __forceinline__ uint32_t vtx_excl_sum(uint32_t v, uint32_t* lds, uint32_t& tot) {
  const uint32_t lane = lane_id(), wid = threadIdx.x / kWave;
  constexpr uint32_t nw = kVtxThreads / kWave;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == kWave - 1) lds[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    const uint32_t x = lane < nw ? lds[lane] : 0u;
    const uint32_t xi = wave_incl_scan(x);
    if (lane < nw) lds[lane] = xi - x;
    if (lane == nw - 1) lds[nw] = xi;
  }
  __syncthreads();
  const uint32_t r = lds[wid] + inc - v;
  tot = lds[nw];
  __syncthreads();
  return r;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, kWave);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

// The keeper of element i in a bitonic compare-exchange with element i ^ j
// of sub-sequence size k: the smaller key when i is the lower of the pair
// in an ascending run or the upper in a descending one.
__device__ __forceinline__ uint64_t bitonic_keep(uint64_t a, uint64_t b, uint32_t i, uint32_t j,
                                                 uint32_t k) {
  const bool take_min = ((i & j) == 0) == ((i & k) == 0);
  return take_min ? (a < b ? a : b) : (a < b ? b : a);
}

// Ascending bitonic sort of s_key[0..M) (M a power of two, at most kVtxMax;
// s_key[M..kVtxMax) hold padding) by all kVtxThreads threads.  Thread t
// keeps elements 4t..4t+3 in registers: distances 1 and 2 are exchanged in
// registers, 4..128 by shuffles within the wavefront, and only 256 and more
// through LDS (10 of the 78 steps of a 4096-key sort need a barrier).
__device__ __forceinline__ void vtx_sort(uint64_t* s_key, uint32_t M) {
  static_assert(kVtxMax == 4 * kVtxThreads, "four keys per thread");
  const uint32_t t = threadIdx.x;
  uint64_t v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = s_key[4 * t + r];
  for (uint32_t k = 2; k <= M; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= 4 * kWave) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) s_key[4 * t + r] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t i = 4 * t + r;
          v[r] = bitonic_keep(v[r], s_key[i ^ j], i, j, k);
        }
      } else if (j >= 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t i = 4 * t + r;
          v[r] = bitonic_keep(v[r], shfl_xor_u64(v[r], (int)(j >> 2)), i, j, k);
        }
      } else {
        uint64_t w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t i = 4 * t + r;
          w[r] = bitonic_keep(v[r], v[r ^ j], i, j, k);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = w[r];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) s_key[4 * t + r] = v[r];
  __syncthreads();
}

// Ascending sort of the m <= kVtxThreads unique keys s_key[0..m) by rank:
// each thread counts the keys below its own (broadcast LDS reads, two keys
// per read; s_key[m] must hold padding) and writes its key there.
__device__ __forceinline__ void vtx_rank_sort(uint64_t* s_key, uint32_t m) {
  const uint32_t t = threadIdx.x;
  const uint64_t mine = t < m ? s_key[t] : 0ull;
  uint32_t rank = 0;
  const ulonglong2* p2 = reinterpret_cast<const ulonglong2*>(s_key);
  for (uint32_t j = 0; j < m; j += 2) {
    const ulonglong2 ab = p2[j >> 1];
    rank += (ab.x < mine ? 1u : 0u) + (ab.y < mine ? 1u : 0u);
  }
  __syncthreads();
  if (t < m) s_key[rank] = mine;
  __syncthreads();
}

__device__ void vertices_event(const VtxIn& in, const VtxOut& o, const DevCfg& c, uint32_t e) {
  __shared__ __align__(16) uint64_t s_key[kVtxMax];  // (z0 key, track << 12 | slot)
  __shared__ double s_w[kVtxMax];       // weight 1/var(z0) by selection slot
  __shared__ double s_ws[kVtxMax];      // the same in sorted order
  __shared__ int32_t s_lab[kVtxMax];    // core flag, then cluster (-1: none)
  __shared__ uint32_t s_rank[kVtxMax];  // cores before each entry; then cluster ends
  __shared__ uint32_t s_core[kVtxMax];  // position of each core; then cluster starts
  __shared__ uint32_t s_scan[kVtxThreads / kWave + 1];
  __shared__ uint32_t s_m, s_toff;
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t nthr = kVtxThreads;
  if (tid == 0) {
    s_m = 0;
    s_toff = 0;
  }
  __syncthreads();
  // first track of the event
  uint32_t part = 0;
  for (uint32_t i = tid; i < e; i += nthr) part += in.per_event_tracks[i];
  part = wave_sum(part);
  if (lane_id() == 0 && part) atomicAdd(&s_toff, part);
  __syncthreads();
  const uint32_t toff = s_toff, ntr = in.per_event_tracks[e];
  // selection: keys appended in any order (the sort fixes the order).  A
  // thread takes kSel tracks per round and issues their loads back to back
  // (hit counts first, then the values of the tracks with enough hits), so
  // the latency of one event's thousands of tracks overlaps.
  constexpr int kSel = 16;
  for (uint32_t t0 = tid; t0 < ntr; t0 += nthr * kSel) {
    uint32_t nh[kSel];
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
      const uint32_t t = t0 + (uint32_t)u * nthr;
      nh[u] = t < ntr ? (uint32_t)in.n_hits[toff + t] : 0u;
    }
    float q[kSel], z[kSel], v[kSel];
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
      const uint32_t t = t0 + (uint32_t)u * nthr;
      q[u] = z[u] = v[u] = 0.0f;
      if (t < ntr) {
        const size_t g = toff + t;
        o.track_vertex[g] = -1;
        if ((int)nh[u] >= c.vtx_min_hits) {
          q[u] = in.params[g * 5 + 2];
          z[u] = in.params[g * 5 + 4];
          v[u] = in.cov[g * 15 + 14];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
      const uint32_t t = t0 + (uint32_t)u * nthr;
      const bool ok = t < ntr && (int)nh[u] >= c.vtx_min_hits && fabsf(q[u]) <= c.vtx_qopt_max &&
                      isfinite(z[u]) && isfinite(v[u]) && v[u] > 0.0f;
      if (ok && t < (1u << 20)) {
        const uint32_t slot = atomicAdd(&s_m, 1u);
        if (slot < (uint32_t)kVtxMax) {
          s_key[slot] = ((uint64_t)z_key(z[u]) << 32) | ((uint64_t)t << 12) | slot;
          // the weight of every selected track at once (the clusters' sums
          // below then only add, in their fixed order)
          s_w[slot] = 1.0 / (double)v[u];
        }
      }
    }
  }
  __syncthreads();
  const uint32_t m = s_m;
  if (m > (uint32_t)kVtxMax || ntr > (1u << 20)) {
    if (tid == 0) {
      o.n_vertices[e] = 0;
      atomicMax(&o.summary->max_selected, m);
      atomicCAS((unsigned int*)&o.summary->status, 0u, (unsigned int)PXT_ERR_CAPACITY);
    }
    return;
  }
  uint32_t M = 1;
  while (M < m) M <<= 1;
  for (uint32_t i = m + tid; i < (uint32_t)kVtxMax; i += nthr) s_key[i] = ~0ull;
  __syncthreads();
  if (m <= (uint32_t)kVtxThreads)
    vtx_rank_sort(s_key, m);
  else
    vtx_sort(s_key, M);
  // cores: the neighbours of entry i are the range [first j with
  // zi - zj <= eps, first j > i with zj - zi > eps)
  for (uint32_t i = tid; i < m; i += nthr) {
    const double zi = (double)z_of_key(s_key[i]);
    uint32_t lo = 0, hi = i;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (zi - (double)z_of_key(s_key[mid]) <= c.vtx_eps) hi = mid; else lo = mid + 1;
    }
    const uint32_t first = lo;
    lo = i + 1;
    hi = m;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if ((double)z_of_key(s_key[mid]) - zi <= c.vtx_eps) lo = mid + 1; else hi = mid;
    }
    s_lab[i] = (int32_t)(lo - first) >= c.vtx_min_pts ? 1 : 0;
  }
  __syncthreads();
  // core ranks and positions; each thread owns kVtxPer consecutive entries
  const uint32_t b0 = tid * kVtxPer;
  uint32_t cnt = 0;
#pragma unroll
  for (int q = 0; q < kVtxPer; ++q)
    if (b0 + q < m && s_lab[b0 + q]) ++cnt;
  uint32_t ncore = 0;
  uint32_t r = vtx_excl_sum(cnt, s_scan, ncore);
#pragma unroll
  for (int q = 0; q < kVtxPer; ++q) {
    const uint32_t i = b0 + q;
    if (i < m) {
      s_rank[i] = r;
      if (s_lab[i]) s_core[r++] = i;
    }
  }
  __syncthreads();
  // clusters: a core starts one unless the previous core is within eps
  uint32_t st = 0;
#pragma unroll
  for (int q = 0; q < kVtxPer; ++q) {
    const uint32_t k = b0 + q;
    if (k < ncore) {
      const bool start =
          k == 0 || (double)z_of_key(s_key[s_core[k]]) - (double)z_of_key(s_key[s_core[k - 1]]) >
                        c.vtx_eps;
      st += start ? 1u : 0u;
    }
  }
  uint32_t ncl = 0;
  uint32_t cl = vtx_excl_sum(st, s_scan, ncl);
  // core labels (cluster numbers, increasing with z)
#pragma unroll
  for (int q = 0; q < kVtxPer; ++q) {
    const uint32_t k = b0 + q;
    if (k < ncore) {
      const bool start =
          k == 0 || (double)z_of_key(s_key[s_core[k]]) - (double)z_of_key(s_key[s_core[k - 1]]) >
                        c.vtx_eps;
      if (start) ++cl;
      s_lab[s_core[k]] = (int32_t)(cl - 1);
    }
  }
  __syncthreads();
  // borders and noise (non-core entries read core labels only)
  for (uint32_t i = tid; i < m; i += nthr) {
    const uint32_t rk = s_rank[i];
    const bool is_core = rk < ncore && s_core[rk] == i;
    if (is_core) continue;
    const double zi = (double)z_of_key(s_key[i]);
    int32_t lab = -1;
    double dp = 0.0, dn = 0.0;
    const bool hp = rk > 0, hn = rk < ncore;
    if (hp) dp = zi - (double)z_of_key(s_key[s_core[rk - 1]]);
    if (hn) dn = (double)z_of_key(s_key[s_core[rk]]) - zi;
    const bool okp = hp && dp <= c.vtx_eps, okn = hn && dn <= c.vtx_eps;
    if (okp && (!okn || dp <= dn)) lab = s_lab[s_core[rk - 1]];
    else if (okn) lab = s_lab[s_core[rk]];
    s_lab[i] = lab;
  }
  __syncthreads();
  if (ncl > o.max_per_event) {
    if (tid == 0) {
      o.n_vertices[e] = 0;
      atomicMax(&o.summary->required_per_event, ncl);
      atomicMax(&o.summary->max_selected, m);
      atomicCAS((unsigned int*)&o.summary->status, 0u, (unsigned int)PXT_ERR_CAPACITY);
    }
    return;
  }
  // cluster ranges (contiguous): starts over s_core, ends over s_rank; and
  // the weights in sorted order, so that the sums below stream them
  for (uint32_t i = tid; i < m; i += nthr) {
    s_ws[i] = s_w[s_key[i] & 0xfffu];
    const int32_t lab = s_lab[i];
    if (lab < 0) continue;
    if (i == 0 || s_lab[i - 1] != lab) s_core[lab] = i;
    if (i + 1 == m || s_lab[i + 1] != lab) s_rank[lab] = i;
  }
  __syncthreads();
  // (members read kVs at a time, key and weight independently, so that
  // their LDS loads overlap; the sums still run in sorted order)
  constexpr uint32_t kVs = 8;
  for (uint32_t v = tid; v < ncl; v += nthr) {
    const uint32_t a = s_core[v], b = s_rank[v] + 1;
    double sw = 0.0, swz = 0.0;
    for (uint32_t i0 = a; i0 < b; i0 += kVs) {
      uint64_t k[kVs];
      double w[kVs];
#pragma unroll
      for (uint32_t q = 0; q < kVs; ++q) {
        k[q] = i0 + q < b ? s_key[i0 + q] : 0ull;
        w[q] = i0 + q < b ? s_ws[i0 + q] : 0.0;
      }
#pragma unroll
      for (uint32_t q = 0; q < kVs; ++q) {
        if (i0 + q < b) {
          sw += w[q];
          swz += w[q] * (double)z_of_key(k[q]);
        }
      }
    }
    const double zv = swz / sw;
    double chi2 = 0.0;
    for (uint32_t i0 = a; i0 < b; i0 += kVs) {
      uint64_t k[kVs];
      double w[kVs];
#pragma unroll
      for (uint32_t q = 0; q < kVs; ++q) {
        k[q] = i0 + q < b ? s_key[i0 + q] : 0ull;
        w[q] = i0 + q < b ? s_ws[i0 + q] : 0.0;
      }
#pragma unroll
      for (uint32_t q = 0; q < kVs; ++q) {
        if (i0 + q < b) {
          const double rz = (double)z_of_key(k[q]) - zv;
          chi2 += w[q] * rz * rz;
        }
      }
    }
    const uint32_t bl = b - 1;
    const size_t slot = (size_t)e * o.max_per_event + v;
    o.z[slot] = (float)zv;
    o.z_err[slot] = (float)sqrt(1.0 / sw);
    o.chi2[slot] = (float)chi2;
    o.n_tracks[slot] = bl - a + 1;
  }
  // every member's vertex, by all threads (the sums above run one thread
  // per cluster)
  for (uint32_t i = tid; i < m; i += nthr) {
    const int32_t lab = s_lab[i];
    if (lab >= 0) o.track_vertex[toff + (uint32_t)((s_key[i] >> 12) & 0xfffffu)] = lab;
  }
  if (tid == 0) {
    o.n_vertices[e] = ncl;
    atomicAdd(&o.summary->n_vertices, ncl);
    atomicMax(&o.summary->required_per_event, ncl);
    atomicMax(&o.summary->max_selected, m);
  }
}

__device__ __forceinline__ void k_vtx_begin_body(const VtxOut& o) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    o.summary->status = 0;
    o.summary->n_vertices = 0;
    o.summary->required_per_event = 0;
    o.summary->max_selected = 0;
  }
}

// One block per event (blocks past n_events leave); when the tracks' own
// status is not ok, no vertices and that status in the summary.
__device__ __forceinline__ void vertices_block(const VtxIn& in, const VtxOut& o,
                                               const DevCfg& c) {
  const uint32_t e = blockIdx.x;
  if (e >= in.n_events) return;
  if (in.counts && in.counts->status != 0) {
    if (threadIdx.x == 0) {
      o.n_vertices[e] = 0;
      if (e == 0) o.summary->status = in.counts->status;
    }
    return;
  }
  vertices_event(in, o, c, e);
}

__global__ void k_vtx_begin(VtxOut o) { k_vtx_begin_body(o); }

__global__ __launch_bounds__(kVtxThreads) void k_vertices(VtxIn in, VtxOut o, DevCfg c) {
  vertices_block(in, o, c);
}

}  // namespace pxt
