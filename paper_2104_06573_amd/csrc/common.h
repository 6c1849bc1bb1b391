// Device-side types and wavefront primitives shared by the pxt kernels.
//
// Everything here targets gfx950 (CDNA4): 64-lane wavefronts, 64-bit ballot
// masks, LDS for cross-wave exchange.  The whole library is compiled with
// -ffp-contract=off so that every double-precision cut is evaluated with the
// rounding of the written expression (no fused multiply-adds), which is what
// makes the cut decisions reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pxt.h"

namespace pxt {

constexpr int kMaxLayers = PXT_MAX_LAYERS;
constexpr int kMaxOuterPerLayer = 8;
constexpr int kMaxHits = PXT_MAX_TUPLE_HITS;   // hits per n-tuplet
constexpr int kMaxCells = kMaxHits - 1;        // doublets per n-tuplet
constexpr uint32_t kPad = PXT_PAD;
constexpr int kWave = 64;
constexpr float kPiF = 3.14159265358979f;
constexpr int kQueue = 128;                    // LDS queue entries per wavefront
constexpr uint32_t kSmallFit = 8192;           // calls with at most this many tracks: one fit launch
constexpr uint32_t kCompactBlocksMax = 4096;   // grid cap of the doublet stage

// Counters kept in device memory for one call (zeroed by k_clear).
enum Ctr : int {
  C_STATUS = 0,      // int32 pxt_status found on the device
  C_NBINS,           // number of phi bins of the batch (host-known)
  C_NBINNED,         // hits with a valid layer id
  C_ND,              // doublets
  C_NWORDS,          // link-mask words
  C_WSTRIDE,         // link-mask words per doublet
  C_NLINKS,          // links
  C_NTUP,            // raw n-tuplets
  C_NSURV,           // n-tuplets surviving the cleaning
  C_NFP64,           // tuples refitted in FP64
  C_NROOT,           // root doublets of the n-tuplet search
  C_REQ_D,           // required sizes on overflow
  C_REQ_W,
  C_REQ_T,
  C_REQ_K,
  C_FITN0,           // survivors of length class k (3, 4, 5+ hits) at C_FITN0 + 3 + k
  C_TICKET0 = C_FITN0 + kMaxHits + 1,  // tile tickets of the single-pass scans
  C_TICKET_END = C_TICKET0 + 8,
  C_NCTR = C_TICKET_END
};

// Physics and tuning constants, passed by value to the kernels.
struct DevCfg {
  int n_layers;
  int nphi;
  float phi_scale;                          // nphi / (2 pi)
  float kmax_f;
  int layer_kind[kMaxLayers];
  int n_outer[kMaxLayers];                  // pairs leaving each layer
  int outer[kMaxLayers][kMaxOuterPerLayer]; // their outer layers, table order
  double kmax, z0max, arz, d0max;
  double kmax2, arz2;                       // squares, for the fast forms
  double c_kappa, sigma_u, sigma_z, sigma_r, x_over_x0, pt_max, pt_fp64;
  uint32_t cap_doublets, cap_words, cap_tuples;
  int link_kernel;                          // 0 thread, 1 lane group, 2 wave
  int bin_lds;                              // binning by one block per event
  int q_win, q_far, q_far_min;              // r-z angle prefilter of the links (angle
                                            // units): window, anti-parallel window, and
                                            // the |angle| below which the latter cannot hold
  // output selection and quality flags
  int min_hits;                             // shorter survivors are not output
  float q_chi2;                             // LOOSE: chi2 per ndf at most
  float q_qopt_max;                         // STRICT: |q/pT| at most (1/pT_min)
  float q_d0_max, q_z0_max;                 // STRICT: |d0|, |z0| at most
  // vertices
  double vtx_eps;
  int vtx_min_pts, vtx_min_hits;
  float vtx_qopt_max;                       // 1/pT_min in single precision
};

struct CallDesc;

// Device arenas of one context.
struct Ws {
  const CallDesc* call;   // descriptor of the current call
  uint32_t* ctr;          // [C_NCTR]
  uint32_t* evt_off;      // [E + 1] (follows the descriptor)
  uint32_t* keys;         // [H]   bin key of each input hit
  uint32_t* bin_cnt;      // [nbins + 1]
  uint32_t* bin_off;      // [nbins + 1]
  uint32_t* rmax;         // [E * L] largest hit radius per layer (float bits)
  float* rasin;           // [E * L] turning angle to that radius (inf: any)
  // binned hits
  float4* bh;             // (x, y, z, phi): one load per candidate
  double* br;             // transverse radius in FP64
  uint32_t* bidx;         // event-local input index
  uint32_t* bevt;         // event id
  uint8_t* blay;          // layer id
  // doublets
  uint32_t* dcnt;         // [H + 1] doublets per inner hit
  uint32_t* cell_off;     // [H + 1] first doublet of each inner hit
  uint2* cio;             // [D] (inner, outer) binned hits: one store, one load
  uint64_t* masks;        // [W] link masks, C_WSTRIDE words per doublet
  uint8_t* has_inner;     // [D]
  uint8_t* has_out;       // [D] the doublet has an outer link
  int16_t* th;            // [D + 16] r-z angle of each doublet in angle units (the link
                          // prefilter's stream)
  uint32_t* roots;        // [D] root doublets, ascending
  uint32_t* rcnt;         // [D + 1] n-tuplets per root doublet
  uint32_t* roff;         // [D + 1]
  // n-tuplets
  uint32_t* thit;         // [T][8] binned hits of each n-tuplet (kPad-padded)
  uint32_t* tcell;        // [T][8] its doublets (7 used, kPad-padded)
  // staged doublets: per-wavefront record regions over roots .. fp64_list,
  // which hold nothing until the links are done
  uint32_t* stage;
  uint32_t stage_words;
  uint32_t* dwn;          // [blocks * 4] records per wavefront region (the doublet
                          // staging, then the n-tuplet walk)
  uint8_t* tn;            // [T] hits
  double* tscore;         // [T]
  // cleaning
  uint64_t* bkey;         // [D] smallest order key of the tuples through it (call-tagged)
  uint64_t* best;         // [D] best tuple through each doublet: call epoch << 32 | tuple
  uint32_t* evt_surv;     // [E + 1] first survivor of each event
  uint4* trow;            // [T][4] staged n-tuplet rows (hits, doublets)
  uint2* tmeta;           // [T] staged row: root, index among its paths | hits << 28
  uint32_t* surv;         // [T]
  uint32_t* sfit;         // [3][T] survivor indices per length class (the fitting order)
  uint32_t* fp64_list;    // [T]
  // scan scratch
  uint64_t* scan_status;  // [max tiles] status words of the single-pass scan
  uint32_t* epoch;        // [1] call counter (never cleared)
};


// ------------------------------------------------------------------------
// wavefront primitives

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= (uint32_t)d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Exclusive block-wide prefix sum; `tot` receives the block total.
// lds must hold blockDim.x / 64 + 1 words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds,
                                                    uint32_t& tot) {
  const uint32_t lane = lane_id();
  const uint32_t wid = threadIdx.x / kWave;
  const uint32_t nw = blockDim.x / kWave;
  uint32_t inc = wave_incl_scan(v);
  if (lane == kWave - 1) lds[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < nw ? lds[lane] : 0u;
    uint32_t wi = wave_incl_scan(w);
    if (lane < nw) lds[lane] = wi - w;
    if (lane == nw - 1) lds[nw] = wi;
  }
  __syncthreads();
  uint32_t res = lds[wid] + inc - v;
  tot = lds[nw];
  __syncthreads();
  return res;
}

// Append `want` (0 or 1) items per lane to a global counter with one atomic
// per wavefront; returns this lane's slot (valid when want != 0).
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool want) {
  const uint64_t m = __ballot(want);
  if (m == 0) return 0;
  const uint32_t leader = __ffsll((unsigned long long)m) - 1;
  const uint32_t below = __popcll(m & ((1ull << lane_id()) - 1ull));
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __shfl(base, leader, kWave);
  return base + below;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, (uint32_t)__shfl_xor(v, d, kWave));
  return v;
}

// XCD-aware logical block index.  Consecutive workgroups of a dispatch go
// round-robin to the 8 XCDs of the chip; with this remap each XCD receives
// a contiguous range of logical blocks, so the contiguous item chunks it
// processes (doublets of the same events) share that XCD's L2.  Identity
// unless the grid is a multiple of 8.
__device__ __forceinline__ uint32_t xcd_block() {
  const uint32_t b = blockIdx.x, n = gridDim.x;
  if (n % 8u) return b;
  return (b % 8u) * (n / 8u) + b / 8u;
}

__device__ __forceinline__ void set_status(uint32_t* ctr, int st) {
  atomicCAS(&ctr[C_STATUS], 0u, (uint32_t)st);
}

__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t* a, uint32_t n,
                                                    uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Number of entries of the sorted a[0..n) below v.
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* a, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace pxt
