// libpxt: C ABI of the pixel-track reconstruction core (see include/pxt.h).
//
// Host side: context creation (one device allocation carved into arenas,
// sized from the configured capacities), argument validation, the launch
// sequence of one call on the caller's stream, and debug dumps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "host_copy.h"
#include "rechits.h"

using namespace pxt;

struct pxt_ctx {
  int device = 0;
  pxt_config cfg{};
  DevCfg dc{};
  void* arena = nullptr;
  size_t arena_bytes = 0;
  Ws ws{};
  // ring of pinned host slots holding each call's descriptor and event
  // offsets; a slot is rewritten only after the call that used it has
  // consumed it, so the host may run up to kSlots calls ahead
  static constexpr int kSlots = 4;
  char* h_slots = nullptr;
  size_t slot_bytes = 0;
  hipEvent_t slot_free[kSlots] = {};
  bool slot_pending[kSlots] = {};
  int next_slot = 0;
  // HIP graphs of the launch sequence, one per slot and binning kernel set
  // (graph mode), captured at their first use
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[kSlots][2] = {};
  hipGraphExec_t gexec[kSlots][2] = {};
  int n_cu = 256;
  // calls made on this context: the scan status words carry a 30-bit tag of
  // (call, scan), which repeats after 2^27 calls, so they are reset every
  // kEpochReset calls (a stale word is then at most that many calls old)
  uint64_t calls = 0;
  static constexpr uint64_t kEpochReset = 1ull << 26;
  std::string err;
  // per-stage timing
  bool timing = false;
  bool timed_valid = false;
  hipEvent_t ev[PXT_N_STAGES + 1] = {};
  bool stage_run[PXT_N_STAGES] = {};
  // last call, for the debug dumps
  bool have_last = false;
  uint32_t last_events = 0;
  std::vector<uint32_t> last_offsets;
};

namespace {

thread_local std::string g_create_err;

int fail(pxt_ctx* c, int st, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return st;
}

#define HIP_OR_FAIL(ctx, call)                                                 \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return fail((ctx), PXT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t n) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * std::max<size_t>(n, 1);
    return p;
  }
};

size_t desc_bytes() { return align_up(sizeof(CallDesc), 64); }
size_t slot_bytes_for(const pxt_config& c) {
  return desc_bytes() + sizeof(uint32_t) * ((size_t)c.max_events + 1);
}

// Largest number of elements any scan of a call covers, in scan tiles.
size_t scan_tiles(const pxt_config& c) {
  const size_t nbins = (size_t)c.max_events * (size_t)c.n_layers * (size_t)c.phi_bins;
  const size_t n = std::max({nbins, (size_t)c.max_hits, (size_t)c.max_doublets,
                             (size_t)c.max_tuples});
  // (the per-event binning takes one tile per event)
  // single-pass doublets: one tile per blockDim/group_lanes binned hits
  const size_t gpb = (size_t)std::max(1, c.block_size / std::max(1, c.group_lanes));
  return std::max({(n + kTile - 1) / kTile + 1, (size_t)c.max_hits / gpb + 2,
                   (size_t)c.max_events + 1});
}

void carve(Carver& cv, const pxt_config& c, Ws& w) {
  const size_t H = c.max_hits, D = c.max_doublets, Wd = c.max_link_words, T = c.max_tuples;
  const size_t nbins = (size_t)c.max_events * (size_t)c.n_layers * (size_t)c.phi_bins;
  const size_t E = c.max_events;
  char* call = cv.take<char>(slot_bytes_for(c));
  w.call = reinterpret_cast<const CallDesc*>(call);
  w.evt_off = call ? reinterpret_cast<uint32_t*>(call + desc_bytes()) : nullptr;
  w.ctr = cv.take<uint32_t>(C_NCTR);
  w.keys = cv.take<uint32_t>(H);
  w.bin_cnt = cv.take<uint32_t>(nbins + 1);
  w.bin_off = cv.take<uint32_t>(nbins + 1);
  w.rmax = cv.take<uint32_t>(E * c.n_layers);
  w.rasin = cv.take<float>(E * c.n_layers);
  w.bh = cv.take<float4>(H);
  w.br = cv.take<double>(H);
  w.bidx = cv.take<uint32_t>(H);
  w.bevt = cv.take<uint32_t>(H);
  w.blay = cv.take<uint8_t>(H);
  w.dcnt = cv.take<uint32_t>(H + 1);
  w.cell_off = cv.take<uint32_t>(H + 1);
  w.cio = cv.take<uint2>(D);
  w.has_inner = cv.take<uint8_t>(D);
  w.has_out = cv.take<uint8_t>(D + 16);  // read 16 flags at a time
  w.th = cv.take<int16_t>(D + 16);  // aligned 16-byte reads may pass the end by 7
  // the election slots keep their contents from call to call (tagged with
  // the call), so they lie outside the doublet staging span below
  w.bkey = cv.take<uint64_t>(D);
  w.best = cv.take<uint64_t>(D);
  // the link masks come first in the staging span: the link kernels write
  // them only after the doublet scatter has read the staged records
  w.masks = cv.take<uint64_t>(Wd);
  w.roots = cv.take<uint32_t>(D);
  w.rcnt = cv.take<uint32_t>(D + 1);
  w.roff = cv.take<uint32_t>(D + 1);
  w.thit = cv.take<uint32_t>(8 * T);
  w.tcell = cv.take<uint32_t>(8 * T);
  w.tn = cv.take<uint8_t>(T);
  w.tscore = cv.take<double>(T);
  w.evt_surv = cv.take<uint32_t>(E + 1);
  w.trow = cv.take<uint4>(4 * T);
  w.tmeta = cv.take<uint2>(T);
  w.surv = cv.take<uint32_t>(T);
  w.sfit = cv.take<uint32_t>(3 * T);
  w.fp64_list = cv.take<uint32_t>(T);
  // the staging buffer of the doublets spans masks .. fp64_list
  w.stage = reinterpret_cast<uint32_t*>(w.masks);
  w.stage_words = cv.base ? (uint32_t)std::min<size_t>(
                                 (size_t)(reinterpret_cast<char*>(w.fp64_list + T) -
                                          reinterpret_cast<char*>(w.masks)) /
                                     sizeof(uint32_t),
                                 0xfffffffeu)
                           : 0u;
  w.dwn = cv.take<uint32_t>((size_t)kCompactBlocksMax * (256 / kWave));
  w.scan_status = cv.take<uint64_t>(scan_tiles(c));
  w.epoch = cv.take<uint32_t>(1);
}

int validate_config(const pxt_config* c, std::string& why) {
  if (!(c->c_kappa > 0)) return why = "c_kappa must be > 0", 1;
  if (c->n_layers < 1 || c->n_layers > PXT_MAX_LAYERS) return why = "n_layers out of range", 1;
  if (c->n_pairs < 0 || c->n_pairs > PXT_MAX_PAIRS) return why = "n_pairs out of range", 1;
  int per_layer[PXT_MAX_LAYERS] = {0};
  for (int i = 0; i < c->n_pairs; ++i) {
    const int a = c->pair_inner[i], b = c->pair_outer[i];
    if (a < 0 || a >= c->n_layers || b < 0 || b >= c->n_layers || a == b)
      return why = "layer pair out of range", 1;
    if (++per_layer[a] > kMaxOuterPerLayer) return why = "more than 8 pairs leave one layer", 1;
  }
  for (int l = 0; l < c->n_layers; ++l)
    if (c->layer_kind[l] != PXT_LAYER_BARREL && c->layer_kind[l] != PXT_LAYER_DISK)
      return why = "layer_kind must be 0 or 1", 1;
  if (!(c->kmax > 0 && c->z0max > 0 && c->arz > 0 && c->d0max > 0))
    return why = "cuts must be > 0", 1;
  if (!(c->sigma_u > 0 && c->sigma_z > 0 && c->sigma_r > 0 && c->x_over_x0 > 0 && c->pt_max > 0))
    return why = "fit constants must be > 0", 1;
  if (c->max_events < 1 || c->max_hits < 1 || c->max_doublets < 1 || c->max_link_words < 1 ||
      c->max_tuples < 1)
    return why = "capacities must be >= 1", 1;
  if ((uint64_t)c->max_hits >= 0xffffffffull || (uint64_t)c->max_doublets >= 0xfffffff0ull ||
      (uint64_t)c->max_tuples * 8ull >= 0xfffffff0ull)
    return why = "capacity too large for 32-bit indices", 1;
  if (c->phi_bins < 16 || c->phi_bins > 4096) return why = "phi_bins out of 16..4096", 1;
  if ((uint64_t)c->max_events * c->n_layers * c->phi_bins >= 0x7fffffffull)
    return why = "max_events * n_layers * phi_bins too large", 1;
  if (c->block_size < 64 || c->block_size > 256 || c->block_size % 64)
    return why = "block_size must be 64, 128, 192 or 256", 1;
  if (!(c->pt_fp64 > 0)) return why = "pt_fp64 must be > 0", 1;
  if (c->group_lanes != 4 && c->group_lanes != 8 && c->group_lanes != 16 &&
      c->group_lanes != 32 && c->group_lanes != 64)
    return why = "group_lanes must be 4, 8, 16, 32 or 64", 1;
  if (c->link_kernel < 0 || c->link_kernel > 2) return why = "link_kernel must be 0, 1 or 2", 1;
  if (c->use_graph != 0 && c->use_graph != 1) return why = "use_graph must be 0 or 1", 1;
  if (c->doublet_mode < 0 || c->doublet_mode > 2) return why = "doublet_mode must be 0, 1 or 2", 1;
  if (c->min_hits < 3 || c->min_hits > PXT_MAX_TUPLE_HITS) return why = "min_hits out of 3..8", 1;
  if (!(c->q_chi2 > 0 && c->q_pt_min > 0 && c->q_d0_max > 0 && c->q_z0_max > 0))
    return why = "quality limits must be > 0", 1;
  if (!(c->vtx_eps > 0 && c->vtx_pt_min > 0) || c->vtx_min_pts < 1 || c->vtx_min_hits < 3 ||
      c->vtx_min_hits > PXT_MAX_TUPLE_HITS)
    return why = "vertex constants out of range", 1;
  return 0;
}

void make_devcfg(const pxt_config& c, DevCfg& d) {
  std::memset(&d, 0, sizeof(d));
  d.n_layers = c.n_layers;
  d.nphi = c.phi_bins;
  d.phi_scale = (float)(c.phi_bins / (2.0 * M_PI));
  d.kmax_f = (float)c.kmax;
  for (int l = 0; l < c.n_layers; ++l) d.layer_kind[l] = c.layer_kind[l];
  for (int i = 0; i < c.n_pairs; ++i) {
    const int a = c.pair_inner[i];
    d.outer[a][d.n_outer[a]++] = c.pair_outer[i];
  }
  d.kmax = c.kmax;
  d.kmax2 = c.kmax * c.kmax;
  d.arz2 = c.arz * c.arz;
  d.z0max = c.z0max;
  d.arz = c.arz;
  d.d0max = c.d0max;
  d.c_kappa = c.c_kappa;
  d.sigma_u = c.sigma_u;
  d.sigma_z = c.sigma_z;
  d.sigma_r = c.sigma_r;
  d.x_over_x0 = c.x_over_x0;
  d.pt_max = c.pt_max;
  d.pt_fp64 = c.pt_fp64;
  d.cap_doublets = c.max_doublets;
  d.cap_words = c.max_link_words;
  d.cap_tuples = c.max_tuples;
  d.link_kernel = c.link_kernel;
  d.bin_lds = (uint32_t)c.n_layers * (uint32_t)c.phi_bins <= kBinLdsBins;
  d.min_hits = c.min_hits;
  d.q_chi2 = c.q_chi2;
  d.q_qopt_max = (float)(1.0 / (double)c.q_pt_min);
  d.q_d0_max = c.q_d0_max;
  d.q_z0_max = c.q_z0_max;
  d.vtx_eps = c.vtx_eps;
  d.vtx_min_pts = c.vtx_min_pts;
  d.vtx_min_hits = c.vtx_min_hits;
  d.vtx_qopt_max = (float)(1.0 / c.vtx_pt_min);
  // L1 holds only if the r-z directions of the two doublets differ by at
  // most asin(arz) or by at least pi - asin(arz).  The FP32 angles carry an
  // error below 1e-6 rad (inputs rounded to FP32: < 1.2e-7; atan2f: a few
  // ulp), so a margin of 1e-5 rad keeps a prefilter on them a strict
  // superset of the FP64 decision.  The stored angles are those rounded to
  // units of (pi/2) / 32767 rad (within one unit each), so the windows in
  // units widen by two: |ta - tc| <= w rad gives at most floor(w / unit) + 2
  // units, >= f rad at least ceil(f / unit) - 2.  arz >= 1 leaves it open.
  const double unit = (M_PI / 2.0) / 32767.0;
  if (c.arz < 1.0) {
    const double a = std::asin(c.arz) + 1e-5;
    d.q_win = (int)std::floor(a / unit) + 2;
    d.q_far = (int)std::ceil((M_PI - a) / unit) - 2;
  } else {
    d.q_win = 65536;
    d.q_far = 0;
  }
  d.q_far_min = d.q_far - 32767;
}

// Blocks of a single-pass scan over at most max_n entries.
uint32_t scan_grid(uint64_t max_n) {
  return (uint32_t)std::max<uint64_t>(1, (max_n + kTile - 1) / kTile);
}

// Single-pass exclusive scan of n = *n_dev entries; `max_n` bounds *n_dev
// (grid size); scan_id is the scan's index within one call (distinct per
// call site, below 8).
void launch_scan1(const Ws& w, const uint32_t* in, uint32_t* out, const uint32_t* n_dev,
                  uint32_t* total_dst, uint64_t max_n, uint32_t scan_id, hipStream_t s) {
  hipLaunchKernelGGL(k_scan1, dim3(scan_grid(max_n)), dim3(kScanThreads1), 0, s, in, out, n_dev,
                     total_dst, w, scan_id);
}


const char* const kStageNames[PXT_N_STAGES] = {
    "clear",       "prep",       "bin_scan",    "fill",       "doublet_count",
    "doublet_scan", "doublet_fill", "mask_clear", "links",    "roots",
    "tuple_count", "tuple_scan", "tuple_fill",  "score",      "best",
    "survive",     "fit32",      "fit64",       "finish",     "vertices"};

// Marks the start of stage i when timing is on (c == nullptr: no timing).
struct StageMarks {
  pxt_ctx* c;
  hipStream_t s;
  void mark(int i) {
    if (!c || !c->timing) return;
    (void)hipEventRecord(c->ev[i], s);
    c->stage_run[i] = true;
  }
};

uint32_t grid_for(uint64_t items, int bs, uint32_t cap_blocks) {
  uint64_t g = (items + bs - 1) / bs;
  if (g < 1) g = 1;
  return (uint32_t)std::min<uint64_t>(g, cap_blocks);
}

// Grid of the chunked group kernels: a multiple of 8 blocks (an equal share
// per XCD), about four items per lane group, at most cap_blocks.
uint32_t grid_chunked(uint64_t items, int bs, int G, uint32_t cap_blocks) {
  const uint64_t groups = (items + 3) / 4;
  uint64_t g = (groups * G + bs - 1) / bs;
  g = std::max<uint64_t>(8, (g + 7) / 8 * 8);
  return (uint32_t)std::min<uint64_t>(g, cap_blocks / 8 * 8);
}

template <bool FILL>
void launch_doublets(int G, dim3 grid, dim3 block, hipStream_t s, const Ws& w, const DevCfg& d) {
  switch (G) {
    case 4: hipLaunchKernelGGL((k_doublets<4, FILL>), grid, block, 0, s, w, d); break;
    case 8: hipLaunchKernelGGL((k_doublets<8, FILL>), grid, block, 0, s, w, d); break;
    case 16: hipLaunchKernelGGL((k_doublets<16, FILL>), grid, block, 0, s, w, d); break;
    case 64: hipLaunchKernelGGL((k_doublets<64, FILL>), grid, block, 0, s, w, d); break;
    default: hipLaunchKernelGGL((k_doublets<32, FILL>), grid, block, 0, s, w, d); break;
  }
}

// kernel template over the group width
#define PXT_LAUNCH_G(K, G, grid, block, s, ...)                                  \
  do {                                                                           \
    switch (G) {                                                                 \
      case 4: hipLaunchKernelGGL((K<4>), grid, block, 0, s, __VA_ARGS__); break;   \
      case 8: hipLaunchKernelGGL((K<8>), grid, block, 0, s, __VA_ARGS__); break;   \
      case 16: hipLaunchKernelGGL((K<16>), grid, block, 0, s, __VA_ARGS__); break; \
      case 64: hipLaunchKernelGGL((K<64>), grid, block, 0, s, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL((K<32>), grid, block, 0, s, __VA_ARGS__); break; \
    }                                                                            \
  } while (0)

// Blocks of a kernel that all compute units hold at once (from its register
// and LDS footprint), as a multiple of 8 (an equal share per XCD): the grid
// of a grid-stride kernel whose blocks get equal shares of the work, so that
// no second, partial round of blocks trails the first.  Cached per kernel and
// block size in a fixed table (no allocation on this path).
uint32_t resident_grid(const void* kernel, int bs, int n_cu) {
  struct Entry {
    const void* kernel;
    int bs, nb;
  };
  static std::mutex mu;
  static Entry cache[32];
  static int used = 0;
  int nb = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; ++i)
      if (cache[i].kernel == kernel && cache[i].bs == bs) nb = cache[i].nb;
    if (nb == 0) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, bs, 0) != hipSuccess ||
          nb < 1)
        nb = 1;
      if (used < 32) cache[used++] = Entry{kernel, bs, nb};
    }
  }
  return std::max<uint32_t>(8, (uint32_t)nb * (uint32_t)n_cu / 8u * 8u);
}

void launch_links(int G, dim3 grid, dim3 block, hipStream_t s, const Ws& w, const DevCfg& d) {
  if (d.link_kernel == 0) {
    hipLaunchKernelGGL(k_links_thread, grid, block, 0, s, w, d);
    return;
  }
  if (d.link_kernel == 2) {
    hipLaunchKernelGGL(k_links_wave, grid, block, 0, s, w, d);
    return;
  }
  switch (G) {
    case 4: hipLaunchKernelGGL((k_links<4>), grid, block, 0, s, w, d); break;
    case 8: hipLaunchKernelGGL((k_links<8>), grid, block, 0, s, w, d); break;
    case 16: hipLaunchKernelGGL((k_links<16>), grid, block, 0, s, w, d); break;
    case 64: hipLaunchKernelGGL((k_links<64>), grid, block, 0, s, w, d); break;
    default: hipLaunchKernelGGL((k_links<32>), grid, block, 0, s, w, d); break;
  }
}

// The kernels of one call on stream s, after its descriptor is in place.
// In graph mode the sequence is captured once per slot: work sizes come
// from the capacities and every kernel reads the call's actual sizes from
// the descriptor; in direct mode the grids are sized from this call's hits
// (H) and events (E).  c supplies the stage timing (nullptr: none).
void enqueue_path(pxt_ctx* c, const pxt_config& cfg, const Ws& w, const DevCfg& d, int n_cu,
                  hipStream_t s, bool graph_mode, uint32_t H, uint32_t E, bool bin_lds) {
  const int bs = cfg.block_size;
  const uint32_t persist = (uint32_t)n_cu * 8u;
  if (graph_mode) {
    H = cfg.max_hits;
    E = cfg.max_events;
  }
  const uint32_t nbins = E * (uint32_t)cfg.n_layers * (uint32_t)cfg.phi_bins;
  StageMarks sm{c, s};
  const bool timed = c && c->timing && !graph_mode;
  if (timed)
    for (int i = 0; i < PXT_N_STAGES; ++i) c->stage_run[i] = false;
  if (timed) sm.mark(0);
  const bool bin_glob = !bin_lds, bin_ev = bin_lds;  // the call's binning kernels
  const uint64_t nclear = std::max<uint64_t>(bin_glob ? nbins + 1 : E, C_NCTR);
  hipLaunchKernelGGL(k_clear, dim3(grid_for(nclear, 256, persist)), dim3(256), 0, s, w, d);
  hipLaunchKernelGGL(k_slots_clear, dim3(grid_for(cfg.max_doublets, 256, persist)), dim3(256), 0,
                     s, w, d);
  if (H > 0) {
    if (timed) sm.mark(1);
    if (bin_glob) {
      const uint32_t gh1 = grid_for(H, 256, persist);
      hipLaunchKernelGGL(k_prep, dim3(gh1), dim3(256), 0, s, w, d);
      if (timed) sm.mark(2);
      launch_scan1(w, w.bin_cnt, w.bin_off, w.ctr + C_NBINS, w.ctr + C_NBINNED, nbins, 0, s);
      if (timed) sm.mark(3);
      hipLaunchKernelGGL(k_fill, dim3(gh1), dim3(256), 0, s, w);
      hipLaunchKernelGGL(k_rmax,
                         dim3(grid_for((uint64_t)E * cfg.n_layers * kWave, 256, persist)),
                         dim3(256), 0, s, w, d);
    }
    if (bin_ev) {
      // one block per event (in direct mode its time shows under prep)
      hipLaunchKernelGGL(k_bin_events, dim3(std::max<uint32_t>(1, E)), dim3(kBinThreads),
                         sizeof(uint32_t) * (size_t)cfg.n_layers * (size_t)cfg.phi_bins, s, w, d);
    }
    const int G = cfg.group_lanes;
    // (the staging pair keeps the full persistent grid: measured faster for
    // the scatter than the resident-block grid)
    const uint32_t gh = grid_chunked(H, bs, G, std::min<uint32_t>(persist, kCompactBlocksMax));
    if (cfg.doublet_mode == 1) {
      // one pass (its time shows under doublet_fill)
      const uint32_t gpb = (uint32_t)(bs / G);
      if (timed) sm.mark(6);
      PXT_LAUNCH_G(k_doublets1, G,
                   dim3((uint32_t)std::max<uint64_t>(1, ((uint64_t)H + gpb - 1) / gpb)), dim3(bs),
                   s, w, d);
    } else {
      if (timed) sm.mark(4);
      if (cfg.doublet_mode == 2)
        PXT_LAUNCH_G(k_dstage, G, dim3(gh), dim3(bs), s, w, d);
      else
        launch_doublets<false>(G, dim3(gh), dim3(bs), s, w, d);
      if (timed) sm.mark(5);
      launch_scan1(w, w.dcnt, w.cell_off, w.ctr + C_NBINNED, w.ctr + C_ND, H, kDoubletScan, s);
      if (timed) sm.mark(6);
      if (cfg.doublet_mode == 2)
        PXT_LAUNCH_G(k_dscatter, G, dim3(gh), dim3(bs), s, w, d);
      else
        launch_doublets<true>(G, dim3(gh), dim3(bs), s, w, d);
    }
    if (timed) sm.mark(7);
    const uint32_t gd = grid_for(cfg.max_doublets, bs, persist);
    if (cfg.link_kernel == 1) hipLaunchKernelGGL(k_zero_words, dim3(gd), dim3(256), 0, s, w, d);
    if (timed) sm.mark(8);
    uint32_t gl;
    if (cfg.link_kernel == 1)
      gl = grid_chunked((uint64_t)H * 16, bs, G, persist);
    else
      gl = std::min(std::max<uint32_t>(8, gd / 8 * 8),
                    resident_grid(cfg.link_kernel == 0 ? (const void*)k_links_thread
                                                       : (const void*)k_links_wave,
                                  bs, n_cu));
    launch_links(G, dim3(gl), dim3(bs), s, w, d);
    if (timed) sm.mark(9);
    hipLaunchKernelGGL(k_roots, dim3(scan_grid(cfg.max_doublets)), dim3(kScanThreads1), 0, s, w,
                       6u);
    if (timed) sm.mark(10);
    // (the walk and the move share one grid: a wavefront's staging region
    // and roots are the same in both)
    const uint32_t gtu = std::min({gd, resident_grid((const void*)k_tuples<false>, bs, n_cu),
                                   kCompactBlocksMax * (256u / kWave) / (uint32_t)(bs / kWave)});
    hipLaunchKernelGGL(k_tuples<false>, dim3(gtu), dim3(bs), 0, s, w, d);
    if (timed) sm.mark(11);
    launch_scan1(w, w.rcnt, w.roff, w.ctr + C_NROOT, w.ctr + C_NTUP, cfg.max_doublets, 3, s);
    if (timed) sm.mark(12);
    hipLaunchKernelGGL(k_tuples<true>, dim3(gtu), dim3(bs), 0, s, w, d);
    const uint32_t gt = grid_for(cfg.max_tuples, bs, persist);
    if (timed) sm.mark(13);
    hipLaunchKernelGGL(k_score, dim3(std::min(gt, resident_grid((const void*)k_score, bs, n_cu))),
                       dim3(bs), 0, s, w, d);
    if (timed) sm.mark(14);
    hipLaunchKernelGGL(k_best, dim3(std::min(gt, resident_grid((const void*)k_best, bs, n_cu))),
                       dim3(bs), 0, s, w, d);
    if (timed) sm.mark(15);
    // survivors, the fitting order (one list per length class) and each
    // event's first survivor
    hipLaunchKernelGGL(k_survive,
                       dim3((uint32_t)(((uint64_t)cfg.max_tuples + kSurvThreads - 1) / kSurvThreads)),
                       dim3(kSurvThreads), 0, s, w, d);
    if (timed) sm.mark(16);
    {
      // fits of 3 and of 4 hits, then the rarer longer ones together (one
      // thread per tuple of the capacity)
      const uint32_t gf = grid_for(cfg.max_tuples, 256, 0xffffffffu);
      hipLaunchKernelGGL(k_fit_small, dim3(kSmallFit / 256 + 2), dim3(256), 0, s, w, d);
      hipLaunchKernelGGL(k_fit32<3>, dim3(gf), dim3(256), 0, s, w, d);
      hipLaunchKernelGGL(k_fit32<4>, dim3(gf), dim3(256), 0, s, w, d);
      hipLaunchKernelGGL(k_fit32<0>, dim3(gf), dim3(256), 0, s, w, d);
    }
    if (timed) sm.mark(17);
    hipLaunchKernelGGL(k_fit64, dim3(grid_for(cfg.max_tuples, 64, (uint32_t)n_cu)), dim3(64),
                       0, s, w, d);
  }
  if (timed) sm.mark(18);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, w);
  // vertices of the call's tracks (the kernels leave at once when the call
  // has no vertex buffers)
  if (timed) sm.mark(19);
  hipLaunchKernelGGL(k_vertices_call, dim3(std::max<uint32_t>(1, E)), dim3(kVtxThreads), 0, s,
                     w, d);
  if (timed) {
    (void)hipEventRecord(c->ev[PXT_N_STAGES], s);
    c->timed_valid = true;
  }
}

// One call of a context: its descriptor and event offsets from the pinned
// slot, then the kernels.
void enqueue(pxt_ctx* c, hipStream_t s, int slot, bool graph_mode, uint32_t H, uint32_t E) {
  const size_t copy = graph_mode ? c->slot_bytes : desc_bytes() + sizeof(uint32_t) * (E + 1);
  const char* hs = c->h_slots + (size_t)slot * c->slot_bytes;
  (void)hipMemcpyAsync(const_cast<CallDesc*>(c->ws.call), hs, copy, hipMemcpyHostToDevice, s);
  const bool bin_lds = reinterpret_cast<const CallDesc*>(hs)->bin_lds != 0;
  enqueue_path(c, c->cfg, c->ws, c->dc, c->n_cu, s, graph_mode, H, E, bin_lds);
}

int validate_vertices(const pxt_vertices* v, uint32_t E, std::string& why) {
  if (!v->summary || (E > 0 && !v->n_vertices)) return why = "null vertex summary / counts", 1;
  if (E > 0 && (!v->track_vertex || (v->max_per_event > 0 &&
                                     (!v->z || !v->z_err || !v->chi2 || !v->n_tracks))))
    return why = "null vertex buffer", 1;
  return 0;
}

VtxOut make_vtx_out(const pxt_vertices* v) {
  return VtxOut{v->max_per_event, v->z, v->z_err, v->chi2, v->n_tracks, v->n_vertices,
                v->track_vertex, v->summary};
}

// Checks of one call's input and output descriptions against cfg.
int validate_call(const pxt_config& cfg, const pxt_hits* in, const pxt_tracks* out,
                  std::string& why) {
  if (!in || !out) return why = "null argument", 1;
  const uint32_t E = in->n_events;
  if (E > cfg.max_events) return why = "n_events above max_events", 1;
  if (!in->event_offsets) return why = "null event_offsets", 1;
  if (in->event_offsets[0] != 0) return why = "event_offsets[0] != 0", 1;
  for (uint32_t e = 0; e < E; ++e)
    if (in->event_offsets[e + 1] < in->event_offsets[e]) return why = "decreasing event_offsets", 1;
  const uint32_t H = in->event_offsets[E];
  if (H > cfg.max_hits) return why = "more hits than max_hits", 1;
  if (H > 0 && (!in->x || !in->y || !in->z || !in->layer)) return why = "null hit array", 1;
  if (!out->counts || (E > 0 && !out->per_event_tracks))
    return why = "null counts / per_event_tracks", 1;
  if (out->capacity > 0 && (!out->hit_idx || !out->n_hits || !out->event_id || !out->params ||
                            !out->cov || !out->chi2 || !out->flags))
    return why = "null track buffer", 1;
  if (out->vertices && validate_vertices(out->vertices, E, why)) return 1;
  return 0;
}

CallDesc make_desc(const pxt_hits* in, const pxt_tracks* out, const DevCfg& d) {
  CallDesc desc{};
  uint32_t largest = 0;
  for (uint32_t e = 0; e < in->n_events; ++e)
    largest = std::max(largest, in->event_offsets[e + 1] - in->event_offsets[e]);
  desc.bin_lds = d.bin_lds && (in->n_events >= kBinLdsEvents || largest <= kBinLdsHits);
  desc.n_events = in->n_events;
  desc.n_hits = in->event_offsets[in->n_events];
  desc.x = in->x;
  desc.y = in->y;
  desc.z = in->z;
  desc.layer = in->layer;
  desc.out = OutPtrs{out->capacity, out->hit_idx, out->n_hits, out->event_id, out->params,
                     out->cov, out->chi2, out->flags, out->per_event_tracks, out->counts};
  desc.has_vtx = out->vertices ? 1u : 0u;
  if (out->vertices) desc.vtx = make_vtx_out(out->vertices);
  return desc;
}

// ------------------------------------------- calls without allocation --
// pxt_reconstruct_static carves the arenas of one call from this buffer
// instead of a context's allocation.  In host code `scratch` names a
// host-side stand-in: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[PXT_STATIC_SCRATCH_BYTES];

// A call's descriptor and event offsets, passed by value to the kernel
// that writes them where the other kernels read them.
struct StaticCall {
  CallDesc desc;
  uint32_t offsets[PXT_STATIC_MAX_EVENTS + 1];
};

__global__ void k_set_call(CallDesc* dst, uint32_t* evt_off, StaticCall sc, uint32_t n_off,
                           uint32_t* epoch) {
  if (threadIdx.x == 0) {
    *dst = sc.desc;
    *epoch = 0u;
  }
  for (uint32_t i = threadIdx.x; i < n_off; i += blockDim.x) evt_off[i] = sc.offsets[i];
}

struct StaticDevice {
  std::once_flag once;
  hipError_t err = hipSuccess;
  void* ptr = nullptr;  // device address of `scratch` on this device
  int n_cu = 256;
};

constexpr int kStaticDevicesMax = 64;
StaticDevice g_static[kStaticDevicesMax];

}  // namespace

namespace pxt {

// ------------------------------------------------ results to host memory --
// (server lanes; see host_copy.h)

// n 32-bit words, as 16-byte vectors where both sides allow it
__device__ __forceinline__ void copy_words(uint32_t* __restrict__ d, const uint32_t* __restrict__ s,
                                           size_t n, size_t tid, size_t stride) {
  const bool vec = ((reinterpret_cast<uintptr_t>(d) | reinterpret_cast<uintptr_t>(s)) & 15u) == 0;
  size_t head = 0;
  if (vec) {
    const size_t n4 = n / 4;
    for (size_t i = tid; i < n4; i += stride)
      reinterpret_cast<uint4*>(d)[i] = reinterpret_cast<const uint4*>(s)[i];
    head = n4 * 4;
  }
  for (size_t i = head + tid; i < n; i += stride) d[i] = s[i];
}

__global__ __launch_bounds__(256) void k_copy_out(pxt_tracks dev, uint32_t n_events,
                                                  HostTracks host) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const pxt_counts* kc = dev.counts;
  const uint32_t n = kc->status == 0 ? min(kc->n_tracks, dev.capacity) : 0u;
  static_assert(sizeof(pxt_counts) % 4 == 0, "counts as words");
  copy_words(reinterpret_cast<uint32_t*>(host.counts), reinterpret_cast<const uint32_t*>(kc),
             sizeof(pxt_counts) / 4, tid, stride);
  copy_words(host.per_event_tracks, dev.per_event_tracks, n_events, tid, stride);
  copy_words(host.hit_idx, dev.hit_idx, 8ull * n, tid, stride);
  copy_words(reinterpret_cast<uint32_t*>(host.params),
             reinterpret_cast<const uint32_t*>(dev.params), 5ull * n, tid, stride);
  copy_words(reinterpret_cast<uint32_t*>(host.cov), reinterpret_cast<const uint32_t*>(dev.cov),
             15ull * n, tid, stride);
  copy_words(reinterpret_cast<uint32_t*>(host.chi2), reinterpret_cast<const uint32_t*>(dev.chi2),
             2ull * n, tid, stride);
  for (size_t i = tid; i < n; i += stride) {
    host.n_hits[i] = dev.n_hits[i];
    host.flags[i] = dev.flags[i];
  }
}

hipError_t launch_copy_out(const pxt_tracks& dev, uint32_t n_events, const HostTracks& host,
                           hipStream_t s) {
  // enough threads for a full batch's tracks in a few rounds; the kernel
  // reads the actual count
  const uint32_t blocks = std::max<uint32_t>(
      1u, std::min<uint32_t>(1024u, (uint32_t)(((uint64_t)dev.capacity * 2u + 255u) / 256u)));
  hipLaunchKernelGGL(k_copy_out, dim3(blocks), dim3(256), 0, s, dev, n_events, host);
  return hipGetLastError();
}

}  // namespace pxt

extern "C" {

int pxt_abi_version(void) { return PXT_ABI_VERSION; }

const char* pxt_status_str(int s) {
  switch (s) {
    case PXT_OK: return "ok";
    case PXT_ERR_INVALID_ARG: return "invalid argument";
    case PXT_ERR_CAPACITY: return "capacity exceeded";
    case PXT_ERR_HIP: return "HIP runtime error";
    case PXT_ERR_OOM: return "out of device memory";
    case PXT_ERR_BUSY: return "busy";
    case PXT_ERR_PATH: return "link-graph path longer than 8 hits";
    case PXT_ERR_NOT_READY: return "not ready";
    default: return "unknown status";
  }
}

const char* pxt_last_error(const pxt_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int pxt_config_defaults(pxt_config* cfg) {
  if (!cfg) return PXT_ERR_INVALID_ARG;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->max_events = 64;
  cfg->max_hits = 1u << 20;
  cfg->max_doublets = 1u << 24;
  cfg->max_link_words = 1u << 26;
  cfg->max_tuples = 1u << 22;
  cfg->phi_bins = 256;
  cfg->block_size = 256;
  cfg->group_lanes = 8;
  cfg->link_kernel = 0;
  cfg->use_graph = 0;
  cfg->doublet_mode = 2;
  cfg->pt_fp64 = 1e9;  // no refit by pT: the refined FP32 solve holds at any pT
  cfg->min_hits = 3;
  cfg->q_chi2 = 5.0f;
  cfg->q_pt_min = 0.5f;
  cfg->q_d0_max = 0.05f;
  cfg->q_z0_max = 15.0f;
  cfg->vtx_eps = 0.02;
  cfg->vtx_min_pts = 6;
  cfg->vtx_min_hits = 4;
  cfg->vtx_pt_min = 0.5;
  return PXT_OK;
}

int pxt_rechits(const double* modules, uint32_t n_modules, uint32_t max_per_module,
                const pxt_clusters* in, const pxt_rechits_out* out, void* stream) {
  if (!modules || !in || !out) return fail(nullptr, PXT_ERR_INVALID_ARG, "null argument");
  if (n_modules < 1 || n_modules > 65535)
    return fail(nullptr, PXT_ERR_INVALID_ARG, "n_modules out of 1..65535");
  if (max_per_module < 1) return fail(nullptr, PXT_ERR_INVALID_ARG, "max_per_module must be >= 1");
  const uint64_t nmod = (uint64_t)in->n_events * n_modules;
  if (nmod + 1 >= 0xffffffffull)
    return fail(nullptr, PXT_ERR_INVALID_ARG, "n_events * n_modules too large");
  if (!out->module_start || !out->hit_offsets || !out->status)
    return fail(nullptr, PXT_ERR_INVALID_ARG, "null offsets / status buffer");
  if (in->n_clusters > 0 &&
      (!in->event_offsets || !in->module || !in->pixel_offsets || !in->pix_u || !in->pix_v ||
       !in->charge || in->n_events == 0))
    return fail(nullptr, PXT_ERR_INVALID_ARG, "null cluster array or no events");
  if (in->n_clusters > 0 && (!out->x || !out->y || !out->z || !out->layer || !out->module ||
                             !out->cluster))
    return fail(nullptr, PXT_ERR_INVALID_ARG, "null hit buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const RhIn ri{in->n_events, in->n_clusters, in->event_offsets, in->module, in->pixel_offsets,
                in->pix_u, in->pix_v, in->charge};
  const RhOut ro{out->capacity, out->x,       out->y,           out->z,
                 out->layer,    out->module,  out->cluster,     out->module_start,
                 out->hit_offsets, out->status};
  const uint32_t n = (uint32_t)nmod;
  hipLaunchKernelGGL(k_rh_zero, dim3(grid_for((uint64_t)n + 1, 256, 2048)), dim3(256), 0, s, ro,
                     n);
  const uint32_t E = in->n_events;
  if (in->n_clusters > 0) {
    const uint32_t g = grid_for(in->n_clusters, 256, 4096);
    hipLaunchKernelGGL(k_rh_count, dim3(g), dim3(256), 0, s, ri, ro, n_modules);
  }
  if (E > 0)
    hipLaunchKernelGGL(k_rh_event_offsets, dim3(E), dim3(kRhEvThreads), 0, s, ro, E, n_modules,
                       max_per_module);
  hipLaunchKernelGGL(k_rh_events, dim3(1), dim3(kRhScanThreads), 0, s, ro, E, n_modules);
  if (E > 0)
    hipLaunchKernelGGL(k_rh_absolute, dim3(grid_for((uint64_t)E * n_modules, 256, 2048)),
                       dim3(256), 0, s, ro, E, n_modules);
  if (in->n_clusters > 0) {
    const uint32_t g = grid_for(in->n_clusters, 256, 4096);
    hipLaunchKernelGGL(k_rh_hits, dim3(g), dim3(256), 0, s, ri, ro, modules, n_modules,
                       max_per_module);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(nullptr, PXT_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  return PXT_OK;
}

int pxt_find_vertices(const pxt_config* cfg, uint32_t n_events, const pxt_tracks* tracks,
                      const pxt_vertices* out, void* stream) {
  if (!cfg || !tracks || !out) return fail(nullptr, PXT_ERR_INVALID_ARG, "null argument");
  std::string why;
  if (validate_config(cfg, why)) return fail(nullptr, PXT_ERR_INVALID_ARG, why);
  if (n_events > 0 && (!tracks->per_event_tracks || !tracks->n_hits || !tracks->params ||
                       !tracks->cov))
    return fail(nullptr, PXT_ERR_INVALID_ARG, "null track buffer");
  if (validate_vertices(out, n_events, why)) return fail(nullptr, PXT_ERR_INVALID_ARG, why);
  DevCfg dc;
  make_devcfg(*cfg, dc);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const VtxOut vo = make_vtx_out(out);
  const VtxIn vi{n_events, tracks->per_event_tracks, tracks->n_hits, tracks->params, tracks->cov,
                 tracks->counts};
  hipLaunchKernelGGL(k_vtx_begin, dim3(1), dim3(64), 0, s, vo);
  if (n_events > 0)
    hipLaunchKernelGGL(k_vertices, dim3(n_events), dim3(kVtxThreads), 0, s, vi, vo, dc);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(nullptr, PXT_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  return PXT_OK;
}

int pxt_create(const pxt_config* cfg, int hip_device, pxt_ctx** out) {
  if (!cfg || !out) return fail(nullptr, PXT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::string why;
  if (validate_config(cfg, why)) return fail(nullptr, PXT_ERR_INVALID_ARG, why);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return fail(nullptr, PXT_ERR_INVALID_ARG, "no such HIP device");
  pxt_ctx* c = new (std::nothrow) pxt_ctx();
  if (!c) return fail(nullptr, PXT_ERR_OOM, "host allocation failed");
  c->device = hip_device;
  c->cfg = *cfg;
  make_devcfg(*cfg, c->dc);
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete c;
    return fail(nullptr, PXT_ERR_HIP, "hipSetDevice failed");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  Carver size_pass;
  carve(size_pass, *cfg, c->ws);
  c->arena_bytes = size_pass.off + 256;
  if (hipMalloc(&c->arena, c->arena_bytes) != hipSuccess) {
    delete c;
    return fail(nullptr, PXT_ERR_OOM, "hipMalloc of " + std::to_string(c->arena_bytes) + " bytes failed");
  }
  Carver real;
  real.base = static_cast<char*>(c->arena);
  carve(real, *cfg, c->ws);
  // the scan status words and the call counter start from zero once; no
  // other arena is ever initialised
  if (hipMemset(c->ws.scan_status, 0, sizeof(uint64_t) * scan_tiles(*cfg)) != hipSuccess ||
      hipMemset(c->ws.epoch, 0, sizeof(uint32_t)) != hipSuccess) {
    pxt_destroy(c);
    return fail(nullptr, PXT_ERR_HIP, "arena initialisation failed");
  }
  c->slot_bytes = slot_bytes_for(*cfg);
  bool ok = hipHostMalloc((void**)&c->h_slots, c->slot_bytes * pxt_ctx::kSlots,
                          hipHostMallocDefault) == hipSuccess;
  for (int i = 0; ok && i < pxt_ctx::kSlots; ++i)
    ok = hipEventCreateWithFlags(&c->slot_free[i], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    pxt_destroy(c);
    return fail(nullptr, PXT_ERR_HIP, "pinned staging / stream creation failed");
  }
  *out = c;
  return PXT_OK;
}

void pxt_destroy(pxt_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (int i = 0; i < pxt_ctx::kSlots; ++i) {
    for (int v = 0; v < 2; ++v) {
      if (c->gexec[i][v]) (void)hipGraphExecDestroy(c->gexec[i][v]);
      if (c->graph[i][v]) (void)hipGraphDestroy(c->graph[i][v]);
    }
    if (c->slot_free[i]) (void)hipEventDestroy(c->slot_free[i]);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int i = 0; i <= PXT_N_STAGES; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->h_slots) (void)hipHostFree(c->h_slots);
  if (c->arena) (void)hipFree(c->arena);
  delete c;
}

int pxt_reconstruct(pxt_ctx* c, const pxt_hits* in, pxt_tracks* out, void* stream) {
  if (!c) return PXT_ERR_INVALID_ARG;
  const pxt_config& cfg = c->cfg;
  std::string why;
  if (validate_call(cfg, in, out, why)) return fail(c, PXT_ERR_INVALID_ARG, why);
  const uint32_t E = in->n_events;
  const uint32_t H = in->event_offsets[E];
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_OR_FAIL(c, hipSetDevice(c->device));

  // descriptor + offsets -> pinned slot (after its previous user read it)
  const int slot = c->next_slot;
  c->next_slot = (slot + 1) % pxt_ctx::kSlots;
  if (c->slot_pending[slot]) HIP_OR_FAIL(c, hipEventSynchronize(c->slot_free[slot]));
  char* hs = c->h_slots + (size_t)slot * c->slot_bytes;
  const CallDesc desc = make_desc(in, out, c->dc);
  std::memcpy(hs, &desc, sizeof(desc));
  std::memcpy(hs + desc_bytes(), in->event_offsets, sizeof(uint32_t) * (E + 1));

  if (c->calls > 0 && c->calls % pxt_ctx::kEpochReset == 0) {
    const uint64_t n = scan_tiles(cfg);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s,
                       c->ws.scan_status, n, 0ull);
  }
  c->calls++;
  if (cfg.use_graph) {
    const int v = desc.bin_lds ? 1 : 0;
    if (!c->gexec[slot][v]) {
      HIP_OR_FAIL(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      enqueue(c, c->cap_stream, slot, true, 0, 0);
      hipGraph_t g = nullptr;
      const hipError_t e1 = hipStreamEndCapture(c->cap_stream, &g);
      if (e1 != hipSuccess || !g)
        return fail(c, PXT_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e1));
      c->graph[slot][v] = g;
      HIP_OR_FAIL(c, hipGraphInstantiate(&c->gexec[slot][v], g, nullptr, nullptr, 0));
    }
    HIP_OR_FAIL(c, hipGraphLaunch(c->gexec[slot][v], s));
    c->timed_valid = false;
  } else {
    enqueue(c, s, slot, false, H, E);
  }
  HIP_OR_FAIL(c, hipGetLastError());
  HIP_OR_FAIL(c, hipEventRecord(c->slot_free[slot], s));
  c->slot_pending[slot] = true;
  c->have_last = true;
  c->last_events = E;
  c->last_offsets.assign(in->event_offsets, in->event_offsets + E + 1);
  return PXT_OK;
}

int pxt_debug_dump(pxt_ctx* c, int what, uint32_t* dst, uint64_t cap, uint64_t* count,
                   void* stream) {
  if (!c) return PXT_ERR_INVALID_ARG;
  if (!count || (cap > 0 && !dst)) return fail(c, PXT_ERR_INVALID_ARG, "null argument");
  if (!c->have_last) return fail(c, PXT_ERR_INVALID_ARG, "no previous reconstruct call");
  if (what < PXT_DUMP_DOUBLETS || what > PXT_DUMP_RAW)
    return fail(c, PXT_ERR_INVALID_ARG, "unknown dump");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipStreamSynchronize(s));
  const Ws& w = c->ws;
  uint32_t ctr[C_NCTR];
  HIP_OR_FAIL(c, hipMemcpy(ctr, w.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
  if (ctr[C_STATUS]) return fail(c, PXT_ERR_INVALID_ARG, "last call ended with a device status");
  const uint32_t nb = ctr[C_NBINNED], nd = ctr[C_ND], nt = ctr[C_NTUP];
  std::vector<uint32_t> bidx(nb), bevt(nb);
  if (nb) {
    HIP_OR_FAIL(c, hipMemcpy(bidx.data(), w.bidx, 4ull * nb, hipMemcpyDeviceToHost));
    HIP_OR_FAIL(c, hipMemcpy(bevt.data(), w.bevt, 4ull * nb, hipMemcpyDeviceToHost));
  }
  std::vector<uint32_t> rows;
  if (what == PXT_DUMP_DOUBLETS || what == PXT_DUMP_LINKS) {
    std::vector<uint32_t> cin(nd), cout(nd);
    if (nd) {
      std::vector<uint2> cio(nd);
      HIP_OR_FAIL(c, hipMemcpy(cio.data(), w.cio, 8ull * nd, hipMemcpyDeviceToHost));
      for (uint32_t k = 0; k < nd; ++k) {
        cin[k] = cio[k].x;
        cout[k] = cio[k].y;
      }
    }
    if (what == PXT_DUMP_DOUBLETS) {
      rows.reserve(3ull * nd);
      for (uint32_t k = 0; k < nd; ++k) {
        rows.push_back(bevt[cin[k]]);
        rows.push_back(bidx[cin[k]]);
        rows.push_back(bidx[cout[k]]);
      }
    } else {
      // mask words of the doublets with links (the only ones the link
      // kernels are bound to leave defined); their count follows from the
      // outer hit's range of doublets
      std::vector<uint32_t> cell_off(nb + 1), mw(nd);
      std::vector<uint8_t> has_out(nd);
      HIP_OR_FAIL(c, hipMemcpy(cell_off.data(), w.cell_off, 4ull * (nb + 1), hipMemcpyDeviceToHost));
      if (nd) HIP_OR_FAIL(c, hipMemcpy(has_out.data(), w.has_out, nd, hipMemcpyDeviceToHost));
      for (uint32_t k = 0; k < nd; ++k)
        mw[k] = has_out[k] ? (cell_off[cout[k] + 1] - cell_off[cout[k]] + 63u) >> 6 : 0u;
      const uint32_t nwords = ctr[C_NWORDS];
      std::vector<uint64_t> masks(nwords);
      if (nwords)
        HIP_OR_FAIL(c, hipMemcpy(masks.data(), w.masks, 8ull * nwords, hipMemcpyDeviceToHost));
      for (uint32_t k = 0; k < nd; ++k) {
        const uint32_t b = cout[k], k0 = cell_off[b];
        for (uint32_t wd = 0; wd < mw[k]; ++wd) {
          uint64_t m = masks[(size_t)wd * nd + k];
          while (m) {
            const int bit = __builtin_ctzll(m);
            m &= m - 1;
            const uint32_t d2 = k0 + wd * 64u + (uint32_t)bit;
            rows.push_back(bevt[cin[k]]);
            rows.push_back(bidx[cin[k]]);
            rows.push_back(bidx[b]);
            rows.push_back(bidx[cout[d2]]);
          }
        }
      }
    }
  } else {
    const uint32_t T = c->cfg.max_tuples;
    const uint32_t n = std::min(nt, T);
    std::vector<uint32_t> th(8ull * n);
    if (n) HIP_OR_FAIL(c, hipMemcpy(th.data(), w.thit, 4ull * 8 * n, hipMemcpyDeviceToHost));
    rows.reserve(9ull * n);
    for (uint32_t t = 0; t < n; ++t) {
      rows.push_back(bevt[th[(size_t)t * 8]]);
      for (int j = 0; j < 8; ++j) {
        const uint32_t h = th[(size_t)t * 8 + j];
        rows.push_back(h == kPad ? kPad : bidx[h]);
      }
    }
  }
  const uint64_t width = what == PXT_DUMP_DOUBLETS ? 3 : (what == PXT_DUMP_LINKS ? 4 : 9);
  const uint64_t nrows = rows.size() / width;
  *count = nrows;
  const uint64_t ncopy = std::min(nrows, cap);
  if (ncopy) std::memcpy(dst, rows.data(), sizeof(uint32_t) * width * ncopy);
  return PXT_OK;
}

int pxt_set_timing(pxt_ctx* c, int enable) {
  if (!c) return PXT_ERR_INVALID_ARG;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  if (enable && !c->ev[0])
    for (int i = 0; i <= PXT_N_STAGES; ++i) HIP_OR_FAIL(c, hipEventCreate(&c->ev[i]));
  c->timing = enable != 0;
  c->timed_valid = false;
  return PXT_OK;
}

int pxt_stage_times(pxt_ctx* c, float* ms, int cap, int* n_stages) {
  if (!c) return PXT_ERR_INVALID_ARG;
  if (!n_stages || (cap > 0 && !ms)) return fail(c, PXT_ERR_INVALID_ARG, "null argument");
  if (!c->timed_valid) return fail(c, PXT_ERR_INVALID_ARG, "no timed call");
  *n_stages = PXT_N_STAGES;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipEventSynchronize(c->ev[PXT_N_STAGES]));
  for (int i = 0; i < PXT_N_STAGES && i < cap; ++i) {
    ms[i] = 0.0f;
    if (!c->stage_run[i]) continue;
    int j = i + 1;
    while (j < PXT_N_STAGES && !c->stage_run[j]) ++j;
    float t = 0.0f;
    HIP_OR_FAIL(c, hipEventElapsedTime(&t, c->ev[i], c->ev[j]));
    ms[i] = t;
  }
  return PXT_OK;
}

const char* pxt_stage_name(int i) {
  return (i >= 0 && i < PXT_N_STAGES) ? kStageNames[i] : nullptr;
}

int pxt_reconstruct_static(const pxt_config* cfg, int hip_device, const pxt_hits* in,
                           pxt_tracks* out, void* stream) {
  if (!cfg) return fail(nullptr, PXT_ERR_INVALID_ARG, "null config");
  std::string why;
  if (validate_config(cfg, why)) return fail(nullptr, PXT_ERR_INVALID_ARG, why);
  if (validate_call(*cfg, in, out, why)) return fail(nullptr, PXT_ERR_INVALID_ARG, why);
  const uint32_t E = in->n_events;
  if (E > PXT_STATIC_MAX_EVENTS)
    return fail(nullptr, PXT_ERR_CAPACITY,
                "n_events above PXT_STATIC_MAX_EVENTS (" +
                    std::to_string(PXT_STATIC_MAX_EVENTS) + ")");
  Carver size_pass;
  Ws w{};
  carve(size_pass, *cfg, w);
  if (size_pass.off > (size_t)PXT_STATIC_SCRATCH_BYTES)
    return fail(nullptr, PXT_ERR_CAPACITY,
                "the configured capacities need " + std::to_string(size_pass.off) +
                    " bytes of arenas, above PXT_STATIC_SCRATCH_BYTES (" +
                    std::to_string((size_t)PXT_STATIC_SCRATCH_BYTES) + ")");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev ||
      hip_device >= kStaticDevicesMax)
    return fail(nullptr, PXT_ERR_INVALID_ARG, "no such HIP device");
  if (hipSetDevice(hip_device) != hipSuccess)
    return fail(nullptr, PXT_ERR_HIP, "hipSetDevice failed");
  StaticDevice& sd = g_static[hip_device];
  std::call_once(sd.once, [&sd, hip_device]() {
    sd.err = hipGetSymbolAddress(&sd.ptr, HIP_SYMBOL(scratch));
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, hip_device) ==
            hipSuccess && n > 0)
      sd.n_cu = n;
  });
  if (sd.err != hipSuccess || !sd.ptr)
    return fail(nullptr, PXT_ERR_HIP,
                std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(sd.err));
  Carver real;
  real.base = static_cast<char*>(sd.ptr);
  carve(real, *cfg, w);
  DevCfg dc;
  make_devcfg(*cfg, dc);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the buffer keeps the previous call's contents: the scan status words
  // and the call counter start again from zero, the rest is never read
  // before this call writes it
  const uint64_t ntiles = scan_tiles(*cfg);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(ntiles, 256, 1024)), dim3(256), 0, s,
                     w.scan_status, ntiles, 0ull);
  StaticCall sc{};
  sc.desc = make_desc(in, out, dc);
  std::memcpy(sc.offsets, in->event_offsets, sizeof(uint32_t) * (E + 1));
  hipLaunchKernelGGL(k_set_call, dim3(1), dim3(64), 0, s, const_cast<CallDesc*>(w.call),
                     w.evt_off, sc, E + 1, w.epoch);
  enqueue_path(nullptr, *cfg, w, dc, sd.n_cu, s, false, in->event_offsets[E], E,
               sc.desc.bin_lds != 0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(nullptr, PXT_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  return PXT_OK;
}

}  // extern "C"
