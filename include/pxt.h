/*
 * pxt -- pixel-track reconstruction core on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpxt.so.  The library implements the Tracks module of the
 * heterogeneous pixel reconstruction described in "Porting CMS Heterogeneous
 * Pixel Reconstruction to Kokkos" (arXiv:2104.06573), Sec. 2: from the 3-D
 * pixel hits of an event it forms hit n-tuplets and fits each one to obtain
 * track parameters.  The steps run on the GPU in hand-written HIP kernels:
 *
 *   per-layer phi binning of the hits (counting sort),
 *   doublets: hit pairs on allowed layer pairs passing geometric cuts,
 *   cellular-automaton links between doublets that share a hit,
 *   n-tuplets: every root-to-leaf path of the link graph with 3..8 hits,
 *   duplicate cleaning: each doublet keeps only its best n-tuplet,
 *   broken-line helix fit of every surviving n-tuplet.
 *
 * The paper states only what the module produces (n-tuplets from hits, and
 * their fitted track parameters); the cut definitions, cleaning rule and fit
 * formulation implemented here are the readings documented with the
 * library.  The paper's performance lessons are built in: all device memory
 * is allocated once per context (its memory-pool result, Sec. 5), arenas are
 * never default-initialised (its View-initialisation result, Sec. 4.2), and
 * many events of uneven size go through one launch sequence (its
 * concurrent-events result, Sec. 5).
 *
 * Conventions
 *  - Every function returns a pxt_status (0 = PXT_OK).  No exception or
 *    abort crosses the ABI.  pxt_last_error() gives a message.
 *  - Calls that take a stream are asynchronous on that HIP stream
 *    (hipStream_t passed as void*; NULL = the null stream).  Their return
 *    code covers argument validation and launch only.  Conditions found on
 *    the device (capacity overflow, a path longer than 8 hits) are written
 *    to pxt_counts.status together with the required sizes; read it after
 *    synchronising the stream.  On such a status every output of that call
 *    is invalid (never silently truncated): grow the capacities and retry.
 *  - Units: cm, GeV.  The field is along +z.
 *  - A context is used by one host thread at a time.  Calls on one context
 *    must be ordered on one stream.
 */
#ifndef PXT_H
#define PXT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PXT_ABI_VERSION 3

#define PXT_MAX_LAYERS 16
#define PXT_MAX_PAIRS 32
#define PXT_MAX_TUPLE_HITS 8
#define PXT_PAD 0xffffffffu

typedef enum pxt_status {
  PXT_OK = 0,
  PXT_ERR_INVALID_ARG = 1, /* null pointer, size or config out of range   */
  PXT_ERR_CAPACITY = 2,    /* a capacity was exceeded; see required[]     */
  PXT_ERR_HIP = 3,         /* a HIP runtime call failed                   */
  PXT_ERR_OOM = 4,         /* device allocation failed at create          */
  PXT_ERR_BUSY = 5,        /* server queue full / no free slot            */
  PXT_ERR_PATH = 6,        /* a link-graph path longer than 8 hits        */
  PXT_ERR_NOT_READY = 7    /* pxt_poll: result not complete yet           */
} pxt_status;

enum { PXT_LAYER_BARREL = 0, PXT_LAYER_DISK = 1 };

/* Geometry, cuts, fit constants, capacities and tuning.
 * Physics fields define the result; tuning fields never change it. */
typedef struct pxt_config {
  /* --- physics -------------------------------------------------------- */
  double c_kappa;                    /* curvature [1/cm] = c_kappa / pT [GeV] */
  int32_t n_layers;                  /* layer ids are 0..n_layers-1          */
  int32_t layer_kind[PXT_MAX_LAYERS];/* PXT_LAYER_BARREL / PXT_LAYER_DISK    */
  int32_t n_pairs;                   /* allowed (inner, outer) layer pairs   */
  int32_t pair_inner[PXT_MAX_PAIRS];
  int32_t pair_outer[PXT_MAX_PAIRS];
  double kmax;      /* doublet/link curvature cut [1/cm]                      */
  double z0max;     /* doublet longitudinal impact cut [cm]                   */
  double arz;       /* link r-z alignment cut (sine of the turning angle)     */
  double d0max;     /* link transverse impact cut [cm]                        */
  double sigma_u;   /* r-phi resolution [cm]                                  */
  double sigma_z;   /* barrel z resolution [cm]                               */
  double sigma_r;   /* disk r resolution [cm]                                 */
  double x_over_x0; /* material per layer at normal incidence [X0]           */
  double pt_max;    /* momentum cap of the scattering estimate [GeV]          */
  /* --- capacities (summed over one call's batch) ---------------------- */
  uint32_t max_events;
  uint32_t max_hits;
  uint32_t max_doublets;
  uint32_t max_link_words;  /* 64-bit link-mask words: doublets times
                               ceil(largest hit out-degree / 64), usually
                               1-2 per doublet at PU~50, up to ~8 at PU~200 */
  uint32_t max_tuples;      /* raw n-tuplets before cleaning               */
  /* --- tuning ------------------------------------------------------------ */
  int32_t phi_bins;         /* phi bins per layer, 16..4096.  Up to 12288
                               bins over all layers, a call of 8 events or
                               more (or of events of at most 8192 hits)
                               is binned by one block per event in LDS;
                               otherwise by device-wide kernels (same
                               result either way)                          */
  int32_t block_size;       /* threads per block of the per-item kernels   */
  int32_t group_lanes;      /* lanes per item in doublet/link kernels:
                               4, 8, 16, 32 or 64                          */
  int32_t link_kernel;      /* link step: 0 one thread per doublet,
                               1 one lane group per doublet, 2 one
                               wavefront per 64 doublets with their
                               candidates spread over its lanes           */
  int32_t use_graph;        /* 1: replay the launch sequence as a HIP
                               graph captured at the first call (stage
                               timing is then unavailable)                */
  int32_t doublet_mode;     /* doublet step: 0 count, scan and fill, each
                               pass evaluating the cuts; 1 one pass, the
                               accepted pairs of each tile of
                               block_size/group_lanes inner hits staged in
                               LDS, tiles chained by look-back (least
                               latency on small batches); 2 count and stage
                               the pairs in device memory, scan, scatter
                               (most throughput on large batches).  All
                               modes give the same results.               */
  double pt_fp64;           /* fit tuples with pT_ref above this in FP64
                               (default 1e9 GeV: none; the FP32 transverse
                               solve is refined once against its FP64
                               residual, which holds at any pT; ill-
                               conditioned or non-finite fits are refitted
                               in FP64 regardless)                        */
  /* --- output selection and track quality (pxt_tracks.flags) ---------- */
  int32_t min_hits;         /* tracks with fewer hits are not output:
                               3 keeps triplets and longer, 4 gives
                               quadruplets and longer only (3..8).  The
                               cleaning is unchanged: a shorter n-tuplet
                               never outranks a longer one.              */
  float q_chi2;             /* PXT_FLAG_LOOSE: chi2 / ndf at most this in
                               both planes (ndf n-3 transverse, at least
                               1; n-2 longitudinal)                       */
  float q_pt_min;           /* PXT_FLAG_STRICT: pT at least [GeV]          */
  float q_d0_max;           /* PXT_FLAG_STRICT: |d0| at most [cm]          */
  float q_z0_max;           /* PXT_FLAG_STRICT: |z0| at most [cm]          */
  /* --- vertices (pxt_tracks.vertices, pxt_find_vertices) -------------- */
  double vtx_eps;           /* z0 neighbour distance [cm]                  */
  int32_t vtx_min_pts;      /* neighbours (itself included) of a core      */
  int32_t vtx_min_hits;     /* tracks used: at least this many hits ...    */
  double vtx_pt_min;        /* ... and pT at least this [GeV]              */
} pxt_config;

/* pxt_tracks.flags bits */
#define PXT_FLAG_FP64 1u   /* fitted on the FP64 path                        */
#define PXT_FLAG_LOOSE 2u  /* parameters finite, chi2/ndf within q_chi2      */
#define PXT_FLAG_STRICT 4u /* LOOSE, pT >= q_pt_min, |d0| <= q_d0_max,
                              |z0| <= q_z0_max                               */

/* One call's input: a ragged batch of events in structure-of-arrays form.
 * x, y, z, layer are DEVICE pointers with event_offsets[n_events] entries;
 * event e owns [event_offsets[e], event_offsets[e+1]).  event_offsets is a
 * HOST pointer (non-decreasing, starting at 0).  Hits whose layer id is
 * outside 0..n_layers-1 take part in nothing. */
typedef struct pxt_hits {
  uint32_t n_events;
  const uint32_t* event_offsets; /* host, [n_events + 1]            */
  const float* x;                /* device, [n_hits]                */
  const float* y;
  const float* z;
  const int16_t* layer;          /* device, [n_hits]                */
  const int16_t* module;         /* device or NULL; not used        */
} pxt_hits;

/* Device-written summary of one call.  required[] holds the sizes a retry
 * needs when status == PXT_ERR_CAPACITY:
 *   required[0] doublets, [1] link-mask words, [2] raw n-tuplets,
 *   [3] output tracks. */
typedef struct pxt_counts {
  int32_t status;
  uint32_t n_tracks;
  uint32_t n_doublets;
  uint32_t n_links;
  uint32_t n_raw_tuples;
  uint32_t n_fp64;          /* tracks fitted on the FP64 path              */
  uint32_t n_hits_binned;   /* hits with a valid layer id                  */
  uint32_t n_link_words;    /* 64-bit link-mask words used                 */
  uint64_t required[4];
} pxt_counts;

/* Caller-owned DEVICE output buffers, each with room for `capacity` tracks.
 * Tracks come out in unspecified order.  hit_idx holds event-local
 * input-order hit indices in path order (increasing radius), padded with
 * PXT_PAD.  params = (phi0, d0, q/pT, cot theta, z0) at the point of closest
 * approach to the transverse origin; d0 > 0 when the origin is left of the
 * direction of motion.  cov = packed lower triangle of the 5x5 covariance
 * (row-major: (0,0),(1,0),(1,1),(2,0),...).  chi2 = (transverse, long.).
 * flags: PXT_FLAG_* bits.  per_event_tracks[e] receives the number of
 * tracks of event e (zero for every event when the call fails).  counts
 * receives the summary. */
/* Vertices of a call's tracks (the Vertices module that follows the Tracks
 * module in the paper's chain, Sec. 2 and Fig. 1; the paper gives no
 * algorithm).  Reading: one-dimensional density-based clustering (DBSCAN)
 * of z0 over the tracks with at least vtx_min_hits hits and pT at least
 * vtx_pt_min (|q/pT| <= 1/vtx_pt_min compared in single precision), finite
 * z0 and a positive variance of z0.  Two tracks are neighbours when their
 * z0 differ by at most vtx_eps (difference of the single-precision values
 * in double precision); a core has at least vtx_min_pts neighbours, itself
 * included; connected cores form a cluster; a non-core track with a core
 * neighbour joins its nearest core's cluster (ties: the lower core), the
 * rest belong to no vertex.  Per cluster, over its tracks in increasing
 * (z0, index) order, in double precision: w = 1/var(z0), z = sum(w z0) /
 * sum(w), z_err = sqrt(1/sum(w)), chi2 = sum(w (z0 - z)^2), rounded to
 * single precision on output.
 *
 * Caller-owned DEVICE buffers.  Event e's vertices are at
 * [e * max_per_event, e * max_per_event + n_vertices[e]), in increasing z.
 * track_vertex[k] = the vertex (index within its event) of output track k,
 * or -1.  An event with more than PXT_VTX_MAX_TRACKS selected tracks or
 * more than max_per_event vertices gets none: summary->status =
 * PXT_ERR_CAPACITY with the sizes it needs in max_selected and
 * required_per_event.  If the tracks themselves failed (pxt_counts.status
 * not PXT_OK), summary->status carries that status and nothing is written. */
#define PXT_VTX_MAX_TRACKS 4096
typedef struct pxt_vertex_summary {
  int32_t status;
  uint32_t n_vertices;          /* over all events                     */
  uint32_t required_per_event;  /* largest vertex count of an event    */
  uint32_t max_selected;        /* largest selected-track count        */
} pxt_vertex_summary;

typedef struct pxt_vertices {
  uint32_t max_per_event;
  float* z;                     /* [n_events][max_per_event] */
  float* z_err;
  float* chi2;
  uint32_t* n_tracks;           /* tracks in each vertex      */
  uint32_t* n_vertices;         /* [n_events]                 */
  int32_t* track_vertex;        /* [track capacity]           */
  pxt_vertex_summary* summary;  /* [1]                        */
} pxt_vertices;

typedef struct pxt_tracks {
  uint32_t capacity;
  uint32_t* hit_idx;          /* [capacity][8]  */
  uint8_t* n_hits;            /* [capacity]     */
  uint32_t* event_id;         /* [capacity]     */
  float* params;              /* [capacity][5]  */
  float* cov;                 /* [capacity][15] */
  float* chi2;                /* [capacity][2]  */
  uint8_t* flags;             /* [capacity]     */
  uint32_t* per_event_tracks; /* [n_events]     */
  pxt_counts* counts;         /* [1]            */
  const pxt_vertices* vertices; /* HOST struct of device buffers, or NULL:
                                   when set, the call also finds the
                                   vertices of its tracks               */
} pxt_tracks;

typedef struct pxt_ctx pxt_ctx;

/* Version of this ABI (PXT_ABI_VERSION). */
int pxt_abi_version(void);

/* Static message for a status code. */
const char* pxt_status_str(int status);

/* Message of the last failing call on ctx (or of the last failing create
 * on this thread when ctx is NULL).  Valid until the next call. */
const char* pxt_last_error(const pxt_ctx* ctx);

/* Fill *cfg with the defaults of the tuning and capacity fields (physics
 * fields zeroed).  Returns PXT_ERR_INVALID_ARG if cfg is NULL. */
int pxt_config_defaults(pxt_config* cfg);

/* Create a context on HIP device `hip_device`: validates cfg and allocates
 * every device arena once from its capacities (no allocation happens per
 * call afterwards).  *out receives the context.  Errors:
 * PXT_ERR_INVALID_ARG (bad config), PXT_ERR_OOM, PXT_ERR_HIP. */
int pxt_create(const pxt_config* cfg, int hip_device, pxt_ctx** out);

/* Free the context and its arenas (synchronises its device first). */
void pxt_destroy(pxt_ctx* ctx);

/* Run the whole path on a batch of events (n_events == 1 is the plain
 * one-event path).  Asynchronous on `hip_stream`; the host reads only
 * in->event_offsets, which may be reused as soon as the call returns.
 * Errors returned directly: PXT_ERR_INVALID_ARG (null pointers, n_events
 * above max_events, more hits than max_hits, decreasing offsets),
 * PXT_ERR_HIP.  Device-side conditions go to out->counts->status. */
int pxt_reconstruct(pxt_ctx* ctx, const pxt_hits* in, pxt_tracks* out,
                    void* hip_stream);

/* Debug dumps of the last pxt_reconstruct on ctx, in a form the tests can
 * put in canonical order.  Synchronises `hip_stream`.  Rows of uint32:
 *   PXT_DUMP_DOUBLETS:  (event, inner hit, outer hit)        3 words
 *   PXT_DUMP_LINKS:     (event, hit a, hit b, hit c)         4 words
 *   PXT_DUMP_RAW:       (event, 8 padded hits)               9 words
 * with event-local input-order hit indices.  dst is HOST memory of `cap`
 * rows; *count receives the number of rows that exist (rows beyond cap are
 * not written; call again with a larger buffer).
 * Errors: PXT_ERR_INVALID_ARG, PXT_ERR_HIP. */
enum { PXT_DUMP_DOUBLETS = 0, PXT_DUMP_LINKS = 1, PXT_DUMP_RAW = 2 };
int pxt_debug_dump(pxt_ctx* ctx, int what, uint32_t* dst, uint64_t cap,
                   uint64_t* count, void* hip_stream);

/* Per-stage timing.  With timing enabled, pxt_reconstruct records a HIP
 * event on the call's stream before each stage and after the last one, so
 * a stage's duration is that of its kernels on the device.  Meant for
 * profiling runs; adds one event record per stage.  Returns
 * PXT_ERR_INVALID_ARG for a NULL ctx. */
int pxt_set_timing(pxt_ctx* ctx, int enable);

/* Durations in milliseconds of the stages of the last call made with timing
 * enabled (synchronises on its last event).  ms is HOST memory of cap
 * floats; *n_stages receives the number of stages (PXT_N_STAGES).  Stages
 * skipped by that call (an empty batch) read 0.  Errors:
 * PXT_ERR_INVALID_ARG (no timed call yet, null pointers), PXT_ERR_HIP. */
#define PXT_N_STAGES 20
int pxt_stage_times(pxt_ctx* ctx, float* ms, int cap, int* n_stages);

/* Static name of stage i (0 <= i < PXT_N_STAGES), or NULL. */
const char* pxt_stage_name(int stage);

/* Vertices of tracks already in device memory (for example the outputs of
 * an earlier pxt_reconstruct), by the reading given with pxt_vertices; the
 * same kernels run at the end of pxt_reconstruct when pxt_tracks.vertices
 * is set.  Uses cfg's vtx_* fields only (validated as by pxt_create).
 * tracks: DEVICE buffers of the tracks of n_events events, grouped by event
 * in event order with per_event_tracks[e] tracks each (n_hits, params and
 * cov are read; tracks->counts may be NULL, else its status must be PXT_OK
 * or the call only reports it).  Asynchronous on hip_stream; allocates
 * nothing.  Errors: PXT_ERR_INVALID_ARG, PXT_ERR_HIP (message from
 * pxt_last_error(NULL)). */
int pxt_find_vertices(const pxt_config* cfg, uint32_t n_events, const pxt_tracks* tracks,
                      const pxt_vertices* out, void* hip_stream);

/* ------------------------------------------------------------------ */
/* RecHits: pixel clusters to 3-D hits (the paper's RecHits module,      */
/* Sec. 2: it estimates the 3-D position of each cluster, forming hits;  */
/* its Fig. 3 limits each module's cluster count and turns the counts    */
/* into the modules' first-hit offsets).  The output is the input of     */
/* pxt_reconstruct.                                                      */
/*                                                                      */
/* Reading, per event: c[m] = the clusters of module m, limited to       */
/* max_per_module; module_start = running sum of c (one array over all  */
/* events, so the hits of all events are contiguous, in event and module */
/* order); a cluster's rank among the earlier clusters of its module     */
/* decides whether it makes a hit (rank < max_per_module) and where      */
/* (module_start + rank); its local position is the charge-weighted      */
/* centroid of its pixel centres, u = u0 + pitch_u * (sum q (iu + 1/2) / */
/* sum q), v likewise (double precision, pixels in order); the 3-D hit:  */
/* barrel module, the tangent-plane point r n + u t projected radially   */
/* onto the cylinder of radius r, (r c - u s, r s + u c) r / sqrt(r r +  */
/* u u), z = z_c + v; disk module, ((r + u) c - v s, (r + u) s + v c,    */
/* z_disk); rounded to single precision.  A cluster without charge makes */
/* a hit with layer -1 at the origin (it takes part in nothing).         */
/*                                                                      */
/* Module table: DEVICE float64 [n_modules][10] rows (layer id, kind 0   */
/* barrel / 1 disk, cos phi_c, sin phi_c, r (barrel radius / disk ring   */
/* centre), z (module centre / disk plane), u0, v0 (local position of    */
/* pixel (0, 0)'s corner), pitch_u, pitch_v), cm.                        */

typedef struct pxt_clusters {
  uint32_t n_events;
  uint32_t n_clusters;
  const uint32_t* event_offsets; /* DEVICE [n_events + 1] clusters of each event */
  const uint16_t* module;        /* DEVICE [n_clusters]: within an event,
                                    non-decreasing (grouped by module)   */
  const uint32_t* pixel_offsets; /* DEVICE [n_clusters + 1] pixel ranges */
  const uint16_t* pix_u;         /* DEVICE pixel column, row, charge     */
  const uint16_t* pix_v;
  const uint16_t* charge;
} pxt_clusters;

typedef struct pxt_rechits_out {
  uint32_t capacity;             /* hits                                  */
  float* x;                      /* DEVICE [capacity]                     */
  float* y;
  float* z;
  int16_t* layer;
  uint16_t* module;
  uint32_t* cluster;             /* the cluster each hit comes from       */
  uint32_t* module_start;        /* DEVICE [n_events * n_modules + 1]     */
  uint32_t* hit_offsets;         /* DEVICE [n_events + 1]                 */
  int32_t* status;               /* DEVICE [1]: PXT_OK, PXT_ERR_CAPACITY
                                    (more hits than capacity: only the
                                    offsets are valid), PXT_ERR_INVALID_ARG
                                    (a module id out of range or clusters
                                    not grouped by module)               */
} pxt_rechits_out;

/* Asynchronous on hip_stream; allocates nothing.  Errors returned
 * directly: PXT_ERR_INVALID_ARG (null pointers, n_modules out of 1..65535,
 * max_per_module 0), PXT_ERR_HIP (message from pxt_last_error(NULL)). */
int pxt_rechits(const double* modules, uint32_t n_modules, uint32_t max_per_module,
                const pxt_clusters* in, const pxt_rechits_out* out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the same
 * computation as pxt_reconstruct on a context created from the same cfg,
 * with no context and no allocation.  Every arena of the call is carved from
 * one library-owned device buffer of PXT_STATIC_SCRATCH_BYTES per device,
 * which each device that ran such a call holds until the process ends; the
 * first call on a device only looks up the buffer's address.  cfg is
 * validated as by pxt_create; its capacities must fit the buffer and
 * in->n_events must not exceed PXT_STATIC_MAX_EVENTS, else
 * PXT_ERR_CAPACITY is returned before anything is launched (the message,
 * from pxt_last_error(NULL), gives the bytes the capacities need).  Always
 * direct launches (cfg->use_graph is ignored), no stage timing, no debug
 * dumps.  Asynchronous on `hip_stream` like pxt_reconstruct, with the same
 * input/output contract and device status in out->counts.  All calls on one
 * device share the buffer and keep nothing from one call to the next: calls
 * that overlap on one device (different streams, or host threads without
 * ordering) race and give wrong results; order them on one stream.  Other
 * errors: PXT_ERR_INVALID_ARG, PXT_ERR_HIP (message from
 * pxt_last_error(NULL), thread-local). */
#define PXT_STATIC_SCRATCH_BYTES (64u << 20)
#define PXT_STATIC_MAX_EVENTS 64
int pxt_reconstruct_static(const pxt_config* cfg, int hip_device, const pxt_hits* in,
                           pxt_tracks* out, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching over several concurrent lanes.          */
/*                                                                      */
/* A server owns n_lanes contexts, each with its own HIP stream, device   */
/* input/output buffers and pinned staging.  pxt_submit (any thread)     */
/* copies one event's hits from HOST memory into the server and returns a */
/* ticket at once; a dispatcher thread forms a batch from the pending     */
/* events whenever a lane is free, admitting events while the batch fits */
/* the lane's arena capacities (events, hits, and doublets estimated from */
/* hits), and runs copy-in, reconstruction and copy-out on that lane's    */
/* stream while the other lanes' batches are on the device.  A batch that */
/* overflows a capacity on the device is re-run one event at a time, so  */
/* an oversize event fails alone (status PXT_ERR_CAPACITY) without        */
/* affecting the others.  Results are the same as for the event alone.   */

typedef struct pxt_server pxt_server;

typedef struct pxt_server_config {
  int32_t n_lanes;          /* concurrent batches (1..16)                 */
  uint32_t queue_depth;     /* pending events accepted; beyond: BUSY      */
  uint32_t max_batch_events;/* events per batch (<= cfg max_events)       */
  uint32_t doublets_per_hit;/* admission estimate of doublets per hit     */
} pxt_server_config;

/* Caller-owned HOST buffers receiving one event's tracks (same layouts as
 * pxt_tracks, for this event only; event_id is implicit).  On return
 * status, n_tracks (tracks of the event, also when above capacity: then
 * nothing is copied and status is PXT_ERR_CAPACITY) and the timing fields
 * are set. */
typedef struct pxt_event_tracks {
  uint32_t capacity;
  uint32_t* hit_idx;   /* [capacity][8]  */
  uint8_t* n_hits;     /* [capacity]     */
  float* params;       /* [capacity][5]  */
  float* cov;          /* [capacity][15] */
  float* chi2;         /* [capacity][2]  */
  uint8_t* flags;      /* [capacity]     */
  uint32_t n_tracks;
  int32_t status;
  double latency_us;   /* submit to results on the host                 */
  double queue_us;     /* submit to the start of its batch              */
  uint32_t batch_events;/* events in the batch it ran in                */
} pxt_event_tracks;

typedef struct pxt_server_stats {
  uint64_t submitted, completed, failed, rejected, batches;
  uint64_t events_in_batches;   /* sum of batch sizes                    */
  uint64_t solo_retries;        /* events re-run alone after an overflow */
  uint64_t delivered;           /* events handed over by pxt_poll        */
  /* sums over the completed events of the time each spent, in us:
   * queued (arrival to admission into a batch), staging and launch
   * (admission to the batch's calls issued), device (to the counts back
   * on the host; for a batch of at most 32768 hits, copied back by one
   * kernel, the tracks too), copy-back of the tracks (larger batches);
   * over the delivered events: delivery (tracks on the host to
   * pxt_poll's return), and the whole latency (arrival to pxt_poll's
   * return) */
  double sum_queue_us, sum_launch_us, sum_device_us, sum_copyback_us;
  double sum_deliver_us, sum_latency_us;
} pxt_server_stats;

/* Create a server on HIP device `hip_device`.  cfg gives physics and the
 * capacities of ONE lane (max_events, max_hits, ...); every lane allocates
 * its arenas at creation (n_lanes times cfg's footprint).  Errors:
 * PXT_ERR_INVALID_ARG, PXT_ERR_OOM, PXT_ERR_HIP. */
int pxt_server_create(const pxt_config* cfg, const pxt_server_config* scfg,
                      int hip_device, pxt_server** out);

/* Submit one event; x, y, z, layer are HOST arrays of n_hits entries and
 * are copied before return.  *ticket identifies the event for pxt_poll.
 * Errors: PXT_ERR_INVALID_ARG (null pointers, n_hits above the lane's
 * max_hits), PXT_ERR_BUSY (queue full). */
int pxt_submit(pxt_server* s, const float* x, const float* y, const float* z,
               const int16_t* layer, uint32_t n_hits, uint64_t* ticket);

/* Wait up to timeout_ms (negative: forever) for the event's result and copy
 * it into *out; the ticket is released once the result has been delivered.
 * With out->capacity == 0 and out->hit_idx == NULL the tracks are not
 * copied: status, n_tracks and the timings are set and the ticket is
 * released.  A finished event's tracks wait in its lane's pinned result
 * buffers (two sets per lane) until it is polled: a lane whose two sets
 * both hold unpolled events takes no new batch.
 * Returns PXT_OK, PXT_ERR_NOT_READY (timeout; the ticket stays valid),
 * PXT_ERR_CAPACITY (out->capacity is below the event's track count, which
 * is written to out->n_tracks; nothing is copied and the ticket stays
 * valid: poll again with buffers of at least that many tracks) or
 * PXT_ERR_INVALID_ARG (unknown ticket, null buffers).  The event's own
 * status is in out->status: PXT_ERR_CAPACITY there means the event itself
 * overflowed the lane's arenas (it has no tracks; the ticket is released). */
int pxt_poll(pxt_server* s, uint64_t ticket, pxt_event_tracks* out, int timeout_ms);

/* Open-loop replay for measuring the server: arrival i submits event
 * event_of_arrival[i] of a pool (HOST SoA arrays x, y, z, layer with
 * pool_offsets[n_pool + 1]) at arrival_us[i] (non-decreasing, us after
 * the call starts; a full queue is retried, the wait counting as
 * latency), from the calling thread, while a second native thread polls
 * the events in arrival order without copying their tracks.  results[i]
 * (HOST, n entries) receives status, n_tracks, batch_events, queue_us and
 * latency_us (from the scheduled arrival to the hand-over).  Returns when
 * every event is done.  Errors: PXT_ERR_INVALID_ARG (null pointers, an
 * event index or size out of range, decreasing arrival times). */
int pxt_server_replay(pxt_server* s, uint32_t n, const uint32_t* event_of_arrival,
                      const double* arrival_us, uint32_t n_pool, const uint32_t* pool_offsets,
                      const float* x, const float* y, const float* z, const int16_t* layer,
                      pxt_event_tracks* results);

/* Counters since creation. */
int pxt_server_get_stats(pxt_server* s, pxt_server_stats* out);

/* Finish the batches in flight, drop the events still queued (their status
 * becomes PXT_ERR_BUSY), stop the dispatcher and free everything. */
void pxt_server_destroy(pxt_server* s);

#ifdef __cplusplus
}
#endif

#endif /* PXT_H */
