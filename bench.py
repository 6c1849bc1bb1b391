"""Throughput benchmark of the pixel-track reconstruction path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--trials T]

A step is one pxt_reconstruct call over one batch of synthetic events already
resident in HBM: the whole path (binning, doublets, links, n-tuplets,
cleaning, fit, output).  The timed region is K steps in T trials, each trial
bracketed by device synchronisation; value = events/s of the batched PU~50
path over all K steps (64 events per batch, several batches in flight on
their own streams), with the trials' mean and sample standard deviation
beside it.  The same run prints, in the same JSON line:

* the PU~50 batched rate with the host->device copy of the hits and the
  device->host copy of the tracks inside the timed loop (pinned buffers,
  async on each batch's stream) -- the paper counts the per-event copy;
* the PU~200 batched (32 events per batch) and plain legs;
* the plain path (one event per call, synchronised per event);
* the paper's two scheduling levers measured natively: k one-event contexts
  on k streams (concurrent events) and a context created per event (no
  memory pool);
* a per-stage breakdown from HIP events on the library's stream, the HBM
  roofline by the method's algorithmic bytes (whole path and the dominant
  kernel), the measured streaming-copy bandwidth as a second denominator and
  the counter bytes of the last profile while the kernels are unchanged;
* the serving leg (Poisson arrivals over a PU 30..140 mix, continuous
  batching) and the CPU oracle on the host cores.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VTX_SLOTS = 256  # vertex slots per event
HOST_WORKERS = 16  # the GPU machine's CPU share for one GPU
WORKLOADS = {
    # name: (generator recipe, events per batch, description)
    "pu50": ("pu50", 64, "PU~50 events: 1500 tracks, 10 vertices, 4 barrel layers + 3 disks "
                         "per side, 5% noise hits"),
    "pu200": ("pu200", 32, "PU~200 events: 6000 tracks, 40 vertices, 4 barrel layers + 3 disks "
                           "per side, 15% noise hits"),
}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--trials", type=int, default=8, help="the K steps are timed as T trials")
    ap.add_argument("--workload", default="pu50", choices=sorted(WORKLOADS),
                    help="workload of the headline value")
    ap.add_argument("--batch", type=int, default=0, help="events per batch (default per workload)")
    ap.add_argument("--pool", type=int, default=2, help="distinct batches cycled through")
    ap.add_argument("--plain-events", type=int, default=512,
                    help="one-event calls timed on the plain path (cycled over the pool); 0 "
                         "skips the plain legs and the ablations")
    ap.add_argument("--pu200-steps", type=int, default=100)
    ap.add_argument("--no-pu200", action="store_true")
    ap.add_argument("--no-rechits", action="store_true")
    ap.add_argument("--rechits-steps", type=int, default=200)
    ap.add_argument("--no-pcie", action="store_true")
    ap.add_argument("--no-ablations", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="events for the CPU baseline (cycled over the pool)")
    ap.add_argument("--cpu-sample-1t", type=int, default=64,
                    help="events for the one-thread CPU figure")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--phi-bins", type=int, default=1024,
                    help="phi bins per layer (1024: fewer doublet candidates than 256 or "
                         "512, and still held in LDS by the per-event binning at 10 layers)")
    ap.add_argument("--group-lanes", type=int, default=8)
    ap.add_argument("--link-kernel", type=int, default=0,
                    help="0 thread per doublet (the fastest with batches in flight at PU~50 "
                         "and PU~200), 1 lane group + queue, 2 wavefront + queue")
    ap.add_argument("--doublet-mode", type=int, default=2,
                    help="batched path: 0 count/scan/fill, 1 one pass (LDS records), "
                         "2 count+stage/scan/scatter")
    ap.add_argument("--latency-doublet-mode", type=int, default=1,
                    help="plain (one event per call) and served paths: the one-pass mode has "
                         "the least latency on a few events")
    ap.add_argument("--graph", type=int, default=1, help="replay the launch sequence as a HIP graph")
    ap.add_argument("--inflight", type=int, default=4,
                    help="batches in flight: contexts, each on its own stream, taking turns")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate (Hz)")
    ap.add_argument("--serve-events", type=int, default=10000)
    ap.add_argument("--serve-pool", type=int, default=96, help="distinct events cycled through")
    ap.add_argument("--serve-lanes", type=int, default=4)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--served-child", action="store_true",
                    help="(internal) run only the serving leg and print its JSON entry")
    ap.add_argument("--vertices", type=int, default=1,
                    help="find the vertices of the tracks in every step (the serving leg "
                         "returns tracks only)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 512 MiB device copy first (calibrates HBM byte counters)")
    return ap.parse_args(argv)


def batch_caps(kind, n_events, max_hits):
    """Context capacities for batches of n_events events of workload `kind`
    holding at most max_hits hits (the timed configuration; the GPU parity
    tests use the same)."""
    per_ev_d = 100_000 if kind == "pu50" else 1_700_000
    per_ev_w = per_ev_d * (4 if kind == "pu50" else 8)  # link-mask words
    per_ev_t = 8_000 if kind == "pu50" else 200_000
    return dict(max_events=n_events, max_hits=max_hits + 1024,
                max_doublets=per_ev_d * n_events, max_link_words=per_ev_w * n_events,
                max_tuples=per_ev_t * n_events, max_tracks=per_ev_t * n_events)


def _gen_one(a):
    import eventgen
    return eventgen.generate(a[0], a[1])


def _gen_clusters(a):
    import eventgen
    from eventgen import clusters
    ev = eventgen.generate(a[0], a[1])
    c = clusters.make_clusters(ev, a[1])
    c.pop("hit_of_cluster")
    return c


def gen_clusters(kind, n, seed0, workers=1):
    """Pixel clusters of events seed0 .. seed0+n-1 (the RecHits input)."""
    args = [(kind, seed0 + i) for i in range(n)]
    if workers <= 1:
        return [_gen_clusters(a) for a in args]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(workers, n),
                             mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_gen_clusters, args))


def rechits_leg(torch, pxt, clusters, args):
    """pxt_rechits on one batch of clusters, timed over --rechits-steps
    calls: events/s, and the step's algorithmic bytes (module id and pixel
    range per cluster, 6 bytes per pixel read; 20 bytes per hit and the
    per-module counters and offsets written) against the HBM peak."""
    from eventgen import clusters as C
    table = C.module_table()
    dev, ev = pxt.upload_clusters(clusters)
    nc = int(ev[-1])
    E = len(clusters)
    rh = pxt.RecHits(table, E, nc)
    limit = 1024
    for _ in range(5):
        rh.launch(dev, E, nc, limit)
    torch.cuda.synchronize()
    status = rh.read(E)[0]
    assert status == 0, status
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.rechits_steps):
        rh.launch(dev, E, nc, limit)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.rechits_steps
    npix = int(dev["pixel_offsets"][-1].item())
    nh = int(rh.hit_offsets[E].item())
    byts = 6 * nc + 6 * npix + 20 * nh + 12 * E * table.shape[0]
    gbs = byts / (ms * 1e-3) / 1e9
    return {"workload": "pixel clusters of the %d PU~50 events of one batch (%d clusters, "
                        "%d pixels, %d modules)" % (E, nc, npix, table.shape[0]),
            "events_per_s": round(E / (ms * 1e-3), 2), "ms_per_step": round(ms, 5),
            "steps": args.rechits_steps, "hits": nh, "algorithmic_bytes": int(byts),
            "achieved_gbs": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 5)}


def gen_events(kind, n, seed0, workers=1):
    """Events seed0 .. seed0+n-1 of workload `kind` (in processes when
    workers > 1; the generator is seeded per event, so the result is the
    same)."""
    args = [(kind, seed0 + i) for i in range(n)]
    if workers <= 1 or n <= 2:
        return [_gen_one(a) for a in args]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(workers, n),
                             mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_gen_one, args, chunksize=max(1, n // (4 * workers))))


# Algorithmic HBM bytes: what the method must move, every product written
# once by its producer and read once by its consumer.  Per event (or batch):
#   14 Nh  hits in (x, y, z f32, layer i16)
#   48 Nh  binned hits written and read (24 B each)
#   16 Nd  doublets (inner, outer hit) written and read
#    8 (Nh + Nd)  incoming-doublet CSR (offsets per hit, entries) w + r
#    8 Nl  links written and read
#   66 Nt  raw n-tuplets written and read (8 hit ids + length, 33 B)
#   12 nbar Nk  hit coordinates gathered by the fit
#  120 Nk  tracks out (8 hit ids, 5 parameters, 15 covariances, 2 chi2, ...)
# and, when the vertices are found, 17 Nk (hit count, q/pT, z0, var(z0)
# read, vertex of each track written) + 16 Nv (vertices written).
# Nh input hits, Nd doublets, Nl links, Nt raw n-tuplets, Nk tracks, nbar
# mean hits per track, Nv vertices.  Each step's share is what it reads of
# its predecessor's product plus what it writes of its own.
def path_bytes(n):
    Nh, Nd, Nl, Nt, Nk, nbar = n["Nh"], n["Nd"], n["Nl"], n["Nt"], n["Nk"], n["nbar"]
    b = (14 * Nh + 48 * Nh + 16 * Nd + 8 * (Nh + Nd) + 8 * Nl + 66 * Nt
         + 12 * nbar * Nk + 120 * Nk)
    if n.get("Nv") is not None:
        b += 17 * Nk + 16 * n["Nv"]
    return b


def step_bytes(step, n):
    Nh, Nd, Nl, Nt, Nk, nbar = n["Nh"], n["Nd"], n["Nl"], n["Nt"], n["Nk"], n["nbar"]
    table = {
        "binning": 14 * Nh + 24 * Nh,                       # hits read, binned hits written
        "doublets": 24 * Nh + 8 * Nd + 4 * (Nh + Nd),       # binned read, doublets + CSR written
        "links": 8 * Nd + 4 * (Nh + Nd) + 4 * Nl,           # doublets + CSR read, links written
        "ntuplets": 4 * Nl + 33 * Nt,                       # links read, raw n-tuplets written
        "cleaning": 33 * Nt,                                # raw n-tuplets read
        "fit": 12 * nbar * Nk + 120 * Nk,                   # hit gathers, tracks written
    }
    if n.get("Nv") is not None:
        table["vertices"] = 17 * Nk + 16 * n["Nv"]          # track values read, vertices written
    return table.get(step)


# library stages (pxt_stage_name) of each step of the path
STEP_STAGES = {
    # (ingest and binning are one kernel, one block per event, unless the
    # histogram of an event exceeds LDS: then k_prep, the scan and k_fill)
    "binning": ("clear", "prep", "bin_scan", "fill"),
    "doublets": ("doublet_count", "doublet_scan", "doublet_fill"),
    "links": ("mask_clear", "links"),
    "ntuplets": ("roots", "tuple_count", "tuple_scan", "tuple_fill"),
    "cleaning": ("score", "best", "survive"),
    "fit": ("fit32", "fit64", "finish"),
    "vertices": ("vertices",),
}


def stage_kernel(stage, args):
    """The kernel of a single-kernel stage (for the counter lookup)."""
    base = {"prep": "pxt::k_prep", "fill": "pxt::k_fill",
            "doublet_count": "pxt::k_doublets<8, false>",
            "doublet_fill": "pxt::k_doublets<8, true>", "links": "pxt::k_links_thread",
            "score": "pxt::k_score", "best": "pxt::k_best", "fit32": "pxt::k_fit32"}
    kname = base.get(stage)
    if stage == "links" and args.link_kernel == 1:
        kname = "pxt::k_links<%d>" % args.group_lanes
    if stage == "links" and args.link_kernel == 2:
        kname = "pxt::k_links_wave"
    if stage == "doublet_fill" and args.doublet_mode == 1:
        kname = "pxt::k_doublets1<8>"
    if stage == "doublet_fill" and args.doublet_mode == 2:
        kname = "pxt::k_dscatter<8>"
    if stage == "doublet_count" and args.doublet_mode == 2:
        kname = "pxt::k_dstage<8>"
    if stage in ("doublet_count", "doublet_fill"):
        kname = kname.replace("<8", "<%d" % args.group_lanes)
    return kname


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2104_06573_amd", "csrc")
    for f in ("common.h", "cuts.h", "fit.h", "kernels.h", "pxt.hip"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if it is absent or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_pu50_batch64.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    try:
        blob = json.loads(txt.split("```json")[1].split("```")[0])
    except (IndexError, ValueError):
        return None
    if blob.get("source_hash") != kernel_source_hash():
        return None
    return blob["bytes_per_launch"].get(kernel)


def roofline(stages, n, batches_per_s, peak_gbs, copy_gbs, workload, args):
    """HBM roofline by the method's algorithmic bytes: the dominant kernel
    (the link kernel: its step's bytes over its mean launch time) and the
    whole path (bytes per batch times batches per second)."""
    links_ms = stages.get("links", 0.0)
    lb = step_bytes("links", n)
    gbs = lb / (links_ms * 1e-3) / 1e9 if links_ms > 0 else 0.0
    kname = stage_kernel("links", args)
    traffic = None
    if workload == "pu50" and args.link_kernel == 0 and args.group_lanes == 8 and \
            args.batch in (0, 64):
        traffic = measured_traffic(kname)
    pb = path_bytes(n)
    path_gbs = pb * batches_per_s / 1e9
    out = {"kernel": kname, "bound": "hbm", "achieved": round(gbs, 2), "peak": peak_gbs,
           "unit": "GB/s", "frac": round(gbs / peak_gbs, 5), "traffic": traffic,
           "algorithmic_bytes_per_launch": int(lb), "avg_launch_ms": round(links_ms, 5),
           "path": {"algorithmic_bytes_per_batch": int(pb), "achieved": round(path_gbs, 2),
                    "frac": round(path_gbs / peak_gbs, 5)},
           "steps": {}}
    for step, stg in STEP_STAGES.items():
        ms = sum(stages.get(s, 0.0) for s in stg)
        b = step_bytes(step, n)
        if b is None:
            continue
        out["steps"][step] = {"ms": round(ms, 5), "bytes": int(b),
                              "frac": round(b / (ms * 1e-3) / 1e9 / peak_gbs, 5) if ms else None}
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / lb, 3)
    if copy_gbs:
        out["copy_peak_gbs"] = round(copy_gbs, 1)
        out["frac_of_copy_peak"] = round(gbs / copy_gbs, 5)
        out["path"]["frac_of_copy_peak"] = round(path_gbs / copy_gbs, 5)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(events, det, threads):
    """The oracle as it stands, one event per thread over `threads` host
    threads."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda e: oracle.reconstruct(e.x, e.y, e.z, e.layer, det)["status"], events))
    dt = time.perf_counter() - t0
    return len(events) / dt, dt


def host_threads():
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(cores or 1, HOST_WORKERS))


def serving_leg(det, args):
    """Continuous batching over the PU 30..140 mix, driven by the library's
    native replay (arrivals submitted and results released by native
    threads): three runs of Poisson arrivals at --serve-rate, then a
    saturating burst of the same events; phase means from the server's
    counters.  Returns the entry and the pool (for the batched comparison
    on the same mix)."""
    import eventgen
    from paper_2104_06573_amd.serve import Server, poisson_schedule, replay
    pool = eventgen.make_batch("serve", args.serve_pool, seed=11)
    srv = Server(det, n_lanes=args.serve_lanes, max_batch_events=64, doublets_per_hit=40,
                 max_events=64, max_hits=1_400_000, max_doublets=36 << 20,
                 max_link_words=160 << 20, max_tuples=6 << 20, phi_bins=args.phi_bins,
                 group_lanes=args.group_lanes, link_kernel=args.link_kernel, use_graph=1,
                 doublet_mode=args.latency_doublet_mode)
    replay(srv, pool, *poisson_schedule(300, args.serve_rate, len(pool)))      # warm-up
    keep = ("events", "events_per_s", "p50_us", "p99_us", "mean_us", "mean_batch",
            "max_batch", "failed", "phases_us")
    rnd = lambda r: {k: round(r[k], 2) if isinstance(r[k], float) else r[k] for k in keep}
    runs = [rnd(replay(srv, pool, *poisson_schedule(args.serve_events, args.serve_rate,
                                                     len(pool), seed=k)))
            for k in range(3)]
    sat = rnd(replay(srv, pool, *poisson_schedule(args.serve_events, float("inf"), len(pool))))
    st = srv.stats()
    srv.close()
    p50 = [r["p50_us"] for r in runs]
    p99 = [r["p99_us"] for r in runs]
    return {
        "workload": "Poisson arrivals, PU uniform 30..140 (30 tracks per PU unit), pool of %d "
                    "distinct events cycled; native replay (submission and release in "
                    "library threads)" % len(pool),
        "lanes": args.serve_lanes,
        "offered_rate_hz": args.serve_rate,
        "at_rate": runs,
        "at_rate_p50_us_range": [min(p50), max(p50)],
        "at_rate_p99_us_range": [min(p99), max(p99)],
        "saturated": sat,
        "solo_retries": st["solo_retries"],
    }, pool


def served_in_child(args):
    """The serving leg in a process of its own that uses only the library,
    as a serving process would: where torch has already taken the device,
    the lanes share hardware queues with it (measured 28–30k instead of 35k
    events/s saturated).  Returns the entry and the pool."""
    import subprocess
    import eventgen
    cmd = [sys.executable, os.path.abspath(__file__), "--served-child",
           "--serve-rate", str(args.serve_rate), "--serve-events", str(args.serve_events),
           "--serve-pool", str(args.serve_pool), "--serve-lanes", str(args.serve_lanes),
           "--phi-bins", str(args.phi_bins), "--group-lanes", str(args.group_lanes),
           "--link-kernel", str(args.link_kernel),
           "--latency-doublet-mode", str(args.latency_doublet_mode)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not lines:
        raise RuntimeError("serving leg failed (rc %d): %s" % (r.returncode, r.stderr[-2000:]))
    entry = json.loads(lines[-1])
    entry["process"] = "own (library only; the other legs run in the parent)"
    return entry, eventgen.make_batch("serve", args.serve_pool, seed=11)


def mix_batched(torch, pxt, det, pool, args):
    """The batched path (64 events per batch, graph, batches in flight) on
    the serving mix, for the saturated serving rate to be compared with."""
    B = 64
    batches = [[pool[(B * k + j) % len(pool)] for j in range(B)] for k in range(2)]
    caps = dict(max_events=B, max_hits=max(sum(e.n_hits for e in b) for b in batches) + 1024,
                max_doublets=36 << 20, max_link_words=160 << 20, max_tuples=6 << 20,
                max_tracks=6 << 20)
    bat = Batched.__new__(Batched)
    bat.torch = torch
    bat.recs = [pxt.Reconstructor(det, phi_bins=args.phi_bins, group_lanes=args.group_lanes,
                                  link_kernel=args.link_kernel, use_graph=args.graph,
                                  doublet_mode=args.doublet_mode, **caps)
                for _ in range(max(1, args.inflight))]
    bat.streams = [torch.cuda.Stream() for _ in bat.recs]
    bat.dev = [bat.recs[0].upload(b) for b in batches]
    bat.B = B
    bat.caps = caps
    torch.cuda.synchronize()
    bat.check()
    v, ms, st = bat.timed(200, 5, args.trials)
    bat.close()
    return {"events_per_s": round(v, 2), "ms_per_step": round(ms, 4), "trials": st,
            "events_per_batch": B}


def stats(values):
    v = np.asarray(values, np.float64)
    return {"mean": round(float(v.mean()), 2),
            "std": round(float(v.std(ddof=1)), 2) if v.size > 1 else 0.0, "n": int(v.size)}


class Batched:
    """K contexts (batches in flight), each on its own stream, taking the
    steps in turn over a pool of device-resident batches."""

    def __init__(self, torch, pxt, det, kind, batches, args, inflight, doublet_mode, graph):
        self.torch = torch
        B = len(batches[0])
        max_hits = max(sum(e.n_hits for e in b) for b in batches)
        caps = batch_caps(kind, B, max_hits)
        self.recs = [pxt.Reconstructor(det, phi_bins=args.phi_bins,
                                       group_lanes=args.group_lanes,
                                       link_kernel=args.link_kernel, use_graph=graph,
                                       doublet_mode=doublet_mode,
                                       max_vertices_per_event=VTX_SLOTS * args.vertices, **caps)
                     for _ in range(inflight)]
        self.streams = [torch.cuda.Stream() for _ in range(inflight)]
        self.dev = [self.recs[0].upload(b) for b in batches]
        self.B = B
        self.caps = caps
        torch.cuda.synchronize()

    def step(self, i):
        K = len(self.recs)
        self.recs[i % K].launch(*self.dev[i % len(self.dev)], stream=self.streams[i % K])

    def check(self):
        """Status of every context on the first batch (parity is tested
        separately); returns the counts."""
        c0 = None
        for r in self.recs:
            r.launch(*self.dev[0])
            self.torch.cuda.synchronize()
            c = r.read_counts()
            assert c["status"] == 0, c
            assert c0 is None or c == c0, (c, c0)
            c0 = c
        return c0

    def timed(self, steps, warmup, trials, step=None):
        step = step or self.step
        torch = self.torch
        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        T = max(1, min(trials, steps))
        sizes = [steps // T + (1 if i < steps % T else 0) for i in range(T)]
        rates, total_dt, done = [], 0.0, 0
        for n in sizes:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(done, done + n):
                step(i)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rates.append(self.B * n / dt)
            total_dt += dt
            done += n
        return self.B * steps / total_dt, total_dt / steps * 1e3, stats(rates)

    def close(self):
        for r in self.recs:
            r.close()


def pcie_leg(torch, bat, batches, counts, args):
    """Batched PU~50 with the hits copied in from pinned host memory and the
    tracks copied out to it inside the timed loop (async, on each batch's
    stream): the paper counts the per-event input copy."""
    K = len(bat.recs)
    host = []
    for b in batches:
        cat = lambda f, dt: torch.from_numpy(np.ascontiguousarray(
            np.concatenate([getattr(e, f) for e in b]), dt)).pin_memory()
        host.append((cat("x", np.float32), cat("y", np.float32), cat("z", np.float32),
                     cat("layer", np.int16), bat.dev[len(host)][4]))
    dev_in = []
    for k in range(K):
        n = max(h[0].shape[0] for h in host)
        dev_in.append(tuple(torch.empty(n, dtype=d, device="cuda")
                            for d in (torch.float32, torch.float32, torch.float32, torch.int16)))
    nk = counts["n_tracks"]
    outs = []
    for r in bat.recs:
        t = {name: getattr(r, "o_" + name) for name in
             ("hit_idx", "n_hits", "event_id", "params", "cov", "chi2", "flags")}
        outs.append({name: (v, torch.empty((nk,) + tuple(v.shape[1:]), dtype=v.dtype,
                                           pin_memory=True)) for name, v in t.items()})
    ev_bytes = [0]

    def step(i):
        k = i % K
        h = host[i % len(host)]
        s = bat.streams[k]
        x, y, z, l = dev_in[k]
        n = h[0].shape[0]
        with torch.cuda.stream(s):
            for dst, src in zip((x, y, z, l), h[:4]):
                dst[:n].copy_(src, non_blocking=True)
        bat.recs[k].launch(x[:n], y[:n], z[:n], l[:n], h[4], stream=s)
        with torch.cuda.stream(s):
            for dev, hb in outs[k].values():
                hb.copy_(dev[:nk], non_blocking=True)

    v, ms, st = bat.timed(args.steps, args.warmup, args.trials, step=step)
    per_batch = 14 * host[0][0].shape[0] + sum(
        hb.numel() * hb.element_size() for _, hb in outs[0].values())
    return {"events_per_s": round(v, 2), "ms_per_step": round(ms, 4), "trials": st,
            "pcie_bytes_per_batch": int(per_batch),
            "note": "hits copied in and tracks copied out per batch (pinned host buffers, "
                    "async on each batch's stream)"}


def plain_leg(torch, pxt, det, kind, events, args, n_calls, streams=1):
    """One event per call, each call waited for before its context is
    reused; `streams` contexts on their own streams keep that many events
    in flight (the paper's concurrent events)."""
    caps = batch_caps(kind, 2, max(e.n_hits for e in events) + 16)
    caps["max_events"] = 1
    recs = [pxt.Reconstructor(det, phi_bins=args.phi_bins, group_lanes=args.group_lanes,
                              link_kernel=args.link_kernel, use_graph=args.graph,
                              doublet_mode=args.latency_doublet_mode,
                              max_vertices_per_event=VTX_SLOTS * args.vertices, **caps)
            for _ in range(streams)]
    ss = [torch.cuda.Stream() for _ in range(streams)]
    dev = [recs[0].upload([e]) for e in events]
    for i in range(min(4 * streams, len(dev))):
        recs[i % streams].launch(*dev[i % len(dev)], stream=ss[i % streams])
    torch.cuda.synchronize()
    done = [None] * streams
    t0 = time.perf_counter()
    for i in range(n_calls):
        k = i % streams
        if done[k] is not None:
            done[k].synchronize()
        recs[k].launch(*dev[i % len(dev)], stream=ss[k])
        done[k] = torch.cuda.Event()
        done[k].record(ss[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for r in recs:
        r.close()
    return n_calls / dt


def plain_malloc_per_event(torch, pxt, det, kind, events, args, n_calls):
    """One event per call with its context (all device arenas) created and
    destroyed around the call: the paper's memory-pool-disabled mode."""
    caps = batch_caps(kind, 2, max(e.n_hits for e in events) + 16)
    caps["max_events"] = 1
    dev = [pxt.upload_events([e]) for e in events]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_calls):
        r = pxt.Reconstructor(det, phi_bins=args.phi_bins, group_lanes=args.group_lanes,
                              link_kernel=args.link_kernel, use_graph=0,
                              doublet_mode=args.latency_doublet_mode,
                              max_vertices_per_event=VTX_SLOTS * args.vertices, **caps)
        r.launch(*dev[i % len(dev)])
        torch.cuda.synchronize()
        r.close()
    dt = time.perf_counter() - t0
    return n_calls / dt


def copy_peak(torch, nbytes=1 << 30, reps=10):
    """Streaming-copy bandwidth of one large device copy (read + write)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def atomic_rates(torch, pxt, rec, n, stages):
    """Atomic throughput: a ruler (random-address 32-bit integer adds by
    torch's index_add_, over a 64 MiB array and over 64k counters, the size
    of the bin histogram of a 64-event batch) and the rates the path's
    atomic-heavy kernels reach: the binning counts (two LDS adds per hit),
    the election keys (one 64-bit min per raw n-tuplet doublet) and the link
    bits (one 64-bit or per link), each over its stage time."""
    dev = "cuda"
    out = {}
    g = torch.Generator(device="cpu").manual_seed(7)
    for name, size in (("ruler_uncontended_gops", 16 << 20), ("ruler_64k_counters_gops", 1 << 16)):
        n_ops = 1 << 25
        idx = torch.randint(0, size, (n_ops,), generator=g).to(dev)
        src = torch.ones(n_ops, dtype=torch.int32, device=dev)
        dst = torch.zeros(size, dtype=torch.int32, device=dev)
        dst.index_add_(0, idx, src)  # warm-up
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        a.record()
        for _ in range(reps):
            dst.index_add_(0, idx, src)
        b.record()
        torch.cuda.synchronize()
        out[name] = round(n_ops * reps / (a.elapsed_time(b) * 1e-3) / 1e9, 2)
        del idx, src, dst
    raw = rec.dump(pxt.DUMP_RAW)
    cells = int(((raw[:, 1:] != 0xFFFFFFFF).sum(axis=1) - 1).sum()) if raw.shape[0] else 0
    kern = {}
    for stage, ops, what in (("prep", 2 * n["Nh"],
                              "bin counter adds, in LDS (two per hit: count, fill cursor)"),
                             ("score", cells, "64-bit key mins (one per raw n-tuplet doublet)"),
                             ("links", n["Nl"], "64-bit mask ors (one per link)")):
        ms = stages.get(stage, 0.0)
        kern[stage] = {"atomics": int(ops), "what": what, "ms": round(ms, 4),
                       "gops": round(ops / (ms * 1e-3) / 1e9, 2) if ms > 0 else None}
    out["kernels"] = kern
    return out


def path_counts(rec, counts, n_hits, n_events):
    nk = counts["n_tracks"]
    nh = rec.o_n_hits[:nk].cpu().numpy()
    n = {"Nh": n_hits, "Nd": counts["n_doublets"], "Nl": counts["n_links"],
         "Nt": counts["n_raw_tuples"], "Nk": nk, "nbar": float(nh.mean()) if nk else 0.0}
    if rec.vtx is not None:
        summary, _, _ = rec.vtx.read(n_events, 0)
        assert summary["status"] == 0, summary
        n["Nv"] = summary["n_vertices"]
    return n


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (events are independent; a multi-GPU "
              "deployment is one process per GPU). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.served_child:
        import eventgen
        entry, _ = serving_leg(eventgen.DETECTOR, args)
        print(json.dumps(entry), flush=True)
        return
    # every input is generated before the GPU is touched (worker processes)
    kind, batch_default, desc = WORKLOADS[args.workload]
    B = args.batch or batch_default
    flat = gen_events(kind, B * args.pool, 1000, workers=HOST_WORKERS)
    pool = [flat[p * B:(p + 1) * B] for p in range(args.pool)]
    clusters = None
    if not args.no_rechits and args.workload == "pu50":
        clusters = gen_clusters(kind, B, 1000, workers=HOST_WORKERS)
    pu200 = None
    if not args.no_pu200 and args.workload == "pu50":
        f2 = gen_events("pu200", 64, 5000, workers=HOST_WORKERS)
        pu200 = [f2[:32], f2[32:]]

    import torch

    import eventgen
    import paper_2104_06573_amd as pxt

    det = eventgen.DETECTOR
    # the serving leg first, in a child process, before this one touches
    # the device
    served = serve_pool = None
    if not args.no_serve and args.workload == "pu50":
        served, serve_pool = served_in_child(args)
    if args.calib_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    hits_per_event = float(np.mean([e.n_hits for b in pool for e in b]))

    bat = Batched(torch, pxt, det, kind, pool, args, max(1, args.inflight), args.doublet_mode,
                  args.graph)
    c0 = bat.check()
    ev_per_s, ms_per_step, trials = bat.timed(args.steps, args.warmup, args.trials)

    # stage breakdown with HIP events on the library's stream (direct mode:
    # events cannot sit inside the replayed graph)
    trec = pxt.Reconstructor(det, phi_bins=args.phi_bins, group_lanes=args.group_lanes,
                             link_kernel=args.link_kernel, use_graph=0,
                             doublet_mode=args.doublet_mode,
                             max_vertices_per_event=VTX_SLOTS * args.vertices, **bat.caps)
    tb = trec.upload(pool[0])
    stages = trec.stage_times(tb, repeats=5)
    n = path_counts(trec, trec.read_counts(), int(tb[4][-1]), B)
    atomics = atomic_rates(torch, pxt, trec, n, stages)
    trec.close()

    pcie = None
    if not args.no_pcie:
        pcie = pcie_leg(torch, bat, pool, c0, args)
    bat.close()
    del bat

    # plain path: one event per call, synchronised per event
    plain_events = [e for b in pool for e in b]
    plain_ev_s = None
    if args.plain_events > 0:
        plain_ev_s = plain_leg(torch, pxt, det, kind, plain_events, args, args.plain_events)

    ablations = None
    if not args.no_ablations and args.plain_events > 0:
        ablations = {
            "workload": "plain path (one event per call) over the %d %s events of the pool" %
                        (len(plain_events), args.workload),
            "concurrent_events_events_per_s": {
                str(k): round(plain_leg(torch, pxt, det, kind, plain_events, args,
                                        args.plain_events, streams=k), 2)
                for k in (1, 2, 4, 8)},
            "context_per_event_events_per_s": round(
                plain_malloc_per_event(torch, pxt, det, kind, plain_events, args, 32), 2),
        }
        base = ablations["concurrent_events_events_per_s"]["1"]
        ablations["concurrent_events_gain"] = {
            k: round(v / base, 2) for k, v in ablations["concurrent_events_events_per_s"].items()}
        ablations["memory_pool_gain"] = round(base / ablations["context_per_event_events_per_s"], 2)

    p200 = None
    if pu200 is not None:
        b2 = Batched(torch, pxt, det, "pu200", pu200, args, max(1, args.inflight),
                     args.doublet_mode, args.graph)
        b2.check()
        v2, ms2, st2 = b2.timed(args.pu200_steps, 5, args.trials)
        b2.close()
        del b2
        pv2 = (plain_leg(torch, pxt, det, "pu200", [e for b in pu200 for e in b], args, 128)
               if args.plain_events > 0 else None)
        p200 = {"workload": WORKLOADS["pu200"][2] + ", 32 events per batch",
                "hits_per_event": round(float(np.mean([e.n_hits for b in pu200 for e in b])), 1),
                "batched_events_per_s": round(v2, 2), "ms_per_step": round(ms2, 4),
                "steps": args.pu200_steps, "trials": st2,
                "plain_events_per_s": round(pv2, 2) if pv2 else None,
                "batched_over_plain": round(v2 / pv2, 2) if pv2 else None}

    rech = rechits_leg(torch, pxt, clusters, args) if clusters is not None else None
    if served is not None:
        mb = mix_batched(torch, pxt, det, serve_pool, args)
        served["batched_same_mix"] = mb
        served["saturated_over_batched"] = round(
            served["saturated"]["events_per_s"] / mb["events_per_s"], 3)
    # (a counter-calibration run measures its one 512 MiB copy alone)
    cgbs = None if args.calib_copy else copy_peak(torch)
    counts = c0
    out = {
        "metric": "events/s at PU50/PU200 on 1 MI355X (batched/served vs plain)",
        "value": round(ev_per_s, 2),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc + ", %d events per batch" % B,
            "events_per_batch": B,
            "hits_per_event": round(hits_per_event, 1),
            "phi_bins": args.phi_bins,
            "group_lanes": args.group_lanes,
            "batches_in_flight": args.inflight,
            "link_kernel": args.link_kernel,
            "doublet_mode": args.doublet_mode,
            "latency_doublet_mode": args.latency_doublet_mode,
            "hip_graph": bool(args.graph),
            "path": "batched (one launch sequence per batch), inputs resident in HBM",
            "vertices": bool(args.vertices),
        },
        "trials": trials,
        "plain_events_per_s": round(plain_ev_s, 2) if plain_ev_s else None,
        "batched_over_plain": round(ev_per_s / plain_ev_s, 2) if plain_ev_s else None,
        "hits_per_s": round(ev_per_s * hits_per_event, 1),
        "per_batch_counts": dict({k: counts[k] for k in ("n_doublets", "n_links",
                                                         "n_raw_tuples", "n_tracks", "n_fp64")},
                                 **({"n_vertices": n["Nv"]} if "Nv" in n else {})),
        # share of the fitted tracks refitted in FP64 (reference pT above
        # pt_fp64, an ill-conditioned FP32 system or a non-finite result)
        "fp64_fraction": round(counts["n_fp64"] / max(1, counts["n_tracks"]), 5),
        "stage_ms": stages,
    }
    if pcie is not None:
        out["pcie_inclusive"] = pcie
    if p200 is not None:
        out["pu200"] = p200
    if ablations is not None:
        out["ablations"] = ablations
    if rech is not None:
        out["rechits"] = rech
    out["roofline"] = roofline(stages, n, ev_per_s / B, HBM_PEAK_GBS, cgbs, args.workload, args)
    out["atomics"] = atomics
    if served is not None:
        out["served"] = served
    if not args.no_cpu:
        threads = host_threads()
        sample = [plain_events[i % len(plain_events)] for i in range(args.cpu_sample)]
        v, cdt = cpu_baseline(sample, det, threads)
        v1, cdt1 = cpu_baseline([plain_events[i % len(plain_events)]
                                 for i in range(args.cpu_sample_1t)], det, 1)
        out["cpu_baseline"] = {"value": round(v, 2), "unit": "events/s", "cores": threads,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "one_thread_events_per_s": round(v1, 2),
                               "sample": "%d %s events (the %d of the pool cycled), one per "
                                         "thread on %d threads, %.1f s wall; one thread: %d "
                                         "events, %.1f s" %
                                         (len(sample), args.workload, len(plain_events),
                                          threads, cdt, args.cpu_sample_1t, cdt1)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
