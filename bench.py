"""Throughput benchmark of the pixel-track reconstruction path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pu50|pu200]

A step is one pxt_reconstruct call over one batch of synthetic events already
resident in HBM (the whole path: binning, doublets, links, n-tuplets,
cleaning, fit, output).  The timed region is K steps bracketed by device
synchronisation; value = events/s of the batched path.  The same run also
times the plain path (one event per call, synchronised per event, as the
paper's one-concurrent-event mode), a per-stage breakdown from HIP events on
the library's stream, and the CPU oracle on the host cores (one event per
thread) on a bounded sample.  Prints one JSON line.
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
WORKLOADS = {
    # name: (generator recipe, events per batch, description)
    "pu50": ("pu50", 64, "PU~50 events: 1500 tracks, 10 vertices, 4 barrel layers + 3 disks "
                         "per side, 5% noise hits"),
    "pu200": ("pu200", 32, "PU~200 events: 6000 tracks, 40 vertices, 4 barrel layers + 3 disks "
                           "per side, 15% noise hits"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="pu50", choices=sorted(WORKLOADS))
    ap.add_argument("--batch", type=int, default=0, help="events per batch (default per workload)")
    ap.add_argument("--pool", type=int, default=2, help="distinct batches cycled through")
    ap.add_argument("--plain-events", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=160, help="events for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--phi-bins", type=int, default=256)
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
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 512 MiB device copy first (calibrates HBM byte counters)")
    return ap.parse_args()


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


def gen_events(kind, n, seed0):
    import eventgen
    return [eventgen.generate(kind, seed0 + i) for i in range(n)]


# Algorithmic HBM bytes of one launch of each single-kernel stage: every
# array the kernel must read or write, touched once (re-reads of candidates
# from cache are not counted).  Nh binned hits, Nd doublets, Nw link-mask
# words, Nt raw n-tuplets, Nk tracks, nbar mean hits per track.
def algorithmic_bytes(stage, n, doublet_mode=0):
    Nh, Nd, Nw, Nt, Nk = n["Nh"], n["Nd"], n["Nw"], n["Nt"], n["Nk"]
    # staged doublets: a 4-byte record per doublet written by the count
    # pass and read by the scatter
    rec = 4 * Nd if doublet_mode == 2 else 0
    nbar = n["nbar"]
    table = {
        # x, y (8) + layer (2) read, bin key (4) written
        "prep": 14 * Nh,
        # key, x, y, z, layer read (18); binned SoA written (33)
        "fill": 51 * Nh,
        # binned hit read (29), doublet count written (4)
        "doublet_count": 33 * Nh + rec,
        # binned hit read and offset read or written (33); per doublet
        # written: in/out hits, flag, outer hit and r-z angle, the angle
        # again (29).  The one-pass kernel (reported under this stage)
        # moves the same bytes.
        "doublet_fill": 33 * Nh + 29 * Nd + rec,
        # inner-hit coordinates and doublet offsets (24 per hit); per
        # doublet: inner and outer hit, outer hit coordinates and angle,
        # candidate range written (32), its angle read once as a candidate
        # (4), neighbour count and cleaning-election slots written (16);
        # mask words written (8)
        "links": 24 * Nh + 52 * Nd + 8 * Nw,
        # per n-tuplet: hits, doublets, length (61), hit coordinates, score
        # written (8), order key min per doublet (8)
        "score": (69 + 20 * nbar + 8 * (nbar - 1)) * Nt,
        # per n-tuplet: length, score, doublets (37), per doublet the key (8)
        "best": (37 + 8 * (nbar - 1)) * Nt,
        # survivor, n-tuplet, hits and ids read (41 + 17 per hit), record written (126)
        "fit32": (41 + 17 * nbar + 126) * Nk,
    }
    return table.get(stage)


# kernel that implements each single-kernel stage (for the counter lookup)
STAGE_KERNEL = {"prep": "pxt::k_prep", "fill": "pxt::k_fill",
                "doublet_count": "pxt::k_doublets<8, false>",
                "doublet_fill": "pxt::k_doublets<8, true>", "links": "pxt::k_links_thread",
                "score": "pxt::k_score", "best": "pxt::k_best", "fit32": "pxt::k_fit32"}


def stage_kernel(stage, args):
    kname = STAGE_KERNEL.get(stage)
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


def roofline(stages, counts, n_hits, peak_gbs, workload, args):
    """Roofline entry of the dominant single-kernel stage."""
    n = {"Nh": n_hits, "Nd": counts["n_doublets"], "Nw": counts["n_words"],
         "Nt": counts["n_raw_tuples"], "Nk": counts["n_tracks"], "nbar": 3.4}
    cand = {k: v for k, v in stages.items() if algorithmic_bytes(k, n) is not None}
    dom = max(cand, key=cand.get)
    byts = algorithmic_bytes(dom, n, args.doublet_mode)
    gbs = byts / (cand[dom] * 1e-3) / 1e9
    traffic = None
    kname = stage_kernel(dom, args)
    if (workload == "pu50" and kname and args.link_kernel == 0 and args.group_lanes == 8
            and args.batch in (0, 64)):
        traffic = measured_traffic(kname)
    return {"kernel": kname or dom, "bound": "hbm", "achieved": round(gbs, 2), "peak": peak_gbs,
            "unit": "GB/s", "frac": round(gbs / peak_gbs, 5), "traffic": traffic,
            "algorithmic_bytes_per_launch": int(byts), "avg_launch_ms": round(cand[dom], 5)}


def cpu_baseline(events, det):
    """The oracle as it stands, one event per thread over the host cores."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    oracle.lib()
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda e: oracle.reconstruct(e.x, e.y, e.z, e.layer, det)["status"], events))
    dt = time.perf_counter() - t0
    return len(events) / dt, cores, dt


def serving_leg(det, args):
    """Continuous batching under Poisson arrivals (PU 30..140 mix), then a
    saturating burst for the sustained rate."""
    import eventgen
    from paper_2104_06573_amd.serve import Server, poisson_run
    pool = eventgen.make_batch("serve", args.serve_pool, seed=11)
    events = [pool[i % len(pool)] for i in range(args.serve_events)]
    srv = Server(det, n_lanes=args.serve_lanes, max_batch_events=64, doublets_per_hit=40,
                 max_events=64, max_hits=1_400_000, max_doublets=36 << 20,
                 max_link_words=160 << 20, max_tuples=6 << 20, phi_bins=args.phi_bins,
                 group_lanes=args.group_lanes, link_kernel=args.link_kernel, use_graph=1,
                 doublet_mode=args.latency_doublet_mode)
    poisson_run(srv, events[:300], rate_hz=args.serve_rate)          # warm-up
    rep = poisson_run(srv, events, rate_hz=args.serve_rate)
    sat = poisson_run(srv, events, rate_hz=1e7)
    st = srv.stats()
    srv.close()
    keep = ("events", "events_per_s", "p50_us", "p99_us", "mean_us", "mean_batch", "failed")
    return {
        "workload": "Poisson arrivals, PU uniform 30..140 (30 tracks per PU unit), pool of %d "
                    "distinct events cycled" % len(pool),
        "lanes": args.serve_lanes,
        "offered_rate_hz": args.serve_rate,
        "at_rate": {k: round(rep[k], 2) if isinstance(rep[k], float) else rep[k] for k in keep},
        "saturated": {k: round(sat[k], 2) if isinstance(sat[k], float) else sat[k] for k in keep},
        "solo_retries": st["solo_retries"],
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (events are independent; a multi-GPU "
              "deployment is one process per GPU). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    import eventgen
    import paper_2104_06573_amd as pxt

    det = eventgen.DETECTOR
    # the serving leg runs first, before this process creates any other
    # stream: its lanes' streams then get hardware queues of their own
    served = None
    if not args.no_serve and args.workload == "pu50":
        served = serving_leg(det, args)
    if args.calib_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    kind, batch_default, desc = WORKLOADS[args.workload]
    B = args.batch or batch_default
    pool = [gen_events(kind, B, 1000 + 97 * p) for p in range(args.pool)]
    hits_per_event = float(np.mean([e.n_hits for b in pool for e in b]))
    max_hits = max(sum(e.n_hits for e in b) for b in pool)
    K = max(1, args.inflight)
    caps = batch_caps(kind, B, max_hits)
    recs = [pxt.Reconstructor(det, phi_bins=args.phi_bins, group_lanes=args.group_lanes,
                              link_kernel=args.link_kernel, use_graph=args.graph,
                              doublet_mode=args.doublet_mode, **caps)
            for _ in range(K)]
    rec = recs[0]
    streams = [torch.cuda.Stream() for _ in range(K)]
    dev_batches = [rec.upload(b) for b in pool]
    torch.cuda.synchronize()

    def step(i):
        x, y, z, l, offs = dev_batches[i % len(dev_batches)]
        recs[i % K].launch(x, y, z, l, offs, stream=streams[i % K])

    # correctness guard on the first batch (status only; parity is tested)
    step(0)
    torch.cuda.synchronize()
    c0 = rec.read_counts()
    assert c0["status"] == 0, c0
    for r in recs[1:]:
        x, y, z, l, offs = dev_batches[0]
        r.launch(x, y, z, l, offs)
        torch.cuda.synchronize()
        assert r.read_counts() == c0
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    ev_per_s = B * args.steps / dt

    # stage breakdown with HIP events on the library's stream (direct mode:
    # events cannot sit inside the replayed graph)
    trec = pxt.Reconstructor(det, phi_bins=args.phi_bins, group_lanes=args.group_lanes,
                             link_kernel=args.link_kernel, use_graph=0,
                             doublet_mode=args.doublet_mode, **caps)
    stages = trec.stage_times(trec.upload(pool[0]), repeats=5)
    trec.close()

    # plain path: one event per call, synchronised per event
    plain_events = [e for b in pool for e in b][: args.plain_events]
    pcaps = batch_caps(kind, 2, max(e.n_hits for e in plain_events) + 16)
    pcaps["max_events"] = 1
    prec = pxt.Reconstructor(det, phi_bins=args.phi_bins, group_lanes=args.group_lanes,
                             link_kernel=args.link_kernel, use_graph=args.graph,
                             doublet_mode=args.latency_doublet_mode, **pcaps)
    plain_dev = [prec.upload([e]) for e in plain_events]
    for i in range(min(4, len(plain_dev))):
        prec.launch(*plain_dev[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in plain_dev:
        prec.launch(*d)
        torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t0
    plain_ev_s = len(plain_dev) / plain_dt

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
            "path": "batched (one launch sequence per batch)",
        },
        "plain_events_per_s": round(plain_ev_s, 2),
        "batched_over_plain": round(ev_per_s / plain_ev_s, 2),
        "hits_per_s": round(ev_per_s * hits_per_event, 1),
        "per_batch_counts": {k: counts[k] for k in ("n_doublets", "n_links", "n_raw_tuples",
                                                    "n_tracks", "n_fp64")},
        "stage_ms": stages,
    }
    roof = roofline(stages, counts, int(dev_batches[0][4][-1]), HBM_PEAK_GBS, args.workload, args)
    out["roofline"] = roof
    if served is not None:
        out["served"] = served
    if not args.no_cpu:
        sample = [e for b in pool for e in b][: args.cpu_sample]
        v, cores, cdt = cpu_baseline(sample, det)
        out["cpu_baseline"] = {"value": round(v, 2), "unit": "events/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "%d %s events, one per thread, %.1f s wall" %
                                         (len(sample), args.workload, cdt)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
