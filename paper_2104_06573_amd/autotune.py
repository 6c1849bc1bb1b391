"""Autotuner for the tuning fields of pxt_config.

The tuning fields -- phi bins per layer, threads per block, lane-group size,
link kernel, graph replay -- never change the result (the cuts decide, the
phi window only bounds the candidates), only the speed.  The tuner times a
sample batch under each point of a search space, checks that every point
gives the same tracks as the first one, and keeps the fastest.  Results are
cached in a JSON file keyed by the workload bucket (events per batch and
mean hits per event, rounded to powers of two), so a serving process tunes
once per bucket.

    from paper_2104_06573_amd import autotune
    best = autotune.tune(det, events)            # dict of tuning fields
    rec = Reconstructor(det, **caps, **best)
"""

import itertools
import json
import os
import time

import numpy as np

DEFAULT_SPACE = {
    "phi_bins": (64, 128, 256, 512, 1024),
    "group_lanes": (4, 8, 16),
    "link_kernel": (0, 2),
    "doublet_mode": (1, 2),
    "block_size": (128, 256),
}

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def bucket_key(n_events, hits_per_event):
    """Workload bucket: events per batch and hits per event, each rounded
    up to a power of two."""
    e = 1 << max(0, int(np.ceil(np.log2(max(1, n_events)))))
    h = 1 << max(0, int(np.ceil(np.log2(max(1.0, hits_per_event)))))
    return "events%d_hits%d" % (e, h)


def load_cache(path=CACHE_PATH):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(n_events, hits_per_event, path=CACHE_PATH):
    """Cached tuning fields of the bucket, or None."""
    ent = load_cache(path).get(bucket_key(n_events, hits_per_event))
    return None if ent is None else dict(ent["best"])


def _signature(res, n_events):
    """Canonical per-event track tuples and parameters (for invariance)."""
    out = res.numpy()
    sig = []
    for e in range(n_events):
        m = out["event_id"] == e
        h = out["hit_idx"][m].view(np.uint32)
        o = np.lexsort(h.T[::-1]) if h.shape[0] else np.zeros(0, int)
        sig.append((h[o].tobytes(), out["params"][m][o].tobytes()))
    return sig


def tune(det, events, caps=None, space=None, repeats=5, use_graph=1, device=0,
         cache_path=CACHE_PATH, write_cache=True, verify=True, log=None):
    """Time every point of `space` on the batch `events`; returns the best
    tuning fields (dict).  Raises if two points disagree on the tracks."""
    import torch

    from . import Reconstructor
    space = dict(space or DEFAULT_SPACE)
    n = len(events)
    hits = sum(len(e.x) for e in events)
    caps = dict(caps or {})
    caps.setdefault("max_events", n)
    caps.setdefault("max_hits", hits + 1024)
    caps.setdefault("max_doublets", max(1 << 16, 60 * hits))
    caps.setdefault("max_link_words", min(8 * caps["max_doublets"], 0xfffffff0))
    caps.setdefault("max_tuples", max(1 << 14, 8 * hits))
    caps.setdefault("max_tracks", caps["max_tuples"])
    keys = sorted(space)
    results = []
    ref_sig = None
    for vals in itertools.product(*(space[k] for k in keys)):
        point = dict(zip(keys, vals))
        rec = Reconstructor(det, device=device, use_graph=use_graph, **caps, **point)
        batch = rec.upload(events)
        res = rec.run(*batch)
        if res.counts["status"] != 0:
            raise RuntimeError("tuning point %s failed: %s" % (point, res.counts))
        if verify:
            sig = _signature(res, n)
            if ref_sig is None:
                ref_sig = sig
            elif sig != ref_sig:
                raise AssertionError("tuning point %s changed the result" % point)
        for _ in range(2):
            rec.launch(*batch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            rec.launch(*batch)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / repeats * 1e3
        results.append({"point": point, "ms": ms})
        if log:
            log("%s %.3f ms" % (point, ms))
        rec.close()
        del batch
    best = min(results, key=lambda r: r["ms"])
    tuned = dict(best["point"], use_graph=use_graph)
    if write_cache and cache_path:
        cache = load_cache(cache_path)
        cache[bucket_key(n, hits / max(n, 1))] = {
            "best": tuned, "ms": best["ms"], "n_events": n, "hits": hits,
            "results": results,
        }
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return tuned
