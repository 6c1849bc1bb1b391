"""Serving over libpxt's continuous-batching server (pxt_server_* in pxt.h).

    srv = Server(det, n_lanes=4, max_events=64, max_hits=500_000)
    t = srv.submit(ev.x, ev.y, ev.z, ev.layer)       # host arrays
    res = srv.poll(t)                                 # dict of numpy arrays
    report = poisson_run(srv, events, rate_hz=2000)   # p50/p99, events/s

Marshalling only: the server, its dispatcher thread, batching and all
device work are in the native library.
"""

import ctypes
import threading
import time

import numpy as np

from . import (OK, ERR_BUSY, ERR_CAPACITY, ERR_NOT_READY, PxtConfig, PxtError, lib,
               make_config)


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_lanes", ctypes.c_int32), ("queue_depth", ctypes.c_uint32),
                ("max_batch_events", ctypes.c_uint32), ("doublets_per_hit", ctypes.c_uint32)]


class EventTracks(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint32), ("hit_idx", ctypes.c_void_p),
                ("n_hits", ctypes.c_void_p), ("params", ctypes.c_void_p),
                ("cov", ctypes.c_void_p), ("chi2", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("n_tracks", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("latency_us", ctypes.c_double), ("queue_us", ctypes.c_double),
                ("batch_events", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "failed", "rejected",
                                               "batches", "events_in_batches", "solo_retries",
                                               "delivered")] + \
        [(n, ctypes.c_double) for n in ("sum_queue_us", "sum_launch_us", "sum_device_us",
                                        "sum_copyback_us", "sum_deliver_us", "sum_latency_us")]


_bound = False


def _bind():
    global _bound
    if _bound:
        return lib()
    L = lib()
    L.pxt_server_create.argtypes = [ctypes.POINTER(PxtConfig), ctypes.POINTER(ServerConfig),
                                    ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    L.pxt_submit.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [
        ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]
    L.pxt_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(EventTracks),
                           ctypes.c_int]
    L.pxt_server_get_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ServerStats)]
    L.pxt_server_replay.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_uint32] + [ctypes.c_void_p] * 5 + \
        [ctypes.POINTER(EventTracks)]
    L.pxt_server_destroy.argtypes = [ctypes.c_void_p]
    L.pxt_server_destroy.restype = None
    _bound = True
    return L


class Server:
    """A libpxt server on one GPU.  Capacities are per lane."""

    def __init__(self, det, device=0, n_lanes=4, queue_depth=65536, max_batch_events=64,
                 doublets_per_hit=40, max_tracks_per_event=1 << 16, **caps):
        L = _bind()
        caps.setdefault("use_graph", 1)
        self.cfg = make_config(det, **caps)
        sc = ServerConfig(n_lanes, queue_depth, max_batch_events, doublets_per_hit)
        h = ctypes.c_void_p()
        st = L.pxt_server_create(ctypes.byref(self.cfg), ctypes.byref(sc), device,
                                 ctypes.byref(h))
        if st != OK:
            raise PxtError(st, "pxt_server_create")
        self.h = h
        self.cap = int(max_tracks_per_event)
        self._tls = threading.local()

    def _buffers(self):
        b = getattr(self._tls, "buf", None)
        if b is None:
            c = self.cap
            b = dict(hit_idx=np.zeros((c, 8), np.uint32), n_hits=np.zeros(c, np.uint8),
                     params=np.zeros((c, 5), np.float32), cov=np.zeros((c, 15), np.float32),
                     chi2=np.zeros((c, 2), np.float32), flags=np.zeros(c, np.uint8))
            self._tls.buf = b
        return b

    def submit(self, x, y, z, layer):
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        z = np.ascontiguousarray(z, np.float32)
        layer = np.ascontiguousarray(layer, np.int16)
        t = ctypes.c_uint64()
        st = lib().pxt_submit(self.h, x.ctypes.data, y.ctypes.data, z.ctypes.data,
                              layer.ctypes.data, x.shape[0], ctypes.byref(t))
        if st != OK:
            raise PxtError(st, "pxt_submit")
        return t.value

    def poll(self, ticket, timeout_ms=-1):
        """Result of `ticket` (dict of numpy arrays and timings), or None on
        timeout."""
        b = self._buffers()
        et = EventTracks(self.cap, b["hit_idx"].ctypes.data, b["n_hits"].ctypes.data,
                         b["params"].ctypes.data, b["cov"].ctypes.data, b["chi2"].ctypes.data,
                         b["flags"].ctypes.data, 0, 0, 0.0, 0.0, 0)
        st = lib().pxt_poll(self.h, ticket, ctypes.byref(et), timeout_ms)
        if st == ERR_CAPACITY:
            # this thread's buffers are too small for the event: grow them
            # and poll again (the ticket is still valid)
            self.cap = max(self.cap, int(et.n_tracks))
            self._tls.buf = None
            return self.poll(ticket, timeout_ms)
        if st == ERR_NOT_READY:
            return None
        if st != OK:
            raise PxtError(st, "pxt_poll")
        n = et.n_tracks if et.status == OK else 0
        return dict(status=et.status, n_tracks=et.n_tracks, latency_us=et.latency_us,
                    queue_us=et.queue_us, batch_events=et.batch_events,
                    hit_idx=b["hit_idx"][:n].copy(), n_hits=b["n_hits"][:n].copy(),
                    params=b["params"][:n].copy(), cov=b["cov"][:n].copy(),
                    chi2=b["chi2"][:n].copy(), flags=b["flags"][:n].copy())

    def stats(self):
        s = ServerStats()
        lib().pxt_server_get_stats(self.h, ctypes.byref(s))
        return {n: getattr(s, n) for n, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().pxt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def phase_means(before, after):
    """Mean time per event in each serving phase between two stats()
    snapshots (us): queued, staging and launch, device, copy-back,
    delivery, whole latency."""
    dc = max(after["completed"] - before["completed"], 1)
    dd = max(after["delivered"] - before["delivered"], 1)
    out = {k: (after["sum_%s_us" % k] - before["sum_%s_us" % k]) / dc
           for k in ("queue", "launch", "device", "copyback")}
    out.update({k: (after["sum_%s_us" % k] - before["sum_%s_us" % k]) / dd
                for k in ("deliver", "latency")})
    return {k: round(v, 2) for k, v in out.items()}


def replay(srv, pool, event_of_arrival, arrival_us):
    """Native open-loop replay (pxt_server_replay): arrival i submits
    pool[event_of_arrival[i]] at arrival_us[i] from a native thread while a
    second native thread releases the results in arrival order.  Returns
    latency percentiles (us, from the scheduled arrival), sustained
    events/s, mean batch size and the mean time per serving phase."""
    L = _bind()
    offs = np.zeros(len(pool) + 1, np.uint32)
    offs[1:] = np.cumsum([e.n_hits for e in pool])
    cat = lambda f, dt: np.ascontiguousarray(np.concatenate([getattr(e, f) for e in pool]), dt)
    x, y, z, lay = cat("x", np.float32), cat("y", np.float32), cat("z", np.float32), \
        cat("layer", np.int16)
    ev = np.ascontiguousarray(event_of_arrival, np.uint32)
    at = np.ascontiguousarray(arrival_us, np.float64)
    n = ev.shape[0]
    res = (EventTracks * n)()
    before = srv.stats()
    t0 = time.perf_counter()
    st = L.pxt_server_replay(srv.h, n, ev.ctypes.data, at.ctypes.data, len(pool),
                             offs.ctypes.data, x.ctypes.data, y.ctypes.data, z.ctypes.data,
                             lay.ctypes.data, res)
    wall = time.perf_counter() - t0
    if st != OK:
        raise PxtError(st, "pxt_server_replay")
    after = srv.stats()
    lat = np.array([r.latency_us for r in res])
    bsz = np.array([r.batch_events for r in res])
    return dict(events=n, wall_s=wall, events_per_s=n / wall,
                p50_us=float(np.percentile(lat, 50)), p99_us=float(np.percentile(lat, 99)),
                mean_us=float(lat.mean()), mean_batch=float(bsz.mean()),
                max_batch=int(bsz.max()), failed=int(sum(r.status != OK for r in res)),
                n_tracks=[int(r.n_tracks) for r in res], phases_us=phase_means(before, after))


def poisson_schedule(n, rate_hz, n_pool, seed=0):
    """Arrival times (us) of n Poisson arrivals at rate_hz, cycling over a
    pool of n_pool events; rate_hz = inf: all at once (a saturating
    burst)."""
    rng = np.random.default_rng(seed)
    if np.isinf(rate_hz):
        at = np.zeros(n)
    else:
        at = np.cumsum(rng.exponential(1e6 / rate_hz, n))
    return np.arange(n) % n_pool, at


def poisson_run(srv, events, rate_hz, seed=0, keep_results=False):
    """Submit `events` with exponential inter-arrival times at `rate_hz`
    (one arrival thread) while a collector thread polls the results.
    Returns latency percentiles (us), sustained events/s and the results."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, len(events))
    tickets = [None] * len(events)
    results = [None] * len(events)
    submitted = threading.Event()
    order = []
    lock = threading.Lock()

    def arrivals():
        t_next = time.perf_counter()
        for i, ev in enumerate(events):
            t_next += gaps[i]
            while True:
                now = time.perf_counter()
                if now >= t_next:
                    break
                if t_next - now > 2e-4:
                    time.sleep(min(t_next - now - 1e-4, 1e-3))
            while True:
                try:
                    tickets[i] = srv.submit(ev.x, ev.y, ev.z, ev.layer)
                    break
                except PxtError as e:
                    if e.status != ERR_BUSY:
                        raise
                    time.sleep(1e-4)
            with lock:
                order.append(i)
        submitted.set()

    def collector():
        k = 0
        while k < len(events):
            with lock:
                ready = k < len(order)
                i = order[k] if ready else None
            if not ready:
                time.sleep(5e-5)
                continue
            r = srv.poll(tickets[i], -1)
            results[i] = r if keep_results else {kk: r[kk] for kk in
                                                  ("status", "n_tracks", "latency_us",
                                                   "queue_us", "batch_events")}
            k += 1

    t0 = time.perf_counter()
    ta = threading.Thread(target=arrivals)
    tc = threading.Thread(target=collector)
    ta.start()
    tc.start()
    ta.join()
    tc.join()
    wall = time.perf_counter() - t0
    lat = np.array([r["latency_us"] for r in results])
    bsz = np.array([r["batch_events"] for r in results])
    return dict(events=len(events), wall_s=wall, events_per_s=len(events) / wall,
                offered_rate_hz=rate_hz, p50_us=float(np.percentile(lat, 50)),
                p99_us=float(np.percentile(lat, 99)), mean_us=float(lat.mean()),
                mean_batch=float(bsz.mean()), failed=int(sum(r["status"] != OK for r in results)),
                results=results)
