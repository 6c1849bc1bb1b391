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
                                               "batches", "events_in_batches", "solo_retries")]


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
