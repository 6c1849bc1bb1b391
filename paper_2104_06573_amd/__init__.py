"""Python binding of libpxt, the MI355X pixel-track reconstruction core.

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of libpxt.so (built from csrc/ by ``build.py``).  PyTorch provides
device memory and the HIP stream; nothing is computed with it.  If the
library is missing or no GPU is present the calls raise -- there is no CPU
fallback.

    import eventgen, paper_2104_06573_amd as pxt
    rec = pxt.Reconstructor(eventgen.DETECTOR, max_events=1, max_hits=40000)
    ev = eventgen.generate("pu50", 1)
    out = rec.run_numpy([ev])          # uploads, runs, syncs
    out.hit_idx, out.params, out.cov, out.chi2, out.counts
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpxt.so")

MAX_LAYERS = 16
MAX_PAIRS = 32
PAD = 0xFFFFFFFF

OK, ERR_INVALID_ARG, ERR_CAPACITY, ERR_HIP, ERR_OOM, ERR_BUSY, ERR_PATH, ERR_NOT_READY = range(8)
DUMP_DOUBLETS, DUMP_LINKS, DUMP_RAW = 0, 1, 2

# every symbol include/pxt.h declares
EXPORTS = ("pxt_abi_version", "pxt_status_str", "pxt_last_error", "pxt_config_defaults",
           "pxt_create", "pxt_destroy", "pxt_reconstruct", "pxt_debug_dump",
           "pxt_set_timing", "pxt_stage_times", "pxt_stage_name",
           "pxt_server_create", "pxt_submit", "pxt_poll", "pxt_server_get_stats",
           "pxt_server_destroy", "pxt_reconstruct_static", "pxt_find_vertices",
           "pxt_rechits", "pxt_server_replay")
STATIC_SCRATCH_BYTES = 64 << 20
STATIC_MAX_EVENTS = 64
N_STAGES = 20
ABI_VERSION = 3  # layout of the structs below
VTX_MAX_TRACKS = 4096
FLAG_FP64, FLAG_LOOSE, FLAG_STRICT = 1, 2, 4


class PxtConfig(ctypes.Structure):
    _fields_ = [
        ("c_kappa", ctypes.c_double),
        ("n_layers", ctypes.c_int32),
        ("layer_kind", ctypes.c_int32 * MAX_LAYERS),
        ("n_pairs", ctypes.c_int32),
        ("pair_inner", ctypes.c_int32 * MAX_PAIRS),
        ("pair_outer", ctypes.c_int32 * MAX_PAIRS),
        ("kmax", ctypes.c_double), ("z0max", ctypes.c_double),
        ("arz", ctypes.c_double), ("d0max", ctypes.c_double),
        ("sigma_u", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("sigma_r", ctypes.c_double), ("x_over_x0", ctypes.c_double),
        ("pt_max", ctypes.c_double),
        ("max_events", ctypes.c_uint32), ("max_hits", ctypes.c_uint32),
        ("max_doublets", ctypes.c_uint32), ("max_link_words", ctypes.c_uint32),
        ("max_tuples", ctypes.c_uint32),
        ("phi_bins", ctypes.c_int32), ("block_size", ctypes.c_int32),
        ("group_lanes", ctypes.c_int32), ("link_kernel", ctypes.c_int32),
        ("use_graph", ctypes.c_int32), ("doublet_mode", ctypes.c_int32),
        ("pt_fp64", ctypes.c_double),
        ("min_hits", ctypes.c_int32), ("q_chi2", ctypes.c_float),
        ("q_pt_min", ctypes.c_float), ("q_d0_max", ctypes.c_float),
        ("q_z0_max", ctypes.c_float),
        ("vtx_eps", ctypes.c_double), ("vtx_min_pts", ctypes.c_int32),
        ("vtx_min_hits", ctypes.c_int32), ("vtx_pt_min", ctypes.c_double),
    ]


class PxtHits(ctypes.Structure):
    _fields_ = [
        ("n_events", ctypes.c_uint32),
        ("event_offsets", ctypes.c_void_p),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
        ("layer", ctypes.c_void_p), ("module", ctypes.c_void_p),
    ]


class PxtCounts(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("n_tracks", ctypes.c_uint32),
        ("n_doublets", ctypes.c_uint32), ("n_links", ctypes.c_uint32),
        ("n_raw_tuples", ctypes.c_uint32), ("n_fp64", ctypes.c_uint32),
        ("n_hits_binned", ctypes.c_uint32), ("n_link_words", ctypes.c_uint32),
        ("required", ctypes.c_uint64 * 4),
    ]


class PxtVertexSummary(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_vertices", ctypes.c_uint32),
                ("required_per_event", ctypes.c_uint32), ("max_selected", ctypes.c_uint32)]


class PxtVertices(ctypes.Structure):
    _fields_ = [
        ("max_per_event", ctypes.c_uint32),
        ("z", ctypes.c_void_p), ("z_err", ctypes.c_void_p), ("chi2", ctypes.c_void_p),
        ("n_tracks", ctypes.c_void_p), ("n_vertices", ctypes.c_void_p),
        ("track_vertex", ctypes.c_void_p), ("summary", ctypes.c_void_p),
    ]


class PxtTracks(ctypes.Structure):
    _fields_ = [
        ("capacity", ctypes.c_uint32),
        ("hit_idx", ctypes.c_void_p), ("n_hits", ctypes.c_void_p),
        ("event_id", ctypes.c_void_p), ("params", ctypes.c_void_p),
        ("cov", ctypes.c_void_p), ("chi2", ctypes.c_void_p),
        ("flags", ctypes.c_void_p), ("per_event_tracks", ctypes.c_void_p),
        ("counts", ctypes.c_void_p), ("vertices", ctypes.c_void_p),
    ]


class PxtClusters(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_uint32), ("n_clusters", ctypes.c_uint32),
                ("event_offsets", ctypes.c_void_p), ("module", ctypes.c_void_p),
                ("pixel_offsets", ctypes.c_void_p), ("pix_u", ctypes.c_void_p),
                ("pix_v", ctypes.c_void_p), ("charge", ctypes.c_void_p)]


class PxtRechitsOut(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint32), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("layer", ctypes.c_void_p), ("module", ctypes.c_void_p),
                ("cluster", ctypes.c_void_p), ("module_start", ctypes.c_void_p),
                ("hit_offsets", ctypes.c_void_p), ("status", ctypes.c_void_p)]


COUNTS_WORDS = ctypes.sizeof(PxtCounts) // 4

_lib = None


class PxtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("pxt status %d: %s" % (status, msg))
        self.status = status


def lib():
    """Load libpxt.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpxt.so not built: run python -m paper_2104_06573_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.pxt_abi_version.restype = ctypes.c_int
        if L.pxt_abi_version() != ABI_VERSION:
            raise ImportError("libpxt.so ABI %d, binding expects %d: rebuild"
                              % (L.pxt_abi_version(), ABI_VERSION))
        L.pxt_status_str.restype = ctypes.c_char_p
        L.pxt_status_str.argtypes = [ctypes.c_int]
        L.pxt_last_error.restype = ctypes.c_char_p
        L.pxt_last_error.argtypes = [ctypes.c_void_p]
        L.pxt_config_defaults.argtypes = [ctypes.POINTER(PxtConfig)]
        L.pxt_create.argtypes = [ctypes.POINTER(PxtConfig), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_void_p)]
        L.pxt_destroy.argtypes = [ctypes.c_void_p]
        L.pxt_destroy.restype = None
        L.pxt_reconstruct.argtypes = [ctypes.c_void_p, ctypes.POINTER(PxtHits),
                                      ctypes.POINTER(PxtTracks), ctypes.c_void_p]
        L.pxt_debug_dump.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.c_void_p]
        L.pxt_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.pxt_stage_times.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
        L.pxt_stage_name.restype = ctypes.c_char_p
        L.pxt_stage_name.argtypes = [ctypes.c_int]
        L.pxt_reconstruct_static.argtypes = [ctypes.POINTER(PxtConfig), ctypes.c_int,
                                             ctypes.POINTER(PxtHits), ctypes.POINTER(PxtTracks),
                                             ctypes.c_void_p]
        L.pxt_find_vertices.argtypes = [ctypes.POINTER(PxtConfig), ctypes.c_uint32,
                                        ctypes.POINTER(PxtTracks), ctypes.POINTER(PxtVertices),
                                        ctypes.c_void_p]
        L.pxt_rechits.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.POINTER(PxtClusters), ctypes.POINTER(PxtRechitsOut),
                                  ctypes.c_void_p]
        _lib = L
    return _lib


def stage_names():
    return [lib().pxt_stage_name(i).decode() for i in range(N_STAGES)]


def make_config(det, max_events=1, max_hits=1 << 16, max_doublets=1 << 21,
                max_link_words=None, max_tuples=1 << 19, phi_bins=256, block_size=256,
                group_lanes=8, link_kernel=0, use_graph=0, doublet_mode=2, pt_fp64=1e9,
                min_hits=None):
    """pxt_config from a detector dictionary (eventgen.DETECTOR layout)."""
    c = PxtConfig()
    if lib().pxt_config_defaults(ctypes.byref(c)) != OK:
        raise PxtError(ERR_INVALID_ARG, "pxt_config_defaults")
    c.c_kappa = det["c_kappa"]
    layers = sorted(det["layers"], key=lambda l: l["id"])
    c.n_layers = len(layers)
    for l in layers:
        c.layer_kind[l["id"]] = int(l["kind"])
    c.n_pairs = len(det["pairs"])
    for i, (a, b) in enumerate(det["pairs"]):
        c.pair_inner[i] = a
        c.pair_outer[i] = b
    cu, f = det["cuts"], det["fit"]
    c.kmax, c.z0max, c.arz, c.d0max = cu["kmax"], cu["z0max"], cu["arz"], cu["d0max"]
    c.sigma_u, c.sigma_z, c.sigma_r = f["sigma_u"], f["sigma_z"], f["sigma_r"]
    c.x_over_x0, c.pt_max = f["x_over_x0"], f["pt_max"]
    c.max_events = max_events
    c.max_hits = max_hits
    c.max_doublets = max_doublets
    c.max_link_words = (max_link_words if max_link_words is not None
                        else min(4 * max_doublets, 0xfffffff0))
    c.max_tuples = max_tuples
    c.phi_bins = phi_bins
    c.block_size = block_size
    c.group_lanes = group_lanes
    c.link_kernel = link_kernel
    c.use_graph = use_graph
    c.doublet_mode = doublet_mode
    c.pt_fp64 = pt_fp64
    q = det.get("quality")
    if q:
        c.min_hits = q["min_hits"] if min_hits is None else min_hits
        c.q_chi2, c.q_pt_min, c.q_d0_max, c.q_z0_max = (q["chi2"], q["pt_min"], q["d0_max"],
                                                        q["z0_max"])
    elif min_hits is not None:
        c.min_hits = min_hits
    v = det.get("vertex")
    if v:
        c.vtx_eps, c.vtx_min_pts = v["eps"], v["min_pts"]
        c.vtx_min_hits, c.vtx_pt_min = v["min_hits"], v["pt_min"]
    return c


class Result:
    """Outputs of one call (torch device tensors, sliced to n_tracks)."""

    def __init__(self, counts, per_event, hit_idx, n_hits, event_id, params, cov, chi2, flags):
        self.counts = counts
        self.per_event_tracks = per_event
        self.hit_idx = hit_idx
        self.n_hits = n_hits
        self.event_id = event_id
        self.params = params
        self.cov = cov
        self.chi2 = chi2
        self.flags = flags

    def numpy(self):
        import torch  # noqa: F401
        return {k: getattr(self, k).cpu().numpy() for k in
                ("hit_idx", "n_hits", "event_id", "params", "cov", "chi2", "flags",
                 "per_event_tracks")}


def counts_dict(words):
    c = PxtCounts.from_buffer_copy(np.ascontiguousarray(words, np.uint32).tobytes())
    return dict(status=c.status, n_tracks=c.n_tracks, n_doublets=c.n_doublets,
                n_links=c.n_links, n_raw_tuples=c.n_raw_tuples, n_fp64=c.n_fp64,
                n_hits_binned=c.n_hits_binned, n_words=c.n_link_words,
                required=list(c.required))


class VertexBuffers:
    """Device buffers of a pxt_vertices for n_events events and n_tracks
    tracks, V vertex slots per event."""

    def __init__(self, n_events, n_tracks, V, device):
        import torch as t
        self.V = V
        self.z = t.empty((n_events, V), dtype=t.float32, device=device)
        self.z_err = t.empty((n_events, V), dtype=t.float32, device=device)
        self.chi2 = t.empty((n_events, V), dtype=t.float32, device=device)
        self.n_tracks = t.empty((n_events, V), dtype=t.int32, device=device)
        self.n_vertices = t.empty(n_events, dtype=t.int32, device=device)
        self.track_vertex = t.empty(max(n_tracks, 1), dtype=t.int32, device=device)
        self.summary = t.empty(4, dtype=t.int32, device=device)
        self.struct = PxtVertices(V, self.z.data_ptr(), self.z_err.data_ptr(),
                                  self.chi2.data_ptr(), self.n_tracks.data_ptr(),
                                  self.n_vertices.data_ptr(), self.track_vertex.data_ptr(),
                                  self.summary.data_ptr())

    def read(self, n_events, n_tracks):
        """Host copy: summary dict, and per event a dict of z, z_err, chi2,
        n_tracks arrays; track_vertex of the n_tracks tracks."""
        sm = self.summary.cpu().numpy()
        summary = dict(status=int(sm[0]), n_vertices=int(sm[1].view(np.uint32)),
                       required_per_event=int(sm[2].view(np.uint32)),
                       max_selected=int(sm[3].view(np.uint32)))
        nv = self.n_vertices[:n_events].cpu().numpy()
        z, ze, ch, nt = (a[:n_events].cpu().numpy() for a in (self.z, self.z_err, self.chi2,
                                                              self.n_tracks))
        events = [dict(z=z[e, :nv[e]], z_err=ze[e, :nv[e]], chi2=ch[e, :nv[e]],
                       n_tracks=nt[e, :nv[e]]) for e in range(n_events)]
        return summary, events, self.track_vertex[:n_tracks].cpu().numpy()


def find_vertices(cfg, per_event_tracks, n_hits, params, cov, max_per_event, stream=None):
    """pxt_find_vertices on device tensors of tracks grouped by event
    (per_event_tracks int32 [E], n_hits uint8 [T], params float32 [T, 5],
    cov float32 [T, 15]); returns the VertexBuffers (read() for results)."""
    import torch as t
    E = int(per_event_tracks.shape[0])
    T = int(n_hits.shape[0])
    vb = VertexBuffers(max(E, 1), T, int(max_per_event), params.device)
    tr = PxtTracks(T, None, n_hits.data_ptr(), None, params.data_ptr(), cov.data_ptr(), None,
                   None, per_event_tracks.data_ptr(), None, None)
    st = stream or t.cuda.current_stream(params.device)
    rc = lib().pxt_find_vertices(ctypes.byref(cfg), E, ctypes.byref(tr), ctypes.byref(vb.struct),
                                 ctypes.c_void_p(st.cuda_stream))
    if rc != OK:
        raise PxtError(rc, lib().pxt_last_error(None).decode())
    return vb


def upload_clusters(clusters, device=0):
    """Concatenate per-event cluster dicts (module, pixel_offsets from 0,
    pix_u, pix_v, charge) into one device batch; returns a dict of device
    tensors (event_offsets, module, pixel_offsets, pix_u, pix_v, charge)
    and the host cluster offsets of the events."""
    import torch as t
    dev = t.device("cuda", device) if isinstance(device, int) else device
    nc = [len(c["module"]) for c in clusters]
    ev = np.zeros(len(clusters) + 1, np.uint32)
    ev[1:] = np.cumsum(nc)
    po = [np.zeros(1, np.uint32)]
    base = 0
    for c in clusters:
        po.append(np.asarray(c["pixel_offsets"][1:], np.int64) + base)
        base += int(c["pixel_offsets"][-1])
    cat = lambda k, dt: np.ascontiguousarray(
        np.concatenate([c[k] for c in clusters]) if clusters else np.zeros(0), dt)
    to = lambda a: t.from_numpy(a).to(dev)
    # uint16 arrays travel as int16 tensors (same bits)
    return dict(event_offsets=to(ev.view(np.int32)),
                module=to(cat("module", np.uint16).view(np.int16)),
                pixel_offsets=to(np.concatenate(po).astype(np.uint32).view(np.int32)),
                pix_u=to(cat("pix_u", np.uint16).view(np.int16)),
                pix_v=to(cat("pix_v", np.uint16).view(np.int16)),
                charge=to(cat("charge", np.uint16).view(np.int16))), ev


class RecHits:
    """Output buffers of pxt_rechits for up to max_events events of
    n_modules modules and `capacity` hits, with the module table on the
    device."""

    def __init__(self, table, max_events, capacity, device=0):
        import torch as t
        self.torch = t
        dev = t.device("cuda", device) if isinstance(device, int) else device
        self.table = t.from_numpy(np.ascontiguousarray(table, np.float64)).to(dev)
        self.n_modules = int(table.shape[0])
        self.capacity = int(capacity)
        C = max(self.capacity, 1)
        self.x = t.empty(C, dtype=t.float32, device=dev)
        self.y = t.empty(C, dtype=t.float32, device=dev)
        self.z = t.empty(C, dtype=t.float32, device=dev)
        self.layer = t.empty(C, dtype=t.int16, device=dev)
        self.module = t.empty(C, dtype=t.int16, device=dev)
        self.cluster = t.empty(C, dtype=t.int32, device=dev)
        self.module_start = t.empty(max_events * self.n_modules + 1, dtype=t.int32, device=dev)
        self.hit_offsets = t.empty(max_events + 1, dtype=t.int32, device=dev)
        self.status = t.empty(1, dtype=t.int32, device=dev)
        self.max_events = max_events
        self._out = PxtRechitsOut(self.capacity, self.x.data_ptr(), self.y.data_ptr(),
                                  self.z.data_ptr(), self.layer.data_ptr(),
                                  self.module.data_ptr(), self.cluster.data_ptr(),
                                  self.module_start.data_ptr(), self.hit_offsets.data_ptr(),
                                  self.status.data_ptr())

    def launch(self, dev_clusters, n_events, n_clusters, max_per_module, stream=None):
        if n_events > self.max_events:
            raise PxtError(ERR_INVALID_ARG, "more events than the buffers hold")
        d = dev_clusters
        cl = PxtClusters(n_events, n_clusters, d["event_offsets"].data_ptr(),
                         d["module"].data_ptr(), d["pixel_offsets"].data_ptr(),
                         d["pix_u"].data_ptr(), d["pix_v"].data_ptr(), d["charge"].data_ptr())
        st = stream or self.torch.cuda.current_stream(self.x.device)
        rc = lib().pxt_rechits(ctypes.c_void_p(self.table.data_ptr()), self.n_modules,
                               int(max_per_module), ctypes.byref(cl), ctypes.byref(self._out),
                               ctypes.c_void_p(st.cuda_stream))
        if rc != OK:
            raise PxtError(rc, lib().pxt_last_error(None).decode())

    def read(self, n_events):
        """Host copy: status, hit offsets per event, module_start, and the
        hits (x, y, z, layer, module, cluster) of all events."""
        status = int(self.status.cpu().numpy()[0])
        ho = self.hit_offsets[:n_events + 1].cpu().numpy().view(np.uint32).copy()
        ms = self.module_start[:n_events * self.n_modules + 1].cpu().numpy().view(np.uint32)
        n = int(ho[-1]) if status == OK else 0
        hits = dict(x=self.x[:n].cpu().numpy(), y=self.y[:n].cpu().numpy(),
                    z=self.z[:n].cpu().numpy(), layer=self.layer[:n].cpu().numpy(),
                    module=self.module[:n].cpu().numpy().view(np.uint16),
                    cluster=self.cluster[:n].cpu().numpy().view(np.uint32))
        return status, ho, ms.copy(), hits


def upload_events(events, device=0):
    """Concatenate host events (objects with x, y, z, layer arrays) into one
    ragged batch on the device; returns (x, y, z, layer, offsets) with the
    offsets on the host."""
    import torch as t
    dev = t.device("cuda", device) if isinstance(device, int) else device
    offs = np.zeros(len(events) + 1, dtype=np.uint32)
    offs[1:] = np.cumsum([len(e.x) for e in events])
    cat = lambda f, dt: t.from_numpy(np.ascontiguousarray(
        np.concatenate([getattr(e, f) for e in events]) if events else np.zeros(0), dt)).to(dev)
    return (cat("x", np.float32), cat("y", np.float32), cat("z", np.float32),
            cat("layer", np.int16), offs)


class Reconstructor:
    """One libpxt context on one GPU with its output buffers.

    max_tracks is the capacity of the output buffers (caller-owned in the C
    ABI; owned by this object here).
    """

    def __init__(self, det, device=0, max_tracks=1 << 18, max_vertices_per_event=0, **caps):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.cfg = make_config(det, **caps)
        h = ctypes.c_void_p()
        st = lib().pxt_create(ctypes.byref(self.cfg), device, ctypes.byref(h))
        if st != OK:
            raise PxtError(st, lib().pxt_last_error(None).decode())
        self.h = h
        self.max_tracks = int(max_tracks)
        E = int(self.cfg.max_events)
        T = self.max_tracks
        dev = self.device
        self.o_hit_idx = torch.empty((T, 8), dtype=torch.int32, device=dev)
        self.o_n_hits = torch.empty(T, dtype=torch.uint8, device=dev)
        self.o_event_id = torch.empty(T, dtype=torch.int32, device=dev)
        self.o_params = torch.empty((T, 5), dtype=torch.float32, device=dev)
        self.o_cov = torch.empty((T, 15), dtype=torch.float32, device=dev)
        self.o_chi2 = torch.empty((T, 2), dtype=torch.float32, device=dev)
        self.o_flags = torch.empty(T, dtype=torch.uint8, device=dev)
        self.o_per_event = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
        self.o_counts = torch.empty(COUNTS_WORDS, dtype=torch.int32, device=dev)
        self._tracks = PxtTracks(
            T, self.o_hit_idx.data_ptr(), self.o_n_hits.data_ptr(), self.o_event_id.data_ptr(),
            self.o_params.data_ptr(), self.o_cov.data_ptr(), self.o_chi2.data_ptr(),
            self.o_flags.data_ptr(), self.o_per_event.data_ptr(), self.o_counts.data_ptr(), None)
        self.vtx = None
        if max_vertices_per_event > 0:
            self.vtx = VertexBuffers(max(E, 1), T, int(max_vertices_per_event), dev)
            self._tracks.vertices = ctypes.addressof(self.vtx.struct)

    def close(self):
        if getattr(self, "h", None):
            lib().pxt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, stream):
        if stream is None:
            stream = self.torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    def launch(self, x, y, z, layer, offsets, stream=None):
        """Enqueue one call; x, y, z (float32), layer (int16) are device
        tensors, offsets a host uint32 array of n_events + 1 entries."""
        offs = np.ascontiguousarray(offsets, dtype=np.uint32)
        self._offs = offs
        hits = PxtHits(offs.shape[0] - 1, offs.ctypes.data, x.data_ptr(), y.data_ptr(),
                       z.data_ptr(), layer.data_ptr(), None)
        st = lib().pxt_reconstruct(self.h, ctypes.byref(hits), ctypes.byref(self._tracks),
                                   self._stream(stream))
        if st != OK:
            raise PxtError(st, lib().pxt_last_error(self.h).decode())
        return offs.shape[0] - 1

    def launch_static(self, x, y, z, layer, offsets, stream=None):
        """As launch(), through pxt_reconstruct_static: the same config and
        output buffers, arenas in the library's fixed device buffer instead
        of this object's context."""
        offs = np.ascontiguousarray(offsets, dtype=np.uint32)
        self._offs = offs
        hits = PxtHits(offs.shape[0] - 1, offs.ctypes.data, x.data_ptr(), y.data_ptr(),
                       z.data_ptr(), layer.data_ptr(), None)
        st = lib().pxt_reconstruct_static(ctypes.byref(self.cfg), self.device.index or 0,
                                          ctypes.byref(hits), ctypes.byref(self._tracks),
                                          self._stream(stream))
        if st != OK:
            raise PxtError(st, lib().pxt_last_error(None).decode())
        return offs.shape[0] - 1

    def read_counts(self):
        return counts_dict(self.o_counts.cpu().numpy().view(np.uint32))

    def result(self, n_events, counts=None):
        counts = counts or self.read_counts()
        n = counts["n_tracks"] if counts["status"] == OK else 0
        return Result(counts, self.o_per_event[:n_events], self.o_hit_idx[:n], self.o_n_hits[:n],
                      self.o_event_id[:n], self.o_params[:n], self.o_cov[:n], self.o_chi2[:n],
                      self.o_flags[:n])

    def run(self, x, y, z, layer, offsets, stream=None):
        n_events = self.launch(x, y, z, layer, offsets, stream)
        self.torch.cuda.synchronize(self.device)
        return self.result(n_events)

    def upload(self, events):
        """Concatenate host events (objects with x, y, z, layer arrays) into
        one ragged batch on the device; returns (x, y, z, layer, offsets)."""
        return upload_events(events, self.device)

    def run_numpy(self, events):
        x, y, z, layer, offs = self.upload(events)
        return self.run(x, y, z, layer, offs)

    def dump(self, what, stream=None):
        """Debug dump of the last call (rows of uint32, see pxt.h)."""
        width = {DUMP_DOUBLETS: 3, DUMP_LINKS: 4, DUMP_RAW: 9}[what]
        cnt = ctypes.c_uint64(0)
        st = lib().pxt_debug_dump(self.h, what, None, 0, ctypes.byref(cnt), self._stream(stream))
        if st != OK:
            raise PxtError(st, lib().pxt_last_error(self.h).decode())
        buf = np.zeros((int(cnt.value), width), dtype=np.uint32)
        st = lib().pxt_debug_dump(self.h, what, buf.ctypes.data, buf.shape[0], ctypes.byref(cnt),
                                  self._stream(stream))
        if st != OK:
            raise PxtError(st, lib().pxt_last_error(self.h).decode())
        return buf

    def set_timing(self, on):
        st = lib().pxt_set_timing(self.h, 1 if on else 0)
        if st != OK:
            raise PxtError(st, lib().pxt_last_error(self.h).decode())

    def last_stage_times(self):
        """Per-stage device durations (ms) of the last timed call."""
        buf = (ctypes.c_float * N_STAGES)()
        n = ctypes.c_int(0)
        st = lib().pxt_stage_times(self.h, buf, N_STAGES, ctypes.byref(n))
        if st != OK:
            raise PxtError(st, lib().pxt_last_error(self.h).decode())
        return dict(zip(stage_names(), [float(v) for v in buf[:n.value]]))

    def stage_times(self, batch, repeats=5):
        """Mean per-stage durations (ms) over `repeats` timed calls on the
        uploaded batch (x, y, z, layer, offsets)."""
        self.set_timing(True)
        acc = None
        try:
            for _ in range(repeats):
                self.launch(*batch)
                t = self.last_stage_times()
                acc = t if acc is None else {k: acc[k] + t[k] for k in acc}
        finally:
            self.set_timing(False)
        return {k: v / repeats for k, v in acc.items()}
