"""CPU oracle of the pixel-track reconstruction path.

TEST INFRASTRUCTURE ONLY: this package is the independent reference the HIP
library is checked against.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import it; the product package never does.

Two tiers, sharing no code with the HIP library:

* ``pxt_oracle.c`` (built with gcc, FP64, ``-ffp-contract=off``): the whole
  path on one event by the plain definitions -- all hit pairs for doublets,
  all doublet pairs sharing a hit for links, recursive depth-first search
  for n-tuplets, per-doublet best-tuple cleaning, and the broken-line fit
  solved by Householder QR.  Wrapped here through ctypes.
* ``brute.py`` (numpy): O(n^2) doublets and O(n^3) triplets enumerated
  directly over hits, path growth by repeated extension, and the fit by a
  generic least-squares solve.  Used on tiny events to cross-check the C tier.
"""

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pxt_oracle.c")
_LIB = os.path.join(_HERE, "libpxt_oracle.so")
_lock = threading.Lock()
_lib = None

PAD = 0xFFFFFFFF
ITEMS = dict(doublets=0, links=1, raw=2, raw_score=3, keep=4, tracks=5,
             params=6, cov=7, chi2=8, kref=9)
_SHAPES = dict(doublets=(np.uint32, 2), links=(np.uint32, 3), raw=(np.uint32, 8),
               raw_score=(np.float64, 1), keep=(np.uint8, 1), tracks=(np.uint32, 8),
               params=(np.float64, 5), cov=(np.float64, 15), chi2=(np.float64, 2),
               kref=(np.float64, 1))

MAX_LAYERS = 16
MAX_PAIRS = 64


class Config(ctypes.Structure):
    _fields_ = [
        ("c_kappa", ctypes.c_double),
        ("n_layers", ctypes.c_int),
        ("layer_kind", ctypes.c_int * MAX_LAYERS),
        ("n_pairs", ctypes.c_int),
        ("pair_inner", ctypes.c_int * MAX_PAIRS),
        ("pair_outer", ctypes.c_int * MAX_PAIRS),
        ("kmax", ctypes.c_double), ("z0max", ctypes.c_double),
        ("arz", ctypes.c_double), ("d0max", ctypes.c_double),
        ("sigma_u", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("sigma_r", ctypes.c_double), ("x_over_x0", ctypes.c_double),
        ("pt_max", ctypes.c_double),
    ]


class VtxConfig(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("min_pts", ctypes.c_int), ("min_hits", ctypes.c_int),
                ("qopt_max", ctypes.c_float)]


def build(force=False):
    """Compile the C oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path):
    """ctypes handle of an oracle build at `path`, with its signatures set."""
    L = ctypes.CDLL(path)
    L.orc_run.restype = ctypes.c_void_p
    L.orc_run.argtypes = [ctypes.POINTER(Config), ctypes.c_uint32,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p]
    L.orc_status.argtypes = [ctypes.c_void_p]
    L.orc_count.restype = ctypes.c_uint64
    L.orc_count.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_data.restype = ctypes.c_void_p
    L.orc_data.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_free.argtypes = [ctypes.c_void_p]
    d = ctypes.c_double
    L.orc_doublet_ok.argtypes = [ctypes.POINTER(Config)] + [d] * 6
    L.orc_link_ok.argtypes = [ctypes.POINTER(Config)] + [d] * 9
    L.orc_link_terms.argtypes = [ctypes.POINTER(Config)] + [d] * 9 + [ctypes.c_void_p]
    L.orc_fit.argtypes = [ctypes.POINTER(Config), ctypes.c_int] + [ctypes.c_void_p] * 8
    L.orc_rechits.restype = ctypes.c_uint32
    L.orc_rechits.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                              ctypes.c_uint32] + [ctypes.c_void_p] * 12
    L.orc_vertices.restype = ctypes.c_int
    L.orc_vertices.argtypes = [ctypes.POINTER(VtxConfig), ctypes.c_uint32] + \
        [ctypes.c_void_p] * 9 + [ctypes.c_uint32]
    return L


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = load_library(_LIB)
    return _lib


def make_config(det):
    """ctypes config from the detector dictionary (eventgen.DETECTOR layout)."""
    c = Config()
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
    return c


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def reconstruct(x, y, z, layer, det, min_hits=None):
    """Run the whole path on one event.  Returns a dict of numpy arrays:

    doublets [Nd,2], links [Nl,3], raw [Nt,8], raw_score [Nt], keep [Nt],
    tracks [Nk,8], params [Nk,5], cov [Nk,15], chi2 [Nk,2], kref [Nk],
    status (0 ok, 1 path longer than 8 hits).  Hit indices are event-local
    input-order indices; tuples are padded with 0xFFFFFFFF.  Tracks (and
    their params, cov, chi2, kref) with fewer than min_hits hits are left
    out (default: the detector's quality.min_hits, else 3); the cleaning is
    the same, since a shorter n-tuplet never outranks a longer one.
    """
    L = lib()
    cfg = make_config(det)
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    layer = np.ascontiguousarray(layer, np.int16)
    r = L.orc_run(ctypes.byref(cfg), x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(layer))
    if not r:
        raise MemoryError("oracle allocation failed")
    try:
        out = {"status": L.orc_status(r)}
        for name, idx in ITEMS.items():
            dt, w = _SHAPES[name]
            n = L.orc_count(r, idx)
            p = L.orc_data(r, idx)
            if n == 0 or not p:
                a = np.zeros((0, w) if w > 1 else (0,), dtype=dt)
            else:
                nbytes = int(n) * w * np.dtype(dt).itemsize
                buf = (ctypes.c_char * nbytes).from_address(p)
                a = np.frombuffer(buf, dtype=dt).copy()
                a = a.reshape(int(n), w) if w > 1 else a
            out[name] = a
    finally:
        L.orc_free(r)
    if min_hits is None:
        min_hits = (det.get("quality") or {}).get("min_hits", 3)
    if min_hits > 3 and out["tracks"].shape[0]:
        keep = (out["tracks"] != PAD).sum(axis=1) >= min_hits
        for name in ("tracks", "params", "cov", "chi2", "kref"):
            out[name] = out[name][keep]
    return out


def fit(X, Y, Z, kind, det):
    """Broken-line fit of one hit tuple given in path order (float64 arrays).

    kind[i] = 0 barrel, 1 disk.  Returns (params[5], cov[15], chi2[2], kref).
    """
    L = lib()
    cfg = make_config(det)
    X = np.ascontiguousarray(X, np.float64)
    Y = np.ascontiguousarray(Y, np.float64)
    Z = np.ascontiguousarray(Z, np.float64)
    K = np.ascontiguousarray(kind, np.int32)
    p = np.zeros(5); cv = np.zeros(15); ch = np.zeros(2); kr = np.zeros(1)
    rc = L.orc_fit(ctypes.byref(cfg), int(X.shape[0]), _ptr(X), _ptr(Y), _ptr(Z),
                   _ptr(K), _ptr(p), _ptr(cv), _ptr(ch), _ptr(kr))
    if rc != 0:
        raise ValueError("oracle fit failed (%d)" % rc)
    return p, cv, ch, float(kr[0])


def doublet_ok(det, pi, po):
    cfg = make_config(det)
    return bool(lib().orc_doublet_ok(ctypes.byref(cfg), *map(float, pi), *map(float, po)))


def link_ok(det, pa, pb, pc):
    cfg = make_config(det)
    return bool(lib().orc_link_ok(ctypes.byref(cfg), *map(float, pa), *map(float, pb),
                                  *map(float, pc)))


def link_terms(det, pa, pb, pc):
    cfg = make_config(det)
    out = np.zeros(5)
    lib().orc_link_terms(ctypes.byref(cfg), *map(float, pa), *map(float, pb),
                         *map(float, pc), _ptr(out))
    return out


def unpack_cov(c15):
    """5x5 symmetric matrix from the packed lower triangle."""
    m = np.zeros((5, 5))
    k = 0
    for a in range(5):
        for b in range(a + 1):
            m[a, b] = m[b, a] = c15[k]
            k += 1
    return m


def canonical(tuples):
    """Sort rows lexicographically (canonical order of a set of tuples)."""
    t = np.asarray(tuples)
    if t.shape[0] == 0:
        return t
    keys = tuple(t[:, i] for i in range(t.shape[1] - 1, -1, -1))
    return t[np.lexsort(keys)]


def vtx_config(det):
    """Vertex-finding constants of the detector dictionary; qopt_max is
    1/pT_min rounded to single precision (the selection compares single
    precision values)."""
    v = det["vertex"]
    return VtxConfig(float(v["eps"]), int(v["min_pts"]), int(v["min_hits"]),
                     float(np.float32(1.0 / v["pt_min"])))


def vertices(z0, var, qopt, nhits, det=None, cfg=None):
    """Vertices of one event from its tracks' single-precision z0, var(z0),
    q/pT and hit counts (the reading is stated in pxt_oracle.c).  Returns a
    dict: z, z_err, chi2 (float64 [nv]), n_tracks (uint32 [nv]), assign
    (int32 [n], -1 for tracks in no vertex)."""
    L = lib()
    c = cfg if cfg is not None else vtx_config(det)
    z0 = np.ascontiguousarray(z0, np.float32)
    var = np.ascontiguousarray(var, np.float32)
    qopt = np.ascontiguousarray(qopt, np.float32)
    nhits = np.ascontiguousarray(nhits, np.uint8)
    n = z0.shape[0]
    assign = np.zeros(n, np.int32)
    cap = n + 1
    vz = np.zeros(cap); ve = np.zeros(cap); vc = np.zeros(cap)
    vn = np.zeros(cap, np.uint32)
    nv = L.orc_vertices(ctypes.byref(c), n, _ptr(z0), _ptr(var), _ptr(qopt), _ptr(nhits),
                        _ptr(assign), _ptr(vz), _ptr(ve), _ptr(vc), _ptr(vn), cap)
    return {"z": vz[:nv], "z_err": ve[:nv], "chi2": vc[:nv], "n_tracks": vn[:nv],
            "assign": assign}


def event_vertices(o, det):
    """Vertices of an event from the oracle's own reconstruction `o` (the
    dict of reconstruct()), its fitted values rounded to single precision
    as the library hands them over."""
    p = np.asarray(o["params"], np.float32)
    cv = np.asarray(o["cov"], np.float32)
    nh = (np.asarray(o["tracks"]) != PAD).sum(axis=1).astype(np.uint8)
    if p.shape[0] == 0:
        return vertices(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0), det)
    return vertices(p[:, 4], cv[:, 14], p[:, 2], nh, det)


def quality_flags(params, chi2, nhits, det):
    """Quality bits of fitted tracks (the reading stated with the library's
    flags): 2 = LOOSE, finite parameters and chi2 per degree of freedom at
    most the limit in both planes (transverse ndf n-3, at least 1;
    longitudinal n-2); 4 = STRICT, LOOSE with pT, |d0| and |z0| within their
    limits.  Decided in single precision on the values rounded to single
    precision, as the library hands them over."""
    q = det["quality"]
    p = np.asarray(params, np.float64).astype(np.float32).reshape(-1, 5)
    ch = np.asarray(chi2, np.float64).astype(np.float32).reshape(-1, 2)
    n = np.asarray(nhits, np.int64)
    ndf_c = np.maximum(n - 3, 1).astype(np.float32)
    ndf_z = (n - 2).astype(np.float32)
    lim = np.float32(q["chi2"])
    fin = np.all(np.isfinite(p), axis=1)
    with np.errstate(invalid="ignore"):
        loose = fin & (ch[:, 0] <= lim * ndf_c) & (ch[:, 1] <= lim * ndf_z)
        strict = (loose & (np.abs(p[:, 2]) <= np.float32(1.0 / float(np.float32(q["pt_min"]))))
                  & (np.abs(p[:, 1]) <= np.float32(q["d0_max"]))
                  & (np.abs(p[:, 4]) <= np.float32(q["z0_max"])))
    return (loose.astype(np.uint8) * 2) | (strict.astype(np.uint8) * 4)


def rechits(cl, table, max_per_module):
    """3-D hits of one event's clusters (the reading is stated in
    pxt_oracle.c).  cl: dict of module (uint16, grouped or not),
    pixel_offsets (uint32 [nc + 1], from 0), pix_u, pix_v, charge (uint16);
    table: float64 [n_modules, 10].  Returns a dict: module_start (uint32
    [n_modules + 1]), x, y, z (float32), layer (int16), module (uint16),
    cluster (uint32), one entry per hit in module order."""
    L = lib()
    table = np.ascontiguousarray(table, np.float64)
    nm = table.shape[0]
    mod = np.ascontiguousarray(cl["module"], np.uint16)
    nc = mod.shape[0]
    po = np.ascontiguousarray(cl["pixel_offsets"], np.uint32)
    pu = np.ascontiguousarray(cl["pix_u"], np.uint16)
    pv = np.ascontiguousarray(cl["pix_v"], np.uint16)
    q = np.ascontiguousarray(cl["charge"], np.uint16)
    ms = np.zeros(nm + 1, np.uint32)
    cap = max(nc, 1)
    x = np.zeros(cap, np.float32); y = np.zeros(cap, np.float32); z = np.zeros(cap, np.float32)
    lay = np.zeros(cap, np.int16); hm = np.zeros(cap, np.uint16); ch = np.zeros(cap, np.uint32)
    nh = L.orc_rechits(_ptr(table), nm, int(max_per_module), nc, _ptr(mod), _ptr(po), _ptr(pu),
                       _ptr(pv), _ptr(q), _ptr(ms), _ptr(x), _ptr(y), _ptr(z), _ptr(lay),
                       _ptr(hm), _ptr(ch))
    return dict(module_start=ms, x=x[:nh], y=y[:nh], z=z[:nh], layer=lay[:nh], module=hm[:nh],
                cluster=ch[:nh])
