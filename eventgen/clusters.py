"""Synthetic pixel modules and pixel clusters (inputs only).

The detector's layers are tiled with sensor modules, and every hit of a
generated event becomes a cluster of pixels on its module: the input of the
RecHits step, which turns clusters back into 3-D hits.  This module holds
the module table (detector conditions) and the cluster manufacturing; it
contains none of the RecHits arithmetic.

Module frames (all in cm):
* barrel ladder: a flat sensor tangent to the layer cylinder of radius r at
  azimuth phi_c (unit vectors n = (cos phi_c, sin phi_c), t = (-sin phi_c,
  cos phi_c)), centred at z = z_c; local u runs along t, v along z.  A hit
  at (r, phi, z) has u = r tan(phi - phi_c), v = z - z_c;
* disk wedge: a flat sensor in the disk plane z = z_D at azimuth phi_c,
  local u radial from the ring centre radius r_c, v along t.  A hit at
  (x, y) has u = x cos phi_c + y sin phi_c - r_c, v = -x sin phi_c +
  y cos phi_c.
Pixel (iu, iv) covers [u0 + iu pu, u0 + (iu + 1) pu) x [v0 + iv pv, ...).
"""

import numpy as np

from .detector import BARREL, DETECTOR

PITCH_U = 0.01      # cm
PITCH_V = 0.015     # cm
THICKNESS = 0.0285  # cm
LADDER_WIDTH = 1.6  # cm, nominal
BARREL_SEGMENTS = 8
DISK_RINGS = ((4.5, 10.25, 24), (10.25, 16.0, 48))  # (rmin, rmax, wedges)

# module table columns (float64): layer, kind, cos phi_c, sin phi_c, r, z,
# u0, v0, pitch_u, pitch_v (r: barrel radius / disk ring centre; z: centre z
# / disk z)
COLUMNS = ("layer", "kind", "cphi", "sphi", "r", "z", "u0", "v0", "pitch_u", "pitch_v")


def module_table(det=DETECTOR):
    """float64 [n_modules, 10] table, modules ordered by layer id, then
    azimuth sector, then z segment / ring."""
    rows = []
    meta = []
    for l in sorted(det["layers"], key=lambda l: l["id"]):
        if l["kind"] == BARREL:
            r = l["r"]
            nl = int(np.ceil(2 * np.pi * r / LADDER_WIDTH))
            half_u = r * np.tan(np.pi / nl) + PITCH_U
            nu = int(np.ceil(2 * half_u / PITCH_U))
            seg = 2 * l["zmax"] / BARREL_SEGMENTS
            nv = int(np.ceil(seg / PITCH_V))
            for k in range(nl):
                pc = 2 * np.pi * (k + 0.5) / nl
                for j in range(BARREL_SEGMENTS):
                    zc = -l["zmax"] + (j + 0.5) * seg
                    rows.append((l["id"], BARREL, np.cos(pc), np.sin(pc), r, zc,
                                 -nu * PITCH_U / 2, -nv * PITCH_V / 2, PITCH_U, PITCH_V))
                    meta.append((l["id"], k, j, nl))
        else:
            for ring, (r0, r1, nw) in enumerate(DISK_RINGS):
                rc = 0.5 * (r0 + r1)
                half_u = 0.5 * (r1 - r0) + PITCH_U
                half_v = r1 * np.tan(np.pi / nw) + PITCH_V
                nu = int(np.ceil(2 * half_u / PITCH_U))
                nv = int(np.ceil(2 * half_v / PITCH_V))
                for k in range(nw):
                    pc = 2 * np.pi * (k + 0.5) / nw
                    rows.append((l["id"], 1, np.cos(pc), np.sin(pc), rc, l["z"],
                                 -nu * PITCH_U / 2, -nv * PITCH_V / 2, PITCH_U, PITCH_V))
                    meta.append((l["id"], k, ring, nw))
    return np.array(rows, np.float64)


def _module_of(det, table, x, y, z, layer):
    """Module index of each hit (same order as module_table)."""
    phi = np.mod(np.arctan2(y, x), 2 * np.pi)
    r = np.hypot(x, y)
    first = {}
    for i, row in enumerate(table):
        first.setdefault(int(row[0]), i)
    out = np.zeros(x.shape[0], np.int64)
    for l in det["layers"]:
        m = layer == l["id"]
        if not m.any():
            continue
        base = first[l["id"]]
        if l["kind"] == BARREL:
            nl = int(np.ceil(2 * np.pi * l["r"] / LADDER_WIDTH))
            k = np.minimum((phi[m] / (2 * np.pi) * nl).astype(np.int64), nl - 1)
            seg = 2 * l["zmax"] / BARREL_SEGMENTS
            j = np.clip(((z[m] + l["zmax"]) / seg).astype(np.int64), 0, BARREL_SEGMENTS - 1)
            out[m] = base + k * BARREL_SEGMENTS + j
        else:
            off = 0
            idx = np.zeros(int(m.sum()), np.int64)
            rm = r[m]
            pm = phi[m]
            for ring, (r0, r1, nw) in enumerate(DISK_RINGS):
                inr = (rm >= r0) & (rm < r1) if ring + 1 < len(DISK_RINGS) else rm >= r0
                if ring == 0:
                    inr = rm < r1
                k = np.minimum((pm / (2 * np.pi) * nw).astype(np.int64), nw - 1)
                idx[inr] = base + off + k[inr]
                off += nw
            out[m] = idx
    return out


def make_clusters(ev, seed, det=DETECTOR, table=None, samples=48):
    """Pixel clusters of every hit of event `ev`, grouped by module in
    increasing module order (within a module, in input hit order).

    Returns a dict: module (uint16 [nc]), pixel_offsets (uint32 [nc + 1]),
    pix_u, pix_v (uint16), charge (uint16) and hit_of_cluster (int64 [nc],
    the input hit each cluster was made from).  The track is taken as coming
    straight from the origin through the hit: its path through the sensor
    thickness projects onto a segment in (u, v) around the hit's local
    position; `samples` points along it (each jittered by 3 um of
    diffusion) deposit charge in the pixels they fall in."""
    if table is None:
        table = module_table(det)
    rng = np.random.default_rng([7, int(seed)])
    x = ev.x.astype(np.float64)
    y = ev.y.astype(np.float64)
    z = ev.z.astype(np.float64)
    lay = ev.layer.astype(np.int64)
    valid = (lay >= 0) & (lay < len(det["layers"]))
    hits = np.nonzero(valid)[0]
    mod = _module_of(det, table, x[hits], y[hits], z[hits], lay[hits])
    order = np.lexsort((hits, mod))
    hits, mod = hits[order], mod[order]
    T = table[mod]
    cphi, sphi, rr, zz, u0, v0, pu, pv = (T[:, i] for i in range(2, 10))
    barrel = T[:, 1] == BARREL
    r_hit = np.hypot(x[hits], y[hits])
    # local position of the hit
    a = x[hits] * cphi + y[hits] * sphi        # along n
    b = -x[hits] * sphi + y[hits] * cphi       # along t
    u = np.where(barrel, rr * b / a, a - rr)
    v = np.where(barrel, z[hits] - zz, b)
    # projected path through the thickness, track from the origin
    du = np.where(barrel, THICKNESS * b / np.maximum(a, 1e-9),
                  THICKNESS * r_hit / np.maximum(np.abs(z[hits]), 1e-9))
    dv = np.where(barrel, THICKNESS * z[hits] / np.maximum(r_hit, 1e-9), 0.0)
    nu_max = np.round(-2 * u0 / pu).astype(np.int64)
    nv_max = np.round(-2 * v0 / pv).astype(np.int64)
    mods, offs, pus, pvs, qs = [], [0], [], [], []
    tt = (np.arange(samples) + 0.5) / samples - 0.5
    for i in range(hits.size):
        su = u[i] + tt * du[i] + rng.normal(0.0, 3e-4, samples)
        sv = v[i] + tt * dv[i] + rng.normal(0.0, 3e-4, samples)
        iu = np.clip(np.floor((su - u0[i]) / pu[i]).astype(np.int64), 0, nu_max[i] - 1)
        iv = np.clip(np.floor((sv - v0[i]) / pv[i]).astype(np.int64), 0, nv_max[i] - 1)
        key = iu * 65536 + iv
        k, cnt = np.unique(key, return_counts=True)
        mods.append(mod[i])
        pus.append(k // 65536)
        pvs.append(k % 65536)
        qs.append(cnt * 25 + rng.integers(0, 25, cnt.size))
        offs.append(offs[-1] + k.size)
    cat = lambda a, dt: (np.concatenate(a) if a else np.zeros(0)).astype(dt)
    return dict(module=np.array(mods, np.uint16), pixel_offsets=np.array(offs, np.uint32),
                pix_u=cat(pus, np.uint16), pix_v=cat(pvs, np.uint16),
                charge=cat(qs, np.uint16), hit_of_cluster=hits)
