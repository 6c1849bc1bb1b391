"""Seeded synthetic helical-track events for the pixel reconstruction path.

The paper measures on simulated CMS top-pair events at an average pileup of
50 (Sec. 2); that data set is not available, so seeded synthetic events with
the same structure stand in for it: prompt charged helices in a 3.8 T field
crossing a four-layer barrel and three disks per side, with hit smearing,
Highland multiple scattering, hit inefficiency and uniform noise hits.

This module only manufactures inputs (and the truth they were made from).  It
contains none of the reconstruction's arithmetic; both the HIP library and the
CPU oracle take its output as input.  Everything is computed in float64 and
rounded to float32 coordinates and int16 layer ids at the end, then shuffled.

    ev = generate("pu50", seed=7)
    ev.x, ev.y, ev.z      float32[n_hits]
    ev.layer              int16[n_hits]
    ev.track_of_hit       int32[n_hits]  (-1 for noise)
    ev.tracks             dict of float64/int arrays per track (truth)
    ev.track_hits         list of int arrays: hit indices in crossing order
"""

from dataclasses import dataclass, field
import numpy as np

from .detector import (DETECTOR, WORKLOADS, BARREL, DISK, BATCH_TRACKS,
                       SERVE_PILEUP, SERVE_TRACKS_PER_PU)

__all__ = ["DETECTOR", "WORKLOADS", "Event", "generate", "generate_custom",
           "make_batch", "concat_events", "workload_params", "BARREL", "DISK"]

_WORKLOAD_IDS = {"tiny": 1, "pu50": 2, "batch": 3, "serve": 4, "pu200": 5, "vertex": 6}


@dataclass
class Event:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    layer: np.ndarray
    track_of_hit: np.ndarray
    tracks: dict = field(default_factory=dict)
    track_hits: list = field(default_factory=list)
    name: str = ""
    seed: int = 0

    @property
    def n_hits(self):
        return int(self.x.shape[0])


def _layer_table(det):
    return {l["id"]: l for l in det["layers"]}


def _advance(px, py, phi, kappa, s):
    """Transverse position after an arc of length s (numerically stable)."""
    h = 0.5 * kappa * s
    sinc = np.where(np.abs(h) < 1e-8, 1.0 - h * h / 6.0,
                    np.sin(h) / np.where(h == 0.0, 1.0, h))
    ang = phi + h
    return px + s * sinc * np.cos(ang), py + s * sinc * np.sin(ang)


def _arc_to_radius(px, py, phi, kappa, r_target):
    """Smallest positive transverse arc length reaching radius r_target.

    Bisection on [0, s_hi]; the radius grows monotonically over the first
    half turn, which is where every crossing of this detector lies.
    """
    n = px.shape[0]
    big = np.where(np.abs(kappa) > 0, np.pi / np.maximum(np.abs(kappa), 1e-300), 1e9)
    s_hi = np.minimum(big, 100.0)
    s_lo = np.zeros(n)
    for _ in range(90):
        mid = 0.5 * (s_lo + s_hi)
        qx, qy = _advance(px, py, phi, kappa, mid)
        inside = qx * qx + qy * qy < r_target * r_target
        s_lo = np.where(inside, mid, s_lo)
        s_hi = np.where(inside, s_hi, mid)
    return 0.5 * (s_lo + s_hi)


def _scatter(rng, phi, cot, p, cos_inc, x_over_x0):
    """Apply two independent Highland-distributed deflections (beta = 1)."""
    x = x_over_x0 / np.maximum(np.abs(cos_inc), 1e-3)
    theta0 = 0.0136 / p * np.sqrt(x) * (1.0 + 0.038 * np.log(x))
    n = phi.shape[0]
    g1 = rng.standard_normal(n) * theta0
    g2 = rng.standard_normal(n) * theta0
    st = 1.0 / np.sqrt(1.0 + cot * cot)
    ct = cot * st
    cphi, sphi = np.cos(phi), np.sin(phi)
    dx, dy, dz = st * cphi, st * sphi, ct
    e1 = (-sphi, cphi, np.zeros(n))
    e2 = (-ct * cphi, -ct * sphi, st)
    nx = dx + g1 * e1[0] + g2 * e2[0]
    ny = dy + g1 * e1[1] + g2 * e2[1]
    nz = dz + g1 * e1[2] + g2 * e2[2]
    nt = np.sqrt(nx * nx + ny * ny)
    return np.arctan2(ny, nx), nz / nt


def workload_params(name, rng=None):
    """Recipe dict of a named workload ('tiny', 'pu50', 'pu200')."""
    return dict(WORKLOADS[name])


def generate_custom(params, rng, det=DETECTOR, name="custom", seed=0):
    """Generate one event from an explicit recipe dict and a numpy Generator."""
    lt = _layer_table(det)
    c_kappa = det["c_kappa"]
    fitc = det["fit"]
    nt = int(params["n_tracks"])
    layers = tuple(params["layers"])
    barrels = [l for l in sorted(layers) if lt[l]["kind"] == BARREL]
    barrels.sort(key=lambda l: lt[l]["r"])
    disks_pos = sorted([l for l in layers if lt[l]["kind"] == DISK and lt[l]["z"] > 0],
                       key=lambda l: lt[l]["z"])
    disks_neg = sorted([l for l in layers if lt[l]["kind"] == DISK and lt[l]["z"] < 0],
                       key=lambda l: -lt[l]["z"])

    # --- track kinematics -------------------------------------------------
    nv = max(1, int(params["n_vertices"]))
    vz = rng.normal(0.0, params["vertex_sigma"], nv)
    vtx_of_track = rng.integers(0, nv, nt)
    zv = vz[vtx_of_track]
    if params["pt_spectrum"] == "loguniform":
        pt = np.exp(rng.uniform(np.log(params["pt_lo"]), np.log(params["pt_hi"]), nt))
    else:  # dN/dpT ~ pT^-3 above pt_lo, capped
        u = rng.uniform(0.0, 1.0, nt)
        pt = np.minimum(params["pt_lo"] / np.sqrt(1.0 - u), params["pt_hi"])
    eta = rng.uniform(-params["eta_max"], params["eta_max"], nt)
    if params.get("phi_spacing"):
        phi = rng.uniform(-np.pi, np.pi) + 2.0 * np.pi * np.arange(nt) / nt
        phi = np.mod(phi + np.pi, 2.0 * np.pi) - np.pi
    else:
        phi = rng.uniform(-np.pi, np.pi, nt)
    q = np.where(rng.uniform(0.0, 1.0, nt) < 0.5, -1.0, 1.0)
    cot = np.sinh(eta)
    p_tot = pt * np.sqrt(1.0 + cot * cot)
    truth = dict(pt=pt.copy(), q=q.copy(), phi=phi.copy(), cot=cot.copy(),
                 zv=zv.copy(), eta=eta.copy(), vertex=vtx_of_track.copy(),
                 vertex_z=vz.copy())

    # --- propagation ------------------------------------------------------
    px = np.zeros(nt)
    py = np.zeros(nt)
    pz = zv.copy()
    cur_phi = phi.copy()
    cur_cot = cot.copy()
    kappa = -q * c_kappa / pt
    alive = np.ones(nt, dtype=bool)
    hx, hy, hz, hl, ht = [], [], [], [], []
    eff = params["efficiency"]
    do_smear = params["smear"]
    do_ms = params["scatter"]

    def record(mask, x, y, z, lid):
        keep = mask & (rng.uniform(0.0, 1.0, nt) < eff) if eff < 1.0 else mask.copy()
        idx = np.nonzero(keep)[0]
        if idx.size == 0:
            return
        xs, ys, zs = x[idx].copy(), y[idx].copy(), z[idx].copy()
        if do_smear:
            r = np.hypot(xs, ys)
            ph = np.arctan2(ys, xs)
            if lt[lid]["kind"] == BARREL:
                ph = ph + rng.standard_normal(idx.size) * fitc["sigma_u"] / r
                zs = zs + rng.standard_normal(idx.size) * fitc["sigma_z"]
                rr = r
            else:
                ph = ph + rng.standard_normal(idx.size) * fitc["sigma_u"] / r
                rr = r + rng.standard_normal(idx.size) * fitc["sigma_r"]
            xs, ys = rr * np.cos(ph), rr * np.sin(ph)
        hx.append(xs); hy.append(ys); hz.append(zs)
        hl.append(np.full(idx.size, lid, dtype=np.int16)); ht.append(idx.astype(np.int32))

    def set_state(mask, s):
        nonlocal px, py, pz
        qx, qy = _advance(px, py, cur_phi, kappa, s)
        px = np.where(mask, qx, px)
        py = np.where(mask, qy, py)
        pz = np.where(mask, pz + cur_cot * s, pz)
        cur_phi[:] = np.where(mask, cur_phi + kappa * s, cur_phi)

    n_crossed = np.zeros(nt, dtype=np.int64)
    skip_first = not params.get("scatter_first", True)

    def apply_ms(mask, cos_inc):
        nonlocal kappa
        first = n_crossed == 0
        n_crossed[mask] += 1
        if not do_ms:
            return
        if skip_first:
            # no material at a track's first crossing: the fitted direction at
            # the first hit is then the production direction
            mask = mask & ~first
        nphi, ncot = _scatter(rng, cur_phi, cur_cot, p_tot, cos_inc, fitc["x_over_x0"])
        cur_phi[:] = np.where(mask, nphi, cur_phi)
        cur_cot[:] = np.where(mask, ncot, cur_cot)
        pt_new = p_tot / np.sqrt(1.0 + cur_cot * cur_cot)
        kappa = np.where(mask, -q * c_kappa / pt_new, kappa)

    in_barrel = alive.copy()
    for lid in barrels:
        L = lt[lid]
        s = _arc_to_radius(px, py, cur_phi, kappa, L["r"])
        zc = pz + cur_cot * s
        hit = in_barrel & (np.abs(zc) < L["zmax"])
        in_barrel &= hit
        set_state(hit, s)
        record(hit, px, py, pz, lid)
        rr = np.maximum(np.hypot(px, py), 1e-12)
        st = 1.0 / np.sqrt(1.0 + cur_cot * cur_cot)
        cos_inc = st * (np.cos(cur_phi) * px + np.sin(cur_phi) * py) / rr
        apply_ms(hit, cos_inc)

    for disks, sgn in ((disks_pos, 1.0), (disks_neg, -1.0)):
        going = alive & (np.sign(cur_cot) == sgn) & (cur_cot != 0.0)
        r_out = max(lt[l]["rmax"] for l in disks) if disks else 0.0
        for lid in disks:
            L = lt[lid]
            s = np.where(going, (L["z"] - pz) / np.where(cur_cot == 0.0, 1.0, cur_cot), 0.0)
            # the disk must be reached before the track leaves the tracker
            # radially (no re-entry of loopers)
            s_exit = _arc_to_radius(px, py, cur_phi, kappa, r_out)
            going &= s <= s_exit
            ok = going & (s > 0.0)
            qx, qy = _advance(px, py, cur_phi, kappa, np.where(ok, s, 0.0))
            rc = np.hypot(qx, qy)
            hit = ok & (rc >= L["rmin"]) & (rc <= L["rmax"])
            gone = ok & (rc > L["rmax"])
            set_state(ok, np.where(ok, s, 0.0))
            record(hit, px, py, pz, lid)
            st = 1.0 / np.sqrt(1.0 + cur_cot * cur_cot)
            apply_ms(hit, cur_cot * st)
            going &= ~gone

    if hx:
        sx = np.concatenate(hx); sy = np.concatenate(hy); sz = np.concatenate(hz)
        sl = np.concatenate(hl); st_ = np.concatenate(ht)
    else:
        sx = sy = sz = np.zeros(0); sl = np.zeros(0, np.int16); st_ = np.zeros(0, np.int32)

    # --- noise ------------------------------------------------------------
    n_noise = int(round(params["noise_fraction"] * sx.shape[0]))
    if n_noise > 0:
        areas = []
        for lid in layers:
            L = lt[lid]
            if L["kind"] == BARREL:
                areas.append(2.0 * np.pi * L["r"] * 2.0 * L["zmax"])
            else:
                areas.append(np.pi * (L["rmax"] ** 2 - L["rmin"] ** 2))
        areas = np.array(areas) / np.sum(areas)
        which = rng.choice(len(layers), size=n_noise, p=areas)
        nph = rng.uniform(-np.pi, np.pi, n_noise)
        nx = np.zeros(n_noise); ny = np.zeros(n_noise); nz = np.zeros(n_noise)
        nl = np.zeros(n_noise, np.int16)
        for k, lid in enumerate(layers):
            m = which == k
            cnt = int(m.sum())
            if cnt == 0:
                continue
            L = lt[lid]
            if L["kind"] == BARREL:
                r = np.full(cnt, L["r"])
                nz[m] = rng.uniform(-L["zmax"], L["zmax"], cnt)
            else:
                r = np.sqrt(rng.uniform(L["rmin"] ** 2, L["rmax"] ** 2, cnt))
                nz[m] = L["z"]
            nx[m] = r * np.cos(nph[m]); ny[m] = r * np.sin(nph[m]); nl[m] = lid
        sx = np.concatenate([sx, nx]); sy = np.concatenate([sy, ny])
        sz = np.concatenate([sz, nz]); sl = np.concatenate([sl, nl])
        st_ = np.concatenate([st_, np.full(n_noise, -1, np.int32)])

    # --- float32 rounding and shuffle ---------------------------------------
    perm = rng.permutation(sx.shape[0])
    x = sx[perm].astype(np.float32)
    y = sy[perm].astype(np.float32)
    z = sz[perm].astype(np.float32)
    layer = sl[perm].astype(np.int16)
    toh = st_[perm].astype(np.int32)

    # truth hit lists in crossing order (increasing radius along the track)
    order = np.argsort(toh, kind="stable")
    hits_sorted = order[toh[order] >= 0]
    tk = toh[hits_sorted]
    track_hits = [np.zeros(0, np.int64) for _ in range(nt)]
    if hits_sorted.size:
        bounds = np.searchsorted(tk, np.arange(nt + 1))
        r64 = np.hypot(x.astype(np.float64), y.astype(np.float64))
        for t in range(nt):
            h = hits_sorted[bounds[t]:bounds[t + 1]]
            track_hits[t] = h[np.argsort(r64[h], kind="stable")]
    return Event(x=x, y=y, z=z, layer=layer, track_of_hit=toh, tracks=truth,
                 track_hits=track_hits, name=name, seed=seed)


def generate(name, seed, n_tracks=None, det=DETECTOR, **overrides):
    """Generate event `seed` of workload `name` ('tiny', 'pu50', 'pu200').

    The stream is numpy.random.default_rng([workload id, seed]).
    """
    params = workload_params(name)
    if n_tracks is not None:
        params["n_tracks"] = int(n_tracks)
        if name != "tiny":
            params["n_vertices"] = max(1, int(round(n_tracks / 150.0)))
    params.update(overrides)
    rng = np.random.default_rng([_WORKLOAD_IDS[name], int(seed)])
    return generate_custom(params, rng, det=det, name=name, seed=seed)


def make_batch(kind, n_events, seed, det=DETECTOR):
    """A list of events of a ragged mix.

    kind = 'batch'  : track count U{300..3000}, pu50 distributions
    kind = 'serve'  : PU U{30..140}, 30 tracks per PU unit
    kind = 'pu50' / 'pu200' / 'tiny' : fixed-size events, seeds seed..seed+n-1
    """
    if kind in ("pu50", "pu200", "tiny"):
        return [generate(kind, seed * 100003 + i, det=det) for i in range(n_events)]
    rng = np.random.default_rng([_WORKLOAD_IDS[kind], int(seed), 0])
    events = []
    for i in range(n_events):
        if kind == "batch":
            ntr = int(rng.integers(BATCH_TRACKS[0], BATCH_TRACKS[1] + 1))
        elif kind == "serve":
            ntr = SERVE_TRACKS_PER_PU * int(rng.integers(SERVE_PILEUP[0], SERVE_PILEUP[1] + 1))
        else:
            raise ValueError(kind)
        params = workload_params("pu50")
        params["n_tracks"] = ntr
        params["n_vertices"] = max(1, int(round(ntr / 150.0)))
        erng = np.random.default_rng([_WORKLOAD_IDS[kind], int(seed), i + 1])
        events.append(generate_custom(params, erng, det=det, name=kind, seed=i))
    return events


def concat_events(events):
    """Concatenate events into one ragged SoA batch.

    Returns (x, y, z, layer, offsets) with offsets uint32[n_events + 1].
    """
    offs = np.zeros(len(events) + 1, dtype=np.uint32)
    offs[1:] = np.cumsum([e.n_hits for e in events])
    cat = lambda a: np.concatenate(a) if a else np.zeros(0)
    x = cat([e.x for e in events]).astype(np.float32)
    y = cat([e.y for e in events]).astype(np.float32)
    z = cat([e.z for e in events]).astype(np.float32)
    layer = cat([e.layer for e in events]).astype(np.int16)
    return x, y, z, layer, offs


def vertex_track_lists(seed, n_events=8, max_tracks=3000):
    """Seeded synthetic track lists for the vertex step alone (inputs only):
    per event, arrays z0, var(z0), q/pT (float32) and hit counts (uint8) of
    tracks drawn around a few vertices (z ~ N(0, 5 cm), track spread
    0.002-0.05 cm) plus uniform background, on a coarse 1/512 cm grid in
    every second event (exact distances and ties), with edge cases mixed in:
    an empty event, a one-track event, identical z0 values, +-0.0, NaN z0,
    zero and negative variances, 3-hit tracks and |q/pT| around the cut."""
    rng = np.random.default_rng([_WORKLOAD_IDS["vertex"], int(seed)])
    out = []
    for e in range(n_events):
        if e == 0:
            n = 0
        elif e == 1:
            n = 1
        else:
            n = int(rng.integers(2, max_tracks))
        nv = int(rng.integers(1, 41))
        vz = rng.normal(0.0, 5.0, nv)
        z = vz[rng.integers(0, nv, n)] + rng.normal(0.0, 1.0, n) * rng.uniform(0.002, 0.05, n)
        bg = rng.uniform(0.0, 1.0, n) < 0.2
        z[bg] = rng.uniform(-15.0, 15.0, int(bg.sum()))
        if e % 2 == 0:
            z = np.round(z * 512.0) / 512.0
        z = z.astype(np.float32)
        var = (rng.uniform(0.001, 0.03, n) ** 2).astype(np.float32)
        qopt = rng.uniform(-3.3, 3.3, n).astype(np.float32)
        nh = rng.integers(3, 7, n).astype(np.uint8)
        if n > 20:
            z[:6] = z[6]                       # identical values
            z[7] = np.float32(-0.0)
            z[8] = np.float32(0.0)
            z[9] = np.float32(np.nan)
            var[10] = 0.0
            var[11] = -1e-4
            qopt[12] = np.float32(2.0)          # exactly 1 / 0.5 GeV
            qopt[13] = np.nextafter(np.float32(2.0), np.float32(3.0))
        out.append(dict(z0=z, var=var, qopt=qopt, nhits=nh))
    return out
