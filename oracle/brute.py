"""Brute-force numpy tier of the CPU oracle (tiny events only).

TEST INFRASTRUCTURE ONLY.  It recomputes the reconstruction of one event by
a route different from the C tier: doublets over the full O(n^2) hit-pair
matrix, links over the full O(n^3) hit-triple tensor, tuples by growing all
paths one link at a time, cleaning by a global sort, and the broken-line fit
by a generic least-squares solve (numpy.linalg.lstsq) instead of Householder
QR.  The cut formulas are the readings stated in pxt_oracle.c; they are
evaluated here with the same operation order in float64.
"""

import numpy as np

PAD = 0xFFFFFFFF


def _pair_mask(det, layer):
    n = layer.shape[0]
    m = np.zeros((n, n), dtype=bool)
    for a, b in det["pairs"]:
        m |= (layer[:, None] == a) & (layer[None, :] == b)
    return m


def doublets(x, y, z, layer, det):
    """All (i, o) with an allowed layer pair passing D1..D4; row-sorted."""
    X = x.astype(np.float64); Y = y.astype(np.float64); Z = z.astype(np.float64)
    R = np.sqrt(X * X + Y * Y)
    c = det["cuts"]
    Xi, Yi, Zi, Ri = X[:, None], Y[:, None], Z[:, None], R[:, None]
    Xo, Yo, Zo, Ro = X[None, :], Y[None, :], Z[None, :], R[None, :]
    d1 = Ro > Ri
    dr = Ro - Ri
    d2 = np.abs(Zi * dr - Ri * (Zo - Zi)) <= c["z0max"] * dr
    cr = Xi * Yo - Yi * Xo
    dx = Xo - Xi; dy = Yo - Yi
    chord = np.sqrt(dx * dx + dy * dy)
    d3 = 2.0 * np.abs(cr) <= c["kmax"] * Ri * Ro * chord
    d4 = Xi * Xo + Yi * Yo > 0.0
    ok = _pair_mask(det, layer) & d1 & d2 & d3 & d4
    i, o = np.nonzero(ok)
    return np.stack([i, o], axis=1).astype(np.uint32), ok


def _link_terms(X, Y, Z, a, b, c, det):
    cu = det["cuts"]
    Ra = np.sqrt(X[a] * X[a] + Y[a] * Y[a])
    Rb = np.sqrt(X[b] * X[b] + Y[b] * Y[b])
    Rc = np.sqrt(X[c] * X[c] + Y[c] * Y[c])
    dra = Rb - Ra; dza = Z[b] - Z[a]; drb = Rc - Rb; dzb = Z[c] - Z[b]
    t0 = np.abs(dra * dzb - dza * drb)
    lab = np.sqrt(dra * dra + dza * dza)
    lbc = np.sqrt(drb * drb + dzb * dzb)
    t1 = cu["arz"] * lab * lbc
    ux = X[b] - X[a]; uy = Y[b] - Y[a]; vx = X[c] - X[a]; vy = Y[c] - Y[a]
    wx = X[c] - X[b]; wy = Y[c] - Y[b]
    cr = ux * vy - uy * vx
    nab = np.sqrt(ux * ux + uy * uy)
    nac = np.sqrt(vx * vx + vy * vy)
    nbc = np.sqrt(wx * wx + wy * wy)
    t2 = 2.0 * np.abs(cr)
    t3 = cu["kmax"] * nab * nbc * nac
    D = 2.0 * cr
    uu = ux * ux + uy * uy; vv = vx * vx + vy * vy
    with np.errstate(divide="ignore", invalid="ignore"):
        ox = (vy * uu - uy * vv) / D
        oy = (ux * vv - vx * uu) / D
        Rr = np.sqrt(ox * ox + oy * oy)
        cx = X[a] + ox; cy = Y[a] + oy
        dc = np.sqrt(cx * cx + cy * cy)
        aa = X[a] * X[a] + Y[a] * Y[a]
        ao = X[a] * ox + Y[a] * oy
        d0 = np.abs(aa + 2.0 * ao) / (dc + Rr)
        dline = np.abs(X[a] * vy - Y[a] * vx) / nac
    d0 = np.where(D == 0.0, dline, d0)
    return t0, t1, t2, t3, d0


def links(x, y, z, layer, det, dmask):
    """All hit triples (a, b, c) with doublets (a,b), (b,c) passing L1..L3."""
    X = x.astype(np.float64); Y = y.astype(np.float64); Z = z.astype(np.float64)
    out = []
    for b in range(dmask.shape[0]):
        ia = np.nonzero(dmask[:, b])[0]
        ic = np.nonzero(dmask[b, :])[0]
        if ia.size == 0 or ic.size == 0:
            continue
        a = np.repeat(ia, ic.size)
        c = np.tile(ic, ia.size)
        bb = np.full(a.size, b)
        t0, t1, t2, t3, d0 = _link_terms(X, Y, Z, a, bb, c, det)
        ok = (t0 <= t1) & (t2 <= t3) & (d0 <= det["cuts"]["d0max"])
        out.append(np.stack([a[ok], bb[ok], c[ok]], axis=1))
    if not out:
        return np.zeros((0, 3), np.uint32)
    return np.concatenate(out).astype(np.uint32)


def tuples(D, L, max_hits=8):
    """All root-to-leaf paths of 3..max_hits hits, grown one link at a time."""
    dset = set(map(tuple, D.tolist()))
    nxt = {}
    has_inner = set()
    for a, b, c in L.tolist():
        nxt.setdefault((a, b), []).append(c)
        has_inner.add((b, c))
    frontier = [list(d) for d in dset if d not in has_inner]
    done = []
    while frontier:
        grown = []
        for p in frontier:
            last = (p[-2], p[-1])
            if last not in nxt:
                if len(p) >= 3:
                    done.append(p)
                continue
            if len(p) + 1 > max_hits:
                raise RuntimeError("path longer than %d hits" % max_hits)
            for c in nxt[last]:
                grown.append(p + [c])
        frontier = grown
    out = np.full((len(done), 8), PAD, dtype=np.uint32)
    for i, p in enumerate(done):
        out[i, :len(p)] = p
    return out


def scores(T, x, y, z, det):
    X = x.astype(np.float64); Y = y.astype(np.float64); Z = z.astype(np.float64)
    s = np.zeros(T.shape[0])
    for i, t in enumerate(T):
        h = t[t != PAD].astype(np.int64)
        acc = 0.0
        for j in range(1, len(h) - 1):
            t0, t1, _, _, d0 = _link_terms(X, Y, Z, h[j - 1:j], h[j:j + 1], h[j + 1:j + 2], det)
            q1 = t0[0] / t1[0]
            q2 = d0[0] / det["cuts"]["d0max"]
            acc += q1 * q1 + q2 * q2
        s[i] = acc
    return s


def clean(T, S):
    """Keep mask: a tuple survives iff it is the first, in the global order
    (more hits, lower score, smaller padded hit tuple), among all tuples
    through each of its doublets."""
    n = (T != PAD).sum(axis=1)
    order = sorted(range(T.shape[0]), key=lambda i: (-int(n[i]), float(S[i]), tuple(T[i].tolist())))
    owner = {}
    for i in order:
        h = T[i, :n[i]].tolist()
        for j in range(len(h) - 1):
            owner.setdefault((h[j], h[j + 1]), i)
    keep = np.ones(T.shape[0], dtype=bool)
    for i in range(T.shape[0]):
        h = T[i, :n[i]].tolist()
        for j in range(len(h) - 1):
            if owner[(h[j], h[j + 1])] != i:
                keep[i] = False
    return keep


# ---------------------------------------------------------------- fit ------

def _g(a, b, k):
    q = a * a + b * b
    return (2.0 * b - k * q) / (1.0 + np.sqrt(1.0 - 2.0 * k * b + k * k * q))


def _arc(a, b, k):
    return a if k == 0.0 else np.arctan2(k * a, 1.0 - k * b) / k


def fit(X, Y, Z, kind, det):
    """Broken-line fit by generic least squares; returns (params, chi2)."""
    f = det["fit"]
    ck = det["c_kappa"]
    n = len(X)
    m = n // 2
    P = np.stack([X, Y], axis=1).astype(np.float64)
    d1 = P[m] - P[0]; d2 = P[n - 1] - P[0]; d3 = P[n - 1] - P[m]
    cr = d1[0] * d2[1] - d1[1] * d2[0]
    k = 2.0 * cr / (np.linalg.norm(d1) * np.linalg.norm(d2) * np.linalg.norm(d3))
    ang = np.arctan2(d2[1], d2[0]) - np.arcsin(np.clip(k * np.linalg.norm(d2) / 2.0, -1, 1))
    t = np.array([np.cos(ang), np.sin(ang)])
    nrm = np.array([-t[1], t[0]])
    E = P - P[0]
    a = E @ t; b = E @ nrm
    mres = np.array([_g(a[i], b[i], k) for i in range(n)])
    s = np.array([_arc(a[i], b[i], k) for i in range(n)])
    tref = (Z[-1] - Z[0]) / (s[-1] - s[0])
    sinT = 1.0 / np.sqrt(1.0 + tref * tref); cosT = tref * sinT
    kabs = max(abs(k), ck / f["pt_max"])
    p = ck / (kabs * sinT)
    x = np.array([f["x_over_x0"] / (sinT if kd == 0 else abs(cosT)) for kd in kind])
    th0 = 0.0136 / p * np.sqrt(x) * (1.0 + 0.038 * np.log(x))
    ds = np.diff(s)
    # transverse: rows of residuals / sigma
    A = np.zeros((2 * n - 2, n + 1)); yv = np.zeros(2 * n - 2)
    A[:n, :n] = np.eye(n) / f["sigma_u"]; yv[:n] = mres / f["sigma_u"]
    for j in range(1, n - 1):
        w = sinT / th0[j]
        r = n + j - 1
        A[r, j + 1] += w / ds[j]; A[r, j] -= w * (1 / ds[j] + 1 / ds[j - 1])
        A[r, j - 1] += w / ds[j - 1]; A[r, n] -= w * (ds[j - 1] + ds[j]) / 2.0
    sol = np.linalg.lstsq(A, yv, rcond=None)[0]
    chi_c = float(np.sum((A @ sol - yv) ** 2))
    mz = Z - Z[0] - tref * (s - s[0])
    B = np.zeros((2 * n - 2, n)); yz = np.zeros(2 * n - 2)
    sz = np.array([f["sigma_z"] if kd == 0 else f["sigma_r"] * abs(tref) for kd in kind])
    B[:n, :n] = np.diag(1.0 / sz); yz[:n] = mz / sz
    for j in range(1, n - 1):
        w = sinT * sinT / th0[j]
        r = n + j - 1
        B[r, j + 1] += w / ds[j]; B[r, j] -= w * (1 / ds[j] + 1 / ds[j - 1])
        B[r, j - 1] += w / ds[j - 1]
    wz = np.linalg.lstsq(B, yz, rcond=None)[0]
    chi_z = float(np.sum((B @ wz - yz) ** 2))
    u0, u1, dk = sol[0], sol[1], sol[n]
    kap = k + dk
    P0 = P[0] + u0 * nrm
    phis = np.arctan2(t[1], t[0]) + (u1 - u0) / ds[0] - dk * ds[0] / 2.0
    tt = np.array([np.cos(phis), np.sin(phis)]); nn = np.array([-tt[1], tt[0]])
    aO = (-P0) @ tt; bO = (-P0) @ nn
    d0 = _g(aO, bO, kap)
    sp = _arc(aO, bO, kap)
    phi0 = np.arctan2(np.sin(phis + kap * sp), np.cos(phis + kap * sp))
    cot = tref + (wz[1] - wz[0]) / ds[0]
    z0 = Z[0] + wz[0] + cot * sp
    return np.array([phi0, d0, -kap / ck, cot, z0]), np.array([chi_c, chi_z])


def reconstruct(x, y, z, layer, det):
    D, dmask = doublets(x, y, z, layer, det)
    L = links(x, y, z, layer, det, dmask)
    T = tuples(D, L)
    S = scores(T, x, y, z, det)
    keep = clean(T, S) if T.shape[0] else np.zeros(0, bool)
    return dict(doublets=D, links=L, raw=T, raw_score=S, keep=keep, tracks=T[keep])


def vertices(z0, var, qopt, nhits, eps, min_pts, min_hits, qopt_max):
    """Vertices by textbook DBSCAN (Ester et al. 1996): the full pairwise
    distance matrix, clusters grown from each unvisited core by breadth-first
    expansion over core neighbours, borders to the nearest core (ties to the
    smaller z0, then the smaller index), weighted means by numpy sums.
    Returns (z, z_err, chi2, n_tracks, assign) with vertices in increasing z."""
    z0 = np.asarray(z0, np.float32)
    var = np.asarray(var, np.float32)
    qopt = np.asarray(qopt, np.float32)
    nhits = np.asarray(nhits)
    n = z0.shape[0]
    sel = ((nhits >= min_hits) & (np.abs(qopt) <= np.float32(qopt_max)) & np.isfinite(z0)
           & np.isfinite(var) & (var > 0))
    idx = np.nonzero(sel)[0]
    z = z0[idx].astype(np.float64)
    dist = np.abs(z[:, None] - z[None, :])
    nb = dist <= eps
    core = nb.sum(axis=1) >= min_pts
    label = -np.ones(idx.size, np.int64)
    k = 0
    for s in range(idx.size):
        if not core[s] or label[s] >= 0:
            continue
        label[s] = k
        queue = [s]
        while queue:
            a = queue.pop(0)
            for b in np.nonzero(nb[a] & core)[0]:
                if label[b] < 0:
                    label[b] = k
                    queue.append(b)
        k += 1
    cores = np.nonzero(core)[0]
    for a in range(idx.size):
        if core[a] or cores.size == 0:
            continue
        d = dist[a, cores]
        ok = d <= eps
        if not ok.any():
            continue
        cand = cores[ok]
        dc = d[ok]
        best = cand[dc == dc.min()]
        # nearest; ties to the smaller z0, then the smaller track index
        best = sorted(best, key=lambda b: (z[b], idx[b]))[0]
        label[a] = label[best]
    # number the clusters by increasing z of their members
    order = sorted(set(label[label >= 0].tolist()), key=lambda c: z[label == c].min())
    ren = {c: i for i, c in enumerate(order)}
    assign = -np.ones(n, np.int32)
    vz, ve, vc, vn = [], [], [], []
    for c in order:
        m = label == c
        assign[idx[m]] = ren[c]
        w = 1.0 / var[idx[m]].astype(np.float64)
        zm = z[m]
        zv = np.sum(w * zm) / np.sum(w)
        vz.append(zv)
        ve.append(np.sqrt(1.0 / np.sum(w)))
        vc.append(np.sum(w * (zm - zv) ** 2))
        vn.append(int(m.sum()))
    return (np.array(vz), np.array(ve), np.array(vc), np.array(vn, np.uint32), assign)


def rechits(cl, table, max_per_module):
    """3-D hits of one event's clusters by a different route: per-cluster
    sums with numpy reduceat, ranks from a stable sort by module, local to
    global through the azimuth (barrel: phi_c + atan2(u, r) on the cylinder
    of radius r; disk: rotation of (r + u, v) by phi_c).  Returns the same
    dict as the C tier."""
    mod = np.asarray(cl["module"], np.int64)
    nc = mod.shape[0]
    nm = table.shape[0]
    cnt = np.bincount(mod, minlength=nm) if nc else np.zeros(nm, np.int64)
    ms = np.concatenate([[0], np.cumsum(np.minimum(cnt, max_per_module))]).astype(np.uint32)
    order = np.argsort(mod, kind="stable")
    rank = np.zeros(nc, np.int64)
    if nc:
        first = np.searchsorted(mod[order], mod[order], side="left")
        rank[order] = np.arange(nc) - first
    po = np.asarray(cl["pixel_offsets"], np.int64)
    q = np.asarray(cl["charge"], np.float64)
    pu = np.asarray(cl["pix_u"], np.float64) + 0.5
    pv = np.asarray(cl["pix_v"], np.float64) + 0.5
    nh = int(ms[-1])
    out = dict(module_start=ms, x=np.zeros(nh, np.float32), y=np.zeros(nh, np.float32),
               z=np.zeros(nh, np.float32), layer=np.zeros(nh, np.int16),
               module=np.zeros(nh, np.uint16), cluster=np.zeros(nh, np.uint32))
    for i in range(nc):
        if rank[i] >= max_per_module:
            continue
        h = int(ms[mod[i]] + rank[i])
        a, b = po[i], po[i + 1]
        Q = q[a:b].sum()
        out["module"][h] = mod[i]
        out["cluster"][h] = i
        if not Q > 0:
            out["layer"][h] = -1
            continue
        T = table[mod[i]]
        u = T[6] + T[8] * (np.dot(q[a:b], pu[a:b]) / Q)
        v = T[7] + T[9] * (np.dot(q[a:b], pv[a:b]) / Q)
        pc = np.arctan2(T[3], T[2])
        if T[1] == 0:
            ph = pc + np.arctan2(u, T[4])
            out["x"][h], out["y"][h], out["z"][h] = T[4] * np.cos(ph), T[4] * np.sin(ph), T[5] + v
        else:
            R = np.hypot(T[4] + u, v)
            ph = pc + np.arctan2(v, T[4] + u)
            out["x"][h], out["y"][h], out["z"][h] = R * np.cos(ph), R * np.sin(ph), T[5]
        out["layer"][h] = int(T[0])
    return out
