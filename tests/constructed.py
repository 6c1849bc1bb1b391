"""Hand-built events whose cleaning outcome and scores are fixed by geometry.

Shared by the oracle pins (CPU) and the GPU parity tests.  Nothing here
calls the oracle or the library: the expected values are computed by a
route of their own -- the r-z turning angle from arctan2, the transverse
impact from the algebraic circle x^2 + y^2 + D x + E y + F = 0 solved in
exact rational arithmetic (the origin's distance from that circle is
|F| / (|C| + R), |C| and R taken to 50 digits) -- from the float32
coordinates the event actually carries.
"""

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

from tests import helix_util as hx


class Ev:
    def __init__(self, x, y, z, layer):
        self.x = np.asarray(x, np.float32)
        self.y = np.asarray(y, np.float32)
        self.z = np.asarray(z, np.float32)
        self.layer = np.asarray(layer, np.int16)

    @property
    def n_hits(self):
        return int(self.x.shape[0])


def event(points, layers):
    p = np.asarray(points, np.float64)
    return Ev(p[:, 0], p[:, 1], p[:, 2], layers)


def _hit(ev, i):
    return float(ev.x[i]), float(ev.y[i]), float(ev.z[i])


def rz_sine(pa, pb, pc):
    """Sine of the turning angle of the r-z segments a->b->c (arctan2 route)."""
    ra, rb, rc = (np.sqrt(p[0] * p[0] + p[1] * p[1]) for p in (pa, pb, pc))
    t1 = np.arctan2(pb[2] - pa[2], rb - ra)
    t2 = np.arctan2(pc[2] - pb[2], rc - rb)
    return float(np.sin(t2 - t1))


def impact_exact(pa, pb, pc):
    """Distance of the transverse origin from the circle through three
    points: the circle x^2 + y^2 + D x + E y + F = 0 solved exactly (Cramer's
    rule over rationals); |C|^2 - R^2 = F, so the distance is
    |F| / (|C| + R)."""
    getcontext().prec = 50
    P = [(Fraction(p[0]), Fraction(p[1])) for p in (pa, pb, pc)]
    M = [[x, y, Fraction(1)] for x, y in P]
    rhs = [-(x * x + y * y) for x, y in P]

    def det3(m):
        return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
                - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))

    d = det3(M)
    sol = []
    for k in range(3):
        mk = [row[:] for row in M]
        for i in range(3):
            mk[i][k] = rhs[i]
        sol.append(det3(mk) / d)
    D, E, F = sol
    c2 = (D * D + E * E) / 4
    r2 = c2 - F
    dec = lambda q: Decimal(q.numerator) / Decimal(q.denominator)
    C = dec(c2).sqrt()
    R = dec(r2).sqrt()
    return float(abs(dec(F)) / (C + R))


def triple_score_expected(det, ev, i, j, k):
    """(rz sine / arz)^2 + (impact / d0max)^2 of hits i, j, k of ev."""
    pa, pb, pc = _hit(ev, i), _hit(ev, j), _hit(ev, k)
    q1 = rz_sine(pa, pb, pc) / det["cuts"]["arz"]
    q2 = impact_exact(pa, pb, pc) / det["cuts"]["d0max"]
    return q1 * q1 + q2 * q2


def scored_quadruplet(det):
    """Four hits on layers 0..3 lying on a circle that passes 0.06 cm from
    the origin (pT 2 GeV), with r-z segments turning by +0.009 and then
    -0.006 rad: a quadruplet whose two triples both carry an r-z term and
    an impact term."""
    k = det["c_kappa"] / 2.0
    phi0, d0 = 0.3, 0.06
    radii = (2.9, 6.8, 10.9, 16.0)
    xy = [hx.point(phi0, d0, k, 0.0, 0.0, hx.arc_at_radius(phi0, d0, k, r))[:2]
          for r in radii]
    alpha = 0.5
    turns = (0.0, 0.009, -0.006)
    z = [1.0]
    ang = alpha
    for i in range(1, 4):
        ang = alpha + sum(turns[:i])
        z.append(z[-1] + (radii[i] - radii[i - 1]) * np.tan(ang))
    pts = [(xy[i][0], xy[i][1], z[i]) for i in range(4)]
    return event(pts, [0, 1, 2, 3])


def impact_decides(det):
    """Two triplets sharing the doublet (a, b) whose third hits are mirror
    images in y: identical radius and z, so identical r-z terms, but
    transverse impacts of about 0.053 and 0.0007 cm.  The larger impact sits
    at the lower hit index, so a score without the impact term would tie and
    the index order would pick the wrong one.  Returns (event, winner)."""
    beta, gam = 0.002, 0.004
    a = (2.9, 0.0, 1.0)
    b = (6.8 * np.cos(beta), 6.8 * np.sin(beta), 2.95)
    c_small = (10.9 * np.cos(gam), 10.9 * np.sin(gam), 5.0)
    c_large = (10.9 * np.cos(gam), -10.9 * np.sin(gam), 5.0)
    ev = event([a, b, c_large, c_small], [0, 1, 2, 2])
    return ev, (0, 1, 3)


def exact_tie(det, low_first):
    """Two triplets with bitwise-equal scores: a and b on the +x axis and the
    third hits mirrored in y, so every difference in the cuts and the score
    changes only in sign.  Only the hit-index order can decide; the winner
    is the one whose third hit has the lower index.  low_first puts the
    +y hit first.  Returns (event, winner)."""
    gam = 0.003
    a = (2.9, 0.0, 0.5)
    b = (6.8, 0.0, 1.3)
    cp = (10.9 * np.cos(gam), 10.9 * np.sin(gam), 2.2)
    cm = (10.9 * np.cos(gam), -10.9 * np.sin(gam), 2.2)
    pts = [a, b, cp, cm] if low_first else [a, b, cm, cp]
    return event(pts, [0, 1, 2, 2]), (0, 1, 2)


def chain_detector(det, n_layers):
    """A barrel-only detector of n_layers layers at radii 3, 4, ... cm, each
    layer paired with the next: a straight radial track crosses all of them
    and forms one path of n_layers hits."""
    d = dict(det)
    d["layers"] = [{"id": i, "kind": 0, "r": 3.0 + i, "zmax": 30.0} for i in range(n_layers)]
    d["pairs"] = [(i, i + 1) for i in range(n_layers - 1)]
    return d


def chain_event(n_layers, phi=0.7, slope=0.25, z0=0.5):
    pts = [((3.0 + i) * np.cos(phi), (3.0 + i) * np.sin(phi), z0 + slope * (3.0 + i))
           for i in range(n_layers)]
    return event(pts, list(range(n_layers)))


def longer_beats_lower_score(det):
    """The scored quadruplet plus a hit on layer 2 that makes a triplet
    (0, 1, 4) sharing the quadruplet's first doublet with a much lower score
    (a straight continuation of the first doublet, 0.004 rad off in phi) and
    no continuation of its own: only the length rule keeps the quadruplet.
    Returns (event, winner)."""
    q = scored_quadruplet(det)
    a = (float(q.x[0]), float(q.y[0]), float(q.z[0]))
    b = (float(q.x[1]), float(q.y[1]), float(q.z[1]))
    ra, rb = np.hypot(a[0], a[1]), np.hypot(b[0], b[1])
    alpha = np.arctan2(b[2] - a[2], rb - ra)
    pa, pb = np.arctan2(a[1], a[0]), np.arctan2(b[1], b[0])
    rc = 10.9
    pc = pb + (pb - pa) * (rc - rb) / (rb - ra) - 0.004
    c2 = (rc * np.cos(pc), rc * np.sin(pc), b[2] + (rc - rb) * np.tan(alpha))
    pts = [(q.x[i], q.y[i], q.z[i]) for i in range(4)] + [c2]
    return event(pts, [0, 1, 2, 3, 2]), (0, 1, 2, 3)


def tie_detector(det):
    """The standard cuts and fit constants on four barrel layers, two of them
    at the same radius 2.9 cm (ids 0 and 1), paired (1,2), (0,2), (2,3) in
    that order: the doublets of layer 1 come before those of layer 0."""
    d = dict(det)
    d["layers"] = [{"id": 0, "kind": 0, "r": 2.9, "zmax": 26.5},
                   {"id": 1, "kind": 0, "r": 2.9, "zmax": 26.5},
                   {"id": 2, "kind": 0, "r": 6.8, "zmax": 26.5},
                   {"id": 3, "kind": 0, "r": 10.9, "zmax": 26.5}]
    d["pairs"] = [(1, 2), (0, 2), (2, 3)]
    return d


def tie_across_roots(det):
    """Two triplets sharing their outer doublet (b, c), b and c on the +x
    axis, their first hits mirror images in y on the two same-radius layers
    of tie_detector: bitwise-equal scores, different root doublets.  The
    lexicographically smaller tuple starts at hit 0 (layer 0), whose root
    doublet comes second in doublet order, so keeping the first tuple met
    would pick the wrong one.  Returns (event, detector, winner)."""
    gam = 0.002
    p = (2.9 * np.cos(gam), 2.9 * np.sin(gam), 0.4)
    pm = (2.9 * np.cos(gam), -2.9 * np.sin(gam), 0.4)
    b = (6.8, 0.0, 1.2)
    c = (10.9, 0.0, 2.1)
    return event([p, pm, b, c], [0, 1, 2, 3]), tie_detector(det), (0, 2, 3)


def rz_threshold_triplet(det, inside, rel=1e-5):
    """Three hits on barrel layers 0..2 on a straight transverse line
    through the origin (no curvature, no impact), whose r-z segments turn
    by an angle with sine arz (1 - rel) (inside: the link holds) or
    arz (1 + rel) (outside: it does not), set for the float32 coordinates
    the event carries: the turn is about 1e-7 rad from the cut, far inside the
    link prefilter's margin, so the prefilter must keep the candidate and
    the exact cut decide it.  Returns (event, sine)."""
    arz = det["cuts"]["arz"]
    phi = 0.7
    radii = (2.9, 6.8, 10.9)
    alpha = 0.3
    target = np.arcsin(arz * (1.0 - rel if inside else 1.0 + rel))
    za, zb = 1.0, 1.0 + (radii[1] - radii[0]) * np.tan(alpha)
    pts = [(r * np.cos(phi), r * np.sin(phi), 0.0) for r in radii]

    def build(zc):
        return event([(pts[0][0], pts[0][1], za), (pts[1][0], pts[1][1], zb),
                      (pts[2][0], pts[2][1], zc)], [0, 1, 2])

    # the third z from the float32 a, b (their rounding moves the first
    # segment's angle), then nudged by float32 ulps onto the intended side
    ev = build(zb + (radii[2] - radii[1]) * np.tan(alpha + target))
    a, b = _hit(ev, 0), _hit(ev, 1)
    rb = np.hypot(b[0], b[1])
    t1 = np.arctan2(b[2] - a[2], rb - np.hypot(a[0], a[1]))
    c = _hit(ev, 2)
    zc = np.float32(b[2] + (np.hypot(c[0], c[1]) - rb) * np.tan(t1 + target))
    for _ in range(64):
        ev = build(float(zc))
        s = rz_sine(_hit(ev, 0), _hit(ev, 1), _hit(ev, 2))
        if (s < arz) == inside and abs(s / arz - 1.0) > 1e-7:
            return ev, s
        zc = np.nextafter(zc, np.float32(-np.inf) if inside else np.float32(np.inf))
    raise RuntimeError("no float32 z on the intended side of the cut")


def _dec(x):
    return Decimal(float(x))


def doublet_curvature_ratio(pa, pb, kmax):
    """2 |xi yo - yi xo| / (kmax ri ro |ab|) of a doublet in 50-digit
    arithmetic from the float32 coordinates: the doublet's curvature cut
    holds when it is at most 1."""
    getcontext().prec = 50
    xi, yi, xo, yo = (_dec(v) for v in (pa[0], pa[1], pb[0], pb[1]))
    cr = abs(xi * yo - yi * xo)
    ri = (xi * xi + yi * yi).sqrt()
    ro = (xo * xo + yo * yo).sqrt()
    ab = ((xo - xi) ** 2 + (yo - yi) ** 2).sqrt()
    return 2 * cr / (_dec(kmax) * ri * ro * ab)


def curvature_threshold_doublet(det, inside, lo=1e-12, hi=1e-9):
    """A layer-0 / layer-1 doublet whose transverse curvature sits within
    [lo, hi] (relative) of kmax, below it (inside: the doublet exists) or
    above: inside the 1e-9 band of the fast squared form, where the
    defining expression decides.  The outer hit's float32 x and y are
    stepped by ulps from the real-valued threshold; the ratio is nearly
    linear in the steps, so for each x step the y step that brings it
    closest to 1 is tried.  Returns (event, ratio - 1)."""
    kmax = det["cuts"]["kmax"]
    phi, ri, ro = 0.4, 2.9, 6.8
    # sin(dphi) = kmax |ab| / 2 with |ab|^2 = ri^2 + ro^2 - 2 ri ro cos(dphi)
    dphi = 0.05
    for _ in range(60):
        ab = np.sqrt(ri * ri + ro * ro - 2 * ri * ro * np.cos(dphi))
        dphi = np.arcsin(kmax * ab / 2.0)
    a = (np.float32(ri * np.cos(phi)), np.float32(ri * np.sin(phi)), np.float32(1.0))
    bx0 = np.float32(ro * np.cos(phi + dphi))
    by0 = np.float32(ro * np.sin(phi + dphi))
    bz = np.float32(1.0 + (ro - ri) * 0.3)
    ux, uy = np.spacing(bx0), np.spacing(by0)

    def ratio(i, j):
        b = (bx0 + np.float32(i) * ux, by0 + np.float32(j) * uy)
        return b, float(doublet_curvature_ratio(a, b, kmax) - 1)

    _, q0 = ratio(0, 0)
    alpha = ratio(1, 0)[1] - q0
    beta = ratio(0, 1)[1] - q0
    best = None
    for i in range(-3000, 3001):
        j0 = int(round(-(q0 + alpha * i) / beta))
        for j in (j0 - 1, j0, j0 + 1):
            b, q = ratio(i, j)
            if (q < 0) == inside and lo <= abs(q) <= hi:
                if best is None or abs(q) < abs(best[1]):
                    best = (b, q)
    if best is None:
        raise RuntimeError("no float32 outer hit within the band")
    (bx, by), q = best
    return event([a, (bx, by, bz)], [0, 1]), q


def impact_exact_dec(pa, pb, pc):
    """impact_exact to 50 digits (a Decimal)."""
    getcontext().prec = 50
    P = [(Fraction(float(p[0])), Fraction(float(p[1]))) for p in (pa, pb, pc)]
    (x1, y1), (x2, y2), (x3, y3) = P
    # the circle x^2 + y^2 + D x + E y + F = 0 through the three points
    a11, a12, b1 = x2 - x1, y2 - y1, -((x2 * x2 + y2 * y2) - (x1 * x1 + y1 * y1))
    a21, a22, b2 = x3 - x1, y3 - y1, -((x3 * x3 + y3 * y3) - (x1 * x1 + y1 * y1))
    det = a11 * a22 - a12 * a21
    D = (b1 * a22 - a12 * b2) / det
    E = (a11 * b2 - b1 * a21) / det
    F = -(x1 * x1 + y1 * y1) - D * x1 - E * y1
    c2 = (D * D + E * E) / 4
    dec = lambda q: Decimal(q.numerator) / Decimal(q.denominator)
    return abs(dec(F)) / (dec(c2).sqrt() + dec(c2 - F).sqrt())


def impact_threshold_triplet(det, inside, lo=1e-12, hi=1e-9):
    """Three hits on barrel layers 0..2 of a helix of pT about 2 GeV (the
    curvature cut holds with room) on a straight r-z line (the r-z cut holds
    exactly), whose transverse impact sits within [lo, hi] (relative) of
    d0max, below it (inside: the link holds) or above: inside the 1e-9 band
    of the impact cut's division-free form, where the defining expression
    decides.  The third hit's float32 x and y are stepped by ulps; the
    impact is nearly linear in the steps, so for each x step the y step
    that brings it closest to d0max is tried.  Returns (event, d0 / d0max
    - 1)."""
    d0max = det["cuts"]["d0max"]
    k = det["c_kappa"] / 2.0
    phi0 = 0.3
    radii = (2.9, 6.8, 10.9)
    xy = [hx.point(phi0, d0max, k, 0.0, 0.0, hx.arc_at_radius(phi0, d0max, k, r))[:2]
          for r in radii]
    z = [1.0 + 0.5 * (r - radii[0]) for r in radii]
    a = (np.float32(xy[0][0]), np.float32(xy[0][1]))
    b = (np.float32(xy[1][0]), np.float32(xy[1][1]))
    cx0, cy0 = np.float32(xy[2][0]), np.float32(xy[2][1])
    ux, uy = np.spacing(cx0), np.spacing(cy0)
    ref = Decimal(float(d0max))

    def rel(i, j):
        c = (cx0 + np.float32(i) * ux, cy0 + np.float32(j) * uy)
        return c, float(impact_exact_dec(a, b, c) / ref - 1)

    _, q0 = rel(0, 0)
    alpha = rel(1, 0)[1] - q0
    beta = rel(0, 1)[1] - q0
    best = None
    for i in range(-4000, 4001):
        j0 = int(round(-(q0 + alpha * i) / beta))
        for j in (j0 - 1, j0, j0 + 1):
            c, q = rel(i, j)
            if (q < 0) == inside and lo <= abs(q) <= hi:
                if best is None or abs(q) < abs(best[1]):
                    best = (c, q)
    if best is None:
        raise RuntimeError("no float32 third hit within the band")
    c, q = best
    pts = [(a[0], a[1], z[0]), (b[0], b[1], z[1]), (c[0], c[1], z[2])]
    return event(pts, [0, 1, 2]), q


def rz_ratio_exact(pa, pb, pc, arz):
    """|sin| of the r-z turn a -> b -> c over arz, to 50 digits from the
    float32 coordinates (the cross product of the r-z segments over their
    lengths): the link's r-z cut holds when it is at most 1."""
    getcontext().prec = 50
    r = [(_dec(p[0]) ** 2 + _dec(p[1]) ** 2).sqrt() for p in (pa, pb, pc)]
    z = [_dec(p[2]) for p in (pa, pb, pc)]
    dra, dza = r[1] - r[0], z[1] - z[0]
    drb, dzb = r[2] - r[1], z[2] - z[1]
    t0 = abs(dra * dzb - dza * drb)
    return t0 / ((dra * dra + dza * dza).sqrt() * (drb * drb + dzb * dzb).sqrt() * _dec(arz))


def rz_band_triplet(det, inside, lo=1e-12, hi=1e-9):
    """rz_threshold_triplet with the turn's sine within [lo, hi] (relative)
    of arz: inside the 1e-9 band of the r-z cut's squared form, where the
    defining expression decides.  The float32 z of the middle and outer hits
    are stepped by ulps (the ratio is nearly linear in the steps; for each
    middle step the outer step closest to the cut is tried).  Returns
    (event, ratio - 1)."""
    arz = det["cuts"]["arz"]
    ev0, _ = rz_threshold_triplet(det, inside)
    a, b, c = _hit(ev0, 0), _hit(ev0, 1), _hit(ev0, 2)
    zb0, zc0 = np.float32(b[2]), np.float32(c[2])
    ub, uc = np.spacing(zb0), np.spacing(zc0)

    def rel(i, j):
        zb = zb0 + np.float32(i) * ub
        zc = zc0 + np.float32(j) * uc
        q = float(rz_ratio_exact(a, (b[0], b[1], zb), (c[0], c[1], zc), arz) - 1)
        return (zb, zc), q

    _, q0 = rel(0, 0)
    alpha = rel(1, 0)[1] - q0
    beta = rel(0, 1)[1] - q0
    best = None
    for i in range(-3000, 3001):
        j0 = int(round(-(q0 + alpha * i) / beta))
        for j in (j0 - 1, j0, j0 + 1):
            zz, q = rel(i, j)
            if (q < 0) == inside and lo <= abs(q) <= hi:
                if best is None or abs(q) < abs(best[1]):
                    best = (zz, q)
    if best is None:
        raise RuntimeError("no float32 z pair within the band")
    (zb, zc), q = best
    return event([a, (b[0], b[1], zb), (c[0], c[1], zc)], [0, 1, 2]), q


def link_curvature_ratio(pa, pb, pc, kmax):
    """Curvature of the transverse circle through three hits over kmax,
    2 |(b - a) x (c - a)| / (|ab| |bc| |ac| kmax), to 50 digits from the
    float32 coordinates: the link's curvature cut holds when it is at most
    1."""
    getcontext().prec = 50
    A, B, C = ([_dec(p[0]), _dec(p[1])] for p in (pa, pb, pc))
    cr = abs((B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]))
    ab = ((B[0] - A[0]) ** 2 + (B[1] - A[1]) ** 2).sqrt()
    bc = ((C[0] - B[0]) ** 2 + (C[1] - B[1]) ** 2).sqrt()
    ac = ((C[0] - A[0]) ** 2 + (C[1] - A[1]) ** 2).sqrt()
    return 2 * cr / (ab * bc * ac * _dec(kmax))


def curvature_band_triplet(det, inside, lo=1e-12, hi=1e-9):
    """Three hits on barrel layers 0..2 of a circle of curvature kmax that
    passes 0.05 cm from the origin (so the doublets' circles through the
    origin are 3-11 % below kmax and the impact cut holds with room), on a
    straight r-z line, whose circle's curvature sits within [lo, hi]
    (relative) of kmax, below (inside: the link holds) or above: inside the
    1e-9 band of the curvature cut's squared form.  The third hit's float32
    x and y are stepped by ulps as in impact_threshold_triplet.  Returns
    (event, ratio - 1)."""
    kmax = det["cuts"]["kmax"]
    phi0, d0 = 0.3, -0.05
    radii = (2.9, 6.8, 10.9)
    xy = [hx.point(phi0, d0, kmax, 0.0, 0.0, hx.arc_at_radius(phi0, d0, kmax, r))[:2]
          for r in radii]
    z = [1.0 + 0.5 * (r - radii[0]) for r in radii]
    a = (np.float32(xy[0][0]), np.float32(xy[0][1]))
    b = (np.float32(xy[1][0]), np.float32(xy[1][1]))
    cx0, cy0 = np.float32(xy[2][0]), np.float32(xy[2][1])
    ux, uy = np.spacing(cx0), np.spacing(cy0)

    def rel(i, j):
        c = (cx0 + np.float32(i) * ux, cy0 + np.float32(j) * uy)
        return c, float(link_curvature_ratio(a, b, c, kmax) - 1)

    _, q0 = rel(0, 0)
    alpha = rel(1, 0)[1] - q0
    beta = rel(0, 1)[1] - q0
    best = None
    for i in range(-3000, 3001):
        j0 = int(round(-(q0 + alpha * i) / beta))
        for j in (j0 - 1, j0, j0 + 1):
            c, q = rel(i, j)
            if (q < 0) == inside and lo <= abs(q) <= hi:
                if best is None or abs(q) < abs(best[1]):
                    best = (c, q)
    if best is None:
        raise RuntimeError("no float32 third hit within the band")
    c, q = best
    pts = [(a[0], a[1], z[0]), (b[0], b[1], z[1]), (c[0], c[1], z[2])]
    return event(pts, [0, 1, 2]), q
