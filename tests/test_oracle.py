"""Pins of the CPU oracle against geometry, closed forms and brute force.

None of these tests compares the oracle with a retyped copy of its own
formulas: each cut is checked on hits constructed from the geometric quantity
it is meant to bound (with the constructed value placed on both sides of the
threshold), whole events are checked against the generator's truth where the
answer is known in closed form, the C tier is checked against the brute-force
numpy tier (different enumeration, a different solver), and the fit against
exact helices, the circumcircle of three hits, symmetries and pull statistics.
"""

import numpy as np
import pytest

import eventgen
import oracle
from oracle import brute
from tests import helix_util as hx


# ------------------------------------------------------------- doublet cuts --

def _on_line_rz(z0, slope, r, phi=0.3):
    """Hit at radius r on the r-z line z = z0 + slope * r, azimuth phi."""
    return (r * np.cos(phi), r * np.sin(phi), z0 + slope * r)


@pytest.mark.parametrize("z0,ok", [(14.9, True), (-14.9, True), (15.1, False), (-15.1, False),
                                   (0.0, True)])
def test_d2_longitudinal_impact(det, z0, ok):
    # two hits on a straight r-z line that meets r = 0 at z0; same azimuth so
    # only the z0 window can reject
    hi = _on_line_rz(z0, 1.7, 2.9)
    ho = _on_line_rz(z0, 1.7, 6.8)
    assert oracle.doublet_ok(det, hi, ho) == ok


@pytest.mark.parametrize("pt,ok", [(0.26, True), (0.5, True), (100.0, True), (0.24, False),
                                   (0.1, False)])
def test_d3_curvature_of_circle_through_origin(det, pt, ok):
    # both hits on a circle through the origin with curvature c_kappa / pT
    k = det["c_kappa"] / pt
    for sign in (1.0, -1.0):
        s1 = hx.arc_at_radius(0.7, 0.0, sign * k, 6.8)
        s2 = hx.arc_at_radius(0.7, 0.0, sign * k, 10.9)
        hi = hx.point(0.7, 0.0, sign * k, 0.0, 0.0, s1)
        ho = hx.point(0.7, 0.0, sign * k, 0.0, 0.0, s2)
        assert oracle.doublet_ok(det, hi, ho) == ok


def test_d1_d4_ordering_and_half_plane(det):
    # outer radius must be larger
    assert not oracle.doublet_ok(det, (6.8, 0, 0), (2.9, 0, 0))
    assert oracle.doublet_ok(det, (2.9, 0, 0), (6.8, 0, 0))
    # a straight line through the origin crossing to the opposite side has
    # zero curvature but lies in the other half plane
    assert not oracle.doublet_ok(det, (2.9, 0, 0), (-6.8, 0, 0))


# ---------------------------------------------------------------- link cuts --

@pytest.mark.parametrize("delta,ok", [(0.0, True), (0.0140, True), (-0.0140, True),
                                      (0.0160, False), (-0.0160, False)])
def test_l1_rz_alignment(det, delta, ok):
    # three hits on one radial line (no transverse bending) whose r-z segments
    # turn by angle delta: |cross| / (l_ab l_bc) = |sin delta|
    phi = -1.1
    alpha = 0.8
    ra, za = 3.0, 1.0
    rb, zb = ra + 4.0 * np.cos(alpha), za + 4.0 * np.sin(alpha)
    rc, zc = rb + 5.0 * np.cos(alpha + delta), zb + 5.0 * np.sin(alpha + delta)
    pts = [(r * np.cos(phi), r * np.sin(phi), z) for r, z in ((ra, za), (rb, zb), (rc, zc))]
    t = oracle.link_terms(det, *pts)
    assert t[0] / (t[1] / det["cuts"]["arz"]) == pytest.approx(abs(np.sin(delta)), abs=1e-12)
    assert oracle.link_ok(det, *pts) == ok


@pytest.mark.parametrize("pt,ok", [(0.3, True), (0.26, True), (0.24, False)])
def test_l2_menger_curvature(det, pt, ok):
    # three hits on a circle through the origin of curvature c_kappa / pT and
    # z = 0 (r-z collinear): the Menger curvature is the circle's
    k = det["c_kappa"] / pt
    pts = [hx.point(2.0, 0.0, k, 0.0, 0.0, hx.arc_at_radius(2.0, 0.0, k, r))
           for r in (2.9, 6.8, 10.9)]
    t = oracle.link_terms(det, *pts)
    assert t[2] / (t[3] / det["cuts"]["kmax"]) == pytest.approx(k, rel=1e-9)
    assert t[4] == pytest.approx(0.0, abs=1e-9)
    assert oracle.link_ok(det, *pts) == ok


@pytest.mark.parametrize("d0,ok", [(0.0, True), (0.05, True), (-0.09, True), (0.11, False),
                                   (-0.2, False)])
def test_l3_transverse_impact(det, d0, ok):
    # three hits on a circle that passes at signed distance d0 from the origin
    k = det["c_kappa"] / 2.0
    pts = [hx.point(-0.4, d0, k, 0.0, 0.0, hx.arc_at_radius(-0.4, d0, k, r))
           for r in (2.9, 6.8, 10.9)]
    t = oracle.link_terms(det, *pts)
    assert t[4] == pytest.approx(abs(d0), abs=1e-9)
    assert oracle.link_ok(det, *pts) == ok


def test_l3_straight_line_branch(det):
    # collinear transverse points: the circle degenerates to a line, whose
    # distance from the origin is the impact
    pts = [(x, 0.05, 0.0) for x in (3.0, 7.0, 11.0)]
    t = oracle.link_terms(det, *pts)
    assert t[4] == pytest.approx(0.05, abs=1e-15)


# --------------------------------------------------------- tiers and truth --

def _canon(a):
    return oracle.canonical(np.asarray(a, dtype=np.uint32))


def _compare_tiers(ev, det):
    c = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    b = brute.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert c["status"] == 0
    np.testing.assert_array_equal(_canon(c["doublets"]), _canon(b["doublets"]))
    np.testing.assert_array_equal(_canon(c["links"]), _canon(b["links"]))
    np.testing.assert_array_equal(_canon(c["raw"]), _canon(b["raw"]))
    np.testing.assert_array_equal(_canon(c["tracks"]), _canon(b["tracks"]))
    # the scores are the same formulas in the same order: identical doubles
    oc = np.lexsort(c["raw"].T[::-1]); ob = np.lexsort(b["raw"].T[::-1])
    np.testing.assert_array_equal(c["raw_score"][oc], b["raw_score"][ob])
    return c


@pytest.mark.parametrize("seed", range(40))
def test_tiers_agree_tiny(det, seed):
    ev = eventgen.generate("tiny", seed)
    _compare_tiers(ev, det)


@pytest.mark.parametrize("seed", range(3))
def test_tiers_agree_small_pu50(det, seed):
    # pu50 distributions (smearing, scattering, noise, disks) at 120 tracks
    ev = eventgen.generate("pu50", 1000 + seed, n_tracks=120)
    _compare_tiers(ev, det)


@pytest.mark.parametrize("seed", range(20))
def test_separated_noiseless_tracks_recover_truth(det, seed):
    # tracks spaced 2 pi / 20 in azimuth cannot form cross-track doublets, so
    # the surviving tuples are exactly the generated hit sets, in order
    ev = eventgen.generate("tiny", seed, phi_spacing=True)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    truth = np.full((len(ev.track_hits), 8), oracle.PAD, np.uint32)
    for i, h in enumerate(ev.track_hits):
        truth[i, :len(h)] = h
    np.testing.assert_array_equal(_canon(r["tracks"]), _canon(truth))
    assert r["keep"].all()


def test_tuple_invariants_pu50(det):
    ev = eventgen.generate("pu50", 5)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    R = np.hypot(ev.x.astype(np.float64), ev.y.astype(np.float64))
    for t in r["raw"]:
        h = t[t != oracle.PAD]
        assert 3 <= len(h) <= 8
        assert len(set(ev.layer[h].tolist())) == len(h)
        assert np.all(np.diff(R[h]) > 0)
    # every doublet passes the cut and lies on an allowed pair
    pairs = set(map(tuple, det["pairs"]))
    rng = np.random.default_rng(0)
    for i, o in r["doublets"][rng.choice(len(r["doublets"]), 300, replace=False)]:
        assert (int(ev.layer[i]), int(ev.layer[o])) in pairs
        assert oracle.doublet_ok(det, (ev.x[i], ev.y[i], ev.z[i]), (ev.x[o], ev.y[o], ev.z[o]))
    # a survivor shares no doublet with another survivor
    seen = set()
    for t in r["tracks"]:
        h = t[t != oracle.PAD].tolist()
        for j in range(len(h) - 1):
            assert (h[j], h[j + 1]) not in seen
            seen.add((h[j], h[j + 1]))


def test_cleaning_prefers_longer_then_lower_score(det):
    # a quadruplet and a triplet sharing their first doublet: the longer wins;
    # two triplets sharing a doublet: the better-aligned one wins
    k = det["c_kappa"] / 3.0
    quad = [hx.point(0.2, 0.0, k, 0.5, 1.0, hx.arc_at_radius(0.2, 0.0, k, r))
            for r in (2.9, 6.8, 10.9, 16.0)]
    # a fake third hit slightly off in z on layer 2
    fake = (quad[2][0], quad[2][1], quad[2][2] + 0.02)
    pts = quad + [fake]
    x = np.array([p[0] for p in pts], np.float32)
    y = np.array([p[1] for p in pts], np.float32)
    z = np.array([p[2] for p in pts], np.float32)
    layer = np.array([0, 1, 2, 3, 2], np.int16)
    r = oracle.reconstruct(x, y, z, layer, det)
    got = _canon(r["tracks"])
    assert got.shape[0] == 1 and list(got[0][:4]) == [0, 1, 2, 3]
    # drop the real layer-3 hit: two triplets 0-1-2 and 0-1-4 compete
    r2 = oracle.reconstruct(x[[0, 1, 2, 4]], y[[0, 1, 2, 4]], z[[0, 1, 2, 4]],
                            layer[[0, 1, 2, 4]], det)
    got = _canon(r2["tracks"])
    assert got.shape[0] == 1 and list(got[0][:3]) == [0, 1, 2]


# ---------------------------------------------------------------------- fit --

FLOORS = np.array([1.0, 0.01, 0.001, 0.1, 1.0])


@pytest.mark.parametrize("case", range(12))
def test_fit_recovers_exact_helix(det, case):
    rng = np.random.default_rng(case)
    phi0 = rng.uniform(-np.pi, np.pi)
    d0 = rng.uniform(-0.05, 0.05) if case % 3 else 0.0
    pt = np.exp(rng.uniform(np.log(0.5), np.log(50.0)))
    q = 1.0 if case % 2 else -1.0
    k = -q * det["c_kappa"] / pt
    z0 = rng.uniform(-5, 5)
    # cot(theta) within what keeps the outermost hit (arc length below 16.5
    # cm at these curvatures) inside the barrel's |z| < 26.5 cm
    cot = rng.uniform(-1.0, 1.0) * (26.0 - abs(z0)) / 16.5
    X, Y, Z = hx.barrel_hits(phi0, d0, k, cot, z0)
    assert (np.abs(Z) < 26.5).all()
    p, cov, chi2, kref = oracle.fit(X, Y, Z, [0, 0, 0, 0], det)
    truth = np.array([phi0, d0, q / pt, cot, z0])
    err = np.abs(p - truth)
    err[0] = abs(hx.wrap(p[0] - phi0))
    assert np.all(err <= 1e-9 * np.maximum(np.abs(truth), FLOORS)), (p, truth)
    assert chi2[0] == pytest.approx(0.0, abs=1e-12) and chi2[1] == pytest.approx(0.0, abs=1e-12)
    # covariance: symmetric positive definite
    C = oracle.unpack_cov(cov)
    assert np.all(np.linalg.eigvalsh(C) > 0)


def test_fit_triplet_is_circumcircle(det):
    rng = np.random.default_rng(3)
    for _ in range(20):
        pts = rng.uniform(-1, 1, (3, 2)) * 0.05 + np.array([[2.9, 0.0], [6.8, 0.3], [10.9, 0.9]])
        z = np.array([0.3, 1.1, 2.0])
        p, cov, chi2, kref = oracle.fit(pts[:, 0], pts[:, 1], z, [0, 0, 0], det)
        a, b, c = pts
        cr = (b - a)[0] * (c - a)[1] - (b - a)[1] * (c - a)[0]
        menger = 2 * cr / (np.linalg.norm(b - a) * np.linalg.norm(c - b) * np.linalg.norm(c - a))
        assert chi2[0] == pytest.approx(0.0, abs=1e-10)
        assert -p[2] * det["c_kappa"] == pytest.approx(menger, rel=1e-9)
        # the fitted circle passes through all three points
        center_dir = np.array([-np.sin(p[0]), np.cos(p[0])])
        pca = -p[1] * center_dir
        center = pca + center_dir / menger
        for q in pts:
            assert np.linalg.norm(q - center) == pytest.approx(1 / abs(menger), rel=1e-9)


def test_fit_straight_line_limit(det):
    X, Y, Z = hx.barrel_hits(0.3, 0.0, -det["c_kappa"] / 1e4, 0.2, 1.0)
    p, cov, chi2, kref = oracle.fit(X, Y, Z, [0, 0, 0, 0], det)
    assert np.all(np.isfinite(p)) and np.all(np.isfinite(cov))
    assert abs(p[2]) < 1e-3 and p[0] == pytest.approx(0.3, abs=1e-9)


def test_fit_symmetries(det):
    X, Y, Z = hx.barrel_hits(0.4, 0.02, 0.004, 0.7, 2.0)
    rng = np.random.default_rng(0)
    X = X + rng.normal(0, 1e-3, 4); Y = Y + rng.normal(0, 1e-3, 4); Z = Z + rng.normal(0, 2e-3, 4)
    kind = [0, 0, 0, 0]
    p, cov, chi2, _ = oracle.fit(X, Y, Z, kind, det)
    # rotation by alpha shifts phi0 only
    al = 0.9
    Xr = X * np.cos(al) - Y * np.sin(al); Yr = X * np.sin(al) + Y * np.cos(al)
    pr, covr, chi2r, _ = oracle.fit(Xr, Yr, Z, kind, det)
    assert hx.wrap(pr[0] - p[0] - al) == pytest.approx(0.0, abs=1e-9)
    np.testing.assert_allclose(pr[1:], p[1:], rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(chi2r, chi2, rtol=1e-6, atol=1e-12)
    # z -> -z flips cot(theta) and z0
    pz, _, chi2z, _ = oracle.fit(X, Y, -Z, kind, det)
    np.testing.assert_allclose(pz[[0, 1, 2]], p[[0, 1, 2]], rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(pz[[3, 4]], -p[[3, 4]], rtol=1e-10, atol=1e-14)
    # y -> -y mirrors: phi0, d0 and the charge change sign
    pm, _, _, _ = oracle.fit(X, -Y, Z, kind, det)
    np.testing.assert_allclose(pm[[0, 1, 2]], -p[[0, 1, 2]], rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(pm[[3, 4]], p[[3, 4]], rtol=1e-9, atol=1e-13)


def test_fit_tiers_agree(det):
    for seed in range(3):
        ev = eventgen.generate("pu50", 2000 + seed, n_tracks=100)
        r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
        kinds = {l["id"]: l["kind"] for l in det["layers"]}
        for t, prm, ch in zip(r["tracks"], r["params"], r["chi2"]):
            h = t[t != oracle.PAD]
            kd = [kinds[int(l)] for l in ev.layer[h]]
            pb, cb = brute.fit(ev.x[h].astype(float), ev.y[h].astype(float),
                               ev.z[h].astype(float), kd, det)
            err = np.abs(pb - prm)
            err[0] = abs(hx.wrap(pb[0] - prm[0]))
            assert np.all(err <= 1e-7 * np.maximum(np.abs(prm), FLOORS)), (pb, prm)
            np.testing.assert_allclose(cb, ch, rtol=1e-5, atol=1e-6)


def test_fit_pulls_and_chi2(det):
    # fits of true hit sets with smearing and scattering: the oracle's
    # covariance describes the spread of (fit - truth)
    pulls, chic, chiz, ndfc, ndfz = [], [], [], [], []
    kinds = {l["id"]: l["kind"] for l in det["layers"]}
    for seed in range(6):
        ev = eventgen.generate("pu50", 3000 + seed, noise_fraction=0.0, efficiency=1.0,
                               scatter_first=False)
        tr = ev.tracks
        for i, h in enumerate(ev.track_hits):
            if len(h) < 4:
                continue
            kd = [kinds[int(l)] for l in ev.layer[h]]
            p, cov, ch, _ = oracle.fit(ev.x[h].astype(float), ev.y[h].astype(float),
                                       ev.z[h].astype(float), kd, det)
            truth = np.array([tr["phi"][i], 0.0, tr["q"][i] / tr["pt"][i], tr["cot"][i], tr["zv"][i]])
            d = p - truth
            d[0] = hx.wrap(d[0])
            sig = np.sqrt(np.diag(oracle.unpack_cov(cov)))
            pulls.append(d / sig)
            chic.append(ch[0]); chiz.append(ch[1])
            ndfc.append(len(h) - 3); ndfz.append(len(h) - 2)
    pulls = np.array(pulls)
    mean = pulls.mean(axis=0)
    rms = pulls.std(axis=0)
    assert np.all(np.abs(mean) < 0.1), mean
    assert np.all((rms > 0.9) & (rms < 1.12)), rms
    assert np.mean(chic) / np.mean(ndfc) == pytest.approx(1.0, abs=0.3)
    assert np.mean(chiz) / np.mean(ndfz) == pytest.approx(1.0, abs=0.3)
