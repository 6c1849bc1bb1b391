"""Pins of the oracle's RecHits step (the paper's RecHits module, Sec. 2:
the 3-D position of each cluster; Fig. 3: each module's cluster count is
limited and the counts become the modules' first-hit offsets).

Geometry is pinned by what the module frames mean, not by the formulas: a
barrel hit lies on its layer cylinder at azimuth phi_c + atan(u/r), a disk
hit at distance sqrt((r_c + u)^2 + v^2) and azimuth phi_c + atan2(v, r_c + u)
in the disk plane; a single pixel puts the hit at the pixel centre, a charge
split 1:3 over two pixels at 3/4 of the way.  The limit and offsets are
pinned on a hand-built list, the whole step against a brute-force route on
generated events, and the round trip hit -> cluster -> hit to the pixel
size."""

import numpy as np
import pytest

import eventgen
import oracle
from eventgen import clusters as C
from oracle import brute

TABLE = C.module_table()


def _one(mod, pixels, max_per_module=1024):
    u = np.array([p[0] for p in pixels], np.uint16)
    v = np.array([p[1] for p in pixels], np.uint16)
    q = np.array([p[2] for p in pixels], np.uint16)
    cl = dict(module=np.array([mod], np.uint16), pixel_offsets=np.array([0, len(pixels)], np.uint32),
              pix_u=u, pix_v=v, charge=q)
    return oracle.rechits(cl, TABLE, max_per_module)


def _barrel_module(layer):
    return int(np.nonzero((TABLE[:, 0] == layer) & (TABLE[:, 1] == 0))[0][5])


def _disk_module(layer):
    return int(np.nonzero(TABLE[:, 0] == layer)[0][7])


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
@pytest.mark.parametrize("iu,iv", [(0, 0), (37, 200), (80, 441)])
def test_barrel_single_pixel_on_the_cylinder(layer, iu, iv):
    m = _barrel_module(layer)
    T = TABLE[m]
    nu = int(round(-2 * T[6] / T[8]))
    iu = min(iu, nu - 1)
    h = _one(m, [(iu, iv, 100)])
    u = T[6] + (iu + 0.5) * T[8]
    v = T[7] + (iv + 0.5) * T[9]
    x, y, z = float(h["x"][0]), float(h["y"][0]), float(h["z"][0])
    assert np.hypot(x, y) == pytest.approx(T[4], abs=2e-6)
    phi_c = np.arctan2(T[3], T[2])
    assert np.arctan2(y, x) == pytest.approx(phi_c + np.arctan(u / T[4]), abs=3e-7)
    assert z == pytest.approx(T[5] + v, abs=2e-6)
    assert h["layer"][0] == layer and h["module"][0] == m and h["cluster"][0] == 0


@pytest.mark.parametrize("layer", [4, 6, 8])
def test_disk_single_pixel(layer):
    m = _disk_module(layer)
    T = TABLE[m]
    iu, iv = 100, 50
    h = _one(m, [(iu, iv, 7)])
    u = T[6] + (iu + 0.5) * T[8]
    v = T[7] + (iv + 0.5) * T[9]
    x, y = float(h["x"][0]), float(h["y"][0])
    assert np.hypot(x, y) == pytest.approx(np.hypot(T[4] + u, v), abs=2e-6)
    phi_c = np.arctan2(T[3], T[2])
    d = np.arctan2(y, x) - (phi_c + np.arctan2(v, T[4] + u))
    assert abs((d + np.pi) % (2 * np.pi) - np.pi) < 3e-7
    assert float(h["z"][0]) == np.float32(T[5])


def test_charge_weighted_centroid():
    # charges 1:3 on pixels iu and iu + 1: the centroid is 3/4 of the way
    m = _barrel_module(1)
    T = TABLE[m]
    h2 = _one(m, [(40, 10, 25), (41, 10, 75)])
    u = T[6] + (40 + 0.5 + 0.75) * T[8]
    phi_c = np.arctan2(T[3], T[2])
    assert np.arctan2(float(h2["y"][0]), float(h2["x"][0])) == pytest.approx(
        phi_c + np.arctan(u / T[4]), abs=3e-7)
    # and along v: equal charges on three rows give the middle row
    h3 = _one(m, [(40, 10, 9), (40, 11, 9), (40, 12, 9)])
    assert float(h3["z"][0]) == pytest.approx(T[5] + T[7] + 11.5 * T[9], abs=2e-6)


def test_zero_charge_cluster_takes_part_in_nothing():
    h = _one(_barrel_module(0), [(3, 3, 0)])
    assert h["layer"][0] == -1 and h["x"][0] == 0 and h["cluster"][0] == 0


def test_limit_and_offsets():
    # modules 2 (5 clusters), 4 (1), 7 (3); limit 3: module 2 keeps its
    # first three clusters, the offsets are the running sum of 0,0,3,0,1,...
    mods = [2, 2, 2, 2, 2, 4, 7, 7, 7]
    cl = dict(module=np.array(mods, np.uint16),
              pixel_offsets=np.arange(len(mods) + 1, dtype=np.uint32),
              pix_u=np.full(len(mods), 5, np.uint16), pix_v=np.full(len(mods), 5, np.uint16),
              charge=np.full(len(mods), 10, np.uint16))
    h = oracle.rechits(cl, TABLE, 3)
    ms = h["module_start"]
    assert list(ms[:10]) == [0, 0, 0, 3, 3, 4, 4, 4, 7, 7]
    assert ms[-1] == 7
    assert list(h["cluster"]) == [0, 1, 2, 5, 6, 7, 8]
    assert list(h["module"]) == [2, 2, 2, 4, 7, 7, 7]
    # no limit: every cluster makes a hit
    assert oracle.rechits(cl, TABLE, 1024)["module_start"][-1] == 9
    # the rank counts earlier clusters of the module whatever the order
    cl2 = dict(cl, module=np.array([7, 2, 7, 2, 4, 2, 7, 2, 2], np.uint16))
    h2 = oracle.rechits(cl2, TABLE, 3)
    assert list(h2["cluster"]) == [1, 3, 5, 4, 0, 2, 6]


@pytest.mark.parametrize("seed", range(3))
def test_brute_route_agrees(seed):
    ev = eventgen.generate("pu50", 60 + seed, n_tracks=200)
    cl = C.make_clusters(ev, seed, table=TABLE)
    for lim in (1024, 2):
        a = oracle.rechits(cl, TABLE, lim)
        b = brute.rechits(cl, TABLE, lim)
        for k in ("module_start", "layer", "module", "cluster"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
        for k in ("x", "y", "z"):
            np.testing.assert_allclose(a[k], b[k], rtol=0, atol=4e-6, err_msg=k)


def test_round_trip_to_the_pixel_size():
    ev = eventgen.generate("pu50", 64)
    cl = C.make_clusters(ev, 64, table=TABLE)
    h = oracle.rechits(cl, TABLE, 1024)
    src = cl["hit_of_cluster"][h["cluster"]]
    d = np.hypot(h["x"] - ev.x[src], h["y"] - ev.y[src])
    assert np.all(h["layer"] == ev.layer[src])
    assert np.percentile(d, 99) < C.PITCH_U and np.percentile(np.abs(h["z"] - ev.z[src]), 99) < C.PITCH_V
