"""Pins of the oracle's vertex finding (the paper's Vertices module, Sec. 2,
Fig. 1: vertices formed from the pixel tracks), read as one-dimensional
density-based clustering (DBSCAN) of the tracks' z0 with a weighted mean per
cluster (the reading is stated in oracle/pxt_oracle.c).

Each pin fixes the result by construction: exact closed forms on constructed
track lists (with values exactly representable in single precision), the
neighbour and core thresholds on both sides, the border tie rule, the
selection boundaries, a brute-force DBSCAN by a different route on random
lists, and the generator's truth vertices on noiseless and on PU~50 events.
"""

from fractions import Fraction

import numpy as np
import pytest

import eventgen
import oracle
from oracle import brute

EPS = 0.0625  # 1/16: neighbour distances exactly representable
CFG = oracle.VtxConfig(EPS, 3, 4, np.float32(2.0))


def _run(z, var=None, qopt=None, nh=None, cfg=CFG):
    z = np.asarray(z, np.float32)
    n = z.shape[0]
    var = np.full(n, 1e-4, np.float32) if var is None else np.asarray(var, np.float32)
    qopt = np.full(n, 0.5, np.float32) if qopt is None else np.asarray(qopt, np.float32)
    nh = np.full(n, 4, np.uint8) if nh is None else np.asarray(nh, np.uint8)
    return oracle.vertices(z, var, qopt, nh, cfg=cfg)


def test_two_groups_closed_form():
    z = [2.0] * 6 + [-1.0] * 5
    var = [4e-4] * 6 + [1e-4] * 5
    v = _run(z, var)
    assert list(v["n_tracks"]) == [5, 6]
    np.testing.assert_array_equal(v["z"], [-1.0, 2.0])
    assert v["chi2"][0] == 0.0 and v["chi2"][1] == 0.0
    w1 = 1.0 / float(np.float32(1e-4))
    w2 = 1.0 / float(np.float32(4e-4))
    np.testing.assert_allclose(v["z_err"], [np.sqrt(1.0 / (5 * w1)), np.sqrt(1.0 / (6 * w2))],
                               rtol=1e-14)
    assert list(v["assign"]) == [1] * 6 + [0] * 5


def test_weighted_mean_and_chi2_exact():
    z = np.array([0.0, 0.015625, 0.046875], np.float32)
    var = np.array([1e-4, 2e-4, 4e-4], np.float32)
    v = _run(z, var)
    assert len(v["z"]) == 1
    w = [Fraction(1) / Fraction(float(s)) for s in var]
    zz = [Fraction(float(q)) for q in z]
    zv = sum(a * b for a, b in zip(w, zz)) / sum(w)
    chi2 = sum(a * (b - zv) ** 2 for a, b in zip(w, zz))
    assert v["z"][0] == pytest.approx(float(zv), rel=1e-15)
    assert v["chi2"][0] == pytest.approx(float(chi2), rel=1e-12)
    assert v["z_err"][0] == pytest.approx(float(1 / sum(w)) ** 0.5, rel=1e-15)


def test_core_threshold():
    # the middle track has 3 neighbours (itself included), the ends 2
    z = [0.0, EPS, 2 * EPS]
    v = _run(z)
    assert list(v["n_tracks"]) == [3] and list(v["assign"]) == [0, 0, 0]
    v4 = _run(z, cfg=oracle.VtxConfig(EPS, 4, 4, np.float32(2.0)))
    assert len(v4["z"]) == 0 and list(v4["assign"]) == [-1, -1, -1]


def test_neighbour_distance_is_inclusive():
    base = [0.0, 0.0, 0.0]
    at = _run(base + [EPS])
    assert list(at["n_tracks"]) == [4]
    past = _run(base + [np.nextafter(np.float32(EPS), np.float32(1))])
    assert list(past["n_tracks"]) == [3] and past["assign"][3] == -1


def test_chain_of_cores_is_one_vertex_and_a_gap_splits():
    z = np.arange(12, dtype=np.float32) * np.float32(EPS / 2)  # span 0.34 cm > eps
    v = _run(z)
    assert list(v["n_tracks"]) == [12]
    z2 = np.concatenate([z[:6], z[6:] + np.float32(4 * EPS)])
    v2 = _run(z2)
    assert list(v2["n_tracks"]) == [6, 6]


def test_border_tie_goes_to_the_lower_vertex():
    # cores at -EPS and +EPS (2 EPS apart: two clusters), each held up by two
    # tracks 1.5 EPS out; the track at 0 has 3 neighbours (not a core at
    # min_pts 4) and is exactly EPS from both cores
    e = EPS
    z = [-1.5 * e, -1.5 * e, -e, 0.0, e, 1.5 * e, 1.5 * e]
    v = _run(z, cfg=oracle.VtxConfig(EPS, 4, 4, np.float32(2.0)))
    assert list(v["n_tracks"]) == [4, 3]
    assert list(v["assign"]) == [0, 0, 0, 0, 1, 1, 1]


def test_nearest_core_wins_a_border():
    # as above with the upper core moved to 0.75 EPS: the track at 0 joins it
    e = EPS
    z = [-1.5 * e, -1.5 * e, -e, 0.0, 0.75 * e, 1.5 * e, 1.5 * e]
    v = _run(z, cfg=oracle.VtxConfig(EPS, 4, 4, np.float32(2.0)))
    assert list(v["n_tracks"]) == [3, 4]
    assert list(v["assign"]) == [0, 0, 0, 1, 1, 1, 1]


def test_selection_boundaries():
    z = [0.0] * 8
    nh = [4, 4, 4, 4, 3, 4, 4, 4]
    qopt = [0.5, -2.0, 2.0, 0.5, 0.5, np.nextafter(np.float32(2.0), np.float32(3)), 0.5, 0.5]
    var = [1e-4] * 6 + [0.0, np.nan]
    v = _run(z, var, qopt, nh)
    # |q/pT| == qopt_max kept; 3 hits, |q/pT| above, zero or NaN variance dropped
    assert list(v["assign"]) == [0, 0, 0, 0, -1, -1, -1, -1]
    zn = [0.0, 0.0, 0.0, np.nan]
    assert list(_run(zn)["assign"]) == [0, 0, 0, -1]


def test_isolated_tracks_are_noise():
    v = _run([0.0, 1.0, 2.0, 3.0])
    assert len(v["z"]) == 0 and np.all(v["assign"] == -1)


def test_empty():
    v = _run(np.zeros(0))
    assert len(v["z"]) == 0 and v["assign"].shape == (0,)


@pytest.mark.parametrize("seed", range(40))
def test_brute_dbscan_agrees(seed):
    rng = np.random.default_rng([91, seed])
    nv = rng.integers(1, 8)
    centres = rng.uniform(-1.0, 1.0, nv)
    n = int(rng.integers(0, 120))
    z = (centres[rng.integers(0, nv, n)] + rng.normal(0, 0.02, n)).astype(np.float32)
    # coarse grid: many exact distances and ties
    if seed % 2:
        z = (np.round(z * 64) / 64).astype(np.float32)
    var = rng.uniform(1e-5, 1e-3, n).astype(np.float32)
    qopt = rng.uniform(-3, 3, n).astype(np.float32)
    nh = rng.integers(3, 6, n).astype(np.uint8)
    cfg = oracle.VtxConfig(EPS, int(rng.integers(2, 6)), 4, np.float32(2.0))
    v = oracle.vertices(z, var, qopt, nh, cfg=cfg)
    bz, be, bc, bn, ba = brute.vertices(z, var, qopt, nh, cfg.eps, cfg.min_pts, cfg.min_hits,
                                        cfg.qopt_max)
    np.testing.assert_array_equal(v["assign"], ba)
    np.testing.assert_array_equal(v["n_tracks"], bn)
    np.testing.assert_allclose(v["z"], bz, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(v["z_err"], be, rtol=1e-12)
    np.testing.assert_allclose(v["chi2"], bc, rtol=1e-9, atol=1e-12)


def test_noiseless_event_gives_the_true_vertex(det):
    # tiny events: one vertex, noiseless helices, every track a quadruplet;
    # z0 is the vertex z up to the single-precision hits
    for seed in range(5):
        ev = eventgen.generate("tiny", 40 + seed)
        o = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
        v = oracle.event_vertices(o, det)
        nh = (o["tracks"] != oracle.PAD).sum(axis=1)
        sel = (nh >= 4) & (np.abs(o["params"][:, 2]) <= 1 / det["vertex"]["pt_min"])
        assert len(v["z"]) == 1
        assert abs(v["z"][0] - ev.tracks["vertex_z"][0]) < 1e-4
        assert v["n_tracks"][0] == sel.sum() and np.all(v["assign"][sel] == 0)


@pytest.mark.slow
def test_pu50_truth_vertices_found(det):
    # every resolvable truth vertex with at least 8 selected tracks of its
    # own is found within 0.01 cm, and no more than a few extra vertices
    # appear
    for seed in range(3):
        ev = eventgen.generate("pu50", 900 + seed)
        o = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
        v = oracle.event_vertices(o, det)
        vz = ev.tracks["vertex_z"]
        nh = (o["tracks"] != oracle.PAD).sum(axis=1)
        sel = (nh >= 4) & (np.abs(o["params"][:, 2]) <= 1 / det["vertex"]["pt_min"])
        owner = []
        for t in o["tracks"][sel]:
            h = t[t != oracle.PAD]
            tid = np.unique(ev.track_of_hit[h])
            owner.append(ev.tracks["vertex"][tid[0]] if tid.size == 1 and tid[0] >= 0 else -1)
        owner = np.array(owner)
        for k, zt in enumerate(vz):
            # resolvable: no other truth vertex within 0.2 cm (about ten
            # times the z0 resolution of these tracks)
            isolated = np.sort(np.abs(vz - zt))[1] >= 0.2 if len(vz) > 1 else True
            if (owner == k).sum() >= 8 and isolated:
                assert np.min(np.abs(v["z"] - zt)) < 0.01, (seed, k, zt, v["z"])
        assert len(v["z"]) <= len(vz) + 3
