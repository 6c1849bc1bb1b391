"""Checks of the synthetic event generator (inputs of both sides)."""

import numpy as np
import pytest

import eventgen


def test_seeded_reproducible():
    a = eventgen.generate("pu50", 11)
    b = eventgen.generate("pu50", 11)
    for f in ("x", "y", "z", "layer", "track_of_hit"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    c = eventgen.generate("pu50", 12)
    assert not np.array_equal(a.x[:100], c.x[:100])


def test_dtypes_and_sizes():
    ev = eventgen.generate("pu50", 1)
    assert ev.x.dtype == np.float32 and ev.layer.dtype == np.int16
    assert 5500 < ev.n_hits < 7200
    ev = eventgen.generate("pu200", 1)
    assert 24000 < ev.n_hits < 31000
    assert ((ev.track_of_hit < 0).sum() / ev.n_hits) == pytest.approx(0.15 / 1.15, abs=0.01)


def test_hits_on_layer_surfaces():
    det = eventgen.DETECTOR
    lt = {l["id"]: l for l in det["layers"]}
    ev = eventgen.generate("pu50", 2)
    r = np.hypot(ev.x.astype(np.float64), ev.y.astype(np.float64))
    for lid, L in lt.items():
        m = ev.layer == lid
        if L["kind"] == eventgen.BARREL:
            assert np.all(np.abs(r[m] - L["r"]) < 1e-5)
            assert np.all(np.abs(ev.z[m]) <= L["zmax"])
        else:
            assert np.all(ev.z[m] == np.float32(L["z"]))
            assert np.all((r[m] > L["rmin"] - 0.01) & (r[m] < L["rmax"] + 0.01))


def test_noiseless_hits_have_generated_curvature():
    # three hits of a noiseless helix from the origin: their Menger curvature
    # is c_kappa / pT, up to float32 rounding of the coordinates
    det = eventgen.DETECTOR
    for seed in range(5):
        ev = eventgen.generate("tiny", seed)
        for t, h in enumerate(ev.track_hits):
            p = np.stack([ev.x[h], ev.y[h]], 1).astype(np.float64)
            a, b, c = p[0], p[1], p[3]
            cr = (b - a)[0] * (c - a)[1] - (b - a)[1] * (c - a)[0]
            k = 2 * cr / (np.linalg.norm(b - a) * np.linalg.norm(c - b) * np.linalg.norm(c - a))
            kt = -ev.tracks["q"][t] * det["c_kappa"] / ev.tracks["pt"][t]
            assert k == pytest.approx(kt, rel=2e-3)


def test_truth_hits_ordered_by_radius():
    ev = eventgen.generate("pu200", 3)
    r = np.hypot(ev.x.astype(np.float64), ev.y.astype(np.float64))
    for h in ev.track_hits[:500]:
        assert np.all(np.diff(r[h]) > 0)
        assert len(set(ev.layer[h].tolist())) == len(h)


def test_batch_mix_sizes():
    evs = eventgen.make_batch("batch", 8, seed=1)
    assert len(evs) == 8
    x, y, z, layer, offs = eventgen.concat_events(evs)
    assert offs[-1] == x.shape[0] and offs.dtype == np.uint32
    assert all(offs[i + 1] - offs[i] == evs[i].n_hits for i in range(8))
