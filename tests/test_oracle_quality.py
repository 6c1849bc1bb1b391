"""Pins of the output policy and the track-quality flags (readings stated
with the library's pxt_config and pxt_tracks.flags).

The flags are single-precision decisions on the fitted values; each limit is
tested exactly at the threshold (kept) and one single-precision step beyond
it (dropped), for every bit and plane.  The quadruplets-only policy is
pinned by the property it rests on: cleaning the raw n-tuplets with the
triplets removed first keeps exactly the same longer tracks as cleaning
everything and dropping the triplets afterwards (brute-force cleaning by a
global sort, on PU~50 events)."""

import numpy as np

import eventgen
import oracle
from oracle import brute


def _up(x):
    return np.nextafter(np.float32(x), np.float32(np.inf))


def _flags(p, ch, n, det):
    return oracle.quality_flags(np.array(p, np.float32)[None], np.array(ch, np.float32)[None],
                                np.array([n]), det)[0]


def test_loose_chi2_limits(det):
    good = [0.0, 0.01, 0.5, 0.1, 1.0]
    # four hits: transverse ndf 1, longitudinal ndf 2; limit 5 per ndf
    assert _flags(good, [5.0, 10.0], 4, det) & 2
    assert not _flags(good, [_up(5.0), 10.0], 4, det) & 2
    assert not _flags(good, [5.0, _up(10.0)], 4, det) & 2
    # triplets: transverse ndf taken as 1, longitudinal 1
    assert _flags(good, [5.0, 5.0], 3, det) & 2
    assert not _flags(good, [0.0, _up(5.0)], 3, det) & 2
    # six hits: 3 and 4 degrees of freedom
    assert _flags(good, [15.0, 20.0], 6, det) & 2
    assert not _flags(good, [_up(15.0), 20.0], 6, det) & 2
    for i in range(5):
        bad = list(good)
        bad[i] = np.nan
        assert _flags(bad, [0.0, 0.0], 4, det) == 0


def test_strict_limits(det):
    base = [0.0, 0.01, 0.5, 0.1, 1.0]
    assert _flags(base, [0.0, 0.0], 4, det) == 6
    for i, at in ((2, 2.0), (2, -2.0), (1, 0.05), (1, -0.05), (4, 15.0), (4, -15.0)):
        p = list(base)
        p[i] = at
        assert _flags(p, [0.0, 0.0], 4, det) == 6, (i, at)
        p[i] = np.sign(at) * _up(abs(at))
        assert _flags(p, [0.0, 0.0], 4, det) == 2, (i, at)
    # strict needs loose
    assert _flags(base, [_up(5.0), 0.0], 4, det) == 0


def test_quadruplets_only_equals_cleaning_without_triplets(det):
    for seed in range(3):
        ev = eventgen.generate("pu50", 120 + seed, n_tracks=250)
        o3 = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det, min_hits=3)
        o4 = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det, min_hits=4)
        T, S = o3["raw"], o3["raw_score"]
        long_ = (T != oracle.PAD).sum(axis=1) >= 4
        keep = brute.clean(T[long_], S[long_])
        want = oracle.canonical(T[long_][keep])
        np.testing.assert_array_equal(oracle.canonical(o4["tracks"]), want)
        assert (o3["tracks"] != oracle.PAD).sum(axis=1).min() == 3  # triplets were there
        n4 = (o3["tracks"] != oracle.PAD).sum(axis=1) >= 4
        np.testing.assert_array_equal(o4["params"], o3["params"][n4])
