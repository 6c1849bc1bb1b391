"""Pins of the oracle's cleaning score and order, and of its path-length
limit, on hand-built events (tests/constructed.py).

The score of a tuple is the sum over its consecutive hit triples of
(r-z turning sine / arz)^2 + (transverse impact / d0max)^2; each test below
fails under a plausible mistake in it: a dropped square, a dropped impact
term, a reversed or missing index tie-break, a path limit off by one.
"""

import numpy as np
import pytest

import oracle
from tests import constructed as cs


def _row(t):
    return tuple(int(v) for v in t[t != oracle.PAD])


def _score_of(r, hits):
    for t, s in zip(r["raw"], r["raw_score"]):
        if _row(t) == hits:
            return s
    raise AssertionError("tuple %s not found in %s" % (hits, [_row(t) for t in r["raw"]]))


def test_score_closed_form_on_a_quadruplet(det):
    ev = cs.scored_quadruplet(det)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert r["status"] == 0
    assert [_row(t) for t in r["raw"]] == [(0, 1, 2, 3)]
    e1 = cs.triple_score_expected(det, ev, 0, 1, 2)
    e2 = cs.triple_score_expected(det, ev, 1, 2, 3)
    # both terms of both triples are sizeable: a dropped square or a dropped
    # impact term moves the sum by far more than the tolerance
    q1 = cs.rz_sine(*[(float(ev.x[i]), float(ev.y[i]), float(ev.z[i])) for i in (0, 1, 2)])
    assert abs(q1) / det["cuts"]["arz"] > 0.5
    assert 0.5 < cs.impact_exact(*[(float(ev.x[i]), float(ev.y[i]), float(ev.z[i]))
                                   for i in (0, 1, 2)]) / det["cuts"]["d0max"] < 0.7
    assert _score_of(r, (0, 1, 2, 3)) == pytest.approx(e1 + e2, rel=1e-10)


def test_score_closed_form_on_its_triplets(det):
    # the same hits as two separate triplets (layer 3 removed, then layer 0)
    ev = cs.scored_quadruplet(det)
    for keep in ((0, 1, 2), (1, 2, 3)):
        sub = cs.Ev(ev.x[list(keep)], ev.y[list(keep)], ev.z[list(keep)], ev.layer[list(keep)])
        r = oracle.reconstruct(sub.x, sub.y, sub.z, sub.layer, det)
        assert [_row(t) for t in r["raw"]] == [(0, 1, 2)]
        assert _score_of(r, (0, 1, 2)) == pytest.approx(
            cs.triple_score_expected(det, sub, 0, 1, 2), rel=1e-10)


def test_cleaning_decided_by_the_impact_term(det):
    ev, winner = cs.impact_decides(det)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert sorted(_row(t) for t in r["raw"]) == [(0, 1, 2), (0, 1, 3)]
    s2, s3 = _score_of(r, (0, 1, 2)), _score_of(r, (0, 1, 3))
    # the r-z terms are equal, so the scores differ by the impact terms only
    d2 = cs.impact_exact(*[(float(ev.x[i]), float(ev.y[i]), float(ev.z[i])) for i in (0, 1, 2)])
    d3 = cs.impact_exact(*[(float(ev.x[i]), float(ev.y[i]), float(ev.z[i])) for i in (0, 1, 3)])
    d0max = det["cuts"]["d0max"]
    assert s2 - s3 == pytest.approx((d2 / d0max) ** 2 - (d3 / d0max) ** 2, rel=1e-9)
    assert d2 > 10 * d3
    assert [_row(t) for t in r["tracks"]] == [winner]


@pytest.mark.parametrize("low_first", [True, False])
def test_exact_tie_goes_to_the_lower_hit_tuple(det, low_first):
    ev, winner = cs.exact_tie(det, low_first)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert sorted(_row(t) for t in r["raw"]) == [(0, 1, 2), (0, 1, 3)]
    # bitwise-equal scores: only the index order can decide
    assert _score_of(r, (0, 1, 2)) == _score_of(r, (0, 1, 3))
    assert [_row(t) for t in r["tracks"]] == [winner]


def test_longest_path_is_kept(det):
    d8 = cs.chain_detector(det, 8)
    ev = cs.chain_event(8)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, d8)
    assert r["status"] == 0
    assert [_row(t) for t in r["tracks"]] == [tuple(range(8))]
    assert np.all(np.isfinite(r["params"]))


def test_path_longer_than_eight_hits_is_an_error(det):
    d9 = cs.chain_detector(det, 9)
    ev = cs.chain_event(9)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, d9)
    assert r["status"] == 1  # ORC_ERR_PATH_TOO_LONG
    # and the same track on eight of the nine layers is fine
    keep = np.arange(8)
    r8 = oracle.reconstruct(ev.x[keep], ev.y[keep], ev.z[keep], ev.layer[keep], d9)
    assert r8["status"] == 0 and len(r8["tracks"]) == 1


def test_longer_tuple_beats_a_lower_score(det):
    ev, winner = cs.longer_beats_lower_score(det)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert sorted(_row(t) for t in r["raw"]) == [(0, 1, 2, 3), (0, 1, 4)]
    assert _score_of(r, (0, 1, 4)) < 0.2 * _score_of(r, (0, 1, 2, 3))
    assert [_row(t) for t in r["tracks"]] == [winner]


def test_exact_tie_across_roots(det):
    ev, d, winner = cs.tie_across_roots(det)
    r = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, d)
    rows = [_row(t) for t in r["raw"]]
    assert sorted(rows) == [(0, 2, 3), (1, 2, 3)]
    # the loser's root doublet is met first
    assert rows[0] == (1, 2, 3)
    assert _score_of(r, (0, 2, 3)) == _score_of(r, (1, 2, 3))
    assert [_row(t) for t in r["tracks"]] == [winner]


@pytest.mark.parametrize("inside", [True, False])
def test_rz_cut_at_its_threshold(det, inside):
    # a straight transverse line through the origin whose r-z segments turn
    # by an angle with sine within 1e-5 of arz (set on the float32
    # coordinates, checked by the arctan2 route): the link exists exactly
    # when the sine is below arz
    ev, s = cs.rz_threshold_triplet(det, inside)
    arz = det["cuts"]["arz"]
    assert (s < arz) == inside and abs(s / arz - 1.0) < 2e-5
    o = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert len(o["doublets"]) == 2
    assert len(o["links"]) == (1 if inside else 0)
    assert len(o["tracks"]) == (1 if inside else 0)


@pytest.mark.parametrize("inside", [True, False])
def test_doublet_curvature_cut_in_its_band(det, inside):
    # a doublet whose curvature is within 1e-9 of kmax (from 50-digit
    # arithmetic on its float32 coordinates): the oracle keeps it exactly
    # when it is below
    ev, q = cs.curvature_threshold_doublet(det, inside)
    assert (q < 0) == inside and 1e-12 <= abs(q) <= 1e-9
    o = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert len(o["doublets"]) == (1 if inside else 0)


@pytest.mark.parametrize("inside", [True, False])
def test_link_impact_cut_in_its_band(det, inside):
    # a triplet whose transverse impact is within 1e-9 of d0max (from exact
    # rational arithmetic on its float32 coordinates), the other cuts
    # holding with room: the oracle links it exactly when it is below
    ev, q = cs.impact_threshold_triplet(det, inside)
    assert (q < 0) == inside and 1e-12 <= abs(q) <= 1e-9
    o = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert len(o["doublets"]) == 2
    assert len(o["links"]) == (1 if inside else 0)


@pytest.mark.parametrize("inside", [True, False])
def test_link_rz_cut_in_its_band(det, inside):
    # a triplet whose r-z turn has a sine within 1e-9 of arz (50-digit
    # arithmetic on its float32 coordinates): linked exactly when below
    ev, q = cs.rz_band_triplet(det, inside)
    assert (q < 0) == inside and 1e-12 <= abs(q) <= 1e-9
    o = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert len(o["doublets"]) == 2
    assert len(o["links"]) == (1 if inside else 0)


@pytest.mark.parametrize("inside", [True, False])
def test_link_curvature_cut_in_its_band(det, inside):
    # a triplet whose circle's curvature is within 1e-9 of kmax (50-digit
    # arithmetic on its float32 coordinates), the doublet and impact cuts
    # holding with room: linked exactly when below
    ev, q = cs.curvature_band_triplet(det, inside)
    assert (q < 0) == inside and 1e-12 <= abs(q) <= 1e-9
    o = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, det)
    assert len(o["doublets"]) == 2
    assert len(o["links"]) == (1 if inside else 0)
