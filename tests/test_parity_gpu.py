"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Doublets, links, raw n-tuplets and surviving tracks must be identical sets
per event (bit-exact after canonical sorting); fitted parameters must agree
with the FP64 oracle within 1e-4 relative to max(|value|, floor) with floors
phi0 1 rad, d0 0.01 cm, q/pT 0.001 /GeV, cot(theta) 0.1, z0 1 cm; the
covariance diagonal within 1e-3 relative (its square roots).
"""

import numpy as np
import pytest

import eventgen
import oracle
from tests import constructed as cs
from tests.compare import (FIT_RTOL, canon_rows, correlations, fit_errors, match_tracks,
                           oracle_events, per_event_rows)

pytestmark = pytest.mark.gpu

DET = eventgen.DETECTOR


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def make_rec(det=DET, **kw):
    import paper_2104_06573_amd as pxt
    caps = dict(max_events=64, max_hits=1 << 20, max_doublets=1 << 22, max_link_words=1 << 24,
                max_tuples=1 << 20, max_tracks=1 << 19)
    caps.update(kw)
    return pxt.Reconstructor(det, **caps)


def run_and_dump(rec, events):
    import paper_2104_06573_amd as pxt
    res = rec.run_numpy(events)
    assert res.counts["status"] == 0, res.counts
    out = res.numpy()
    dumps = {k: rec.dump(v) for k, v in (("d", pxt.DUMP_DOUBLETS), ("l", pxt.DUMP_LINKS),
                                          ("r", pxt.DUMP_RAW))}
    return res, out, dumps


def check_events(events, res, out, dumps, check_cov=True, fit_stats=None, det=DET, oref=None):
    """Every event of a call against the oracle: doublets, links, raw
    n-tuplets (when dumps are given) and tracks bit-exact; fits within
    FIT_RTOL; covariance diagonal (square roots) within 1e-3 relative and
    its correlation coefficients within 1e-3; chi2 within 2e-3."""
    n = len(events)
    if oref is None:
        oref = oracle_events(events, det)
    if dumps is not None:
        D = per_event_rows(dumps["d"], n)
        L = per_event_rows(dumps["l"], n)
        R = per_event_rows(dumps["r"], n)
    tot_tracks = 0
    for e, ev in enumerate(events):
        o = oref[e]
        assert o["status"] == 0
        if dumps is not None:
            np.testing.assert_array_equal(D[e], canon_rows(o["doublets"]),
                                          err_msg="doublets ev%d" % e)
            np.testing.assert_array_equal(L[e], canon_rows(o["links"]), err_msg="links ev%d" % e)
            np.testing.assert_array_equal(R[e], canon_rows(o["raw"]), err_msg="raw tuples ev%d" % e)
        gh, gp, gc, gx, gf, oh, op, oc, ox = match_tracks(out, o, e)
        np.testing.assert_array_equal(gh, oh, err_msg="tracks ev%d" % e)
        assert int(out["per_event_tracks"][e]) == oh.shape[0]
        tot_tracks += oh.shape[0]
        if oh.shape[0] == 0:
            continue
        err = fit_errors(gp, op)
        if fit_stats is not None:
            fit_stats.append(err)
        bad = np.nonzero(err.max(axis=1) > FIT_RTOL)[0]
        assert bad.size == 0, ("fit ev%d" % e, err[bad[:5]], gp[bad[:5]], op[bad[:5]], gf[bad[:5]])
        if check_cov:
            diag = [0, 2, 5, 9, 14]
            sg = np.sqrt(gc[:, diag].astype(np.float64))
            so = np.sqrt(oc[:, diag])
            np.testing.assert_allclose(sg, so, rtol=1e-3, err_msg="cov diag ev%d" % e)
            np.testing.assert_allclose(correlations(gc), correlations(oc), rtol=0, atol=1e-3,
                                       err_msg="cov correlations ev%d" % e)
            np.testing.assert_allclose(gx, ox, rtol=2e-3, atol=2e-3, err_msg="chi2 ev%d" % e)
    assert res.counts["n_tracks"] == tot_tracks


def test_tiny_batch(torch):
    events = [eventgen.generate("tiny", s) for s in range(24)]
    rec = make_rec()
    res, out, dumps = run_and_dump(rec, events)
    check_events(events, res, out, dumps)


def test_separated_tracks_recover_truth(torch):
    events = [eventgen.generate("tiny", s, phi_spacing=True) for s in range(8)]
    rec = make_rec()
    res = rec.run_numpy(events).numpy()
    for e, ev in enumerate(events):
        m = res["event_id"] == e
        got = canon_rows(res["hit_idx"][m].view(np.uint32))
        truth = np.full((len(ev.track_hits), 8), 0xFFFFFFFF, np.uint32)
        for i, h in enumerate(ev.track_hits):
            truth[i, :len(h)] = h
        np.testing.assert_array_equal(got, canon_rows(truth))


def test_pu50_batch(torch):
    events = [eventgen.generate("pu50", 100 + s) for s in range(3)]
    rec = make_rec()
    res, out, dumps = run_and_dump(rec, events)
    stats = []
    check_events(events, res, out, dumps, fit_stats=stats)
    err = np.concatenate(stats)
    print("pu50 fit rel. error max", err.max(axis=0), "p99.9", np.percentile(err, 99.9, axis=0),
          "fp64 fraction %.4f" % (res.counts["n_fp64"] / max(res.counts["n_tracks"], 1)))


def test_pu200_event(torch):
    events = [eventgen.generate("pu200", 7)]
    rec = make_rec(max_doublets=3 << 20, max_link_words=24 << 20)
    res, out, dumps = run_and_dump(rec, events)
    stats = []
    check_events(events, res, out, dumps, fit_stats=stats)
    err = np.concatenate(stats)
    print("pu200 fit rel. error max", err.max(axis=0), "p99.9", np.percentile(err, 99.9, axis=0),
          "fp64 fraction %.4f" % (res.counts["n_fp64"] / max(res.counts["n_tracks"], 1)))


def test_fp64_refit_by_pt(torch):
    """The FP64 refit path at parity: with pt_fp64 = 2 GeV every track above
    2 GeV of reference pT is refitted in FP64 (FP64 flag set) and all fits
    still match the oracle; the refitted tracks' parameters also match those
    of the default configuration (FP32 with one refinement step)."""
    import paper_2104_06573_amd as pxt
    events = [eventgen.generate("pu50", 300 + s) for s in range(2)]
    oref = oracle_events(events, DET)
    rec = make_rec(pt_fp64=2.0)
    res, out, dumps = run_and_dump(rec, events)
    check_events(events, res, out, dumps, oref=oref)
    n64 = int(np.count_nonzero(out["flags"] & pxt.FLAG_FP64))
    assert n64 == res.counts["n_fp64"]
    hi = int(np.count_nonzero(np.abs(out["params"][:, 2]) < 1 / 2.5))
    assert n64 >= hi > 0, (n64, hi)
    base = make_rec().run_numpy(events).numpy()
    for e in range(len(events)):
        ga = match_tracks(out, oref[e], e)
        gb = match_tracks(base, oref[e], e)
        np.testing.assert_array_equal(ga[0], gb[0])
        assert (fit_errors(ga[1], gb[1].astype(np.float64)) <= FIT_RTOL).all()
    print("fp64 refits with pt_fp64 = 2 GeV: %d of %d tracks" % (n64, res.counts["n_tracks"]))


def _tracks_by_event(out, n):
    rows = []
    for e in range(n):
        m = out["event_id"] == e
        h = out["hit_idx"][m].view(np.uint32)
        o = np.lexsort(h.T[::-1]) if h.shape[0] else np.zeros(0, int)
        rows.append((h[o], out["params"][m][o], out["cov"][m][o]))
    return rows


def test_batch_equivalence(torch):
    # each event's result is the same alone, in a ragged batch, and in any
    # order of the batch (tracks bit-exact; fits bit-exact: same code)
    events = eventgen.make_batch("batch", 6, seed=3)
    rec = make_rec()
    batch = _tracks_by_event(rec.run_numpy(events).numpy(), len(events))
    perm = [4, 0, 5, 2, 1, 3]
    permuted = _tracks_by_event(rec.run_numpy([events[i] for i in perm]).numpy(), len(events))
    for e, ev in enumerate(events):
        alone = _tracks_by_event(rec.run_numpy([ev]).numpy(), 1)[0]
        for other in (batch[e], permuted[perm.index(e)]):
            np.testing.assert_array_equal(alone[0], other[0])
            np.testing.assert_array_equal(alone[1], other[1])
            np.testing.assert_array_equal(alone[2], other[2])


@pytest.mark.parametrize("phi_bins,block,group,lk,mode", [
    (16, 256, 16, 0, 0), (64, 64, 64, 1, 1), (1024, 128, 32, 1, 2), (4096, 256, 16, 1, 0),
    (256, 192, 64, 0, 2), (256, 64, 16, 0, 1), (256, 256, 16, 2, 0), (128, 64, 32, 2, 1),
    (512, 192, 16, 2, 2), (256, 256, 8, 0, 0), (64, 128, 8, 1, 1), (128, 256, 4, 0, 1)])
def test_tuning_invariance(torch, phi_bins, block, group, lk, mode):
    events = [eventgen.generate("pu50", 55), eventgen.generate("tiny", 3)]
    ref = _tracks_by_event(make_rec().run_numpy(events).numpy(), 2)
    got = _tracks_by_event(make_rec(phi_bins=phi_bins, block_size=block, group_lanes=group,
                                    link_kernel=lk, doublet_mode=mode).run_numpy(events).numpy(), 2)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


class _Ev:
    def __init__(self, x, y, z, layer):
        self.x = np.asarray(x, np.float32)
        self.y = np.asarray(y, np.float32)
        self.z = np.asarray(z, np.float32)
        self.layer = np.asarray(layer, np.int16)


# 256 phi bins: binning by one block per event; 4096: the histogram of an
# event exceeds LDS and the binning takes the global-atomic kernels
@pytest.mark.parametrize("phi_bins", [256, 4096])
def test_edge_cases(torch, phi_bins):
    tiny = eventgen.generate("tiny", 1)
    empty = _Ev([], [], [], [])
    one_layer = _Ev(tiny.x[tiny.layer == 0], tiny.y[tiny.layer == 0], tiny.z[tiny.layer == 0],
                    tiny.layer[tiny.layer == 0])
    bad_layers = _Ev(tiny.x, tiny.y, tiny.z, np.where(np.arange(tiny.n_hits) % 3 == 0, -1,
                                                      np.where(np.arange(tiny.n_hits) % 3 == 1,
                                                               99, tiny.layer)))
    dup = _Ev(np.concatenate([tiny.x, tiny.x[:10]]), np.concatenate([tiny.y, tiny.y[:10]]),
              np.concatenate([tiny.z, tiny.z[:10]]), np.concatenate([tiny.layer, tiny.layer[:10]]))
    events = [empty, tiny, one_layer, empty, bad_layers, dup, empty]
    rec = make_rec(phi_bins=phi_bins)
    res, out, dumps = run_and_dump(rec, events)
    check_events(events, res, out, dumps)
    # an empty batch
    import paper_2104_06573_amd as pxt
    x = torch.zeros(1, device="cuda")
    lay = torch.zeros(1, dtype=torch.int16, device="cuda")
    r = rec.run(x, x, x, lay, np.zeros(1, np.uint32))
    assert r.counts["status"] == 0 and r.counts["n_tracks"] == 0
    r = rec.run(x, x, x, lay, np.zeros(4, np.uint32))
    assert r.counts["status"] == 0 and r.counts["n_tracks"] == 0


def _dense_middle_event(seed=5, n_out=600):
    # one barrel-1 hit joined to a few barrel-0 hits and to n_out barrel-2
    # hits, all within the doublet cuts: a hit whose out-doublets need
    # several link-mask words (a stride above one)
    rng = np.random.default_rng(seed)
    r0, r1, r2 = 2.9, 6.8, 10.9
    p0 = rng.uniform(-0.01, 0.01, 5)
    p2 = rng.uniform(-0.05, 0.05, n_out)
    x = np.concatenate([r0 * np.cos(p0), [r1], r2 * np.cos(p2)])
    y = np.concatenate([r0 * np.sin(p0), [0.0], r2 * np.sin(p2)])
    z = np.concatenate([rng.uniform(-1, 1, 5), [0.0], rng.uniform(-3, 3, n_out)])
    lay = np.concatenate([np.zeros(5), [1], np.full(n_out, 2)])
    return _Ev(x, y, z, lay)


@pytest.mark.parametrize("lk", [0, 1, 2])
def test_dense_middle_hit(torch, lk):
    events = [_dense_middle_event(), eventgen.generate("tiny", 4)]
    rec = make_rec(link_kernel=lk)
    res, out, dumps = run_and_dump(rec, events)
    o = oracle.reconstruct(events[0].x, events[0].y, events[0].z, events[0].layer, DET)
    assert np.bincount(np.asarray(o["doublets"])[:, 0]).max() > 512
    check_events(events, res, out, dumps)


def _runs_are_grouped(rows):
    # rows (event, inner hit, outer hit) in device order: every inner hit's
    # doublets form one contiguous run
    key = rows[:, 0].astype(np.int64) * (1 << 32) + rows[:, 1]
    starts = np.concatenate([[True], key[1:] != key[:-1]])
    return np.unique(key).size == int(starts.sum())


@pytest.mark.parametrize("group,block", [(4, 256), (8, 256), (16, 128), (64, 64)])
def test_doublet_modes(torch, group, block):
    # the one-pass and staged doublet kernels, from their records and from
    # their recompute paths (the dense hit's 600 doublets exceed the
    # record's 9-bit index, so its tile or block evaluates the cuts again),
    # give the two-pass results: doublets grouped by inner hit, and the same
    # doublets, links, n-tuplets and tracks.  (Hits within a phi bin are
    # binned in arrival order, so the raw order varies from run to run.)
    events = [eventgen.generate("pu50", 21), _dense_middle_event(), eventgen.generate("tiny", 5)]
    n = len(events)
    ref = None
    for mode in (0, 1, 2):
        rec = make_rec(group_lanes=group, block_size=block, doublet_mode=mode)
        res, out, dumps = run_and_dump(rec, events)
        assert _runs_are_grouped(np.asarray(dumps["d"]).reshape(-1, 3)), mode
        if ref is None:
            check_events(events, res, out, dumps)
            ref = ({k: per_event_rows(dumps[k], n) for k in ("d", "l", "r")},
                   _tracks_by_event(out, n))
            continue
        for k in ("d", "l", "r"):
            for e, (a, b) in enumerate(zip(ref[0][k], per_event_rows(dumps[k], n))):
                np.testing.assert_array_equal(a, b, err_msg="%s ev%d mode %d" % (k, e, mode))
        for a, b in zip(ref[1], _tracks_by_event(out, n)):
            np.testing.assert_array_equal(a[0], b[0])


def test_capacity_overflow_and_retry(torch):
    import paper_2104_06573_amd as pxt
    events = [eventgen.generate("pu50", 9)]
    o = oracle.reconstruct(events[0].x, events[0].y, events[0].z, events[0].layer, DET)
    nd, nt, nk = len(o["doublets"]), len(o["raw"]), len(o["tracks"])
    # link-mask words: one stride per doublet, ceil(largest out-degree / 64)
    outdeg = np.bincount(np.asarray(o["doublets"])[:, 0])
    nw = nd * int((outdeg.max() + 63) // 64)
    for caps, idx, need in ((dict(max_doublets=nd - 1), 0, nd),
                            (dict(max_link_words=nw - 1), 1, nw),
                            (dict(max_tuples=nt - 1), 2, nt),
                            (dict(max_tracks=nk - 1), 3, nk)):
        rec = make_rec(**caps)
        r = rec.run_numpy(events)
        assert r.counts["status"] == pxt.ERR_CAPACITY, (caps, r.counts)
        assert r.counts["required"][idx] == need, (caps, r.counts)
        assert r.counts["n_tracks"] == 0
    for mode in (0, 1):  # the two-pass and one-pass kernels (mode 2 above)
        r = make_rec(max_doublets=nd - 1, doublet_mode=mode).run_numpy(events)
        assert r.counts["status"] == pxt.ERR_CAPACITY and r.counts["required"][0] == nd, r.counts
    rec = make_rec(max_doublets=nd, max_tuples=nt, max_tracks=nk)
    r = rec.run_numpy(events)
    assert r.counts["status"] == 0 and r.counts["n_tracks"] == nk
    # at exactly the raw n-tuplet capacity the n-tuplet walk's staging
    # regions (the capacity split over the grid's wavefronts) are too small
    # and every wavefront walks its roots again: still the oracle's tracks
    check_events(events, r, r.numpy(), None, check_cov=False, oref=[o])
    # the context recovers after an overflow on the next call
    rec2 = make_rec(max_doublets=nd - 1)
    assert rec2.run_numpy(events).counts["status"] == pxt.ERR_CAPACITY
    assert rec2.run_numpy([eventgen.generate("tiny", 2)]).counts["status"] == 0


def test_invalid_arguments(torch):
    import paper_2104_06573_amd as pxt
    rec = make_rec(max_events=2, max_hits=1000)
    ev = eventgen.generate("tiny", 0)
    x, y, z, lay, offs = rec.upload([ev, ev, ev])
    with pytest.raises(pxt.PxtError) as e:
        rec.launch(x, y, z, lay, offs)
    assert e.value.status == pxt.ERR_INVALID_ARG
    with pytest.raises(pxt.PxtError):
        rec.launch(x, y, z, lay, np.array([0, 50, 40], np.uint32))
    big = eventgen.generate("pu50", 0)
    x, y, z, lay, offs = rec.upload([big])
    with pytest.raises(pxt.PxtError):
        rec.launch(x, y, z, lay, offs)


def test_graph_replays_match_direct(torch):
    # the launch sequence captured once per staging slot and replayed for
    # batches of different sizes must give exactly the direct-mode results;
    # eager work and synchronisations sit between the replays
    batches = [eventgen.make_batch("batch", n, seed=20 + n) for n in (3, 1, 5, 2, 4, 1, 3)]
    batches.append([eventgen.generate("tiny", 4)])
    # the binning of each call by one block per event (eight events or
    # more, or only small ones) or by the global kernels (a few large
    # events), in turn on the same context (a graph per slot and kernel set)
    batches += [eventgen.make_batch("batch", 9, seed=40), [eventgen.generate("pu200", 41)],
                [eventgen.generate("pu50", 42 + s) for s in range(2)],
                [eventgen.generate("pu200", 43), eventgen.generate("tiny", 44)],
                eventgen.make_batch("batch", 8, seed=45)]
    direct = make_rec()
    graph = make_rec(use_graph=1)
    for i, evs in enumerate(batches):
        ref = direct.run_numpy(evs)
        got = graph.run_numpy(evs)
        assert got.counts == ref.counts, (i, got.counts, ref.counts)
        a = _tracks_by_event(ref.numpy(), len(evs))
        b = _tracks_by_event(got.numpy(), len(evs))
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x[0], y[0])
            np.testing.assert_array_equal(x[1], y[1])
            np.testing.assert_array_equal(x[2], y[2])
        np.testing.assert_array_equal(ref.numpy()["per_event_tracks"],
                                      got.numpy()["per_event_tracks"])
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
    # a graph replay also overflows cleanly and recovers
    small = make_rec(use_graph=1, max_doublets=1000)
    r = small.run_numpy([eventgen.generate("pu50", 3)])
    assert r.counts["status"] == 2
    assert small.run_numpy([eventgen.generate("tiny", 5)]).counts["status"] == 0


@pytest.mark.parametrize("use_graph", [0, 1])
def test_election_slots_across_calls(torch, use_graph):
    """The cleaning's per-doublet slots are tagged with the call rather than
    cleared: 300 calls alternating two different batches on one context
    (across the tag's wrap after 256 calls and its full reset) give every
    time the tracks of the first call of that batch, which match the
    oracle."""
    a = [eventgen.generate("pu50", 400 + s) for s in range(2)]
    b = [eventgen.generate("pu50", 410 + s) for s in range(3)]
    rec = make_rec(use_graph=use_graph)
    up = [rec.upload(a), rec.upload(b)]
    ref = []
    for i, evs in enumerate((a, b)):
        r = rec.run(*up[i])
        check_events(evs, r, r.numpy(), None, check_cov=False)
        ref.append((r.counts, _tracks_by_event(r.numpy(), len(evs))))
    for call in range(2, 300):
        i = call % 2
        r = rec.run(*up[i])
        counts, tracks = ref[i]
        assert r.counts == counts, (call, r.counts, counts)
        if call % 16 == 0 or call > 250:
            for x, y in zip(tracks, _tracks_by_event(r.numpy(), len(up[i][4]) - 1)):
                np.testing.assert_array_equal(x[0], y[0])
                np.testing.assert_array_equal(x[1], y[1])


def test_constructed_cleaning_cases(torch):
    # hand-built events whose winner is fixed by geometry (tests/constructed):
    # the score's closed form, the impact term deciding, the length rule
    # beating a lower score, bitwise-equal scores decided by the hit order
    # (within one root and across roots), the longest path of 8 hits
    cases = [(cs.scored_quadruplet(DET), DET), (cs.impact_decides(DET)[0], DET),
             (cs.longer_beats_lower_score(DET)[0], DET), (cs.exact_tie(DET, True)[0], DET),
             (cs.exact_tie(DET, False)[0], DET)]
    ev, d, _ = cs.tie_across_roots(DET)
    cases.append((ev, d))
    cases.append((cs.chain_event(8), cs.chain_detector(DET, 8)))
    for mode in (0, 1, 2):
        for ev, d in cases:
            rec = make_rec(det=d, max_events=4, max_hits=4096, max_doublets=1 << 16,
                           max_tuples=1 << 14, max_tracks=1 << 14, doublet_mode=mode)
            res, out, dumps = run_and_dump(rec, [ev])
            check_events([ev], res, out, dumps, det=d)
            rec.close()


@pytest.mark.parametrize("lk", [0, 1, 2])
def test_rz_cut_at_its_threshold(torch, lk):
    # r-z turns within 1e-5 (relative) of the cut on either side: the link
    # prefilter (16-bit angles, widened windows) must keep both candidates
    # and the exact cut decide them as the oracle does
    events = [cs.rz_threshold_triplet(DET, inside)[0] for inside in (True, False)]
    rec = make_rec(link_kernel=lk)
    res, out, dumps = run_and_dump(rec, events)
    check_events(events, res, out, dumps)
    assert res.counts["n_links"] == 1


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_doublet_curvature_cut_in_its_band(torch, mode):
    # doublets within 1e-9 of the curvature cut on either side: inside the
    # fast squared form's band, the defining expression decides, in every
    # doublet kernel as in the oracle
    events = [cs.curvature_threshold_doublet(DET, inside)[0] for inside in (True, False)]
    rec = make_rec(doublet_mode=mode)
    res, out, dumps = run_and_dump(rec, events)
    check_events(events, res, out, dumps)
    assert res.counts["n_doublets"] == 1


def test_link_impact_cut_in_its_band(torch):
    # triplets within 1e-9 of the impact cut on either side: inside the
    # division-free form's band, the defining expression decides, in every
    # link kernel as in the oracle (one event per triplet)
    events = [cs.impact_threshold_triplet(DET, inside)[0] for inside in (True, False)]
    # and the same for the r-z and curvature cuts' squared forms
    events += [cs.rz_band_triplet(DET, inside)[0] for inside in (True, False)]
    events += [cs.curvature_band_triplet(DET, inside)[0] for inside in (True, False)]
    for lk in (0, 1, 2):
        rec = make_rec(link_kernel=lk)
        res, out, dumps = run_and_dump(rec, events)
        check_events(events, res, out, dumps)
        assert res.counts["n_links"] == 3
        rec.close()


def test_path_longer_than_eight_hits(torch):
    import paper_2104_06573_amd as pxt
    d9 = cs.chain_detector(DET, 9)
    ev9 = cs.chain_event(9)
    o = oracle.reconstruct(ev9.x, ev9.y, ev9.z, ev9.layer, d9)
    assert o["status"] == 1
    rec = make_rec(det=d9, max_events=4, max_hits=4096, max_doublets=1 << 16,
                   max_tuples=1 << 14, max_tracks=1 << 14)
    r = rec.run_numpy([eventgen.generate("tiny", 1, det=DET), ev9])
    assert r.counts["status"] == pxt.ERR_PATH, r.counts
    assert r.counts["n_tracks"] == 0
    # the context recovers: the same track on eight of the nine layers
    keep = np.arange(8)
    ev8 = cs.Ev(ev9.x[keep], ev9.y[keep], ev9.z[keep], ev9.layer[keep])
    res, out, dumps = run_and_dump(rec, [ev8])
    check_events([ev8], res, out, dumps, det=d9)


def test_quadruplets_only(torch):
    # min_hits 4: only quadruplets and longer come out, the same ones as the
    # oracle's; doublets, links and raw n-tuplets are unchanged
    det4 = {**DET, "quality": {**DET["quality"], "min_hits": 4}}
    events = [eventgen.generate("pu50", 100 + s) for s in range(3)]
    rec = make_rec(det=det4)
    res, out, dumps = run_and_dump(rec, events)
    assert out["n_hits"].min() >= 4
    check_events(events, res, out, dumps, det=det4)


def test_quality_flags(torch):
    # LOOSE / STRICT bits against the oracle's decisions on its own fitted
    # values; a track whose oracle value lies within the fit tolerance of a
    # limit may go either way and is left out (counted and printed)
    events = [eventgen.generate("pu50", 100 + s) for s in range(3)]
    rec = make_rec()
    res = rec.run_numpy(events)
    assert res.counts["status"] == 0
    out = res.numpy()
    oref = oracle_events(events, DET)
    q = DET["quality"]
    checked = near = 0
    for e in range(len(events)):
        gh, gp, gc, gx, gf, oh, op, oc, ox = match_tracks(out, oref[e], e)
        n = (oh != 0xFFFFFFFF).sum(axis=1)
        want = oracle.quality_flags(op, ox, n, DET)
        ndf_c = np.maximum(n - 3, 1)
        ndf_z = n - 2
        rel = lambda v, lim, fl: np.abs(np.abs(v) - lim) <= 1e-4 * np.maximum(np.abs(v), fl)
        close = (rel(op[:, 2], 1.0 / q["pt_min"], 0.001) | rel(op[:, 1], q["d0_max"], 0.01)
                 | rel(op[:, 4], q["z0_max"], 1.0)
                 | (np.abs(ox[:, 0] - q["chi2"] * ndf_c) <= 2e-3 * (1 + ox[:, 0]))
                 | (np.abs(ox[:, 1] - q["chi2"] * ndf_z) <= 2e-3 * (1 + ox[:, 1])))
        got = gf & 6
        np.testing.assert_array_equal(got[~close], want[~close])
        checked += int((~close).sum())
        near += int(close.sum())
    frac = lambda b: float(np.mean((out["flags"] & b) != 0))
    print("flags: %d tracks compared, %d near a limit; loose %.3f strict %.3f fp64 %.4f" %
          (checked, near, frac(2), frac(4), frac(1)))
    assert checked > 0.99 * (checked + near)
