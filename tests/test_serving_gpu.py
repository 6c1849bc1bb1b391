"""Continuous-batching server: each event's result is the same alone and in
the mix, an oversize event fails alone, and the counters add up."""

import numpy as np
import pytest

import eventgen

pytestmark = pytest.mark.gpu

DET = eventgen.DETECTOR
CAPS = dict(max_events=16, max_hits=1 << 17, max_doublets=1 << 21, max_link_words=1 << 23,
            max_tuples=1 << 18, phi_bins=256)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def _solo(events):
    import paper_2104_06573_amd as pxt
    rec = pxt.Reconstructor(DET, max_tracks=1 << 18, **dict(CAPS, max_events=1))
    out = []
    for ev in events:
        r = rec.run_numpy([ev]).numpy()
        h = r["hit_idx"].view(np.uint32)
        o = np.lexsort(h.T[::-1]) if h.shape[0] else np.zeros(0, int)
        out.append((h[o], r["params"][o], r["cov"][o]))
    rec.close()
    return out


def _canon(res):
    h = res["hit_idx"].view(np.uint32)
    o = np.lexsort(h.T[::-1]) if h.shape[0] else np.zeros(0, int)
    return h[o], res["params"][o], res["cov"][o]


def test_mix_equals_solo(torch):
    from paper_2104_06573_amd.serve import Server, poisson_run
    events = eventgen.make_batch("serve", 24, seed=5)
    solo = _solo(events)
    srv = Server(DET, n_lanes=3, max_batch_events=8, **CAPS)
    # arrivals 50 us apart on average, several times faster than a batch
    # takes on the device: requests arrive while others are on the GPU, so
    # some are admitted together into one batch
    rep = poisson_run(srv, events, rate_hz=20000.0, keep_results=True)
    st = srv.stats()
    srv.close()
    assert rep["failed"] == 0
    assert st["completed"] == len(events) and st["failed"] == 0
    assert max(r["batch_events"] for r in rep["results"]) > 1, st
    for i, (res, ref) in enumerate(zip(rep["results"], solo)):
        got = _canon(res)
        np.testing.assert_array_equal(got[0], ref[0], err_msg="tracks of event %d" % i)
        np.testing.assert_array_equal(got[1], ref[1], err_msg="params of event %d" % i)
        np.testing.assert_array_equal(got[2], ref[2], err_msg="cov of event %d" % i)


def test_burst_is_batched_and_exact(torch):
    # a burst submitted at once is served in multi-event batches
    from paper_2104_06573_amd.serve import Server
    events = [eventgen.generate("pu50", 700 + i, n_tracks=400) for i in range(20)]
    solo = _solo(events)
    srv = Server(DET, n_lanes=2, max_batch_events=8, **CAPS)
    tickets = [srv.submit(e.x, e.y, e.z, e.layer) for e in events]
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["events_in_batches"] / st["batches"] > 1.5, st
    assert max(r["batch_events"] for r in res) > 1
    for r, ref in zip(res, solo):
        assert r["status"] == 0
        got = _canon(r)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])


def test_oversize_event_fails_alone(torch):
    import paper_2104_06573_amd as pxt
    from paper_2104_06573_amd.serve import Server
    small = [eventgen.generate("pu50", 800 + i, n_tracks=150) for i in range(6)]
    big = eventgen.generate("pu200", 3)
    caps = dict(CAPS, max_doublets=400_000, max_link_words=1_600_000)
    srv = Server(DET, n_lanes=1, max_batch_events=8, doublets_per_hit=1, **caps)
    evs = small[:3] + [big] + small[3:]
    tickets = [srv.submit(e.x, e.y, e.z, e.layer) for e in evs]
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert res[3]["status"] == pxt.ERR_CAPACITY
    assert all(r["status"] == 0 for i, r in enumerate(res) if i != 3)
    assert st["failed"] == 1 and st["completed"] == len(evs)
    solo = _solo(small)
    for r, ref in zip(res[:3] + res[4:], solo):
        np.testing.assert_array_equal(_canon(r)[0], ref[0])


def test_poll_timeout_and_unknown_ticket(torch):
    import paper_2104_06573_amd as pxt
    from paper_2104_06573_amd.serve import Server
    srv = Server(DET, n_lanes=1, **CAPS)
    with pytest.raises(pxt.PxtError):
        srv.poll(123456, 0)
    ev = eventgen.generate("tiny", 1)
    t = srv.submit(ev.x, ev.y, ev.z, ev.layer)
    r = None
    while r is None:
        r = srv.poll(t, 10)
    assert r["status"] == 0 and r["n_tracks"] == 20
    srv.close()


def test_native_replay_and_phases(torch):
    # the native replay: a burst of 96 events of the serving mix is admitted
    # into multi-event batches, every event comes back with the track count
    # it has alone, and the phase means add up to about the latency
    from paper_2104_06573_amd.serve import Server, poisson_schedule, replay
    pool = eventgen.make_batch("serve", 12, seed=9)
    solo = _solo(pool)
    srv = Server(DET, n_lanes=2, max_batch_events=16, **CAPS)
    order, at = poisson_schedule(96, float("inf"), len(pool))
    rep = replay(srv, pool, order, at)
    assert rep["failed"] == 0 and rep["max_batch"] > 1
    assert rep["n_tracks"] == [solo[i % len(pool)][0].shape[0] for i in range(96)]
    ph = rep["phases_us"]
    parts = ph["queue"] + ph["launch"] + ph["device"] + ph["copyback"] + ph["deliver"]
    assert abs(parts - ph["latency"]) <= 0.05 * ph["latency"] + 50, ph
    # at a modest rate as well
    order, at = poisson_schedule(48, 5000.0, len(pool), seed=1)
    rep2 = replay(srv, pool, order, at)
    assert rep2["failed"] == 0
    assert rep2["n_tracks"] == [solo[i % len(pool)][0].shape[0] for i in range(48)]
    st = srv.stats()
    srv.close()
    assert st["completed"] == st["delivered"] == 144


def test_release_without_copy(torch):
    import ctypes

    from paper_2104_06573_amd import OK, lib
    from paper_2104_06573_amd.serve import EventTracks, Server
    ev = eventgen.generate("pu50", 3, n_tracks=300)
    solo = _solo([ev])
    srv = Server(DET, n_lanes=1, **CAPS)
    t = srv.submit(ev.x, ev.y, ev.z, ev.layer)
    et = EventTracks(0, None, None, None, None, None, None, 0, 0, 0.0, 0.0, 0)
    assert lib().pxt_poll(srv.h, t, ctypes.byref(et), -1) == OK
    assert et.status == OK and et.n_tracks == solo[0][0].shape[0]
    # the ticket is gone
    with pytest.raises(Exception):
        srv.poll(t, 0)
    srv.close()
