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
