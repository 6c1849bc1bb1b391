"""Oracle parity at the shapes the benchmark times.

The benchmark's batched PU~50 step is a 64-event batch replayed as a HIP
graph (8-lane groups, thread-per-doublet links, staged doublets), with
several contexts taking turns on their own streams; its PU~200 step is a
32-event batch the same way; its plain and served paths run the one-pass
doublet kernel on single events.  Each test below runs exactly such a
configuration (the benchmark's own capacity recipe) and compares every
event with the CPU oracle: doublets, links, raw n-tuplets and tracks
bit-exact, fits within 1e-4 relative, covariances and chi2 as in
test_parity_gpu.  The oracle runs one event per host thread.
"""

import numpy as np
import pytest

import bench
import eventgen
from tests.compare import oracle_events
from tests.test_parity_gpu import check_events

pytestmark = pytest.mark.gpu

DET = eventgen.DETECTOR


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def _rec(kind, events, n_events=None, **tuning):
    import paper_2104_06573_amd as pxt
    if n_events is None:
        caps = bench.batch_caps(kind, len(events), sum(e.n_hits for e in events))
    else:
        caps = bench.batch_caps(kind, n_events, max(e.n_hits for e in events) * n_events)
    caps.update({k: tuning.pop(k) for k in list(tuning) if k.startswith("max_")})
    kw = dict(phi_bins=1024, group_lanes=8, link_kernel=0, use_graph=1, doublet_mode=2)
    kw.update(tuning)
    return pxt.Reconstructor(DET, **caps, **kw)


def _dumps(rec):
    import paper_2104_06573_amd as pxt
    return {k: rec.dump(v) for k, v in (("d", pxt.DUMP_DOUBLETS), ("l", pxt.DUMP_LINKS),
                                         ("r", pxt.DUMP_RAW))}


def _check(rec, events, oref, res=None, dumps=True):
    if res is None:
        res = rec.result(len(events))
    assert res.counts["status"] == 0, res.counts
    check_events(events, res, res.numpy(), _dumps(rec) if dumps else None, oref=oref)
    return res


def test_pu50_batch64_graph_two_contexts(torch):
    # the headline step: 64 PU~50 events, graph replay, replayed twice through
    # one context while a second context runs another batch on its own stream
    a = bench.gen_events("pu50", 64, 1000)
    b = bench.gen_events("pu50", 64, 1097)
    oa = oracle_events(a, DET)
    ob = oracle_events(b, DET)
    ra, rb = _rec("pu50", a), _rec("pu50", b)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    da, db = ra.upload(a), rb.upload(b)
    torch.cuda.synchronize()
    ra.launch(*da, stream=sa)
    rb.launch(*db, stream=sb)
    torch.cuda.synchronize()
    _check(ra, a, oa)
    _check(rb, b, ob)
    # second replays of both graphs, again side by side
    ra.launch(*da, stream=sa)
    rb.launch(*db, stream=sb)
    ra.launch(*da, stream=sa)
    torch.cuda.synchronize()
    _check(ra, a, oa)
    _check(rb, b, ob, dumps=False)


def test_pu200_batch_graph(torch):
    # eight events: the call bins by one block per event (as the benchmark's
    # 32-event batches do), where a single PU~200 event takes the global
    # kernels (test_pu200_event)
    events = bench.gen_events("pu200", 8, 1000)
    oref = oracle_events(events, DET)
    rec = _rec("pu200", events)
    d = rec.upload(events)
    for _ in range(2):
        rec.launch(*d)
        torch.cuda.synchronize()
        res = _check(rec, events, oref)
    print("pu200 x8 graph: %d tracks, fp64 fraction %.4f" %
          (res.counts["n_tracks"], res.counts["n_fp64"] / max(res.counts["n_tracks"], 1)))


def test_ragged_batch64_graph(torch):
    # the ragged mix: 64 events with U{300..3000} tracks each
    # (doublets grow with the square of the hits: the mix's 3000-track events
    # need more than the PU~50 recipe's 100k per event)
    events = eventgen.make_batch("batch", 64, seed=7)
    oref = oracle_events(events, DET)
    rec = _rec("pu50", events, max_doublets=12 << 20, max_link_words=48 << 20)
    d = rec.upload(events)
    rec.launch(*d)
    torch.cuda.synchronize()
    _check(rec, events, oref)


@pytest.mark.parametrize("graph", [0, 1])
def test_latency_mode_single_events(torch, graph):
    # the plain and served paths: one event per call, one-pass doublets
    events = bench.gen_events("pu50", 8, 1000)
    oref = oracle_events(events, DET)
    rec = _rec("pu50", events, n_events=1, doublet_mode=1, use_graph=graph)
    for ev, o in zip(events, oref):
        rec.run_numpy([ev])
        _check(rec, [ev], [o])
