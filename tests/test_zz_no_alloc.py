"""pxt_reconstruct_static (arenas in the library's fixed device buffer, no
allocation) against pxt_reconstruct on a context of the same config: two
calls in a row on the same buffer, the second with a smaller input.  Both
paths run the same kernels, so counts, per-event track counts, hit tuples,
parameters, covariances, chi2 and flags must be identical after putting the
tracks in canonical order."""

import numpy as np
import pytest

import eventgen

pytestmark = pytest.mark.gpu

DET = eventgen.DETECTOR
CAPS = dict(max_events=4, max_hits=32768, max_doublets=400_000, max_link_words=1_600_000,
            max_tuples=32768, max_tracks=32768)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def _canon(out, counts):
    n = counts["n_tracks"]
    h = out["hit_idx"][:n].view(np.uint32)
    key = np.concatenate([out["event_id"][:n, None].view(np.uint32), h], axis=1)
    o = np.lexsort(key.T[::-1]) if n else np.zeros(0, int)
    return {k: out[k][:n][o] for k in ("hit_idx", "n_hits", "event_id", "params", "cov", "chi2",
                                       "flags")}


def _same(a, b, ca, cb, n_events):
    for k in ("status", "n_tracks", "n_doublets", "n_links", "n_raw_tuples", "n_fp64",
              "n_hits_binned", "n_words"):
        assert ca[k] == cb[k], (k, ca[k], cb[k])
    np.testing.assert_array_equal(a["per_event_tracks"][:n_events],
                                  b["per_event_tracks"][:n_events])
    x, y = _canon(a, ca), _canon(b, cb)
    for k in x:
        np.testing.assert_array_equal(x[k], y[k], err_msg=k)


def _run(rec, torch, events, static):
    d = rec.upload(events)
    # outputs poisoned first, so every value compared was written by this call
    for t in (rec.o_hit_idx, rec.o_event_id, rec.o_per_event, rec.o_counts):
        t.fill_(-1)
    for t in (rec.o_params, rec.o_cov, rec.o_chi2):
        t.fill_(float("nan"))
    (rec.launch_static if static else rec.launch)(*d)
    torch.cuda.synchronize()
    counts = rec.read_counts()
    assert counts["status"] == 0, counts
    res = rec.result(len(events), counts).numpy()
    res["per_event_tracks"] = rec.o_per_event.cpu().numpy()
    return res, counts


def test_static_matches_context_two_calls(torch):
    import paper_2104_06573_amd as pxt
    rec = pxt.Reconstructor(DET, use_graph=0, **CAPS)
    big = [eventgen.generate("pu50", 300 + s) for s in range(3)]
    small = [eventgen.generate("tiny", 5)]
    for events in (big, small):
        print("static vs context: %d events, %d hits" %
              (len(events), sum(e.n_hits for e in events)), flush=True)
        ref, cref = _run(rec, torch, events, static=False)
        got, cgot = _run(rec, torch, events, static=True)
        assert cgot["n_tracks"] > 0
        _same(got, ref, cgot, cref, len(events))
    rec.close()


def test_static_rejects_oversize(torch):
    import paper_2104_06573_amd as pxt
    rec = pxt.Reconstructor(DET, use_graph=0, max_events=4, max_hits=32768,
                            max_doublets=4_000_000, max_link_words=16_000_000, max_tuples=32768,
                            max_tracks=1024)
    d = rec.upload([eventgen.generate("tiny", 1)])
    with pytest.raises(pxt.PxtError) as ei:
        rec.launch_static(*d)
    assert ei.value.status == pxt.ERR_CAPACITY
    assert "PXT_STATIC_SCRATCH_BYTES" in str(ei.value)
    rec.close()
