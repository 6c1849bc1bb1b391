"""RecHits on the GPU (pxt_rechits) against the oracle: the clusters of a
ragged batch (PU~50 events, a tiny event, an empty event) become hits with
identical per-module offsets, event offsets, hit order, layer, module and
cluster ids, and bit-identical single-precision x, y, z (both sides sum the
charges in pixel order and use the same operations in double precision:
additions, products, one division and one square root, no transcendental
function).  The module limit is exercised at its default and at 3 (many
modules overflow).  The chain clusters -> hits -> tracks then gives the
oracle's tracks exactly."""

import numpy as np
import pytest

import eventgen
import oracle
from eventgen import clusters as C
from tests.compare import match_tracks

pytestmark = pytest.mark.gpu

DET = eventgen.DETECTOR
TABLE = C.module_table()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


@pytest.fixture(scope="module")
def batch():
    events = [eventgen.generate("pu50", 500 + s) for s in range(4)]
    events.insert(2, eventgen.generate("tiny", 3))
    cls = [C.make_clusters(ev, 500 + i, table=TABLE) for i, ev in enumerate(events)]
    empty = dict(module=np.zeros(0, np.uint16), pixel_offsets=np.zeros(1, np.uint32),
                 pix_u=np.zeros(0, np.uint16), pix_v=np.zeros(0, np.uint16),
                 charge=np.zeros(0, np.uint16), hit_of_cluster=np.zeros(0, np.int64))
    cls.insert(1, empty)
    # one zero-charge cluster
    cls[0]["charge"][cls[0]["pixel_offsets"][5]:cls[0]["pixel_offsets"][6]] = 0
    return cls


def _run(torch, cls, limit, capacity=None):
    import paper_2104_06573_amd as pxt
    dev, ev = pxt.upload_clusters(cls)
    n = int(ev[-1])
    rh = pxt.RecHits(TABLE, len(cls), capacity if capacity is not None else n)
    rh.launch(dev, len(cls), n, limit)
    torch.cuda.synchronize()
    return rh, ev, rh.read(len(cls))


@pytest.mark.parametrize("limit", [1024, 3])
def test_rechits_bit_exact(torch, batch, limit):
    rh, ev, (status, ho, ms, hits) = _run(torch, batch, limit)
    assert status == 0
    NM = TABLE.shape[0]
    off = 0
    dropped = 0
    for e, cl in enumerate(batch):
        o = oracle.rechits(cl, TABLE, limit)
        n = len(o["x"])
        assert ho[e] == off and ho[e + 1] == off + n
        np.testing.assert_array_equal(ms[e * NM:(e + 1) * NM + 1] - off, o["module_start"])
        sl = slice(off, off + n)
        for k in ("x", "y", "z", "layer", "module"):
            np.testing.assert_array_equal(hits[k][sl], o[k], err_msg="%s ev%d" % (k, e))
        np.testing.assert_array_equal(hits["cluster"][sl], o["cluster"] + ev[e])
        dropped += len(cl["module"]) - n
        off += n
    print("limit %d: %d hits, %d clusters over the limit" % (limit, off, dropped))
    if limit == 3:
        assert dropped > 0


def test_rechits_errors(torch, batch):
    import paper_2104_06573_amd as pxt
    # capacity below the hits: status CAPACITY, offsets still valid
    n_all = sum(len(c["module"]) for c in batch)
    rh, ev, (status, ho, ms, hits) = _run(torch, batch, 1024, capacity=n_all - 1)
    assert status == pxt.ERR_CAPACITY and ho[-1] == n_all
    # clusters not grouped by module
    bad = dict(batch[0])
    bad["module"] = bad["module"].copy()[::-1].copy()
    bad["pixel_offsets"] = batch[0]["pixel_offsets"]
    rh, ev, (status, *_rest) = _run(torch, [bad], 1024)
    assert status == pxt.ERR_INVALID_ARG
    # a module id beyond the table
    bad2 = dict(batch[0])
    bad2["module"] = batch[0]["module"].copy()
    bad2["module"][-1] = TABLE.shape[0]
    rh, ev, (status, *_rest) = _run(torch, [bad2], 1024)
    assert status == pxt.ERR_INVALID_ARG


def test_chain_clusters_to_tracks(torch, batch):
    # hits from the GPU's RecHits go straight into pxt_reconstruct; the
    # oracle does the same from its own RecHits
    import paper_2104_06573_amd as pxt
    rh, ev, (status, ho, ms, hits) = _run(torch, batch, 1024)
    assert status == 0
    n = int(ho[-1])
    rec = pxt.Reconstructor(DET, max_events=len(batch), max_hits=n + 16, max_doublets=1 << 20,
                            max_tuples=1 << 16, max_tracks=1 << 16)
    rec.launch(rh.x[:n], rh.y[:n], rh.z[:n], rh.layer[:n], ho)
    torch.cuda.synchronize()
    res = rec.result(len(batch))
    assert res.counts["status"] == 0
    out = res.numpy()
    for e, cl in enumerate(batch):
        o = oracle.rechits(cl, TABLE, 1024)
        orc = oracle.reconstruct(o["x"], o["y"], o["z"], o["layer"], DET)
        gh, gp, gc, gx, gf, oh, op, oc, ox = match_tracks(out, orc, e)
        np.testing.assert_array_equal(gh, oh, err_msg="tracks ev%d" % e)
    rec.close()
