"""Vertex finding on the GPU (pxt_find_vertices and the vertex step at the
end of pxt_reconstruct) against the oracle.

On the same single-precision track values both sides take every decision
(selection, neighbours, cores, borders) identically and sum each cluster in
the same order in double precision, so vertex membership, counts and the
single-precision z, z_err and chi2 must be identical.  The lists come from
the input generator (eventgen.vertex_track_lists: ragged events, vertex
mixtures over a uniform background, exact-distance grids, ties, +-0, NaN,
non-positive variances, the pT cut exactly, empty and one-track events).

Through pxt_reconstruct the vertices are found from the GPU's own fitted
tracks, whose z0 agree with the oracle's only to the fit tolerance, so there
the comparison is by properties: the vertex step equals pxt_find_vertices
on the same tracks, and against the oracle's vertices (from its own tracks)
per-track assignments agree for nearly every track and matched vertices
agree in z within the fit tolerance."""

import numpy as np
import pytest

import eventgen
import oracle
from tests.compare import match_tracks, oracle_events

pytestmark = pytest.mark.gpu

DET = eventgen.DETECTOR


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def _device_lists(torch, lists):
    dev = torch.device("cuda", 0)
    n = np.array([len(e["z0"]) for e in lists], np.int32)
    T = int(n.sum())
    params = np.zeros((T, 5), np.float32)
    cov = np.zeros((T, 15), np.float32)
    if T:
        params[:, 2] = np.concatenate([e["qopt"] for e in lists])
        params[:, 4] = np.concatenate([e["z0"] for e in lists])
        cov[:, 14] = np.concatenate([e["var"] for e in lists])
        nh = np.concatenate([e["nhits"] for e in lists])
    else:
        nh = np.zeros(0, np.uint8)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t(n), t(nh.astype(np.uint8)), t(params), t(cov)


def _check_event(got, tv, o):
    np.testing.assert_array_equal(tv, o["assign"])
    np.testing.assert_array_equal(got["n_tracks"], o["n_tracks"])
    np.testing.assert_array_equal(got["z"], o["z"].astype(np.float32))
    np.testing.assert_array_equal(got["z_err"], o["z_err"].astype(np.float32))
    np.testing.assert_array_equal(got["chi2"], o["chi2"].astype(np.float32))


@pytest.mark.parametrize("seed", range(6))
def test_find_vertices_bit_exact(torch, seed):
    import paper_2104_06573_amd as pxt
    lists = eventgen.vertex_track_lists(seed)
    per, nh, params, cov = _device_lists(torch, lists)
    cfg = pxt.make_config(DET)
    vb = pxt.find_vertices(cfg, per, nh, params, cov, max_per_event=512)
    torch.cuda.synchronize()
    summary, events, tv = vb.read(len(lists), int(per.sum()))
    assert summary["status"] == 0, summary
    off = 0
    nv = 0
    for e, lst in enumerate(lists):
        o = oracle.vertices(lst["z0"], lst["var"], lst["qopt"], lst["nhits"], DET)
        n = len(lst["z0"])
        _check_event(events[e], tv[off:off + n], o)
        off += n
        nv += len(o["z"])
    assert summary["n_vertices"] == nv
    print("seed %d: %d tracks, %d vertices" % (seed, off, nv))


def test_find_vertices_capacity(torch):
    import paper_2104_06573_amd as pxt
    lists = eventgen.vertex_track_lists(3)
    per, nh, params, cov = _device_lists(torch, lists)
    cfg = pxt.make_config(DET)
    want = [len(oracle.vertices(l["z0"], l["var"], l["qopt"], l["nhits"], DET)["z"])
            for l in lists]
    small = max(1, max(want) - 1)
    vb = pxt.find_vertices(cfg, per, nh, params, cov, max_per_event=small)
    torch.cuda.synchronize()
    summary, events, tv = vb.read(len(lists), int(per.sum()))
    assert summary["status"] == pxt.ERR_CAPACITY
    assert summary["required_per_event"] == max(want)
    for e, w in enumerate(want):
        assert len(events[e]["z"]) == (w if w <= small else 0)
    # more selected tracks in one event than the kernel holds
    n = pxt.VTX_MAX_TRACKS + 1
    big = [dict(z0=np.linspace(-1, 1, n).astype(np.float32),
                var=np.full(n, 1e-4, np.float32), qopt=np.full(n, 0.5, np.float32),
                nhits=np.full(n, 4, np.uint8))]
    vb = pxt.find_vertices(cfg, *_device_lists(torch, big), max_per_event=16)
    torch.cuda.synchronize()
    summary, events, tv = vb.read(1, n)
    assert summary["status"] == pxt.ERR_CAPACITY and summary["max_selected"] == n
    assert len(events[0]["z"]) == 0 and np.all(tv == -1)


def _assignment_agreement(events, out, oref, vs):
    """Per event: fraction of matched tracks whose vertex (as a z value) is
    the same on both sides; largest |dz| of vertices built from the same
    track set."""
    agree = tot = 0
    worst = 0.0
    summary, vev, tv = vs
    for e in range(len(events)):
        o = oref[e]
        ov = oracle.event_vertices(o, DET)
        m = out["event_id"] == e
        gidx = np.nonzero(m)[0]
        gh = out["hit_idx"][m].view(np.uint32)
        go = np.lexsort(gh.T[::-1])
        oo = np.lexsort(o["tracks"].T[::-1])
        np.testing.assert_array_equal(gh[go], o["tracks"][oo])
        g_assign = tv[gidx[go]]
        o_assign = ov["assign"][oo]
        agree += int(np.sum(g_assign == o_assign))
        tot += len(go)
        for v in range(len(ov["z"])):
            ot = set(np.nonzero(o_assign == v)[0].tolist())
            gv = np.unique(g_assign[list(ot)]) if ot else []
            if len(gv) == 1 and gv[0] >= 0:
                gt = set(np.nonzero(g_assign == gv[0])[0].tolist())
                if gt == ot:
                    worst = max(worst, abs(float(vev[e]["z"][gv[0]]) - ov["z"][v]))
    return agree / max(tot, 1), worst


@pytest.mark.parametrize("graph", [0, 1])
def test_reconstruct_with_vertices(torch, graph):
    import paper_2104_06573_amd as pxt
    events = [eventgen.generate("pu50", 400 + s) for s in range(4)]
    oref = oracle_events(events, DET)
    rec = pxt.Reconstructor(DET, max_events=8, max_hits=1 << 16, max_doublets=1 << 20,
                            max_tuples=1 << 16, max_tracks=1 << 16, use_graph=graph,
                            max_vertices_per_event=256)
    for _ in range(2):
        res = rec.run_numpy(events)
        assert res.counts["status"] == 0
        out = res.numpy()
        vs = rec.vtx.read(len(events), res.counts["n_tracks"])
        assert vs[0]["status"] == 0, vs[0]
        # the in-path step equals pxt_find_vertices on the same tracks
        vb = pxt.find_vertices(rec.cfg, rec.o_per_event[:len(events)], res.n_hits, res.params,
                               res.cov, max_per_event=256)
        torch.cuda.synchronize()
        alone = vb.read(len(events), res.counts["n_tracks"])
        assert alone[0] == vs[0]
        np.testing.assert_array_equal(alone[2], vs[2])
        for a, b in zip(alone[1], vs[1]):
            for k in a:
                np.testing.assert_array_equal(a[k], b[k])
        frac, worst = _assignment_agreement(events, out, oref, vs)
        print("graph %d: %d vertices, assignment agreement %.5f, worst dz %.2e cm" %
              (graph, vs[0]["n_vertices"], frac, worst))
        assert frac >= 0.995
        assert worst <= 1e-3
    rec.close()


def test_vertices_skip_a_failed_call(torch):
    import paper_2104_06573_amd as pxt
    events = [eventgen.generate("pu50", 7)]
    rec = pxt.Reconstructor(DET, max_events=1, max_hits=1 << 14, max_doublets=1000,
                            max_tuples=1 << 14, max_tracks=1 << 14, max_vertices_per_event=64)
    res = rec.run_numpy(events)
    assert res.counts["status"] == pxt.ERR_CAPACITY
    summary, ev, _ = rec.vtx.read(1, 0)
    assert summary["status"] == pxt.ERR_CAPACITY and len(ev[0]["z"]) == 0
    rec.close()
