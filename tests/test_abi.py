"""C ABI: the library builds, loads and exports every declared symbol, and
argument validation works without touching a GPU."""

import ctypes
import os
import re

import numpy as np

import pytest

import eventgen
import paper_2104_06573_amd as pxt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pxt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(pxt_\w+)\s*\(", src, re.M)))


def test_header_symbols_exported():
    L = pxt.lib()
    names = _declared()
    assert set(names) == set(pxt.EXPORTS), names
    for n in names:
        assert hasattr(L, n), n


def test_version_and_status_strings():
    L = pxt.lib()
    assert L.pxt_abi_version() == pxt.ABI_VERSION == 3
    assert L.pxt_status_str(0) == b"ok"
    assert L.pxt_status_str(2) == b"capacity exceeded"
    assert L.pxt_status_str(99) == b"unknown status"


def test_config_defaults_and_validation():
    L = pxt.lib()
    c = pxt.PxtConfig()
    assert L.pxt_config_defaults(ctypes.byref(c)) == 0
    assert c.phi_bins == 256 and c.block_size == 256 and c.doublet_mode == 2
    assert L.pxt_config_defaults(None) == pxt.ERR_INVALID_ARG
    h = ctypes.c_void_p()
    # physics fields zeroed: rejected before any device call
    assert L.pxt_create(ctypes.byref(c), 0, ctypes.byref(h)) == pxt.ERR_INVALID_ARG
    assert b"c_kappa" in L.pxt_last_error(None)
    good = pxt.make_config(eventgen.DETECTOR)
    for field, bad in (("phi_bins", 8), ("block_size", 100), ("n_layers", 0), ("max_hits", 0),
                       ("arz", 0.0), ("pt_fp64", -1.0), ("doublet_mode", 3),
                       ("doublet_mode", -1)):
        c2 = pxt.make_config(eventgen.DETECTOR)
        setattr(c2, field, bad)
        assert L.pxt_create(ctypes.byref(c2), 0, ctypes.byref(h)) == pxt.ERR_INVALID_ARG, field
    c3 = pxt.make_config(eventgen.DETECTOR)
    c3.pair_inner[0] = 12  # beyond n_layers
    assert L.pxt_create(ctypes.byref(c3), 0, ctypes.byref(h)) == pxt.ERR_INVALID_ARG
    assert good.n_layers == 10 and good.n_pairs == 13


def test_null_arguments_rejected():
    L = pxt.lib()
    assert L.pxt_create(None, 0, None) == pxt.ERR_INVALID_ARG
    assert L.pxt_reconstruct(None, None, None, None) == pxt.ERR_INVALID_ARG
    cnt = ctypes.c_uint64()
    assert L.pxt_debug_dump(None, 0, None, 0, ctypes.byref(cnt), None) == pxt.ERR_INVALID_ARG
    L.pxt_destroy(None)


def test_struct_sizes_match_header():
    # compile a probe of sizeof/offsetof with the host compiler and compare
    import subprocess
    import tempfile
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "pxt.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(pxt_config),
         offsetof(pxt_config, pt_fp64), offsetof(pxt_config, group_lanes),
         offsetof(pxt_config, doublet_mode), offsetof(pxt_config, min_hits),
         offsetof(pxt_config, q_z0_max), offsetof(pxt_config, vtx_eps),
         offsetof(pxt_config, vtx_pt_min), sizeof(pxt_hits), sizeof(pxt_tracks),
         sizeof(pxt_counts), sizeof(pxt_vertices), sizeof(pxt_vertex_summary));
  printf("%zu %zu\n", sizeof(pxt_clusters), sizeof(pxt_rechits_out));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "p")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        got = list(map(int, subprocess.check_output([exe]).split()))
    C = pxt.PxtConfig
    want = [ctypes.sizeof(C), C.pt_fp64.offset, C.group_lanes.offset, C.doublet_mode.offset,
            C.min_hits.offset, C.q_z0_max.offset, C.vtx_eps.offset, C.vtx_pt_min.offset,
            ctypes.sizeof(pxt.PxtHits), ctypes.sizeof(pxt.PxtTracks),
            ctypes.sizeof(pxt.PxtCounts), ctypes.sizeof(pxt.PxtVertices),
            ctypes.sizeof(pxt.PxtVertexSummary), ctypes.sizeof(pxt.PxtClusters),
            ctypes.sizeof(pxt.PxtRechitsOut)]
    assert got == want


def test_server_argument_validation():
    from paper_2104_06573_amd import serve
    L = serve._bind()
    cfg = pxt.make_config(eventgen.DETECTOR)
    h = ctypes.c_void_p()
    bad = serve.ServerConfig(0, 16, 8, 40)
    assert L.pxt_server_create(ctypes.byref(cfg), ctypes.byref(bad), 0,
                               ctypes.byref(h)) == pxt.ERR_INVALID_ARG
    bad = serve.ServerConfig(2, 0, 8, 40)
    assert L.pxt_server_create(ctypes.byref(cfg), ctypes.byref(bad), 0,
                               ctypes.byref(h)) == pxt.ERR_INVALID_ARG
    t = ctypes.c_uint64()
    assert L.pxt_submit(None, None, None, None, None, 0, ctypes.byref(t)) == pxt.ERR_INVALID_ARG
    assert L.pxt_poll(None, 1, None, 0) == pxt.ERR_INVALID_ARG
    L.pxt_server_destroy(None)


def test_static_entry_point_validation():
    # checked on the host before any device call: capacities beyond the
    # fixed buffer, more events than it admits, a bad config
    L = pxt.lib()
    cnt = (ctypes.c_uint32 * 32)()
    per = (ctypes.c_uint32 * 128)()
    out = pxt.PxtTracks(0, None, None, None, None, None, None, None,
                        ctypes.addressof(per), ctypes.addressof(cnt))
    offs = np.zeros(2, np.uint32)
    hits = pxt.PxtHits(1, offs.ctypes.data, None, None, None, None, None)
    big = pxt.make_config(eventgen.DETECTOR, max_events=4, max_doublets=1 << 24)
    assert L.pxt_reconstruct_static(ctypes.byref(big), 0, ctypes.byref(hits), ctypes.byref(out),
                                    None) == pxt.ERR_CAPACITY
    assert b"PXT_STATIC_SCRATCH_BYTES" in L.pxt_last_error(None)
    many = pxt.make_config(eventgen.DETECTOR, max_events=100, max_hits=1024,
                           max_doublets=1024, max_tuples=1024)
    offs2 = np.zeros(101, np.uint32)
    hits2 = pxt.PxtHits(100, offs2.ctypes.data, None, None, None, None, None)
    assert L.pxt_reconstruct_static(ctypes.byref(many), 0, ctypes.byref(hits2),
                                    ctypes.byref(out), None) == pxt.ERR_CAPACITY
    assert b"PXT_STATIC_MAX_EVENTS" in L.pxt_last_error(None)
    bad = pxt.make_config(eventgen.DETECTOR)
    bad.phi_bins = 8
    assert L.pxt_reconstruct_static(ctypes.byref(bad), 0, ctypes.byref(hits), ctypes.byref(out),
                                    None) == pxt.ERR_INVALID_ARG
    assert L.pxt_reconstruct_static(None, 0, ctypes.byref(hits), ctypes.byref(out),
                                    None) == pxt.ERR_INVALID_ARG


def test_output_policy_and_vertex_config_validation():
    L = pxt.lib()
    h = ctypes.c_void_p()
    for field, bad in (("min_hits", 2), ("min_hits", 9), ("q_chi2", 0.0), ("q_pt_min", -1.0),
                       ("vtx_eps", 0.0), ("vtx_min_pts", 0), ("vtx_min_hits", 2),
                       ("vtx_pt_min", 0.0)):
        c = pxt.make_config(eventgen.DETECTOR)
        setattr(c, field, bad)
        assert L.pxt_create(ctypes.byref(c), 0, ctypes.byref(h)) == pxt.ERR_INVALID_ARG, field
        assert L.pxt_find_vertices(ctypes.byref(c), 0, ctypes.byref(pxt.PxtTracks()),
                                   ctypes.byref(pxt.PxtVertices()), None) == pxt.ERR_INVALID_ARG
    good = pxt.make_config(eventgen.DETECTOR)
    # null buffers are rejected before any device call
    assert L.pxt_find_vertices(ctypes.byref(good), 2, ctypes.byref(pxt.PxtTracks()),
                               ctypes.byref(pxt.PxtVertices()), None) == pxt.ERR_INVALID_ARG
    assert L.pxt_find_vertices(None, 0, None, None, None) == pxt.ERR_INVALID_ARG
    d = pxt.make_config({**eventgen.DETECTOR, "quality": None}, min_hits=4)
    assert d.min_hits == 4 and d.q_chi2 == 5.0  # library defaults of the quality limits


def test_rechits_validation():
    L = pxt.lib()
    ms = (ctypes.c_uint32 * 8)()
    out = pxt.PxtRechitsOut(0, None, None, None, None, None, None, ctypes.addressof(ms),
                            ctypes.addressof(ms), ctypes.addressof(ms))
    cl = pxt.PxtClusters(1, 0, None, None, None, None, None, None)
    tab = ctypes.c_void_p(1)
    for nm, lim in ((0, 8), (65536, 8), (10, 0)):
        assert L.pxt_rechits(tab, nm, lim, ctypes.byref(cl), ctypes.byref(out),
                             None) == pxt.ERR_INVALID_ARG
    assert L.pxt_rechits(None, 10, 8, ctypes.byref(cl), ctypes.byref(out), None) == \
        pxt.ERR_INVALID_ARG
    cl2 = pxt.PxtClusters(1, 5, None, None, None, None, None, None)
    assert L.pxt_rechits(tab, 10, 8, ctypes.byref(cl2), ctypes.byref(out), None) == \
        pxt.ERR_INVALID_ARG
    assert b"null" in L.pxt_last_error(None)
