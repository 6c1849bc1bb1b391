"""Host-side logic of bench.py (no GPU): the one-GPU guard, the kernel named
for each stage and mode, the algorithmic byte table and the roofline entry
with the committed traffic summary."""

import argparse
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _args(**kw):
    a = dict(link_kernel=0, group_lanes=8, batch=0, doublet_mode=2)
    a.update(kw)
    return argparse.Namespace(**a)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("stage,kw,name", [
    ("links", {}, "pxt::k_links_thread"),
    ("links", dict(link_kernel=1), "pxt::k_links<8>"),
    ("links", dict(link_kernel=1, group_lanes=16), "pxt::k_links<16>"),
    ("links", dict(link_kernel=2), "pxt::k_links_wave"),
    ("doublet_count", {}, "pxt::k_dstage<8>"),
    ("doublet_fill", {}, "pxt::k_dscatter<8>"),
    ("doublet_fill", dict(doublet_mode=1, group_lanes=4), "pxt::k_doublets1<4>"),
    ("doublet_count", dict(doublet_mode=0), "pxt::k_doublets<8, false>"),
    ("doublet_fill", dict(doublet_mode=0, group_lanes=16), "pxt::k_doublets<16, true>"),
    ("fit32", {}, "pxt::k_fit32"),
])
def test_stage_kernel_names(stage, kw, name):
    assert bench.stage_kernel(stage, _args(**kw)) == name


def test_algorithmic_bytes_table():
    n = dict(Nh=1000, Nd=20000, Nw=30000, Nt=500, Nk=300, nbar=3.4)
    # the staged doublets add one 4-byte record per doublet to each pass
    assert (bench.algorithmic_bytes("doublet_count", n, 2)
            - bench.algorithmic_bytes("doublet_count", n, 0)) == 4 * n["Nd"]
    assert (bench.algorithmic_bytes("doublet_fill", n, 2)
            - bench.algorithmic_bytes("doublet_fill", n, 0)) == 4 * n["Nd"]
    assert bench.algorithmic_bytes("links", n) == 24 * 1000 + 52 * 20000 + 8 * 30000
    assert bench.algorithmic_bytes("no_such_stage", n) is None


def test_roofline_picks_the_slowest_priced_stage():
    stages = {"links": 0.2, "doublet_count": 0.1, "doublet_fill": 0.05, "tuple_scan": 0.9}
    counts = dict(n_doublets=20000, n_words=30000, n_raw_tuples=500, n_tracks=300)
    r = bench.roofline(stages, counts, 1000, bench.HBM_PEAK_GBS, "pu200", _args())
    # tuple_scan has no byte entry, so the links stage is the dominant one
    assert r["kernel"] == "pxt::k_links_thread"
    byts = bench.algorithmic_bytes("links", dict(Nh=1000, Nd=20000, Nw=30000, Nt=500,
                                                 Nk=300, nbar=3.4))
    assert r["algorithmic_bytes_per_launch"] == byts
    assert r["achieved"] == pytest.approx(byts / 0.2e-3 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, abs=1e-5)
    assert r["traffic"] is None  # counters are only taken for the PU~50 workload


def test_measured_traffic_follows_the_source_hash():
    path = os.path.join(ROOT, "profiles", "hbm_traffic_pu50_batch64.md")
    if not os.path.exists(path):
        pytest.skip("no traffic summary committed")
    txt = open(path).read()
    if bench.kernel_source_hash() not in txt:
        # kernels changed since the counters were taken: no traffic figure
        assert bench.measured_traffic("pxt::k_links_thread") is None
    else:
        assert bench.measured_traffic("pxt::k_links_thread") > 0
    assert bench.measured_traffic("pxt::no_such_kernel") is None
