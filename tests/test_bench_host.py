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
])
def test_stage_kernel_names(stage, kw, name):
    assert bench.stage_kernel(stage, _args(**kw)) == name


def test_algorithmic_bytes_follow_the_method_formula():
    n = dict(Nh=1000, Nd=20000, Nl=3000, Nt=500, Nk=300, nbar=3.5)
    total = (14 * 1000 + 48 * 1000 + 16 * 20000 + 8 * (1000 + 20000) + 8 * 3000 + 66 * 500
             + 12 * 3.5 * 300 + 120 * 300)
    assert bench.path_bytes(n) == pytest.approx(total)
    # the steps' shares add up to the whole path
    assert sum(bench.step_bytes(s, n) or 0 for s in bench.STEP_STAGES) == pytest.approx(total)
    # with vertices: the tracks' z0 values read and their vertex written, and
    # the vertices
    nv = dict(n, Nv=40)
    assert bench.path_bytes(nv) == pytest.approx(total + 17 * 300 + 16 * 40)
    assert sum(bench.step_bytes(s, nv) for s in bench.STEP_STAGES) == pytest.approx(
        bench.path_bytes(nv))
    assert bench.step_bytes("links", n) == 8 * 20000 + 4 * (1000 + 20000) + 4 * 3000
    assert bench.step_bytes("no_such_step", n) is None


def test_roofline_entry():
    stages = {"links": 0.2, "doublet_count": 0.1, "doublet_fill": 0.05, "tuple_scan": 0.9}
    n = dict(Nh=10 ** 6, Nd=2 * 10 ** 7, Nl=3 * 10 ** 6, Nt=5 * 10 ** 5, Nk=3 * 10 ** 5, nbar=3.5)
    r = bench.roofline(stages, n, 100.0, bench.HBM_PEAK_GBS, 5000.0, "pu200", _args())
    assert r["kernel"] == "pxt::k_links_thread"
    lb = bench.step_bytes("links", n)
    assert r["algorithmic_bytes_per_launch"] == lb
    assert r["achieved"] == pytest.approx(lb / 0.2e-3 / 1e9, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, abs=1e-5)
    assert r["path"]["achieved"] == pytest.approx(bench.path_bytes(n) * 100.0 / 1e9, rel=1e-4)
    assert r["frac_of_copy_peak"] == pytest.approx(r["achieved"] / 5000.0, abs=1e-5)
    assert r["steps"]["doublets"]["ms"] == pytest.approx(0.15)
    assert r["traffic"] is None  # counters are only taken for the PU~50 workload


def test_trial_statistics():
    st = bench.stats([1.0, 2.0, 3.0])
    assert st == {"mean": 2.0, "std": 1.0, "n": 3}


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
