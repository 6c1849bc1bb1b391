"""The autotuner over a small search space: every point must give the same
tracks (the tuner checks it and raises otherwise), the best point comes
from the space, and the cache entry of the workload bucket records every
point and returns the best one on lookup."""

import pytest

import eventgen

DET = eventgen.DETECTOR


def test_bucket_key():
    from paper_2104_06573_amd import autotune
    assert autotune.bucket_key(64, 6260.0) == "events64_hits8192"
    assert autotune.bucket_key(1, 1.0) == "events1_hits1"
    assert autotune.bucket_key(33, 27404.1) == "events64_hits32768"


@pytest.mark.gpu
def test_tune_small_space(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2104_06573_amd import autotune
    # a batch of 8 events (one-block-per-event binning at 64 bins, the
    # global kernels at 4096), both link kernels, both doublet modes
    events = [eventgen.generate("tiny", s) for s in range(7)] + [eventgen.generate("pu50", 3)]
    space = {"phi_bins": (64, 4096), "group_lanes": (8,), "link_kernel": (0, 2),
             "doublet_mode": (1, 2), "block_size": (256,)}
    path = str(tmp_path / "tuning.json")
    best = autotune.tune(DET, events, space=space, repeats=2, cache_path=path)
    for k, vals in space.items():
        assert best[k] in vals
    hits = sum(len(e.x) for e in events)
    assert autotune.lookup(len(events), hits / len(events), path=path) == best
    entry = autotune.load_cache(path)[autotune.bucket_key(len(events), hits / len(events))]
    assert len(entry["results"]) == 8
    assert entry["ms"] == min(r["ms"] for r in entry["results"])
