"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

A test-only C driver (tests/oracle_driver.c) including the oracle source is
built with gcc -fsanitize=address,undefined and run in a subprocess on
generated events; it must finish cleanly and report the same counts as the
normal build."""

import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import eventgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "orc_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", exe, os.path.join(HERE, "oracle_driver.c"), "-lm"])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,seed,ntr", [("tiny", 0, None), ("tiny", 7, None),
                                           ("pu50", 3, 200), ("pu50", 4, None)])
def test_oracle_clean_under_sanitizers(driver, name, seed, ntr):
    ev = eventgen.generate(name, seed, n_tracks=ntr)
    cfg = oracle.make_config(eventgen.DETECTOR)
    with tempfile.NamedTemporaryFile(suffix=".bin", delete=False) as f:
        f.write(bytes(cfg))
        f.write(np.uint32(ev.n_hits).tobytes())
        for a in (ev.x, ev.y, ev.z):
            f.write(np.ascontiguousarray(a, np.float32).tobytes())
        f.write(np.ascontiguousarray(ev.layer, np.int16).tobytes())
        path = f.name
    try:
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
        out = subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=300)
    finally:
        os.unlink(path)
    assert out.returncode == 0, out.stderr[-2000:]
    vals = list(map(int, out.stdout.split()))
    ref = oracle.reconstruct(ev.x, ev.y, ev.z, ev.layer, eventgen.DETECTOR)
    assert vals[0] == ref["status"]
    assert vals[1:] == [len(ref[k]) for k in oracle.ITEMS]
