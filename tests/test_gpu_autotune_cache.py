"""The autotuner's JSON result cache: a first call times the launch shapes and
records the choice under its key; a second call with the same key sets the
recorded shape without timing anything."""
import json
import sys

import pytest

from paper_2411_05799_amd import native as N
from paper_2411_05799_amd import workloads as W

from _helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def test_autotune_cache_records_then_reuses(tmp_path, monkeypatch):
    print("autotune cache: 64 hexapods, 20-frame timing runs", flush=True)
    sys.stdout.flush()
    cache = str(tmp_path / "tune.json")
    w = W.config2(n_inst=64, n_steps=40)
    with N.World(w) as a:
        rec = a.autotune(steps=20, cache=cache, key="hexapod64")
        assert rec["tried"] and a.get_launch().as_dict() == rec["best"]
    stored = json.load(open(cache))
    assert stored["hexapod64"]["best"] == rec["best"]

    def no_timing(*args):
        raise AssertionError("npx_autotune called although the key is cached")

    monkeypatch.setattr(N.lib(), "npx_autotune", no_timing)
    with N.World(w) as b:
        again = b.autotune(steps=20, cache=cache, key="hexapod64")
        assert again["best"] == rec["best"]
        assert b.get_launch().as_dict() == rec["best"]
