"""npx_step_n_noalloc against npx_step_n, through the C ABI: bit-identical
states on two calls in a row, the second on a smaller world, for the
persistent task-queue launch (whose counters live in the library's static
device array) and the plain grid launch; refusal of a call that needs more
chunk launches than the static counters hold."""
import sys

import numpy as np
import pytest

from paper_2411_05799_amd import native as N
from paper_2411_05799_amd import workloads as W

from _helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

FIELDS = [N.F_BODY, N.F_JOINT, N.F_JOINT_PREV, N.F_STEP, N.F_FLAGS, N.F_TELE]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(w, frames, launch):
    """The same world stepped by npx_step_n and by npx_step_n_noalloc."""
    import torch
    with N.World(w) as a, N.World(w) as b:
        a.set_launch(**launch)
        b.set_launch(**launch)
        s = torch.cuda.Stream()
        a.step_n(frames, stream=s)
        b.step_n_noalloc(frames, stream=s)
        s.synchronize()
        return [a.read_state(f) for f in FIELDS], [b.read_state(f) for f in FIELDS]


@pytest.mark.parametrize("persistent", [1, 0])
def test_noalloc_step_matches_step_n(persistent):
    say(f"case: npx_step_n_noalloc vs npx_step_n, persistent {persistent}")
    launch = dict(lanes_per_instance=32, persistent=persistent, chunk_steps=50, use_graph=1,
                  waves_per_cu=2)
    # first call: 64 hexapods, 250 frames (5 chunk launches)
    ref, got = _pair(W.hexapod_batch(64, seed=71), 250, launch)
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(r, g)
    # second call, smaller: 16 hexapods, 120 frames (3 launches; counters reused)
    ref, got = _pair(W.hexapod_batch(16, seed=72), 120, launch)
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(r, g)
    assert (got[3] == 120).all()


def test_noalloc_refuses_more_chunks_than_counters():
    say("case: npx_step_n_noalloc refusal")
    w = W.hexapod_batch(4, seed=73)
    with N.World(w) as gw:
        gw.set_launch(lanes_per_instance=32, persistent=1, chunk_steps=1)
        before = [gw.read_state(f) for f in FIELDS]
        with pytest.raises(N.NpxError, match="static"):
            gw.step_n_noalloc(4097)
        after = [gw.read_state(f) for f in FIELDS]
        for b, a in zip(before, after):
            np.testing.assert_array_equal(b, a)     # nothing was launched
        gw.step_n_noalloc(4096)                      # exactly the limit is fine
        assert (gw.read_state(N.F_STEP) == 4096).all()
