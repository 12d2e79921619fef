"""A world whose state lives in caller-owned device memory (npx_world_desc.
ext_device_buffers, here torch tensors): the same frames bit for bit as a
world with its own buffers, the tensors holding that state with no copy, the
memory left to its owner at destruction, and refusal of memory the world
cannot use."""
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


def _ext_tensors(w):
    import torch
    I, J = w.n_instances, N.j_max_of(w.morphs)
    return [torch.full(((13 + 2 * J) * I,), float("nan"), dtype=torch.float32, device="cuda"),
            torch.full((I,), -7, dtype=torch.int32, device="cuda"),
            torch.full((I,), -7, dtype=torch.int32, device="cuda"),
            torch.full((4 * I,), float("nan"), dtype=torch.float64, device="cuda")]


@pytest.mark.parametrize("which", [(0, 1, 2, 3), (0, 3)])
def test_ext_state_buffers_match_own_buffers_bitwise(which):
    import torch
    w = W.config2(n_inst=96, n_steps=200)
    say(f"ext buffers {which}: 96 hexapods, 3 x 40 frames")
    ext = _ext_tensors(w)
    ext = [t if k in which else None for k, t in enumerate(ext)]
    with N.World(w) as a, N.World(w, ext=ext) as b:
        s = torch.cuda.Stream()
        for _ in range(3):
            a.step_n(40, stream=s)
            b.step_n(40, stream=s)
            s.synchronize()
            for f in FIELDS:
                np.testing.assert_array_equal(a.read_state(f), b.read_state(f))
        # the tensors are the state: rows of F_BODY, F_JOINT, F_JOINT_PREV in order
        I, J = w.n_instances, b.j_max
        st = np.concatenate([b.read_state(N.F_BODY).reshape(13, I),
                             b.read_state(N.F_JOINT).reshape(J, I),
                             b.read_state(N.F_JOINT_PREV).reshape(J, I)])
        if 0 in which:
            np.testing.assert_array_equal(ext[0].cpu().numpy().reshape(13 + 2 * J, I), st)
        if 1 in which:
            np.testing.assert_array_equal(ext[1].cpu().numpy(), b.read_state(N.F_STEP).ravel())
        if 2 in which:
            np.testing.assert_array_equal(ext[2].cpu().numpy(), b.read_state(N.F_FLAGS).ravel())
        if 3 in which:
            np.testing.assert_array_equal(ext[3].cpu().numpy().reshape(4, I),
                                          b.read_state(N.F_TELE).reshape(4, I))
    # destroyed worlds leave the memory to torch: still usable
    for t in ext:
        if t is not None:
            t.add_(1)
    torch.cuda.synchronize()


def test_ext_state_buffers_refused_when_misaligned():
    import torch
    w = W.config2(n_inst=8, n_steps=10)
    I, J = w.n_instances, N.j_max_of(w.morphs)
    big = torch.zeros((13 + 2 * J) * I + 1, dtype=torch.float32, device="cuda")
    say("ext buffers: a state tensor 4 bytes off 16-byte alignment")
    with pytest.raises(N.NpxError, match="ext_device_buffers"):
        N.World(w, ext=[big[1:]])
    with pytest.raises(ValueError):
        N.World(w, ext=[big])                      # wrong element count (binding check)
