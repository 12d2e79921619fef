"""Range sensors on the GPU (npx_world_ray_ranges) vs the FP64 oracle, through
the C ABI.

Both sides start from the same FP32 state: the GPU's, read back. Tolerance on a
range: 2e-4 m. The ray ends agree to about 1e-6 m (FP32 transforms of
coordinates below 10 m) and the cell crossings to about 1e-6 m, so a range
differs by that over the sine of the angle between ray and ground; a ray
whose oracle range moves by more than half the tolerance when both its ends
are moved by 2e-5 m up or down grazes the ground or a cell corner, its answer
decided by rounding, and is not compared (at most 10% of the rays).
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_05799_amd import native as N
from paper_2411_05799_amd import workloads as W

from _helpers import gpu_available, read_states

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

TOL = 2e-4
SHIFT = 2e-5
SENTINEL = -7.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ranges(gw, ld):
    import torch
    out = torch.full((gw.n_instances, ld), SENTINEL, dtype=torch.float32, device="cuda")
    gw.ray_ranges(out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _compare(ow, gw, got, idx, rays_of, J_of):
    """Compares instances idx; returns (compared, skipped as rounding-decided)."""
    states = read_states(gw, idx, J_of)
    compared = skipped = 0
    worst = 0.0
    for i, st in zip(idx, states):
        rays, links = rays_of(i)
        if len(links) == 0:
            continue
        S, E = ow.ray_ends(i, st, rays, links)
        for k in range(len(links)):
            r = ow.params.ray_range(S[k], E[k])
            up = ow.params.ray_range(S[k] + [0, 0, SHIFT], E[k] + [0, 0, SHIFT])
            dn = ow.params.ray_range(S[k] - [0, 0, SHIFT], E[k] - [0, 0, SHIFT])
            if max(abs(up - r), abs(dn - r)) > TOL / 2:
                skipped += 1
                continue
            compared += 1
            err = abs(float(got[i, k]) - r)
            worst = max(worst, err)
            assert err <= TOL, (i, k, float(got[i, k]), r)
    say(f"  compared {compared}, rounding-decided {skipped}, worst {worst:.2e} m")
    assert skipped <= 0.1 * (compared + skipped)
    return compared, skipped


def test_ray_ranges_hexapods_on_terrain():
    """48 hexapods walking on the 2 cm terrain, each with the six sensor rays
    and 40 random rays on random links (lengths 5 cm to 1 m), after 0 and 300
    frames."""
    say("case: rays / hexapods on terrain")
    w = W.hexapod_batch(48, seed=5)
    m = w.morphs[0]
    r6, l6 = W.sensor_rays(m)
    rr, lr = W.random_rays(m, 40, np.random.default_rng(7))
    rays, links = np.concatenate([r6, rr]), np.concatenate([l6, lr])
    ow = O.OracleWorld(w)
    J = m.n_links - 1
    with N.World(w) as gw:
        gw.set_rays(0, rays, links)
        for frames in (0, 300):
            if frames:
                gw.step_n(frames)
            got = _ranges(gw, 48)
            assert np.all(got[:, len(links):] == SENTINEL)
            n, _ = _compare(ow, gw, got, range(48), lambda i: (rays, links), lambda i: J)
            assert n >= 1500


def test_ray_ranges_uneven_morphologies_limits_and_errors():
    """Uneven morphologies, some with rays (up to the 64 maximum, a zero-length
    ray among them) and some without: only each instance's own entries are
    written, a non-finite state reads NaN, and bad tables, too small a stride
    and a bilinear world are refused."""
    say("case: rays / uneven morphologies, limits, errors")
    w = W.config3(n_inst=40, n_steps=100)
    rng = np.random.default_rng(9)
    tables = {}
    for mi, m in enumerate(w.morphs):
        n = [64, 0, 5][mi % 3]
        if n:
            rays, links = W.random_rays(m, n, rng)
            rays[0, 3:] = rays[0, :3]                      # zero length
            tables[mi] = (rays, links)
    ow = O.OracleWorld(w)
    im = w.inst_morph
    rays_of = lambda i: tables.get(int(im[i]), (np.zeros((0, 6), np.float32), np.zeros(0)))
    J_of = lambda i: w.morphs[int(im[i])].n_links - 1
    with N.World(w) as gw:
        for mi, (rays, links) in tables.items():
            gw.set_rays(mi, rays, links)
        gw.step_n(100)
        got = _ranges(gw, 70)
        for i in range(w.n_instances):
            n = len(rays_of(i)[1])
            assert np.all(got[i, n:] == SENTINEL), i
            if n:
                assert got[i, 0] == 0.0                      # the zero-length ray
        _compare(ow, gw, got, range(w.n_instances), rays_of, J_of)

        # a non-finite state reads NaN on that instance only
        i_bad = next(i for i in range(w.n_instances) if len(rays_of(i)[1]))
        cog = gw.read_state(N.F_COG)
        cog[0, i_bad] = np.nan
        gw.write_state(N.F_COG, cog)
        got2 = _ranges(gw, 70)
        n_bad = len(rays_of(i_bad)[1])
        assert np.all(np.isnan(got2[i_bad, :n_bad]))
        others = [i for i in range(w.n_instances) if i != i_bad]
        np.testing.assert_array_equal(got2[others], got[others])

        import torch
        out = torch.zeros((w.n_instances, 63), device="cuda")
        with pytest.raises(N.NpxError):
            gw.ray_ranges(out)                               # ld below 64
        m0 = w.morphs[0]
        with pytest.raises(N.NpxError):
            gw.set_rays(0, np.zeros((1, 6)), [m0.n_links])   # no such link
        with pytest.raises(N.NpxError):
            gw.set_rays(0, np.zeros((65, 6)), np.zeros(65))  # more than 64
        with pytest.raises(N.NpxError):
            gw.set_rays(0, [[0, 0, 0, math.nan, 0, 0]], [0])
        with pytest.raises(N.NpxError):
            gw.set_rays(0, [[0, 0, 0, 1000.0, 0, 0]], [0])   # > 65,536 cells at 50 /m
        # the refused calls left the tables as they were
        got3 = _ranges(gw, 70)
        np.testing.assert_array_equal(got3[others], got[others])

    wb = W.hexapod_batch(4, seed=1)
    wb.params.hf_bilinear = True
    with N.World(wb) as gw:
        r6, l6 = W.sensor_rays(wb.morphs[0])
        gw.set_rays(0, r6, l6)
        with pytest.raises(N.NpxError):
            _ranges(gw, 6)


def test_ray_ranges_full_size_sampled():
    """The 4,096 hexapods of the benchmark with the six sensor rays each, after
    200 frames in the benchmark's launch shape; 64 sampled instances against
    the oracle, and every range within [0, length]."""
    say("case: rays / 4096 hexapods, sampled")
    w = W.config2()
    m = w.morphs[0]
    rays, links = W.sensor_rays(m)
    lengths = np.linalg.norm(rays[:, 3:] - rays[:, :3], axis=1)
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        gw.set_launch(lanes_per_instance=32)
        gw.set_rays(0, rays, links)
        gw.step_n(200)
        got = _ranges(gw, 6)
        assert np.all(np.isfinite(got))
        assert np.all(got >= 0.0) and np.all(got <= lengths[None, :] * (1 + 1e-6))
        idx = np.random.default_rng(3).choice(w.n_instances, 64, replace=False)
        _compare(ow, gw, got, idx, lambda i: (rays, links), lambda i: m.n_links - 1)
