"""The search's selection step on the device (npx_sur_screen_select): every
candidate's fitness against the formula, and the n_top best in order (equal
fitness by the lower index) against a host sort of the same fitness values;
flagged and non-finite candidates last; argument errors."""
import sys

import numpy as np
import pytest

from paper_2411_05799_amd import native as N

from _helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    lds = 7
    s0 = rng.normal(0, 2, size=(n, lds)).astype(np.float32)
    s1 = s0 + rng.normal(0, 0.5, size=(n, lds)).astype(np.float32)
    ang = rng.uniform(0, 2 * np.pi, n)
    h = np.stack([np.cos(ang), np.sin(ang)], 1).astype(np.float32)
    tau = rng.uniform(0, 50, n).astype(np.float32)
    flags = np.zeros(n, np.int32)
    flags[rng.choice(n, n // 50, replace=False)] = 1
    if n >= 200:
        # exact ties: copies of a few candidates' inputs; and non-finite ends
        for a, b in zip(rng.choice(n // 2, 40, replace=False),
                        rng.choice(np.arange(n // 2, n), 40, replace=False)):
            s0[b], s1[b], h[b], tau[b], flags[b] = s0[a], s1[a], h[a], tau[a], flags[a]
        s1[rng.choice(n, 5, replace=False), 0] = np.nan
    return s0, s1, h, tau, flags


@pytest.mark.parametrize("n,n_top", [(5000, 137), (65536, 3277), (1, 1), (300, 0)])
def test_fitness_and_top_match_the_formula_and_a_host_sort(n, n_top):
    import torch
    say(f"screen select: n {n}, n_top {n_top}")
    s0, s1, h, tau, flags = _inputs(n, seed=n)
    calls, wt = 100, 0.1
    dev = [torch.from_numpy(a).cuda() for a in (s0, s1, h, tau, flags)]
    fit, top = N.screen_select(dev[0], dev[1], dev[2], dev[3], calls, wt, flags=dev[4],
                               n_top=n_top)
    torch.cuda.synchronize()
    fit, top = fit.cpu().numpy(), top.cpu().numpy()
    d = s1.astype(np.float64) - s0.astype(np.float64)
    want = d[:, 0] * h[:, 0] + d[:, 1] * h[:, 1] - wt * tau.astype(np.float64) / calls
    bad = (flags != 0) | ~np.isfinite(want)
    assert np.all(np.isneginf(fit[bad]))
    np.testing.assert_allclose(fit[~bad], want[~bad], rtol=1e-5, atol=1e-5)
    order = np.lexsort((np.arange(n), -fit.astype(np.float64)))
    np.testing.assert_array_equal(top, order[:n_top])
    if n_top > 1:
        assert np.all(np.diff(fit[top]) <= 0)


def test_screen_select_argument_errors():
    import torch
    z = torch.zeros((4, 2), device="cuda")
    with pytest.raises(N.NpxError):
        N.screen_select(z, z, z, z[:, 0].contiguous(), 10, 0.1, n_top=5)   # n_top > n
    with pytest.raises(N.NpxError):
        N.screen_select(z, z, z, z[:, 0].contiguous(), 0, 0.1, n_top=1)    # n_calls < 1
