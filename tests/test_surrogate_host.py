"""Host-side logic of the controller search (no GPU): rankings, rank agreement,
the learning-rate schedule and the start headings used by the fitness."""
import math

import numpy as np

from paper_2411_05799_amd import surrogate as S
from paper_2411_05799_amd import workloads as W


def test_ranks_best_first_ties_by_index():
    f = np.array([0.5, 2.0, -1.0, 2.0, 0.5])
    np.testing.assert_array_equal(S.ranks(f), [2, 0, 4, 1, 3])
    # -inf (a flagged candidate) ranks last
    g = np.array([1.0, -np.inf, 0.0])
    np.testing.assert_array_equal(S.ranks(g), [0, 2, 1])


def test_rank_agreement_identity_reversal_and_random():
    rng = np.random.default_rng(3)
    f = rng.normal(size=2000)
    same = S.rank_agreement(f, f, 100)
    assert same["rank_error"] == 0.0 and same["top_recall"] == 1.0
    assert abs(same["fitness_corr"] - 1.0) < 1e-12
    # reversed order: mean |r - (N-1-r)| / N = (N/2) / N for even N
    rev = S.rank_agreement(-f, f, 100)
    assert abs(rev["rank_error"] - 0.5) < 1e-12 and rev["top_recall"] == 0.0
    # independent rankings: mean |r1 - r2| / N -> 1/3
    other = S.rank_agreement(rng.normal(size=2000), f, 100)
    assert abs(other["rank_error"] - 1.0 / 3.0) < 0.02


def test_cosine_schedule_endpoints_and_midpoint():
    assert S.cosine_lr(0, 100, 1e-3, 1e-5) == 1e-3
    assert abs(S.cosine_lr(100, 100, 1e-3, 1e-5) - 1e-5) < 1e-15
    assert abs(S.cosine_lr(50, 100, 1e-3, 1e-5) - 0.5 * (1e-3 + 1e-5)) < 1e-15
    assert S.cosine_lr(500, 100, 1e-3, 1e-5) == S.cosine_lr(100, 100, 1e-3, 1e-5)


def test_start_heading_is_the_torso_x_axis_on_the_ground():
    w = W.hexapod_batch(8, seed=3, n_steps=10)
    yaw = np.linspace(-3.0, 3.0, 8)
    w.pose[:, 3] = np.cos(yaw / 2)          # rotation about z by yaw
    w.pose[:, 4:6] = 0.0
    w.pose[:, 6] = np.sin(yaw / 2)
    h = S._heading0(w)
    np.testing.assert_allclose(h, np.stack([np.cos(yaw), np.sin(yaw)], 1), atol=1e-6)
    # a tilt about the heading axis leaves the heading unchanged
    q = np.array([math.cos(0.2), math.sin(0.2), 0.0, 0.0])   # 0.4 rad about x
    w.pose[0, 3:7] = q
    np.testing.assert_allclose(S._heading0(w)[0], [1.0, 0.0], atol=1e-6)
