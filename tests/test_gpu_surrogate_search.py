"""The learned surrogate end to end on the GPU: transitions from the step
kernel, training by the library's kernels, held-out error, and what the screen
gains over spending the same plain-simulation budget on random candidates."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def trained():
    from paper_2411_05799_amd import surrogate as S
    say("case: generate 2 x 2048 x 120 transitions, train 12 epochs")
    X, Y, info = S.generate(n_terrains=2, n_inst=2048, n_samples=120, seed=4242)
    assert info["transitions"] == X.shape[0] == Y.shape[0] > 0.95 * 2 * 2048 * 120
    X, Y, n_train = S.split(X, Y, holdout=0.05)
    tr = S.train(X, Y, n_train, epochs=12, batch=4096)
    ev = S.evaluate(tr, X, Y, n_train, X.shape[0])
    yield tr, ev
    tr.net.close()


def test_training_beats_the_mean_predictor_on_held_out_data(trained):
    tr, ev = trained
    assert tr.history[-1] < 0.5 * tr.history[0]
    assert ev["nmse_mean_predictor"] > 0.9
    assert ev["nmse"] < 0.15, ev["nmse"]


def test_screen_gains_over_random_candidates(trained):
    """Same number of plain re-simulations (the top 5% by the surrogate vs a
    random 5%): the screen must find a better best candidate, and its
    re-simulated fitness is exactly the plain method's."""
    from paper_2411_05799_amd import surrogate as S
    from paper_2411_05799_amd import workloads as W
    tr, _ = trained
    say("case: screen 4096 candidates x 100 calls")
    w = W.hexapod_batch(4096, seed=77, hf=W.octave_terrain(2), n_steps=10)
    out = S.screen(w, tr, settle=200, n_calls=100, top_frac=0.05, plain_all=True)
    assert out["resim_matches_plain"]
    f_all, _, _ = S.plain_fitness(w, np.arange(4096), 200, 100)
    rng = np.random.default_rng(0)
    random_best = [np.max(f_all[rng.choice(4096, out["top"], replace=False)]) for _ in range(200)]
    say(f"screen best {out['best_found']:.4f}, random-subset best "
        f"{np.mean(random_best):.4f} (mean), true best {out['best_true']:.4f}, "
        f"rank error {out['rank_error']:.3f}, recall {out['top_recall']:.3f}")
    beaten = float(np.mean(out["best_found"] > np.array(random_best)))
    say(f"screen best beats {100 * beaten:.0f}% of random subsets of the same size")
    assert beaten > 0.5
    assert out["top_recall"] > 0.15          # random choice gives 0.05
    assert out["rank_error"] < 0.3           # random ranking gives 1/3


def test_output_weights_keep_the_delta_scale(trained):
    """Loss weights on output columns are realised in the target scale: the
    de-standardised outputs stay the state change, so a network trained with
    the joint columns nearly ignored predicts the body columns as well as
    the unweighted one and the joint columns still in their own units."""
    from paper_2411_05799_amd import surrogate as S
    tr, ev = trained
    say("case: re-train 12 epochs with joint outputs at weight 1e-3")
    X, Y, _ = S.generate(n_terrains=2, n_inst=2048, n_samples=120, seed=4242)
    X, Y, n_train = S.split(X, Y, holdout=0.05)
    ow = np.ones(49)
    ow[13:] = 1e-3
    tw = S.train(X, Y, n_train, epochs=12, batch=4096, out_weight=ow)
    np.testing.assert_allclose(tw.y_std, tw.y_std_raw / np.sqrt(ow), rtol=1e-6)
    np.testing.assert_allclose(tw.y_std_raw, tr.y_std_raw, rtol=1e-5)
    evw = S.evaluate(tw, X, Y, n_train, X.shape[0])
    body, body_w = np.array(ev["rmse"][:13]), np.array(evw["rmse"][:13])
    say(f"body rmse ratio weighted/unweighted: {np.round(body_w / body, 3).tolist()}")
    assert np.all(body_w < 1.25 * body)
    joint_std = tr.y_std_raw[13:]
    assert np.all(np.array(evw["rmse"][13:]) < 2.0 * joint_std + 1e-6)
    tw.net.close()
