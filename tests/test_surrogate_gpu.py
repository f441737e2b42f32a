"""What the trained surrogate gains over the method without it: trained
on samples the solver produced for one set of capillaries, it predicts
drag, lift and bond hazard for capillaries it has not seen far better than
the best feature-free guess (the training mean), at a fraction of a
microsecond per prediction against the solver's milliseconds per step.
All computation runs in the HIP kernels (solver and surrogate)."""
import numpy as np
import pytest

from helpers import say
from paper_2210_06043_amd import inputs, surrogate

pytestmark = pytest.mark.gpu


def test_surrogate_generalises_to_unseen_capillaries():
    """Trained on the 256 capillaries of the batched workload (600 steps,
    samples every 2 steps), evaluated on 32 capillaries of another draw.
    Drag and hazard: mean squared error (standardised) below half the
    mean-guess error.  Lift depends on the particle's deformation and its
    position under the cell, which the 37 features do not carry: its gain
    is smaller, required below 0.9 of the mean guess."""
    train_cfgs = inputs.config_c3(seed=0, members=256)
    test_cfgs = inputs.config_c3(seed=1, members=32)
    S, ms, first = surrogate.harvest(train_cfgs, 600, every=2)
    X, T, _ = surrogate.features(S, train_cfgs, first)
    S2, _, first2 = surrogate.harvest(test_cfgs, 600, every=2)
    X2, T2, _ = surrogate.features(S2, test_cfgs, first2)
    fx, ft = surrogate.Standardiser(X), surrogate.Standardiser(T)
    net, ms_train = surrogate.train(fx(X), ft(T), steps=1000, batch=4096)
    P = surrogate.predict(net, fx(X2))
    err = np.mean((P - ft(T2)) ** 2, axis=0)
    base = np.mean(ft(T2) ** 2, axis=0)
    say(f"surrogate: {X.shape[0]} training samples ({len(train_cfgs)} capillaries), {X2.shape[0]} held-out "
        f"({len(test_cfgs)}); solver {ms:.3f} ms per ensemble step, training {ms_train:.3f} ms per step")
    say(f"held-out MSE (standardised) drag/lift/hazard {np.round(err, 4).tolist()} vs mean-guess "
        f"{np.round(base, 4).tolist()}")
    assert np.all(np.isfinite(P))
    assert err[0] < 0.5 * base[0] and err[2] < 0.5 * base[2]
    assert err[1] < 0.9 * base[1]


@pytest.mark.timeout(900)
def test_screened_sweep_against_the_solver_alone():
    """The surrogate screening a parameter sweep, with the solver as its
    fallback and its judge: 32 unseen capillaries, each with six particle
    variants (aspect ratio 0.3 / 0.6 / 0.9, rigid or Ca = 1e-4).  Without
    the surrogate every variant is a solver run.  Screened, one solver run
    per capillary (the reference variant) supplies the cell-side features,
    four networks predict the other variants, and a variant whose predicted
    uncertainty exceeds a threshold falls back to the solver.  The
    threshold is chosen on 16 capillaries so that the answers stay within a
    standardised mean squared error of 0.1 on every output; on the other 16
    the screened answers must stay within 0.15 and save solver runs."""
    res = surrogate.screening_study(inputs.config_c3(seed=0, members=256), sweep_seed=1, cells=32, eps=0.1)
    say(f"screening: threshold {res['tau']:.4f}; evaluation error (standardised MSE drag/lift/hazard) "
        f"{np.round(res['eval_error'], 4).tolist()}; {res['eval_runs']} solver runs for {res['eval_answers']} "
        f"variant answers ({res['eval_fallbacks']} fallbacks) = {res['answers_per_run']:.2f} answers per run")
    for tau, err, runs, given in res["calibration"]:
        say(f"  calibration: threshold {tau:.4f} -> worst error {err:.4f}, {runs} runs for {given} answers")
    # answers per hour: the solver alone gives one variant answer per run
    # (runs of the sweep's length at the measured ensemble step time); the
    # screened sweep answers_per_run per solver run (inference takes
    # microseconds per variant)
    solver = 256 * 3600.0 / (600 * res["harvest_ms_per_step"] * 1e-3)
    say(f"variant answers per hour at standardised error <= {res['eps']}: solver alone {solver:.3e}, "
        f"screened {solver * res['answers_per_run']:.3e}")
    assert max(res["eval_error"]) <= 0.15
    assert res["answers_per_run"] > 1.0


@pytest.mark.timeout(600)
def test_surrogate_trained_on_paper_scale_runs():
    """Trained on 1.0e6 samples harvested from 256 paper-scale channels
    (3840 x 240, six cells, the particle's aspect ratio and Ca drawn as in
    the paper-scale draw, the row of cells shifted by up to 150 nodes so
    that the cell-particle distance varies), evaluated on 32 channels of
    another draw: drag below half and hazard below three quarters of the
    mean-guess error; lift, which depends on what the features do not
    carry, below 0.9 of it."""
    res = surrogate.paper_scale_study()
    say(f"paper-scale surrogate: {res['train_samples']} training samples, {res['test_samples']} held-out; solver "
        f"{res['harvest_ms_per_step']:.3f} ms per 256-channel step; held-out MSE drag/lift/hazard "
        f"{np.round(res['err'], 4).tolist()} vs mean guess {np.round(res['mean_guess'], 4).tolist()}")
    assert res["finite"] and res["train_samples"] >= 1_000_000
    e, b = res["err"], res["mean_guess"]
    assert e[0] < 0.5 * b[0] and e[2] < 0.75 * b[2] and e[1] < 0.9 * b[1]
