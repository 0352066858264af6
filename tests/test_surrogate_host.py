"""Host logic of the sweep surrogate (no GPU): inputs over the sweep
ranges, the stable solver parameters of an input row, the target encoding
of a diagnostics record, the error definitions and the trust-threshold
calibration."""
import math

import numpy as np

from paper_1702_04487_amd import surrogate as S


def test_inputs_cover_the_sweep_ranges_deterministically():
    x = S.sample_inputs(4000, 3)
    assert np.array_equal(x, S.sample_inputs(4000, 3))
    assert x[:, 0].min() >= 30 and x[:, 0].max() <= 150
    assert x[:, 1].min() >= 0.005 and x[:, 1].max() <= 0.02
    # sigma log-uniform: its log is uniform, so half the draws lie below the geometric mean
    assert abs(np.mean(x[:, 1] < math.sqrt(0.005 * 0.02)) - 0.5) < 0.03
    for c in (2, 3):
        assert x[:, c].min() >= 5e-5 and x[:, c].max() <= 3e-4
    for c in (4, 5, 6):
        assert x[:, c].min() >= 500 and x[:, c].max() <= 3000 and np.all(x[:, c] == np.floor(x[:, c]))


def test_stable_parameters_respect_both_bounds():
    x = S.sample_inputs(500, 4)
    for row in x:
        p = S.case_params(row)
        assert p["gamma"] * p["sigma"] <= S.GAMMA_SIGMA_MAX * (1 + 1e-12)
        bound = max(p["f_pos"], p["f_neg"]) * 32 ** 2 / (8 * 0.55 * 0.1)
        assert bound <= S.U_CAP * (1 + 1e-12)
        # one factor for both amplitudes: their ratio is kept
        assert p["f_pos"] / p["f_neg"] == np.float64(row[2] / row[3]) or \
            abs(p["f_pos"] / p["f_neg"] - row[2] / row[3]) < 1e-12 * row[2] / row[3]
        assert p["periodic_pulse"] == 1 and p["nozzle_w"] == 32 and p["nozzle_len"] == 256


def test_target_encoding():
    none = dict(breakup_step=-1, v_drop=float("nan"), vol_drop=0, satellite=0)
    assert list(S.targets_of(none, 24000)) == [24000.0, 0.0, 0.0, 0.0]
    drop = dict(breakup_step=6400, v_drop=0.0073, vol_drop=9200, satellite=1)
    assert list(S.targets_of(drop, 24000)) == [6400.0, 0.0073, 9200.0, 1.0]
    lost = dict(breakup_step=16200, v_drop=float("nan"), vol_drop=0, satellite=0)
    assert list(S.targets_of(lost, 24000)) == [16200.0, 0.0, 0.0, 0.0]


def test_scores_and_calibration():
    H = 24000.0
    # breakup (v defined), breakup whose drop left no velocity sample (v = 0),
    # breakup, no breakup predicted as none, no breakup predicted as breakup
    y = np.array([[10000.0, 0.02], [20000.0, 0.0], [5000.0, -0.01], [H, 0.0], [H, 0.0]])
    pred = np.array([[10100.0, 0.0202], [20000.0, 0.001], [6000.0, -0.01], [H, 0.0], [23000.0, 0.003]])
    sc = S.scores(pred, y, H)
    assert list(sc["breakup"]) == [True, True, True, False, False]
    assert list(sc["wrong"]) == [False, False, False, False, True]
    assert np.allclose(sc["et"][:3], [0.01, 0.0, 0.2]) and np.isnan(sc["et"][3:]).all()
    # v is scored only where the target has one: case 1 carries none
    assert np.allclose(sc["ev"][[0, 2]], [0.01, 0.0]) and np.isnan(sc["ev"][[1, 3, 4]]).all()
    spread = np.array([0.1, 0.3, 0.5, 0.05, 0.6])
    # ordered by spread: cases 3, 0, 1, 2, 4.  Prefix ends and their bounds:
    # case 3: nothing defined, no wrong call -> ok; case 0: et .01, ev .01 -> ok;
    # case 1: et {.01, 0} (bound .005 + 1.645 * .005 / sqrt 2 = .0108) -> ok;
    # case 2: et mean .07 -> refused; case 4: a wrong call -> refused
    assert S.calibrate(spread, sc, tol=0.02) == 0.3
    sc_bad = dict(sc, wrong=np.ones(5, bool))
    assert S.calibrate(spread, sc_bad, tol=0.02) == 0.0
    # a prefix whose mean is within tol but whose bound is not is refused:
    # errors 0, .039 have mean .0195 and bound .0195 + 1.645 * .0195 / sqrt 2 = .042
    s2 = np.array([0.1, 0.2])
    sc2 = dict(et=np.array([0.0, 0.039]), ev=np.full(2, np.nan), wrong=np.zeros(2, bool))
    assert S.calibrate(s2, sc2, tol=0.02) == 0.1
    assert S.calibrate(s2, sc2, tol=0.02, z=0.0) == 0.2
    rep = S.summary(sc, spread <= 0.3)
    assert rep["answered"] == 3 and rep["class_accuracy"] == 1.0 and rep["answered_breakup"] == 2
    assert rep["err_breakup_step_n"] == 2 and np.isclose(rep["err_breakup_step_mean"], 0.005)
    assert rep["err_v_drop_n"] == 1 and np.isclose(rep["err_v_drop_mean"], 0.01)


def test_predict_reads_breakup_near_horizon_as_none():
    """A mean breakup step within the band below the horizon is answered as
    no breakup exactly; other rows and the spread pass through."""
    import torch

    class _Net:
        def predict(self, x):
            mean = torch.tensor([[23700.0, 0.0003, 12.0, 0.1], [23000.0, 0.012, 9000.0, 0.2]])
            return mean, torch.tensor([[2.0, 0.004, 0.0, 0.0], [4.0, 0.002, 0.0, 0.0]])

    sur = S.Surrogate.__new__(S.Surrogate)
    sur.net, sur.horizon, sur.y_std = _Net(), 24000.0, np.array([10.0, 0.01, 1.0])
    mean, spread = sur.predict(np.zeros((2, 7)))
    assert list(mean[0]) == [24000.0, 0.0, 0.0, 0.0]              # 23700 >= 0.98 * 24000
    assert np.allclose(mean[1], [23000.0, 0.012, 9000.0, 0.2])    # below the band: unchanged
    assert np.allclose(spread, [0.4, 0.4])                         # max(2/10, .004/.01), max(4/10, .002/.01)
