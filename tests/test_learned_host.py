"""Host-side logic of the selector's training pipeline (no GPU): targets,
initial parameters and the regret/gain summary."""
import math

import numpy as np

from oracle import mlp as M


def test_targets_are_log_ratios_to_the_fastest_timed_class():
    from paper_2206_01784_amd import learned as L
    times = np.array([[2.0, 1.0, np.nan, 4.0] + [np.nan] * 8,
                      [np.nan, 3.0, 3.0, 6.0] + [np.nan] * 8])
    y, mask = L.targets(times)
    assert mask.tolist()[0][:4] == [1, 1, 0, 1] and mask[:, 4:].sum() == 0
    np.testing.assert_allclose(y[0, :4], [math.log(2), 0, 0, math.log(4)], rtol=1e-6)
    np.testing.assert_allclose(y[1, :4], [0, 0, 0, math.log(2)], rtol=1e-6)


def test_glorot_params_match_the_layer_layout():
    from paper_2206_01784_amd import learned as L
    p = L.glorot_params(3)
    assert p.size == M.NUM_PARAMS and p.dtype == np.float32
    blocks = M.unflatten(p.astype(np.float64))
    for name, shape in M.PARAM_SHAPES:
        if len(shape) == 1:
            assert not blocks[name].any(), name
        else:
            a = math.sqrt(6.0 / (shape[0] + shape[1]))
            assert np.abs(blocks[name]).max() <= a and np.abs(blocks[name]).max() > 0.5 * a


def test_summary_regret_and_gain():
    """gain = default / learned (selection included), regret = learned / best
    - 1; inputs of 2^26 keys or more are summarised apart (selection runs
    only there)."""
    from paper_2206_01784_amd import learned as L
    rows = [dict(n=1 << 20, best_ms=1.0, default_ms=2.0, learned_ms=1.0, pick_ms=1.0),
            dict(n=1 << 27, best_ms=2.0, default_ms=2.0, learned_ms=4.0, pick_ms=3.0)]
    s = L.summarize(rows)
    assert s["inputs"] == 2 and s["inputs_selected"] == 1
    assert math.isclose(s["regret_mean"], (0.0 + 1.0) / 2)
    assert math.isclose(s["gain_geomean"], math.sqrt(2.0 * 0.5))
    assert math.isclose(s["gain_geomean_without_selection"], math.sqrt(2.0 * 2.0 / 3.0))
    assert math.isclose(s["best_over_default_geomean"], math.sqrt(2.0))
    assert math.isclose(s["gain_geomean_selected"], 0.5)
    assert math.isclose(s["best_over_default_geomean_selected"], 1.0)
