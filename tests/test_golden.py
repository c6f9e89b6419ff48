"""Defaults of the oracle follow the parameters the paper prints (Fig. 2, sec. 2.1)."""
import json
import os

import oracle as o

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_defaults_follow_fig2():
    cfg = json.load(open(os.path.join(HERE, "golden", "fig2_sample_config.json")))
    D = o.Domain(8, 8, 0.1, 0.1, 0.01, -1.0 * __import__("numpy").ones((9, 9)))
    assert D.p.eps == cfg["epsilon"]
    assert D.p.n_corr == cfg["correctionStepsNum"]
    assert abs(D.p.Bdisp - cfg["dispersion_B"]["value"]) < 1e-16
    assert D.p.ws == cfg["fieldDimensions"]["stillWaterElevation"]
