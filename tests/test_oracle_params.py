"""The oracle's default parameters against the values the paper prints
(tests/golden/paper_parameters.json, each entry with its citation)."""
import json
import math
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def test_oracle_defaults_match_paper(orc):
    g = json.load(open(GOLDEN))
    p = orc.Params()
    for k in ("eta", "r_search0", "r_search1", "r_search2", "r_search3", "r_cut1", "G", "m_star"):
        assert getattr(p, k) == g[k]["value"], k
    assert math.isclose(p.eta0, g["eta0_over_eta"]["value"] * p.eta)
    assert p.r_cut0 == g["r_cut0_timing_runs"]["value"]
    # soft step: 1/64 of an orbit at 1 au (an orbit is one year = 2 pi)
    assert math.isclose(p.dt_soft * 64, g["year_in_time_units"]["value"])
