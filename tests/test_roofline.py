"""The roofline helpers reproduce the printed performance model of the paper
(Sec. 4.3, Table 1): traffic per update, P_max, lightspeed and the ratios."""
import json
import os

import pytest

from paper_2402_13171_amd import roofline

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")


def test_table1_reproduced():
    with open(GOLD) as fh:
        t = json.load(fh)
    assert roofline.bytes_per_lup(4, force_components=3) == t["n_b"]
    l = roofline.lightspeed(1713.0e9, t["n_f"], t["peak_flops_a100"], t["n_b"])
    assert l == pytest.approx(t["lightspeed_a100"], abs=5e-5)
    for row in t["rows"]:
        pmax = roofline.p_max_lups(row["b_S_GBps"] * 1e9, t["n_b"]) / 1e6
        assert pmax == pytest.approx(row["P_max_MLUPS"], abs=0.05)
        pct = 100 * roofline.fraction_of_pmax(row["with_MLUPS"] * 1e6, row["b_S_GBps"] * 1e9, t["n_b"])
        assert pct == pytest.approx(row["ratio_pct"], abs=0.05)


def test_mi355x_rooflines():
    assert roofline.bytes_per_lup(4) == 216
    assert roofline.bytes_per_lup(2) == 108
    assert roofline.p_max_lups(8e12, 216) / 1e6 == pytest.approx(37037.04, abs=0.01)
    assert roofline.p_max_lups(8e12, 108) / 1e6 == pytest.approx(74074.07, abs=0.01)
