"""Pins for the roofline model against the values printed in Section 3.3 and
Table 3 (tests/golden/roofline_spin26.json)."""
import json
import os

import pytest

from oracle import perfmodel as P

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "roofline_spin26.json")))


@pytest.mark.parametrize("arch", ["ivb", "skx"])
def test_spin26_symmspmv_bounds(arch):
    a = G[arch]
    i = P.intensity_symmspmv(a["alpha_symm"], G["nnzr"])
    lo, hi = a["expect_GFs"]
    assert round(P.performance(i, a["copy_GBs"]), 2) == lo
    assert round(P.performance(i, a["load_GBs"]), 2) == hi


@pytest.mark.parametrize("arch", ["ivb", "skx"])
def test_alpha_from_measured_traffic(arch):
    a = G[arch]
    # the traffic is printed to 0.01 B and alpha to 0.001: allow both roundings
    alpha = P.alpha_from_traffic(a["traffic_B_per_nnz"], G["nnzr"])
    assert abs(alpha - a["alpha_spmv"]) <= 0.005 / 8 + 0.0005
    # and the alpha of Table 3 lies inside the printed traffic's rounding interval
    t = 12.0 + 20.0 / G["nnzr"] + 8.0 * a["alpha_symm"]
    assert abs(t - a["traffic_B_per_nnz"]) <= 0.005 + 1e-9


@pytest.mark.parametrize("row", G["table3_optimal"], ids=lambda r: r["matrix"])
def test_table3_optimal_columns(row):
    nnzr = 1.0 / row["alpha_opt"]
    assert P.optimal_alpha_spmv(nnzr) == pytest.approx(row["alpha_opt"], rel=1e-12)
    assert P.intensity_spmv(P.optimal_alpha_spmv(nnzr), nnzr) == pytest.approx(row["I_opt"], rel=1e-9)


def test_symm_intensity_limits():
    # with small alpha SymmSpMV approaches twice the SpMV intensity (Section 3.2)
    nnzr = 27.0
    r = P.intensity_symmspmv(0.0, 1e12) / P.intensity_spmv(0.0, 1e12)
    assert r == pytest.approx(2.0)
    assert P.nnzr_symm(nnzr) == 14.0
    assert P.optimal_alpha_symmspmv(nnzr) == pytest.approx(1 / 14.0)
