"""Host-side summary of the held-out warm-start evaluation: subsets, ratios and the
geometries recorded without a solve."""
import numpy as np
import pytest

from paper_1410_1921_amd import warmstart as WS


def row(seed, plain, warm, conv=(True, True, True, True), ps=(2.0, 8.0), ws=(2.0, 5.0),
        k=(1e-3, 1e-3), d=(0.01, 0.01), dp=(0.01, 0.01), no_path=False):
    r = dict(seed=seed, porosity=0.3, n_fluid=100, plain_steps=list(plain),
             warm_steps=list(warm), plain_s=list(ps), warm_s=list(ws), inference_s=0.5,
             converged=list(conv), warm_used=True, k_plain=k[0], k_warm=k[1],
             deff_plain=d[0], deff_warm=d[1], deff_planes_plain=dp[0], deff_planes_warm=dp[1])
    if no_path:
        r["no_path"] = True
    return r


def test_summary_subsets_and_ratios():
    rows = [row(1, (1000, 100000), (1000, 50000), d=(0.01, 0.0101), dp=(0.01, 0.01001)),
            row(2, (2000, 300000), (2000, 240000)),
            # the solve from rest does not converge: solved, not in the converged subset
            row(3, (60000, 4000000), (60000, 4000000), conv=(False, False, False, False),
                ps=(20.0, 20.0), ws=(20.0, 20.0)),
            row(4, (0, 0), (0, 0), ps=(0.0, 0.0), ws=(0.0, 0.0), no_path=True)]
    s = WS.summary(rows)
    assert s["no_path"] == 1 and s["all"]["n"] == 3 and s["converged"]["n"] == 2
    c = s["converged"]
    assert c["knudsen_steps_ratio"] == pytest.approx(290000 / 400000)
    assert c["knudsen_steps_ratio_median"] == pytest.approx(np.median([0.5, 0.8]))
    assert c["time_plain_s"] == pytest.approx(20.0)
    assert c["time_warm_s"] == pytest.approx(7.0 + 7.0 + 1.0)  # inference counted
    assert c["speedup"] == pytest.approx(20.0 / 15.0)
    assert s["deff_rel_diff_max"] == pytest.approx(0.01)
    assert s["deff_planes_rel_diff_max"] == pytest.approx(1e-3)
    assert s["knudsen_converged"] == [2, 2]
    assert s["all"]["time_plain_s"] == pytest.approx(60.0)


def test_summary_without_converged_rows():
    s = WS.summary([row(3, (60000, 4000000), (60000, 4000000),
                        conv=(False, False, False, False))])
    assert s["converged"] == {} and s["all"]["n"] == 1
