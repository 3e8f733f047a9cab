"""Host logic of the statistical validation driver (no GPU): window selection,
means of the velocity estimators and least-squares slopes of the separations."""
import math

import numpy as np
import pytest

from paper_2208_01525_amd import validation as V


def _rec(eta, xi_w, v2):
    return {"eta": eta, "v2_lag": v2, "v2_pq": math.nan if eta < 231 else 0.3, "f_total": 0.02, "f_p": 0.04,
            "xi_W": xi_w, "xi_p": 1.5 * xi_w, "xi_q": 1.4 * xi_w, "xi_pq": math.inf, "xi_lag": 2.0 * xi_w,
            "gauss_rel": [1e-6, 2e-6]}


def test_asymptotic_window_means_and_slopes():
    recs = [_rec(float(e), 0.2 * e + 3.0, 0.25 + 0.001 * (e % 2)) for e in range(200, 257)]
    a = V.asymptotic(recs, 230.0, 256.0)
    assert a["records"] == 27
    assert a["xi_W_dot"] == approx(0.2) and a["xi_p_dot"] == approx(0.3)
    assert a["xi_lag_dot"] == approx(0.4)
    assert a["xi_pq_dot"] is None                      # no finite pq separations
    v = [0.25 + 0.001 * (e % 2) for e in range(230, 257)]
    assert a["v2_lag"] == approx(np.mean(v))
    assert a["v2_pq"] == approx(0.3)            # NaN records are skipped
    assert a["xi_W_end"] == approx(0.2 * 256 + 3.0)
    assert a["gauss_rel_max"] == 2e-6


def test_asymptotic_empty_window():
    assert V.asymptotic([_rec(1.0, 1.0, 0.1)], 230.0, 256.0) == {"records": 0}


def approx(x):
    return pytest.approx(x, rel=1e-12, abs=1e-12)
