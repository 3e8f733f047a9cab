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


def test_summarize_files_recomputes_per_seed_values(tmp_path):
    """Record files alone give the per-seed slopes and the mean +- std table; the
    Manhattan-length reading scales only the separation slopes, by sqrt(3/2)."""
    import json

    path = tmp_path / "runs.jsonl"
    slopes = {1: 0.20, 2: 0.22, 3: 0.18}
    with open(path, "w") as f:
        for seed, k in slopes.items():
            for e in range(230, 257):
                r = _rec(float(e), k * e + seed, 0.25 + 0.01 * seed)
                f.write(json.dumps({"n": 1024, "era": 0.5, "m_damp": 0.9, "seed": seed, **r}) + "\n")
    groups = V.summarize_files([str(path)])
    per_seed = groups[(1024, 0.5)]
    assert [p["seed"] for p in per_seed] == [1, 2, 3]
    assert [p["xi_W_dot"] for p in per_seed] == [approx(0.20), approx(0.22), approx(0.18)]
    sm = V.summarize(per_seed)
    assert sm["xi_W_dot"][0] == approx(0.20) and sm["xi_W_dot"][1] == approx(0.02)
    assert sm["f_p"][0] == approx(0.04) and sm["v2_lag"][0] == approx(0.27)
    t = V.table(groups)
    row = next(line for line in t.splitlines() if "| xi_W_dot |" in line)
    assert f"{0.2 * math.sqrt(1.5):.4g}" in row
    for key in ("v2_lag", "xi_lag_dot", "f_p"):       # not lengths counted from windings
        row = next(line for line in t.splitlines() if f"| {key} |" in line)
        assert row.rstrip().endswith("|  |"), key
