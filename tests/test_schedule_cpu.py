"""Host-side schedule helpers against Table 3 of the paper (tests/golden/)."""
import os

import pytest

from paper_2208_01525_amd import schedule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3_core_growth.txt")


def rows():
    return [l.split() for l in open(GOLDEN) if l.strip() and l[0] != "#"]


def test_core_growth_beta_matches_table3():
    """Table 3: with the damping phase ending at eta = 5 (Sec. III), growing the radius to
    r_s,max by eta_tr = 343 takes the printed beta_growth (to 1e-4)."""
    for mm, _md, beta_g, _b, eta_tr, rmax in rows():
        got = schedule.core_growth_beta(float(rmax), float(mm), 5.0, float(eta_tr))
        assert got == pytest.approx(float(beta_g), rel=1e-4)


def test_max_radius_matches_table3():
    """a = 1 at the end of the run (eta = 1024) gives r_s,max = (1024/343)^p = 3.0 / 9.0."""
    for mm, _md, _bg, _b, eta_tr, rmax in rows():
        assert schedule.max_radius(float(mm), float(eta_tr), 1024.0) == pytest.approx(float(rmax), rel=0.011)


class Recorder:
    def __init__(self):
        self.calls = []

    def cool(self, n, dt):
        self.calls.append(("cool", n, dt))

    def step(self, n, eta, era_m, s):
        self.calls.append(("step", n, eta, era_m, s))


def test_protocol_segments():
    r = Recorder()
    seg = schedule.run_paper_protocol(r, 0.5, 0.95, 64.0, physical=True, eta_tr=30.0)
    assert r.calls[0] == ("cool", 330, 1.0 / 30.0)
    assert r.calls[1] == ("step", 40, 1.0, 0.95, 0.0)
    assert r.calls[2][0] == "step" and r.calls[2][1] == 250 and r.calls[2][4] < 0
    assert r.calls[3] == ("step", 340, pytest.approx(30.0), 0.5, 1.0)
    assert seg[-1][1] == 64.0
    r = Recorder()
    schedule.run_paper_protocol(r, 2.0 / 3.0, 0.75, 20.0, physical=False)
    assert r.calls[-1] == ("step", 150, 5.0, 2.0 / 3.0, 0.0)
