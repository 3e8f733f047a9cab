"""The paper's full run schedule on a small box (GPU): cooling, damped phase, core growth,
physical evolution (Sec. III, Sec. V), checked through properties that hold at any size."""
import math

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2208_01525_amd")
from paper_2208_01525_amd import schedule  # noqa: E402


@pytest.mark.parametrize("physical", [True, False])
def test_protocol_forms_a_coarsening_network(physical):
    n, eta_end = 64, 32.0
    lat = P.Lattice(P.make_params(n, precision="fp32", eta_ref=eta_end, diag_every=20))
    lat.init_fields(3)
    schedule.run_paper_protocol(lat, 0.5, 0.95, eta_end, physical=physical, eta_tr=18.0)
    recs = lat.diagnostics()
    assert len(recs) >= 10
    for r in recs:
        assert r["flags"] == 0
        assert all(math.isfinite(v) for v in (r["sum_energy"], r["sum_lagrangian"]))
    late = [r for r in recs if r["eta"] > 10]
    # the string network coarsens: fewer pierced plaquettes, larger mean separation
    assert late[-1]["wind_abs"][0] < late[0]["wind_abs"][0]
    assert late[-1]["xi_W"] > late[0]["xi_W"]
    # and it is still a network of both species
    assert late[-1]["wind_abs"][0] > 0 and late[-1]["wind_abs"][1] > 0
