"""Symmetries of the model on the HIP path, through the C ABI.

* Exchange (Sec. II): swapping phi <-> psi, A <-> B and their momenta together
  with the couplings of the two sectors swaps every output.  The update treats
  each sector with the same operations, so the evolved fields, the windings
  and the cell values swap bit for bit; the record's sums add the two
  sectors' terms in the other order (and the interaction weight multiplies
  its factors in the other order), agreeing to the working precision.
* Lattice gauge transform: phi -> e^{i Lambda} phi, Pi -> e^{i Lambda} Pi,
  A_i -> A_i + (Lambda(x+i) - Lambda(x)) / h.  The fields evolve covariantly
  (to the rounding of the transformed inputs), and the windings, cells and
  overlap counts are invariant bit for bit; the energy, Lagrangian and Gauss
  sums are invariant to rounding.
"""
import numpy as np
import pytest

from tests import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2208_01525_amd")

COUP = dict(lam=(2.0, 1.6), e=(1.0, 0.9), sig=(1.0, 1.1), kappa=0.7)
SWAPPED = dict(lam=(1.6, 2.0), e=(0.9, 1.0), sig=(1.1, 1.0), kappa=0.7)


def _swap(st):
    out = st.copy()
    for a, b, n in ((I.PHI, I.PSI, 2), (I.PI, I.PSIDOT, 2), (I.A, I.B, 3), (I.E, I.H, 3)):
        out[a:a + n], out[b:b + n] = st[b:b + n], st[a:a + n]
    return out


def _lattice(geom, precision, coup, **kw):
    nx, ny, nz = geom
    return P.Lattice(P.make_params(nx, ny, nz, precision=precision, eta_ref=9.0, **coup, **kw), device="cuda:0")


def _evolve(geom, precision, coup, st, n=6, d=3):
    lat = _lattice(geom, precision, coup, diag_every=d)
    lat.set_fields(st)
    lat.step(n, 2.0, 0.5, 1.0)
    recs = lat.diagnostics()
    out = lat.get_fields(), lat.get_windings().astype(np.int32), lat.get_cells().astype(np.int32), recs
    lat.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sector_exchange(precision):
    geom = (72, 18, 11)
    st = I.random_full(*geom, 17, link=0.8, mom=0.5)
    if precision == "fp32":
        st = I.to_f32_values(st)
    f, W, cells, recs = _evolve(geom, precision, COUP, st)
    fs, Ws, cells_s, recs_s = _evolve(geom, precision, SWAPPED, _swap(st))
    assert np.array_equal(fs, _swap(f))
    assert np.array_equal(Ws, np.concatenate([W[3:], W[:3]]))
    assert np.array_equal(cells_s, cells[::-1])
    assert len(recs) == len(recs_s) == 2
    # the interaction weight kappa (|phi|^2 - sigma_p^2)(|psi|^2 - sigma_q^2) multiplies its
    # factors in the other order: per-site rounding of the working precision
    rt = 1e-6 if precision == "fp32" else 1e-12
    for r, q in zip(recs, recs_s):
        assert q["wind_abs"] == r["wind_abs"][::-1] and q["pq_count2"] == r["pq_count2"]
        for k in ("sum_energy", "sum_lagrangian", "sum_KL", "sum_GL", "sum_KV", "sum_GV"):
            assert q[k] == pytest.approx(r[k], rel=rt, abs=rt), k
        for a in range(2):
            assert q["gauss_abs"][1 - a] == pytest.approx(r["gauss_abs"][a], rel=1e-9, abs=1e-12)
            assert q["gauss_scale"][1 - a] == pytest.approx(r["gauss_scale"][a], rel=1e-9)


def _gauge(st, lam, h):
    out = st.copy()
    ph = np.exp(1j * lam)
    for c in (I.PHI, I.PSI, I.PI, I.PSIDOT):
        z = (st[c] + 1j * st[c + 1]) * ph
        out[c], out[c + 1] = z.real, z.imag
    for a0 in (I.A, I.B):
        for i, ax in enumerate((2, 1, 0)):
            out[a0 + i] = st[a0 + i] + (np.roll(lam, -1, axis=ax) - lam) / h
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_gauge_transform(precision):
    geom = (64, 16, 12)
    h = 0.5
    st = I.random_full(*geom, 23, link=0.6, mom=0.5)
    lam = I.gauge_function(*geom, 24)
    st_g = _gauge(st, lam, h)
    if precision == "fp32":
        st, st_g = I.to_f32_values(st), I.to_f32_values(st_g)
    f, W, cells, recs = _evolve(geom, precision, COUP, st)
    fg, Wg, cells_g, recs_g = _evolve(geom, precision, COUP, st_g)
    # windings, cells and overlap: invariant bit for bit
    assert np.array_equal(W, Wg) and np.abs(W).sum() > 0
    assert np.array_equal(cells, cells_g)
    for r, q in zip(recs, recs_g):
        assert r["wind_abs"] == q["wind_abs"] and r["pq_count2"] == q["pq_count2"]
    # the evolved fields are the transform of the evolved fields
    tol = 2e-4 if precision == "fp32" else 1e-11
    assert np.abs(_gauge(f, lam, h) - fg).max() < tol
    # gauge-invariant sums
    rt = 1e-4 if precision == "fp32" else 1e-10
    for r, q in zip(recs, recs_g):
        for k in ("sum_energy", "sum_lagrangian"):
            assert q[k] == pytest.approx(r[k], rel=rt), k
        for a in range(2):
            assert q["gauss_scale"][a] == pytest.approx(r["gauss_scale"][a], rel=rt)
