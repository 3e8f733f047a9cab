"""Pins of the oracle's network estimators (`oracle.derive`, Sec. III.A) against
what geometry and the paper fix, independently of how the record was summed:

* the length of a straight string along z through a periodic box is N_z h, so
  a set of them has a length known by counting, and every xi = sqrt(V / L) of
  Sec. III.A with V = N_x N_y N_z h^3 follows;
* the bound-state fractions f_total and f_p are ratios of those counted
  lengths (one bound and several free strings per sector);
* a closed circular string is counted by its Manhattan length: Sigma|W| is
  the number of faces the circle crosses, 2 per lattice line x = i or y = j it
  cuts (about 8R, not 2 pi R), and L = h Sigma|W| (no length correction is
  printed, so none is applied);
* a relaxed static string at critical coupling has energy mu_lat per unit
  length, within the lattice's O(h^2) deficit of the BPS tension 2 pi sigma^2
  (Sec. IV), and with no motion the Lagrangian sums to minus the energy, so
  the Lagrangian estimator xi_L = sqrt(-mu V / sum L) must equal
  sqrt(V / L) sqrt(2 pi sigma^2 / mu_lat).  A dropped h^3, a wrong V or a mu
  that ignores sigma moves it off by far more than the deficit.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import inputs as I


def _record(m, st):
    """The integer-time record of a static configuration (one step at m = 0)."""
    return O.step(m, st.copy(), 1.0, 0.0, 1.0, diag=True)


def test_xi_of_a_straight_string_pair():
    """A vortex / antivortex pair along z: two strings of length N_z h each, so
    xi_p = xi_W = sqrt(N_x N_y N_z h^3 / (2 N_z h)); no q-strings, no bound states."""
    nx, ny, nz = 20, 14, 6
    m = O.model(nx, ny, nz)
    st = I.string_pairs(nx, ny, nz, p_pair=(5, 12, 7))
    d = O.derive(m, _record(m, st))
    h = m.h
    length = 2 * nz * h
    volume = nx * ny * nz * h ** 3
    assert d["L_p"] == pytest.approx(length, rel=1e-15)
    assert d["L_q"] == 0.0 and d["L_pq"] == 0.0
    assert d["xi_p"] == pytest.approx(math.sqrt(volume / length), rel=1e-15)
    assert d["xi_W"] == pytest.approx(math.sqrt(volume / length), rel=1e-15)
    assert d["xi_q"] == math.inf and d["xi_pq"] == math.inf
    assert d["f_total"] == 0.0 and d["f_p"] == 0.0


def test_bound_state_fractions_by_counting():
    """Four p-strings and two q-strings along z, one of them coincident in both sectors
    (a bound (1,1) string), the others at least four cells from any string of the other
    sector.  By counting: L_pq = N_z h, L_p = 3 N_z h, L_q = N_z h, so f_total = 1/5,
    f_p = 1/3 and xi_W = sqrt(V / (5 N_z h))."""
    nx, ny, nz = 24, 16, 5
    m = O.model(nx, ny, nz, overlap_radius=1)
    p = [(4, 4, 1), (10, 4, -1), (4, 10, -1), (10, 10, 1)]
    q = [(4, 4, 1), (4, 7, -1)]
    st = I.string_set(nx, ny, nz, p_vortices=p, q_vortices=q)
    rec = _record(m, st)
    h, Lz = m.h, nz * m.h
    volume = nx * ny * nz * h ** 3
    assert rec["wind_abs"] == (4 * nz, 2 * nz)        # the fixture: straight strings only
    d = O.derive(m, rec)
    assert d["L_pq"] == pytest.approx(Lz, rel=1e-15)
    assert d["L_p"] == pytest.approx(3 * Lz, rel=1e-15)
    assert d["L_q"] == pytest.approx(Lz, rel=1e-15)
    assert d["f_total"] == pytest.approx(1.0 / 5.0, rel=1e-15)
    assert d["f_p"] == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert d["xi_W"] == pytest.approx(math.sqrt(volume / (5 * Lz)), rel=1e-15)
    assert d["xi_p"] == pytest.approx(math.sqrt(volume / (3 * Lz)), rel=1e-15)
    assert d["xi_pq"] == pytest.approx(math.sqrt(volume / Lz), rel=1e-15)
    # a second q pair, one of its strings on a free p-string: two bound strings, and
    # L_p = L_q = 2 N_z h, so f_total = 1/3 and f_p = 1
    q2 = q + [(10, 10, 1), (10, 13, -1)]
    rec2 = _record(m, I.string_set(nx, ny, nz, p_vortices=p, q_vortices=q2))
    assert rec2["wind_abs"] == (4 * nz, 4 * nz)
    d2 = O.derive(m, rec2)
    assert d2["L_pq"] == pytest.approx(2 * Lz, rel=1e-15)
    assert d2["L_q"] == pytest.approx(2 * Lz, rel=1e-15)
    assert d2["f_p"] == pytest.approx(1.0, rel=1e-15)
    assert d2["f_total"] == pytest.approx(1.0 / 3.0, rel=1e-15)


def _relaxed_pair(sig_p):
    """A straight p vortex / antivortex pair along z, 8 length units apart, relaxed by
    the gradient flow at critical coupling (lambda = 2 e^2), kappa = 0, psi in its vacuum."""
    nx, ny, nz = 32, 16, 2
    m = O.model(nx, ny, nz, kappa=0.0, sig=(sig_p, 1.0))
    st = I.string_set(nx, ny, nz, p_vortices=[(7, 7, 1), (23, 7, -1)], sig=(sig_p, 1.0))
    O.cool(m, st, 1500)
    return m, st


@pytest.mark.parametrize("sig_p", [1.0, 1.3])
def test_lagrangian_estimator_of_a_static_string(sig_p):
    """Sec. III.A / IV: xi_L = sqrt(-mu V / sum L), mu = 2 pi sigma_p^2.  For the relaxed pair
    (no motion) sum L h^3 = -E = -mu_lat L, so xi_L = sqrt(V / L) sqrt(2 pi sigma_p^2 / mu_lat),
    and mu_lat is the BPS tension 2 pi sigma_p^2 up to the lattice deficit (under 3 % at
    h = 0.5 for these vevs)."""
    m, st = _relaxed_pair(sig_p)
    h = m.h
    length = 2 * m.nz * h
    volume = m.sites * h ** 3
    mu_bps = 2.0 * math.pi * sig_p ** 2
    mu_lat = O.hamiltonian(m, st) / length
    assert 0.0 < 1.0 - mu_lat / mu_bps < 0.03, mu_lat
    rec = _record(m, st)
    assert rec["wind_abs"] == (2 * m.nz, 0)
    d = O.derive(m, rec)
    assert d["xi_W"] == pytest.approx(math.sqrt(volume / length), rel=1e-15)
    # the relaxed state barely moves in one step: the time-centred kinetic terms are tiny
    assert rec["sum_lag"] == pytest.approx(-mu_lat * length, rel=1e-6)
    assert d["xi_lag"] == pytest.approx(math.sqrt(volume / length) * math.sqrt(mu_bps / mu_lat), rel=1e-6)
    # so xi_L sits within half the tension deficit of the winding estimator
    assert 1.0 < d["xi_lag"] / d["xi_W"] < 1.0 + 0.5 * 0.03


def test_velocity_estimator_of_a_static_string():
    """Sec. III.A: <v^2> = 2R/(1+R), R = sum K L / sum G L; a relaxed static string has
    K = 0 up to the momentum of one step from rest, so <v^2>_L vanishes to that order; the
    interaction weight V_int is zero everywhere when psi sits in its vacuum, so <v^2>_pq
    has a zero denominator and is reported as nan."""
    m, st = _relaxed_pair(1.0)
    d = O.derive(m, _record(m, st))
    assert 0.0 <= d["v2_lag"] < 1e-6
    assert math.isnan(d["v2_pq"])


@pytest.mark.parametrize("radius", [6.3, 9.7])
def test_ring_length_is_the_counted_crossings(radius):
    """A circular p-string of radius R in a z plane crosses each lattice line x = i with
    |i - cx| < R twice and each line y = j likewise; each crossing pierces one face, so
    Sigma|W_p| is that count exactly (about 8R: the Manhattan length of the circle, 4/pi of
    its true length 2 pi R) and L_p = h Sigma|W_p|.  The fixture's phase is not periodic
    in z: across the box's z boundary it winds the other way round the same circle, so
    the periodic box holds the ring and an opposite copy half a box above it (a closed
    string cannot carry net flux through the box), and Sigma|W_p| is twice one ring's."""
    nx = ny = 32
    nz = 8
    m = O.model(nx, ny, nz)
    st = I.ring(nx, ny, nz, radius)
    cx = nx / 2.0 - 0.5
    lines = sum(1 for i in range(nx) if abs(i - cx) < radius)
    count = 2 * lines + 2 * lines                     # x and y lines (cy = cx), one ring
    W = O.windings(m, st)
    assert int(np.abs(W[0]).sum()) == int(np.abs(W[1]).sum()) == 2 * 2 * lines
    assert np.abs(W[2]).sum() == 0                    # no face normal to z is pierced
    assert np.abs(W[3:]).sum() == 0
    # the ring in plane cz and its copy across the z boundary, face by face
    cz = nz // 2 - 1
    assert np.abs(W[:2, cz]).sum() == count and np.abs(W[:2, nz - 1]).sum() == count
    d = O.derive(m, _record(m, st))
    assert d["L_p"] == pytest.approx(m.h * 2 * count, rel=1e-15)
    # the Manhattan length of the circle, against its true length
    assert abs(count - 8 * radius) <= 4
    assert count / (2 * math.pi * radius) == pytest.approx(4 / math.pi, rel=0.08)
