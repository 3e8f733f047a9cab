"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these retypes the oracle's formulas: each checks a closed form, an
exact invariant, a brute-force computation through a different route, or a
value the paper prints.  A dropped term, a wrong sign, index or factor in the
update, the energy, the windings or the overlap fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from tests import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- P1, P2


@pytest.mark.parametrize("era_m,s", [(0.0, 1.0), (0.5, 1.0), (2.0 / 3.0, 0.0), (0.5, -0.26)])
def test_vacuum_is_static_bitwise(era_m, s):
    """P1: phi = psi = sigma with everything else zero is an exact fixed point."""
    m = O.model(6, 5, 4, eta_ref=10.0, sig=(1.0, 1.0))
    st = I.empty(6, 5, 4)
    st[I.PHI] = 1.0
    st[I.PSI] = 1.0
    ref = st.copy()
    O.run(m, st, 7, 1.0, era_m, s)
    assert np.array_equal(st, ref)


def test_pure_gauge_is_static():
    """P2: phi = sigma e^{i Lambda}, h A_i = Lambda(x+i) - Lambda(x) has D_i phi = 0 and
    zero plaquettes, so every force vanishes (covariant Laplacian, current, curl)."""
    nx, ny, nz = 7, 6, 5
    m = O.model(nx, ny, nz, eta_ref=5.0)
    lam_p = I.gauge_function(nx, ny, nz, 3)
    lam_q = I.gauge_function(nx, ny, nz, 4)
    st = I.empty(nx, ny, nz)
    for c, l, a in ((I.PHI, lam_p, I.A), (I.PSI, lam_q, I.B)):
        st[c] = np.cos(l)
        st[c + 1] = np.sin(l)
        for i, ax in enumerate((2, 1, 0)):
            st[a + i] = (np.roll(l, -1, axis=ax) - l) / m.h
    F = O.forces(m, st, 1.0)
    assert np.abs(F).max() < 1e-12
    O.run(m, st, 20, 1.0, 0.5, 1.0)
    assert np.abs(st[I.PI:I.PI + 4]).max() < 1e-12
    assert np.abs(st[I.E:I.E + 6]).max() < 1e-12


# --------------------------------------------------------------- P3


def test_plane_wave_is_exact_leapfrog_solution():
    """P3: with lambda = kappa = e = 0 and no expansion, phi = exp(i(q.x - Omega eta)) is an
    exact solution of the leapfrog when (2/k)^2 sin^2(Omega k/2) = sum_i (2/h)^2 sin^2(q_i h/2)."""
    nx, ny, nz = 8, 6, 5
    m = O.model(nx, ny, nz, lam=(0.0, 0.0), e=(0.0, 0.0), kappa=0.0)
    h, k = m.h, m.k
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    st = I.empty(nx, ny, nz)
    waves = []
    for c, pc, n in ((I.PHI, I.PI, (1, 2, 1)), (I.PSI, I.PSIDOT, (3, 0, 2))):
        q = [2 * np.pi * n[0] / (nx * h), 2 * np.pi * n[1] / (ny * h), 2 * np.pi * n[2] / (nz * h)]
        w2 = sum((2 / h) ** 2 * np.sin(qi * h / 2) ** 2 for qi in q)
        Om = 2 / k * np.arcsin(k * np.sqrt(w2) / 2)
        ph = (q[0] * x + q[1] * y + q[2] * z) * h
        f0 = np.exp(1j * ph)
        pim = f0 * (1 - np.exp(1j * Om * k)) / k     # Pi^{-1/2} = (phi^0 - phi^{-1}) / k
        st[c], st[c + 1] = f0.real, f0.imag
        st[pc], st[pc + 1] = pim.real, pim.imag
        waves.append((c, ph, Om))
    N = 60
    O.run(m, st, N, 1.0, 0.0, 1.0)
    for c, ph, Om in waves:
        exact = np.exp(1j * (ph - Om * N * k))
        assert np.abs(st[c] + 1j * st[c + 1] - exact).max() < 1e-11


# --------------------------------------------------------------- P4


@pytest.mark.parametrize("era_m,s", [(0.5, 1.0), (0.5, 0.0), (0.5, 0.5), (2.0 / 3.0, 0.0), (2.0 / 3.0, 1.0)])
def test_pure_hubble_damping_telescopes(era_m, s):
    """P4: with zero force, (1+delta)Pi' = (1-delta)Pi gives Pi_N = Pi_0 prod (1-delta_n)/(1+delta_n),
    delta_n = p k / eta_n (alpha = 2, a ~ eta^p, p = m/(1-m)).  For integer 2p the product
    telescopes: (eta - p k)/(eta + p k) = eta_{n-p}/eta_{n+p}.  E obeys the same with
    omega = (1 - s) delta, whose factor (1 - s)p must also telescope."""
    nx = 4
    m = O.model(nx, lam=(0.0, 0.0), kappa=0.0, eta_ref=3.0)
    k, eta0, N = m.k, 1.0, 37
    st = I.empty(nx, nx, nx)
    st[I.PHI] = 0.7                  # uniform scalar, no potential: zero scalar force
    st[I.PI] = 0.3
    st[I.PI + 1] = -0.2
    st[I.PSI] = 0.0                  # psi = 0: zero current in sector q
    st[I.H:I.H + 3] = np.array([0.4, -0.1, 0.25])[:, None, None, None]
    pi0 = st[I.PI:I.PI + 2, 0, 0, 0].copy()
    H0 = st[I.H:I.H + 3, 0, 0, 0].copy()
    O.run(m, st, N, eta0, era_m, s)

    def closed(c):
        # prod_{n<N} (eta_n - c k)/(eta_n + c k) = prod_{n<N} f(n - c)/f(n + c), f(t) = eta0 + t k,
        # telescopes for integer 2c to prod_{j<2c} f(j - c)/f(N - c + j)
        f = lambda t: eta0 + t * k
        assert abs(2 * c - round(2 * c)) < 1e-12
        out = 1.0
        for j in range(int(round(2 * c))):
            out *= f(j - c) / f(N - c + j)
        return out

    p = era_m / (1 - era_m)
    # continuum limit: the damped free field has d phi/d eta ~ a^{-2}, here between the
    # half-integer times eta_{-1/2} and eta_{N-1/2} of Pi
    cont = ((eta0 - k / 2) / (eta0 + (N - 0.5) * k)) ** (2 * p)
    assert closed(p) == pytest.approx(cont, rel=0.05)
    assert np.allclose(st[I.PI:I.PI + 2, 1, 2, 3], pi0 * closed(p), rtol=1e-13, atol=0)
    assert np.allclose(st[I.H:I.H + 3, 3, 0, 1], H0 * closed((1 - s) * p), rtol=1e-13, atol=0)
    assert np.all(st[I.PI:I.PI + 2] == st[I.PI:I.PI + 2, :1, :1, :1])   # stays uniform


def test_damping_above_one_follows_the_same_closed_form():
    """R26: the damped phase of Sec. V runs at m_damp = 0.95 from eta = 1, where
    delta = p k / eta with p = 19 exceeds 1 until eta = p k = 1.9.  The printed kick is
    applied as it stands: (1 - delta)/(1 + delta) is then negative (the free momentum flips
    sign every step while its magnitude still shrinks), it erases the momentum at
    eta = p k, and the telescoped product of P4 holds for any delta.  From eta = 1.05 the
    product's 38 factors have no zero: nine negative factors, so the sign is reversed."""
    nx = 4
    era_m = 0.95
    p = era_m / (1 - era_m)
    m = O.model(nx, lam=(0.0, 0.0), kappa=0.0, eta_ref=5.0)
    k = m.k

    def free_momentum(eta0, N):
        st = I.empty(nx, nx, nx)
        st[I.PHI] = 0.7
        st[I.PI] = 0.3
        st[I.PI + 1] = -0.2
        O.run(m, st, N, eta0, era_m, 0.0)
        return st[I.PI:I.PI + 2, 1, 2, 3] / np.array([0.3, -0.2])

    # the first step from eta = 1: (1 - 1.9)/(1 + 1.9)
    assert np.allclose(free_momentum(1.0, 1), -0.9 / 2.9, rtol=1e-14, atol=0)
    # the step from eta = 1.9 multiplies by (1.9 - p k)/(1.9 + p k) = 0 (to rounding of p)
    assert np.abs(free_momentum(1.0, 10)).max() < 1e-14
    # telescoped closed form from eta = 1.05 over N >= 2p steps
    eta0, N = 1.05, 41
    f = lambda t: eta0 + t * k
    closed = 1.0
    for j in range(int(round(2 * p))):
        closed *= f(j - p) / f(N - p + j)
    assert closed < 0
    assert np.allclose(free_momentum(eta0, N), closed, rtol=1e-11, atol=0)


# --------------------------------------------------------------- P5


def _energy_drift(k):
    nx = 8
    st = I.random_full(nx, nx, nx, 11, link=0.3, mom=0.3)
    m = O.model(nx, k=k)
    T = 3.0
    n = int(round(T / k))
    recs = O.run(m, st, n, 1.0, 0.0, 1.0, diag_every=1)
    e = np.array([r["sum_eps"] for r in recs])
    return np.abs(e - e[0]).max() / e[0]


def test_energy_conserved_to_order_k2():
    """P5: at a = 1 (m = 0) the leapfrog conserves the lattice energy to O(k^2): halving k
    divides the maximal deviation by ~4, with no secular drift."""
    d = [_energy_drift(k) for k in (0.1, 0.05, 0.025)]
    assert d[0] < 0.1
    for a, b in zip(d, d[1:]):
        assert 3.3 < a / b < 4.7, d


# --------------------------------------------------------------- P6


@pytest.mark.parametrize("era_m,s", [(0.0, 0.3), (2.0 / 3.0, 0.0), (0.5, 0.0), (0.5, 0.5), (0.5, 1.0)])
def test_gauss_law_exact(era_m, s):
    """P6: the discrete Gauss residual C = div E^{n+1/2} - g_n Im[phi^n* Pi^{n+1/2}],
    g_n = 2 e^2 a^{2s} (1+delta)/(1+omega), is zero to round-off for these schedules."""
    nx = 8
    m = O.model(nx, 7, 6, eta_ref=12.0, e=(1.0, 0.8), lam=(2.0, 1.28))
    st = I.random_phase(nx, 7, 6, 5)
    recs = O.run(m, st, 30, 1.0, era_m, s, diag_every=5)
    for r in recs:
        for a, b in zip(r["gauss_abs"], r["gauss_scale"]):
            assert b > 0
            assert a / b < 5e-14


def test_gauss_law_drift_when_not_exact():
    """P6 (converse): matter era with s = 1 is not exactly Gauss-preserving; the per-step
    defect is O((k/eta)^3) -- small, nonzero, and shrinking at later times."""
    nx = 8
    m = O.model(nx, eta_ref=40.0)
    st = I.random_phase(nx, nx, nx, 6)
    early = O.run(m, st, 20, 1.0, 2.0 / 3.0, 1.0, diag_every=19)
    rel_early = early[-1]["gauss_abs"][0] / early[-1]["gauss_scale"][0]
    assert 1e-9 < rel_early < 1e-2


# --------------------------------------------------------------- P7


def _fd(fun, x0, eps):
    # fourth-order central difference
    return (-fun(x0 + 2 * eps) + 8 * fun(x0 + eps) - 8 * fun(x0 - eps) + fun(x0 - 2 * eps)) / (12 * eps)


def test_forces_are_minus_energy_gradient_brute_force():
    """P7: on an 8^3 box every force equals the negative gradient of the lattice energy,
    by finite differences over all 5120 field degrees of freedom:
      F_phi = -(1/(2 h^3)) dH/dphi,   F_A = -(e^2/h^3) dH/dA."""
    nx = 8
    m = O.model(nx, e=(1.0, 0.7), lam=(2.0, 1.3), sig=(1.0, 0.8), kappa=0.45)
    st = I.random_full(nx, nx, nx, 21)
    F = O.forces(m, st, 1.0)
    h3 = m.h ** 3
    flat = st.reshape(20, -1)
    Ff = F.reshape(10, -1)
    comps = [(0, 0, 0.5), (1, 1, 0.5), (2, 2, 0.5), (3, 3, 0.5)]
    comps += [(8 + i, 4 + i, m.e[0] ** 2) for i in range(3)] + [(11 + i, 7 + i, m.e[1] ** 2) for i in range(3)]
    worst = 0.0
    for cs, cf, scale in comps:
        for s0 in range(flat.shape[1]):
            orig = flat[cs, s0]

            def Hof(v):
                flat[cs, s0] = v
                return O.hamiltonian(m, st)

            g = _fd(Hof, orig, 1e-3)
            flat[cs, s0] = orig
            worst = max(worst, abs(-scale * g / h3 - Ff[cf, s0]))
    assert worst < 2e-6, worst


def test_kick_and_drift_use_the_forces():
    """P7 (time stepping): at m = 0 one step is Pi += k F, E += k F_A, then phi += k Pi, A += k E."""
    nx = 5
    m = O.model(nx, 4, 6)
    st = I.random_full(nx, 4, 6, 2)
    F = O.forces(m, st, 1.0)
    ref = st.copy()
    ref[4:8] += m.k * F[0:4]
    ref[14:20] += m.k * F[4:10]
    ref[0:4] += m.k * ref[4:8]
    ref[8:14] += m.k * ref[14:20]
    O.step(m, st, 1.0, 0.0, 1.0)
    assert np.abs(st - ref).max() < 1e-13


# --------------------------------------------------------------- P8, P9, P10


def test_gauge_covariance():
    """P8: a random lattice gauge transform commutes with the evolution; energy, Lagrangian,
    velocity sums and Gauss residual are invariant and the windings are identical."""
    nx, ny, nz = 8, 7, 6
    m = O.model(nx, ny, nz, eta_ref=8.0)
    st = I.random_phase(nx, ny, nz, 9)
    O.run(m, st, 10, 1.0, 0.5, 1.0)           # develop links and momenta
    lp = I.gauge_function(nx, ny, nz, 31)
    lq = I.gauge_function(nx, ny, nz, 32)

    def transform(s):
        t = s.copy()
        for c, pc, a, l in ((I.PHI, I.PI, I.A, lp), (I.PSI, I.PSIDOT, I.B, lq)):
            for cc in (c, pc):
                z = (s[cc] + 1j * s[cc + 1]) * np.exp(1j * l)
                t[cc], t[cc + 1] = z.real, z.imag
            for i, ax in enumerate((2, 1, 0)):
                t[a + i] = s[a + i] + (np.roll(l, -1, axis=ax) - l) / m.h
        return t

    st2 = transform(st)
    assert np.array_equal(O.windings(m, st), O.windings(m, st2))
    r1 = O.run(m, st, 8, 2.0, 0.5, 1.0, j0=0, diag_every=4)
    r2 = O.run(m, st2, 8, 2.0, 0.5, 1.0, j0=0, diag_every=4)
    assert np.abs(transform(st) - st2).max() < 1e-10
    for a, b in zip(r1, r2):
        for key in ("sum_eps", "sum_lag", "sum_KL", "sum_GL", "sum_KV", "sum_GV"):
            assert abs(a[key] - b[key]) <= 1e-10 * (abs(a[key]) + 1.0)
        assert a["wind_abs"] == b["wind_abs"] and a["pq_count2"] == b["pq_count2"]
        assert np.allclose(a["gauss_abs"], b["gauss_abs"], atol=1e-12)


def _swap(st):
    t = st.copy()
    t[[0, 1, 2, 3]] = st[[2, 3, 0, 1]]
    t[[4, 5, 6, 7]] = st[[6, 7, 4, 5]]
    t[8:11], t[11:14] = st[11:14], st[8:11]
    t[14:17], t[17:20] = st[17:20], st[14:17]
    return t


def test_sector_exchange_symmetry_bitwise():
    """P9: exchanging phi<->psi, A<->B (and momenta) together with lambda_p<->lambda_q,
    e_p<->e_q, sigma_p<->sigma_q exchanges every output (Sec. II)."""
    nx, ny, nz = 6, 5, 7
    kw = dict(eta_ref=6.0, kappa=0.6)
    m1 = O.model(nx, ny, nz, lam=(2.0, 1.5), e=(1.0, 0.8), sig=(1.0, 0.9), **kw)
    m2 = O.model(nx, ny, nz, lam=(1.5, 2.0), e=(0.8, 1.0), sig=(0.9, 1.0), **kw)
    st = I.random_full(nx, ny, nz, 4)
    st2 = _swap(st)
    r1 = O.run(m1, st, 6, 1.0, 0.5, 1.0, diag_every=3)
    r2 = O.run(m2, st2, 6, 1.0, 0.5, 1.0, diag_every=3)
    assert np.array_equal(_swap(st), st2)
    for a, b in zip(r1, r2):
        assert a["gauss_abs"] == b["gauss_abs"][::-1]
        assert a["wind_abs"] == b["wind_abs"][::-1]
        assert a["pq_count2"] == b["pq_count2"]


def test_kappa_zero_decouples_sectors():
    """P10: with kappa = 0 the p sector evolves independently of the q sector."""
    nx = 6
    m = O.model(nx, kappa=0.0, eta_ref=5.0)
    s1 = I.random_full(nx, nx, nx, 7)
    s2 = s1.copy()
    other = I.random_full(nx, nx, nx, 8)
    for c in (2, 3, 6, 7) + tuple(range(11, 14)) + tuple(range(17, 20)):
        s2[c] = other[c]
    O.run(m, s1, 5, 1.0, 0.5, 1.0)
    O.run(m, s2, 5, 1.0, 0.5, 1.0)
    p_planes = [0, 1, 4, 5] + list(range(8, 11)) + list(range(14, 17))
    assert np.array_equal(s1[p_planes], s2[p_planes])
    # and kappa != 0 does couple them
    m.kappa = 0.9
    s3, s4 = I.random_full(nx, nx, nx, 7), s2.copy()
    s4[p_planes] = s3[p_planes]
    O.run(m, s3, 2, 1.0, 0.5, 1.0)
    O.run(m, s4, 2, 1.0, 0.5, 1.0)
    assert not np.array_equal(s3[p_planes], s4[p_planes])


# --------------------------------------------------------------- P11, P12: windings, cells, overlap


def _wrapped(d):
    return (d + np.pi) % (2 * np.pi) - np.pi


def _brute_windings_from_phase(theta):
    """W_z of a pure scalar phase field (A = 0) by walking each xy plaquette and summing
    wrapped phase differences of the angles themselves (no complex products)."""
    t00 = theta
    t10 = np.roll(theta, -1, axis=2)
    t11 = np.roll(np.roll(theta, -1, axis=2), -1, axis=1)
    t01 = np.roll(theta, -1, axis=1)
    loop = _wrapped(t10 - t00) + _wrapped(t11 - t10) + _wrapped(t01 - t11) + _wrapped(t00 - t01)
    return np.rint(loop / (2 * np.pi)).astype(np.int32)


def test_windings_match_brute_force_plaquette_walk():
    """P7 (windings): with A = 0 the gauge-invariant plaquette winding equals the naive
    walk around every xy plaquette of the phase angles; checked on random phases."""
    nx, ny, nz = 9, 8, 5
    m = O.model(nx, ny, nz)
    st = I.random_phase(nx, ny, nz, 12)
    W = O.windings(m, st)
    theta = np.arctan2(st[I.PHI + 1], st[I.PHI])
    assert np.array_equal(W[2], _brute_windings_from_phase(theta))
    # W_x is the (y,z) plaquette: transpose the axes so that (y, z) play (x, y)
    th_yz = np.transpose(theta, (2, 0, 1))          # (x, z, y): axis2 = y, axis1 = z
    assert np.array_equal(np.transpose(W[0], (2, 0, 1)), _brute_windings_from_phase(th_yz))
    assert np.abs(W).max() >= 1


def test_winding_flux_is_conserved_in_every_cell():
    """The windings through the six faces of every cell add to zero (strings do not end)."""
    nx, ny, nz = 8, 7, 6
    m = O.model(nx, ny, nz, eta_ref=5.0)
    st = I.random_phase(nx, ny, nz, 13)
    O.run(m, st, 5, 1.0, 0.5, 1.0)
    st[I.A:I.A + 6] += I.random_full(nx, ny, nz, 1, link=2.0)[I.A:I.A + 6]
    W = O.windings(m, st)
    for sec in range(2):
        Wx, Wy, Wz = W[3 * sec], W[3 * sec + 1], W[3 * sec + 2]
        div = (np.roll(Wx, -1, axis=2) - Wx) + (np.roll(Wy, -1, axis=1) - Wy) + (np.roll(Wz, -1, axis=0) - Wz)
        assert not div.any()


def test_straight_string_pair_winding_and_cells():
    """P11: a straight vortex-antivortex pair along z gives W_z = +1 and -1 at the two core
    plaquettes of every z-plane (sum |W| = 2 N_z), no other winding, and cell value 2 in
    the cells the strings thread (Sec. III.B: a straight string pierces two faces)."""
    nx, ny, nz = 16, 14, 6
    m = O.model(nx, ny, nz)
    st = I.string_pairs(nx, ny, nz, p_pair=(5, 10, 7))
    W = O.windings(m, st)
    assert not W[3:].any()
    Wz = W[2]
    assert (Wz[:, 7, 5] == 1).all() and (Wz[:, 7, 10] == -1).all()
    assert np.abs(W[:3]).sum() == 2 * nz
    n = O.cells(m, W)
    assert (n[0][:, 7, 5] == 2).all() and (n[0][:, 7, 10] == 2).all()
    assert n[0].sum() == 4 * nz and not n[1].any()
    # the same pair, gauge transformed with random links, keeps its windings
    lam = I.gauge_function(nx, ny, nz, 40)
    z = (st[0] + 1j * st[1]) * np.exp(1j * lam)
    st[0], st[1] = z.real, z.imag
    for i, ax in enumerate((2, 1, 0)):
        st[I.A + i] = (np.roll(lam, -1, axis=ax) - lam) / m.h
    assert np.array_equal(O.windings(m, st), W)


@pytest.mark.parametrize("dx,r,expect", [(0, 0, 1), (0, 1, 1), (1, 1, 1), (1, 0, 0), (2, 1, 0), (-1, 1, 1)])
def test_bound_state_overlap(dx, r, expect):
    """P12: coincident p and q string pairs overlap cell for cell (N_pq = 2 N_z, since both
    strings of the pair are bound, and L_p = L_q = 0); displaced by one cell they overlap
    only with the one-cell tolerance; displaced by two cells they do not (Sec. III.B)."""
    nx, ny, nz = 20, 14, 5
    m = O.model(nx, ny, nz, overlap_radius=r)
    st = I.string_pairs(nx, ny, nz, p_pair=(5, 12, 7), q_pair=(5 + dx, 12 + dx, 7))
    W = O.windings(m, st)
    n = O.cells(m, W)
    cp, cq = O.overlap(m, n)
    assert cp == cq == expect * 2 * nz
    # the record-level estimators of the same configuration
    rec = O.step(m, st.copy(), 1.0, 0.0, 1.0, diag=True)
    d = O.derive(m, rec)
    assert rec["pq_count2"] == cp + cq
    if expect:
        assert d["L_p"] == 0.0 and d["L_q"] == 0.0 and d["f_total"] == 1.0
    else:
        assert d["L_pq"] == 0.0 and d["L_p"] == m.h * 2 * nz


# --------------------------------------------------------------- R24 generator, Table 3


def test_initial_phases_follow_splitmix64_vectors():
    """R24: the oracle's random phases are SplitMix64 draws (published reference outputs
    from state 0), top 53 bits as a fraction of 2 pi; moduli are sigma."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.strip() and l[0] != "#"]
    m = O.model(3, 1, 1, sig=(1.0, 0.8))        # 3 sites: draws 0-2 are sector p
    st = O.init_random_phase(m, 0)
    for cnt, hexv in rows:
        r = int(hexv, 16)
        ph = 2 * math.pi * ((r >> 11) * 2.0 ** -53)
        s0 = int(cnt)
        assert st[0].ravel()[s0] == pytest.approx(math.cos(ph), abs=1e-15)
        assert st[1].ravel()[s0] == pytest.approx(math.sin(ph), abs=1e-15)
    assert np.allclose(np.hypot(st[2], st[3]), 0.8)
    assert not st[4:].any()


def test_scale_factor_normalisation_matches_table3():
    """R6: a = (eta/eta_ref)^p with a = 1 at the end of the run (eta_end = 1024) reproduces
    Table 3's maximum radius r_s,max = 1/a(eta_tr) of the physical runs (3.0 and 9.0),
    and the core-growth beta that grows the radius from 1 at eta = 5 to r_s,max."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table3_core_growth.txt")) if l.strip() and l[0] != "#"]
    for mm, _mdamp, beta_g, _beta, eta_tr, rmax in rows:
        mm, beta_g, eta_tr, rmax = float(mm), float(beta_g), float(eta_tr), float(rmax)
        m = O.model(4, eta_ref=1024.0)
        a_tr = O.coefficients(m, eta_tr, mm, 1.0)[0]
        assert 1.0 / a_tr == pytest.approx(rmax, rel=0.011)
        a_start = O.coefficients(m, 5.0, mm, 1.0)[0]
        # comoving radius ~ a^{-beta} under the coupling scaling of Sec. III
        beta_fit = -math.log(rmax) / math.log(a_tr / a_start)
        assert beta_fit == pytest.approx(beta_g, rel=2e-4)


# --------------------------------------------------------------- cells and overlap by brute force


def test_cells_match_face_enumeration_on_random_phases():
    """Cell values on a dense random network, against windings from the plaquette walk of
    the phase angles (all three orientations) summed explicitly over each cell's six faces."""
    nx, ny, nz = 9, 8, 7
    m = O.model(nx, ny, nz)
    st = I.random_phase(nx, ny, nz, 14)
    for sec, c in enumerate((I.PHI, I.PSI)):
        th = np.arctan2(st[c + 1], st[c])                       # (z, y, x)
        Wz = _brute_windings_from_phase(th)                     # xy faces
        Wx = np.transpose(_brute_windings_from_phase(np.transpose(th, (2, 0, 1))), (1, 2, 0))  # yz faces
        Wy = np.transpose(_brute_windings_from_phase(np.transpose(th, (1, 2, 0))), (2, 0, 1))  # zx faces
        brute = np.zeros((nz, ny, nx), dtype=np.int64)
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    faces = [Wx[z, y, x], Wx[z, y, (x + 1) % nx], Wy[z, y, x], Wy[z, (y + 1) % ny, x],
                             Wz[z, y, x], Wz[(z + 1) % nz, y, x]]
                    brute[z, y, x] = sum(abs(int(f)) for f in faces)
        W = O.windings(m, st)
        assert np.array_equal(W[3 * sec:3 * sec + 3], np.stack([Wx, Wy, Wz]))
        assert np.array_equal(O.cells(m, W)[sec], brute)


@pytest.mark.parametrize("r", [0, 1])
def test_overlap_matches_brute_force(r):
    """Overlap counts on random sparse cell arrays, against a direct scan of the
    (2r+1)^3 periodic neighbourhood of every cell."""
    nx, ny, nz = 7, 9, 6
    m = O.model(nx, ny, nz)
    rng = np.random.default_rng(5)
    n = (rng.random((2, nz, ny, nx)) < 0.08).astype(np.int32) * rng.integers(1, 5, size=(2, nz, ny, nx)).astype(np.int32)
    cnt = [0, 0]
    for sec in range(2):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    if n[sec, z, y, x] == 0:
                        continue
                    hit = any(n[1 - sec, (z + dz) % nz, (y + dy) % ny, (x + dx) % nx] > 0
                              for dz in range(-r, r + 1) for dy in range(-r, r + 1) for dx in range(-r, r + 1))
                    cnt[sec] += hit
    assert O.overlap(m, n, r) == tuple(cnt)
    assert cnt[0] > 0


# --------------------------------------------------------------- energy and Lagrangian weights


def _frozen_drift(k, a, s):
    nx = 8
    st = I.random_full(nx, nx, nx, 17, link=0.3, mom=0.3)
    m = O.model(nx, k=k)
    e = []
    for j in range(int(round(2.0 / k))):
        e.append(O.step_coeffs(m, st, 1.0 + j * k, a, 0.0, 0.0, s, diag=True)["sum_eps"])
    e = np.array(e)
    return np.abs(e - e[0]).max() / e[0]


@pytest.mark.parametrize("a,s", [(0.5, 1.0), (1.7, -0.26)])
def test_energy_conserved_at_frozen_expansion(a, s):
    """With the expansion frozen (delta = omega = 0, fixed a != 1) the equations of Sec. III
    conserve eps = K + G + a^{2s} V + a^{-2s} (Kg + Bg) to O(k^2): this pins the a-weights."""
    d = [_frozen_drift(k, a, s) for k in (0.05, 0.025)]
    assert d[0] < 0.05
    assert 3.3 < d[0] / d[1] < 4.7, d


def test_lagrangian_is_kinetic_minus_potential():
    """Lag = T - U and eps = T + U with the same weights: with no motion Lag = -eps,
    with no potential energy Lag = +eps (at a frozen a != 1)."""
    nx = 6
    m = O.model(nx, k=1e-7)
    a, s = 0.6, 1.0
    st = I.random_full(nx, nx, nx, 3)
    st[4:8] = 0.0
    st[14:20] = 0.0
    r = O.step_coeffs(m, st, 1.0, a, 0.0, 0.0, s, diag=True)
    assert r["sum_lag"] == pytest.approx(-r["sum_eps"], rel=1e-9)
    st = I.random_full(nx, nx, nx, 4)
    st[0], st[1], st[2], st[3] = 1.0, 0.0, 1.0, 0.0
    st[8:14] = 0.0
    r = O.step_coeffs(m, st, 1.0, a, 0.0, 0.0, s, diag=True)
    assert r["sum_lag"] == pytest.approx(r["sum_eps"], rel=1e-9)
    assert r["sum_eps"] > 0


def test_velocity_estimator_on_exact_plane_waves():
    """Velocity estimator R = sum K W / sum G W (Sec. III.A) in closed form: with lambda = 0 and
    a negligible gauge coupling, plane waves phi = r_p e^{i(q.x - Omega eta)} (and psi likewise)
    of constant modulus are exact leapfrog solutions with the uniform mass -kappa(r_q^2 - 1).
    Every weight is uniform, so R = sum_sigma r^2 sin^2(Omega k)/k^2 / sum_sigma r^2 w_q^2 with
    the time-centred momentum (Pi^{n-1/2} + Pi^{n+1/2})/2 and w_q^2 = sum_i (2/h)^2 sin^2(q_i h/2)."""
    nx, ny, nz = 8, 6, 5
    kap = 0.5
    m = O.model(nx, ny, nz, lam=(0.0, 0.0), e=(1e-8, 1e-8), kappa=kap)
    h, k = m.h, m.k
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    st = I.empty(nx, ny, nz)
    r = (0.8, 0.7)
    num = den = 0.0
    for sec, (c, pc, n) in enumerate(((I.PHI, I.PI, (1, 2, 1)), (I.PSI, I.PSIDOT, (3, 0, 2)))):
        q = [2 * np.pi * n[0] / (nx * h), 2 * np.pi * n[1] / (ny * h), 2 * np.pi * n[2] / (nz * h)]
        w2 = sum((2 / h) ** 2 * np.sin(qi * h / 2) ** 2 for qi in q)
        mass2 = -kap * (r[1 - sec] ** 2 - 1.0)
        Om = 2 / k * np.arcsin(k * np.sqrt(w2 + mass2) / 2)
        f0 = r[sec] * np.exp(1j * (q[0] * x + q[1] * y + q[2] * z) * h)
        pim = f0 * (1 - np.exp(1j * Om * k)) / k
        st[c], st[c + 1] = f0.real, f0.imag
        st[pc], st[pc + 1] = pim.real, pim.imag
        num += r[sec] ** 2 * np.sin(Om * k) ** 2 / k ** 2
        den += r[sec] ** 2 * w2
    R = num / den
    recs = O.run(m, st, 9, 1.0, 0.0, 1.0, diag_every=4)
    for rec in recs:
        d = O.derive(m, rec)
        assert rec["sum_KL"] / rec["sum_GL"] == pytest.approx(R, rel=1e-9)
        assert rec["sum_KV"] / rec["sum_GV"] == pytest.approx(R, rel=1e-9)
        assert d["v2_pq"] == pytest.approx(2 * R / (1 + R), rel=1e-9)


# --------------------------------------------------------------- P13 static string, P17 stability


def _relaxed_string_pair(scale):
    """A straight vortex / antivortex pair along z, 8 length units apart in a periodic box,
    relaxed by the gradient flow for 50 time units (kappa = 0, psi in its vacuum,
    lambda = 2 e^2: critical coupling).  The energy is then converged to ~1e-5 relative; the
    pair's residual attraction only moves it at the 1e-6 level."""
    h = 0.5 / scale
    nx, ny, nz = 32 * scale, 16 * scale, 2
    m = O.model(nx, ny, nz, h=h, k=0.1 / scale, kappa=0.0)
    st = I.string_pairs(nx, ny, nz, p_pair=(8 * scale - 1, 24 * scale - 1, 8 * scale - 1), core=2.0 * scale)
    O.cool(m, st, 1500 * scale ** 2, (1.0 / 30.0) / scale ** 2)
    return m, st, O.hamiltonian(m, st) / (2.0 * nz * h)


def test_static_string_tension_is_2_pi_sigma_squared():
    """P13: at critical coupling (lambda = 2 e^2, as in Sec. IV) a static string has
    tension 2 pi sigma^2.  The relaxed lattice pair's energy per unit length per string
    approaches it as O(h^2): the deficit shrinks about 4x when h halves.  A wrong factor in
    any term of the energy (gradient, magnetic, potential) moves it off the BPS value."""
    _, _, mu_coarse = _relaxed_string_pair(1)
    _, _, mu_fine = _relaxed_string_pair(2)
    d_coarse = 1.0 - mu_coarse / (2.0 * math.pi)
    d_fine = 1.0 - mu_fine / (2.0 * math.pi)
    assert 0.005 < d_coarse < 0.02, mu_coarse
    assert 0.0 < d_fine < 0.005, mu_fine
    assert 3.5 < d_coarse / d_fine < 4.7, (d_coarse, d_fine)


def test_static_string_stays_put_without_expansion():
    """P13: the relaxed pair is a static solution of the update at m = 0: over 10 time
    units the windings stay on the same plaquettes, the momenta grow no faster than the
    residual force of the relaxed state allows (|pi| <= 2 |F| t; a wrong term in the update
    would make the relaxed state far from a fixed point) and the energy is unchanged."""
    m, st, _ = _relaxed_string_pair(1)
    f0 = np.abs(O.forces(m, st)).max()
    assert f0 < 1e-3
    W0 = O.windings(m, st)
    e0 = O.hamiltonian(m, st)
    O.run(m, st, 100, 1.0, 0.0, 1.0)
    t = 100 * m.k
    assert np.array_equal(O.windings(m, st), W0)
    assert np.abs(st[I.PI:I.PI + 4]).max() < 2.0 * f0 * t
    assert np.abs(st[I.E:I.E + 6]).max() < 2.0 * f0 * t
    assert O.hamiltonian(m, st) == pytest.approx(e0, rel=1e-6)


@pytest.mark.parametrize("factor,stable", [(0.97, True), (1.03, False)])
def test_leapfrog_stability_threshold(factor, stable):
    """P17: the vacuum is stable while k^2 (12/h^2 + a^{2s} mu2_max) < 4, with mu2_max =
    lambda + 2 kappa the heavier eigenvalue of the vacuum mass matrix of Sec. II, and blows
    up just above it (the staggered mode of the heavier scalar combination)."""
    nx = 8
    m = O.model(nx)
    mu2 = 2.0 + 2.0 * 0.9
    a2s = factor * (4.0 / m.k ** 2 - 12.0 / m.h ** 2) / mu2
    st = I.empty(nx, nx, nx)
    st[I.PHI] = 1.0
    st[I.PSI] = 1.0
    st += np.random.default_rng(5).normal(0.0, 1e-6, size=st.shape)
    with np.errstate(all="ignore"):
        for j in range(200):
            O.step_coeffs(m, st, 10.0 + j * m.k, math.sqrt(a2s), 0.0, 0.0, 1.0)
        dev = np.abs(st[[I.PHI, I.PSI]] - 1.0).max()
    if stable:
        assert dev < 1e-4
    else:
        assert not np.isfinite(dev) or dev > 1.0


# --------------------------------------------------------------- diffusive cooling (Sec. III)


def test_cooling_is_a_descending_flow():
    """The cooling equations are the gradient flow of the static lattice energy (with kappa = 0):
    every forward-Euler step of small size lowers it, the vacuum is a fixed point, and the
    kappa coupling plays no part."""
    nx = 8
    m = O.model(nx, kappa=0.9)
    st = I.random_phase(nx, nx, nx, 21)
    st[I.A:I.A + 6] = I.random_full(nx, nx, nx, 22, link=0.3)[I.A:I.A + 6]
    m0 = O.model(nx, kappa=0.0)
    e = [O.hamiltonian(m0, st)]
    for _ in range(40):
        O.cool(m, st, 1, 1.0 / 30.0)
        e.append(O.hamiltonian(m0, st))
    assert all(b < a for a, b in zip(e, e[1:]))
    assert e[-1] < 0.5 * e[0]
    # kappa does not enter
    s1, s2 = I.random_full(6, 5, 4, 3), None
    s2 = s1.copy()
    O.cool(O.model(6, 5, 4, kappa=0.9), s1, 5)
    O.cool(O.model(6, 5, 4, kappa=0.0), s2, 5)
    assert np.array_equal(s1, s2)
    # momenta untouched, vacuum fixed
    assert np.array_equal(s1[4:8], I.random_full(6, 5, 4, 3)[4:8])
    vac = I.empty(5, 5, 5)
    vac[I.PHI] = vac[I.PSI] = 1.0
    ref = vac.copy()
    O.cool(O.model(5), vac, 10)
    assert np.array_equal(vac, ref)


def test_cooling_step_is_forward_euler_of_the_forces():
    """One cooling step moves phi and A by dt times the update's own forces at a = 1, kappa = 0."""
    m = O.model(6, 5, 7, kappa=0.0)
    st = I.random_full(6, 5, 7, 9)
    F = O.forces(m, st, 1.0)
    ref = st.copy()
    ref[0:4] += 0.03 * F[0:4]
    ref[8:14] += 0.03 * F[4:10]
    O.cool(O.model(6, 5, 7, kappa=0.4), st, 1, 0.03)
    assert np.abs(st - ref).max() < 1e-14


# --------------------------------------------------------------- robust-method segments


def _py_components(mark):
    """Brute force: union-find over every pair of marked cells within one cell
    (periodic Chebyshev distance <= 1), in plain Python."""
    nz, ny, nx = mark.shape
    cells = [tuple(c) for c in np.argwhere(mark)]
    idx = {c: i for i, c in enumerate(cells)}
    parent = list(range(len(cells)))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for (z, y, x), i in idx.items():
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    j = idx.get(((z + dz) % nz, (y + dy) % ny, (x + dx) % nx))
                    if j is not None:
                        ra, rb = find(i), find(j)
                        if ra != rb:
                            parent[ra] = rb
    sizes = {}
    for i in range(len(cells)):
        r = find(i)
        sizes[r] = sizes.get(r, 0) + 1
    return sorted(sizes.values(), reverse=True)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_segments_match_brute_force(seed):
    """Connected regions of pq cells on random sparse cell arrays, against a Python
    union-find over all neighbouring pairs (periodic, 26-neighbourhood)."""
    nx, ny, nz = 11, 9, 8
    m = O.model(nx, ny, nz)
    rng = np.random.default_rng(seed)
    n = (rng.random((2, nz, ny, nx)) < 0.12).astype(np.int32) * 2
    mark = np.zeros((nz, ny, nx), dtype=bool)
    for sec in range(2):
        other = n[1 - sec] > 0
        dil = np.zeros_like(other)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    dil |= np.roll(other, (dz, dy, dx), axis=(0, 1, 2))
        mark |= (n[sec] > 0) & dil
    got = O.segments(m, n)
    assert list(got) == _py_components(mark)
    assert got.sum() == mark.sum()


def test_segments_of_bound_string_pairs():
    """A bound straight pair (p and q strings coincident or one cell apart) gives one region
    per string, each threading the box (N_z cells); two cells apart there is none."""
    nx, ny, nz = 20, 14, 9
    m = O.model(nx, ny, nz)
    for dx, expect in ((0, [nz, nz]), (1, [2 * nz, 2 * nz]), (2, [])):
        st = I.string_pairs(nx, ny, nz, p_pair=(5, 12, 7), q_pair=(5 + dx, 12 + dx, 7))
        sizes = O.segments(m, O.cells(m, O.windings(m, st)))
        assert list(sizes) == expect, dx
    r = O.robust(m, [2 * nz, 2 * nz, 3], min_length=2.0)
    assert r["N_pq"] == 2 and r["L_pq"] == 2 * (2 * nz - 1) * 0.5
