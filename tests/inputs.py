"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds none of the method's arithmetic: only random numbers and analytic
test configurations, returned in the host field exchange format
(float64 array of shape (20, nz, ny, nx), x fastest; planes
0-1 phi, 2-3 psi, 4-5 Pi, 6-7 Psi, 8-10 A, 11-13 B, 14-16 E, 17-19 H).
"""
import numpy as np

PHI, PSI, PI, PSIDOT = 0, 2, 4, 6
A, B, E, H = 8, 11, 14, 17


def empty(nx, ny, nz):
    return np.zeros((20, nz, ny, nx), dtype=np.float64)


def random_phase(nx, ny, nz, seed, sig=(1.0, 1.0)):
    """The paper's initial condition (Sec. III): |phi| = sig_p, |psi| = sig_q with
    iid uniform phases; momenta, links and electric fields zero."""
    rng = np.random.default_rng(seed)
    st = empty(nx, ny, nz)
    for sec, c in enumerate((PHI, PSI)):
        th = rng.uniform(0.0, 2.0 * np.pi, size=(nz, ny, nx))
        st[c] = sig[sec] * np.cos(th)
        st[c + 1] = sig[sec] * np.sin(th)
    return st


def random_full(nx, ny, nz, seed, amp=1.0, link=0.6, mom=0.5):
    """Every one of the 20 components random: scalar moduli in [0.2, 1.4) with random
    phases, links ~ N(0, link), momenta and electric fields ~ N(0, mom)."""
    rng = np.random.default_rng(seed)
    st = empty(nx, ny, nz)
    shp = (nz, ny, nx)
    for c in (PHI, PSI):
        r = amp * rng.uniform(0.2, 1.4, size=shp)
        th = rng.uniform(0.0, 2.0 * np.pi, size=shp)
        st[c] = r * np.cos(th)
        st[c + 1] = r * np.sin(th)
    for c in (PI, PSIDOT):
        st[c:c + 2] = rng.normal(0.0, mom, size=(2,) + shp)
    st[A:A + 6] = rng.normal(0.0, link, size=(6,) + shp)
    st[E:E + 6] = rng.normal(0.0, mom, size=(6,) + shp)
    return st


def gauge_function(nx, ny, nz, seed):
    """iid uniform Lambda(x) in [0, 2 pi) for a random lattice gauge transform."""
    return np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi, size=(nz, ny, nx))


def pair_phase(nx, ny, x1, x2, yc):
    """Phase (ny, nx) of a vortex at (x1 + 1/2, yc + 1/2) and an antivortex at
    (x2 + 1/2, yc + 1/2) in lattice units: the difference of the two polar
    angles, which decays away from the pair."""
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    a1 = np.arctan2(y - (yc + 0.5), x - (x1 + 0.5))
    a2 = np.arctan2(y - (yc + 0.5), x - (x2 + 0.5))
    return a1 - a2


def string_pairs(nx, ny, nz, p_pair=None, q_pair=None, core=0.0):
    """Straight strings along z: for each sector, an optional (x1, x2, yc) vortex /
    antivortex pair; the modulus is 1 (or tanh(r / core) if core > 0).  Sectors
    without a pair sit in the vacuum phi = 1.  Links and momenta zero."""
    st = empty(nx, ny, nz)
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    for c, pair in ((PHI, p_pair), (PSI, q_pair)):
        if pair is None:
            st[c] = 1.0
            continue
        x1, x2, yc = pair
        th = pair_phase(nx, ny, x1, x2, yc)
        mod = np.ones((ny, nx))
        if core > 0:
            r1 = np.hypot(x - (x1 + 0.5), y - (yc + 0.5))
            r2 = np.hypot(x - (x2 + 0.5), y - (yc + 0.5))
            mod = np.tanh(r1 / core) * np.tanh(r2 / core)
        st[c] = (mod * np.cos(th))[None]
        st[c + 1] = (mod * np.sin(th))[None]
    return st


def to_f32_values(st):
    """Round every component to the nearest float32 (the values an FP32 lattice holds)."""
    return st.astype(np.float32).astype(np.float64)


def string_set(nx, ny, nz, p_vortices=(), q_vortices=(), sig=(1.0, 1.0)):
    """Straight strings along z: each sector gets the vortices in its list of
    (xc, yc, w), a vortex of winding w at (xc + 1/2, yc + 1/2) in lattice units;
    the phase is the sum of w times the polar angle about each, the modulus sig.
    Windings that add up to zero keep the phase smooth across the periodic
    boundary.  A sector with no vortex sits in its vacuum.  Links and momenta zero."""
    st = empty(nx, ny, nz)
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    for sec, (c, vort) in enumerate(((PHI, p_vortices), (PSI, q_vortices))):
        th = np.zeros((ny, nx))
        for xc, yc, w in vort:
            th += w * np.arctan2(y - (yc + 0.5), x - (xc + 0.5))
        st[c] = (sig[sec] * np.cos(th))[None]
        st[c + 1] = (sig[sec] * np.sin(th))[None]
    return st


def ring(nx, ny, nz, radius, center=None):
    """One closed string in the p sector: a circle of the given radius (lattice units) in
    the plane z = cz about (cx, cy); the phase at a point is the polar angle of (rho - R,
    z - cz) in the half-plane through the ring's axis (rho its distance from the axis),
    so it winds once around the core; modulus 1.  The default centre lies at half-integer
    coordinates so the circle meets no lattice line at a lattice site.  The q sector sits
    in its vacuum; links and momenta zero."""
    cx, cy, cz = center if center is not None else (nx / 2.0 - 0.5, ny / 2.0 - 0.5, nz / 2.0 - 0.5)
    st = empty(nx, ny, nz)
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    rho = np.hypot(x - cx, y - cy)
    th = np.arctan2(z - cz, rho - radius)
    st[PHI], st[PHI + 1] = np.cos(th), np.sin(th)
    st[PSI] = 1.0
    return st
