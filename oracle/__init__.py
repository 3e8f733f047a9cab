"""FP64 CPU oracle for the U(1)xU(1) multitension-string lattice update
(Correia & Martins, arXiv:2208.01525) -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP library:
the arithmetic lives in `oracle.c` (plain C, FP64, no blocking or fusion);
this module only marshals numpy arrays through ctypes and derives the
network estimators from the summed diagnostics.

State format: float64 array of shape (20, nz, ny, nx), x fastest; planes
  0-1 phi (re, im)   2-3 psi   4-5 Pi   6-7 Psi
  8-10 A_{x,y,z}     11-13 B   14-16 E  17-19 H
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Model(ctypes.Structure):
    """Lattice and couplings (Sec. II-III).  Sector 0 is p (phi, A), 1 is q (psi, B)."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("overlap_radius", ctypes.c_int32),
        ("h", ctypes.c_double), ("k", ctypes.c_double),
        ("lam", ctypes.c_double * 2), ("e", ctypes.c_double * 2), ("sig", ctypes.c_double * 2),
        ("kappa", ctypes.c_double), ("eta_ref", ctypes.c_double),
    ]

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def sites(self):
        return self.nx * self.ny * self.nz


class Diag(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_double), ("a", ctypes.c_double),
        ("sum_eps", ctypes.c_double), ("sum_lag", ctypes.c_double),
        ("sum_KL", ctypes.c_double), ("sum_GL", ctypes.c_double),
        ("sum_KV", ctypes.c_double), ("sum_GV", ctypes.c_double),
        ("gauss_abs", ctypes.c_double * 2), ("gauss_scale", ctypes.c_double * 2),
        ("wind_abs", ctypes.c_int64 * 2), ("pq_count2", ctypes.c_int64),
    ]

    def as_dict(self):
        return {
            "eta": self.eta, "a": self.a, "sum_eps": self.sum_eps, "sum_lag": self.sum_lag,
            "sum_KL": self.sum_KL, "sum_GL": self.sum_GL, "sum_KV": self.sum_KV, "sum_GV": self.sum_GV,
            "gauss_abs": tuple(self.gauss_abs), "gauss_scale": tuple(self.gauss_scale),
            "wind_abs": tuple(self.wind_abs), "pq_count2": self.pq_count2,
        }


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        mp = ctypes.POINTER(Model)
        L.orc_forces.argtypes = [mp, dp, ctypes.c_double, dp]
        L.orc_hamiltonian.argtypes = [mp, dp]
        L.orc_hamiltonian.restype = ctypes.c_double
        L.orc_windings.argtypes = [mp, dp, ip]
        L.orc_cells.argtypes = [mp, ip, ip]
        L.orc_overlap.argtypes = [mp, ip, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.orc_init_random_phase.argtypes = [mp, ctypes.c_uint64, dp]
        L.orc_coefficients.argtypes = [mp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_step.argtypes = [mp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Diag)]
        L.orc_step_coeffs.argtypes = [mp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(Diag)]
        L.orc_segments.argtypes = [mp, ip, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]
        L.orc_segments.restype = ctypes.c_int64
        L.orc_cool.argtypes = [mp, dp, ctypes.c_int, ctypes.c_double]
        L.orc_run.argtypes = [mp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int64, ctypes.c_int, ctypes.POINTER(Diag), ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


def model(nx, ny=None, nz=None, *, h=0.5, k=0.1, lam=(2.0, 2.0), e=(1.0, 1.0), sig=(1.0, 1.0),
          kappa=0.9, eta_ref=1.0, overlap_radius=1):
    """Defaults are the paper's production couplings (Sec. IV): lambda = 2, e = 1,
    sigma = 1, kappa = 0.9, dx = 0.5, d eta = 0.1."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    m = Model()
    m.nx, m.ny, m.nz, m.overlap_radius = nx, ny, nz, overlap_radius
    m.h, m.k, m.kappa, m.eta_ref = h, k, kappa, eta_ref
    m.lam[:] = lam
    m.e[:] = e
    m.sig[:] = sig
    return m


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def zeros(m):
    return np.zeros((20,) + m.shape, dtype=np.float64)


def init_random_phase(m, seed):
    st = zeros(m)
    lib().orc_init_random_phase(ctypes.byref(m), ctypes.c_uint64(seed), _dp(st))
    return st


def forces(m, st, An=1.0):
    F = np.zeros((10,) + m.shape, dtype=np.float64)
    lib().orc_forces(ctypes.byref(m), _dp(st), An, _dp(F))
    return F


def hamiltonian(m, st):
    return lib().orc_hamiltonian(ctypes.byref(m), _dp(st))


def coefficients(m, eta, era_m, s):
    """(a, delta, omega, a^{2s}) of the step from eta (Sec. III)."""
    out = np.zeros(4)
    lib().orc_coefficients(ctypes.byref(m), eta, era_m, s, _dp(out))
    return tuple(out)


def step(m, st, eta, era_m, s, diag=False):
    """One leapfrog step in place; returns the integer-time record if asked."""
    d = Diag() if diag else None
    lib().orc_step(ctypes.byref(m), _dp(st), eta, era_m, s, ctypes.byref(d) if diag else None)
    return d.as_dict() if diag else None


def step_coeffs(m, st, eta, a, delta, omega, s, diag=False):
    """One step with explicit scale factor and damping (An = a^{2s})."""
    d = Diag() if diag else None
    lib().orc_step_coeffs(ctypes.byref(m), _dp(st), eta, a, delta, omega, s, ctypes.byref(d) if diag else None)
    return d.as_dict() if diag else None


def run(m, st, n, eta0, era_m, s, j0=0, diag_every=0):
    """n steps from eta0 (eta_j = eta0 + j k); records for (j0 + j) % diag_every == 0."""
    cap = (n // diag_every + 2) if diag_every > 0 else 1
    recs = (Diag * cap)()
    nd = lib().orc_run(ctypes.byref(m), _dp(st), n, eta0, era_m, s, j0, diag_every, recs, cap)
    return [recs[i].as_dict() for i in range(nd)]


def cool(m, st, n, dt=1.0 / 30.0):
    """n forward-Euler steps of the diffusive cooling flow (Sec. III), in place."""
    lib().orc_cool(ctypes.byref(m), _dp(st), n, dt)


def windings(m, st):
    """Signed plaquette windings, int32 (6, nz, ny, nx): p (W_x, W_y, W_z), q (...)."""
    W = np.zeros((6,) + m.shape, dtype=np.int32)
    lib().orc_windings(ctypes.byref(m), _dp(st), _ip(W))
    return W


def cells(m, W):
    """Cell values (total |W| through the six faces), int32 (2, nz, ny, nx)."""
    W = np.ascontiguousarray(W, dtype=np.int32)
    n = np.zeros((2,) + m.shape, dtype=np.int32)
    lib().orc_cells(ctypes.byref(m), _ip(W), _ip(n))
    return n


def overlap(m, n, radius=None):
    """(count_p, count_q) of the fast-method overlap (Sec. III.B)."""
    radius = m.overlap_radius if radius is None else radius
    n = np.ascontiguousarray(n, dtype=np.int32)
    cp, cq = ctypes.c_int64(), ctypes.c_int64()
    lib().orc_overlap(ctypes.byref(m), _ip(n), radius, ctypes.byref(cp), ctypes.byref(cq))
    return cp.value, cq.value


def segments(m, n, radius=None):
    """Sizes (cells) of the connected regions of fast-method pq cells (Sec. III.B robust
    method), sorted in decreasing order."""
    radius = m.overlap_radius if radius is None else radius
    n = np.ascontiguousarray(n, dtype=np.int32)
    cap = m.sites
    sizes = np.zeros(cap, dtype=np.int64)
    k = lib().orc_segments(ctypes.byref(m), _ip(n), radius, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap)
    assert k >= 0
    return np.sort(sizes[:k])[::-1]


def robust(m, sizes, min_length):
    """Robust-method estimators (Sec. III.B, V.B): segments are regions with
    (N_cells - 1) h > min_length; L_pq = sum (N_cells - 1) h, N_pq their number,
    l_pq = L_pq / N_pq, xi_pq = sqrt(V / L_pq)."""
    L = [(s - 1) * m.h for s in sizes if (s - 1) * m.h > min_length]
    Lpq = float(sum(L))
    V = m.sites * m.h ** 3
    return {"N_pq": len(L), "L_pq": Lpq, "l_pq": Lpq / len(L) if L else float("nan"),
            "xi_pq": math.sqrt(V / Lpq) if Lpq > 0 else float("inf")}


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """Threads the oracle uses from now on (results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def derive(m, rec, mu=None):
    """Network estimators from one record (Sec. III.A):
      L_pq = h N_pq,  L_p = h sum|W_p| - L_pq,  L_q likewise
      xi_X = sqrt(V / L_X),  xi_W = sqrt(V / (L_p + L_q + L_pq))
      xi_Lag = sqrt(-mu V / (h^3 sum Lag)) with mu the tension of a basic string:
        2 pi sigma_p^2 for a p-string at critical coupling (Sec. IV) unless given
      f_total = L_pq / (L_pq + L_p + L_q),  f_p = L_pq / L_p
      <v^2> = 2R / (1 + R), R = sum K W / sum G W with W = Lag or Vint.
    A ratio with a zero denominator is reported as nan."""
    h = m.h
    V = m.sites * h ** 3
    if mu is None:
        mu = 2.0 * math.pi * m.sig[0] ** 2

    def ratio(a, b):
        return a / b if b != 0 else float("nan")

    L_pq = h * rec["pq_count2"] / 2.0
    L_p = h * rec["wind_abs"][0] - L_pq
    L_q = h * rec["wind_abs"][1] - L_pq

    def xi(L):
        return math.sqrt(V / L) if L > 0 else float("inf")

    R_L = ratio(rec["sum_KL"], rec["sum_GL"])
    R_pq = ratio(rec["sum_KV"], rec["sum_GV"])
    return {
        "L_p": L_p, "L_q": L_q, "L_pq": L_pq,
        "xi_p": xi(L_p), "xi_q": xi(L_q), "xi_pq": xi(L_pq), "xi_W": xi(L_p + L_q + L_pq),
        "xi_lag": math.sqrt(-mu * V / rec["sum_lag"]) if rec["sum_lag"] < 0 else float("nan"),
        "f_total": ratio(L_pq, L_pq + L_p + L_q), "f_p": ratio(L_pq, L_p),
        "v2_lag": 2 * R_L / (1 + R_L), "v2_pq": 2 * R_pq / (1 + R_pq),
        "gauss_rel": tuple(ratio(a, b) if b != 0 else 0.0 for a, b in zip(rec["gauss_abs"], rec["gauss_scale"])),
    }
