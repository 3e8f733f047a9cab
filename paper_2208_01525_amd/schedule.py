"""Run schedules of the paper's simulations (Sec. III and Sec. V), host side.

* core_growth_beta: the beta < 0 that grows the comoving string radius
  r_s ~ a^{-beta} (couplings scaled as a^{-2(1-beta)}, Sec. III) from 1 at
  eta_start to r_max at eta_tr, with a ~ eta^p, p = m/(1-m) (Sec. V, Table 3).
* max_radius: the radius a physical (beta = 1) string has at eta_tr when
  a = 1 at eta_end (Table 3's r_s,max).
* run_paper_protocol: cooling (eta -10 -> 1, d eta = 1/30), the damped phase
  (eta 1 -> 5 at era m_damp, beta = 0), then either core growth up to eta_tr
  followed by physical evolution, or constant comoving width throughout.
"""
import math


def era_power(era_m):
    return era_m / (1.0 - era_m)


def core_growth_beta(r_max, era_m, eta_start, eta_tr):
    return -math.log(r_max) / (era_power(era_m) * math.log(eta_tr / eta_start))


def max_radius(era_m, eta_tr, eta_end):
    return (eta_end / eta_tr) ** era_power(era_m)


def run_paper_protocol(lat, era_m, m_damp, eta_end, physical=True, eta_tr=None, r_max=None,
                       dt=0.1, cool_from=-10.0, damp_until=5.0):
    """Drive a Lattice (or anything with cool/step) through the paper's schedule.
    The lattice's eta_ref must be eta_end.  Returns the (eta, s) segments run."""
    n_cool = int(round((1.0 - cool_from) * 30))
    lat.cool(n_cool, 1.0 / 30.0)
    segments = []
    n_damp = int(round((damp_until - 1.0) / dt))
    lat.step(n_damp, 1.0, m_damp, 0.0)
    segments.append((1.0, damp_until, m_damp, 0.0))
    eta = damp_until
    if physical:
        eta_tr = eta_tr if eta_tr is not None else 0.5 * (eta + eta_end)
        r_max = r_max if r_max is not None else max_radius(era_m, eta_tr, eta_end)
        beta_g = core_growth_beta(r_max, era_m, eta, eta_tr)
        n_g = int(round((eta_tr - eta) / dt))
        lat.step(n_g, eta, era_m, beta_g)
        segments.append((eta, eta_tr, era_m, beta_g))
        eta = eta + n_g * dt
        n_p = int(round((eta_end - eta) / dt))
        lat.step(n_p, eta, era_m, 1.0)
        segments.append((eta, eta_end, era_m, 1.0))
    else:
        n_p = int(round((eta_end - eta) / dt))
        lat.step(n_p, eta, era_m, 0.0)
        segments.append((eta, eta_end, era_m, 0.0))
    return segments
