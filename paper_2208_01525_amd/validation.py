"""Statistical validation runs of Sec. IV (Tables 1 and 2) on one GPU.

One run: random-phase initial conditions (seed), diffusive cooling from
eta = -10 to 1 (steps of 1/30), a damped phase from eta = 1 to 5 at the
expansion rate m_damp with constant comoving width (s = 0), then
constant-comoving-width evolution (s = 0, the validation's PRS choice) in
the radiation (m = 1/2) or matter (m = 2/3) era up to half a light-crossing
of the box, eta_end = N dx / 2 (256 at 1024^3, dx = 0.5).  Diagnostic
records every `diag_every` steps.

Asymptotic values, as in Tables 1 and 2: the mean over the records with
eta in [eta_lo, eta_end] of <v^2>_L and <v^2>_pq, and the least-squares
slopes d xi / d eta of xi_W, xi_p and xi_pq over the same records (fast
method for the pq lengths).

Command line (one JSON line per run, then one summary line per era):

    python -m paper_2208_01525_amd.validation --n 1024 --era 0.5 --seeds 1 2 3
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import mts as M


def asymptotic(records, eta_lo, eta_hi):
    """Means of the velocity estimators and slopes of the separations over the records
    whose eta lies in [eta_lo, eta_hi]."""
    sel = [r for r in records if eta_lo <= r["eta"] <= eta_hi]
    out = {"records": len(sel)}
    if not sel:
        return out
    eta = np.array([r["eta"] for r in sel])
    for key in ("v2_lag", "v2_pq", "f_total", "f_p"):
        v = np.array([r[key] for r in sel], dtype=np.float64)
        v = v[np.isfinite(v)]
        out[key] = float(v.mean()) if v.size else None
    for key in ("xi_W", "xi_p", "xi_q", "xi_pq", "xi_lag"):
        v = np.array([r[key] for r in sel], dtype=np.float64)
        ok = np.isfinite(v)
        out[key + "_dot"] = float(np.polyfit(eta[ok], v[ok], 1)[0]) if ok.sum() >= 2 else None
        out[key + "_end"] = float(v[ok][-1]) if ok.any() else None
    out["gauss_rel_max"] = float(max(max(r["gauss_rel"]) for r in sel))
    return out


def run(n, era_m, seed, m_damp=0.9, dx=0.5, dt=0.1, diag_every=10, eta_lo=230.0, eta_end=None,
        device="cuda:0", chunk=200, log=sys.stderr):
    """One validation run; returns (records, asymptotic values).  Progress lines go to
    `log` (None: silent)."""
    eta_end = eta_end if eta_end is not None else n * dx / 2.0
    params = M.make_params(n, eta_ref=eta_end, diag_every=diag_every, dx=dx, dt=dt)
    lat = M.Lattice(params, device=device)
    try:
        lat.autotune(2)
        lat.init_fields(seed)
        t0 = time.perf_counter()
        lat.cool(int(round(11.0 * 30.0)), 1.0 / 30.0)
        n_damp = int(round(4.0 / dt))
        lat.step(n_damp, 1.0, m_damp, 0.0)
        records = lat.diagnostics()
        n_evol = int(round((eta_end - 5.0) / dt))
        done = 0
        while done < n_evol:
            c = min(chunk, n_evol - done)
            lat.step(c, 5.0 + done * dt, era_m, 0.0)
            done += c
            records += lat.diagnostics()
            r = records[-1] if records else None
            if log is not None:
                print(f"seed {seed} m {era_m:.3f}: eta {5.0 + done * dt:.1f}, "
                      f"xi_W {r['xi_W'] if r else float('nan'):.2f}, {time.perf_counter() - t0:.0f} s",
                      file=log, flush=True)
    finally:
        lat.close()
    return records, asymptotic(records, eta_lo, eta_end)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--era", type=float, default=0.5)
    ap.add_argument("--m-damp", type=float, default=0.9)
    ap.add_argument("--seeds", type=int, nargs="+", default=[1])
    ap.add_argument("--eta-lo", type=float, default=230.0)
    ap.add_argument("--records", type=str, default=None, help="write every record as JSON lines here")
    a = ap.parse_args(argv)
    per_seed = []
    rec_file = open(a.records, "a") if a.records else None
    for seed in a.seeds:
        eta_lo = a.eta_lo if a.n == 1024 else a.eta_lo * a.n / 1024.0
        records, asym = run(a.n, a.era, seed, m_damp=a.m_damp, eta_lo=eta_lo)
        if rec_file:
            for r in records:
                rec_file.write(json.dumps({"n": a.n, "era": a.era, "seed": seed, **r}) + "\n")
            rec_file.flush()
        line = {"n": a.n, "era": a.era, "m_damp": a.m_damp, "seed": seed, **asym}
        print(json.dumps(line), flush=True)
        per_seed.append(asym)
    summary = {"n": a.n, "era": a.era, "seeds": len(per_seed)}
    for key in ("v2_lag", "v2_pq", "xi_W_dot", "xi_p_dot", "xi_pq_dot", "xi_lag_dot", "f_total"):
        v = np.array([s[key] for s in per_seed if s.get(key) is not None], dtype=np.float64)
        if v.size:
            summary[key] = [float(v.mean()), float(v.std(ddof=1)) if v.size > 1 else math.nan]
    print(json.dumps({"summary": summary}), flush=True)


if __name__ == "__main__":
    main()
