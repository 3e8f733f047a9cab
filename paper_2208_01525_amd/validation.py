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

    python -m paper_2208_01525_amd.validation --n 1024 --era 0.5 --seeds 1 2 3 --records runs.jsonl

--records appends the records of each run's averaging window as JSON lines;
--summarize recomputes the per-seed values and the table of means and
standard deviations from such files alone (no GPU):

    python -m paper_2208_01525_amd.validation --summarize runs.jsonl

The table also gives the separation slopes under the other reading of the
string length (a Manhattan-length correction of 2/3 on L, which scales every
xi and its slope by sqrt(3/2)), labelled as that reading.
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
        device="cuda:0", chunk=200, log=sys.stderr, tune_cache=None):
    """One validation run; returns (records, asymptotic values).  Progress lines go to
    `log` (None: silent)."""
    eta_end = eta_end if eta_end is not None else n * dx / 2.0
    params = M.make_params(n, eta_ref=eta_end, diag_every=diag_every, dx=dx, dt=dt)
    lat = M.Lattice(params, device=device)
    try:
        lat.autotune(2, cache=tune_cache)
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


SUMMARY_KEYS = ("v2_lag", "v2_pq", "xi_W_dot", "xi_p_dot", "xi_pq_dot", "xi_lag_dot", "f_total", "f_p")
MANHATTAN = math.sqrt(1.5)   # xi under L -> (2/3) L
WINDING_SLOPES = ("xi_W_dot", "xi_p_dot", "xi_q_dot", "xi_pq_dot")


def summarize(per_seed):
    """Mean and sample standard deviation over seeds of each asymptotic value."""
    out = {"seeds": len(per_seed)}
    for key in SUMMARY_KEYS:
        v = np.array([s[key] for s in per_seed if s.get(key) is not None], dtype=np.float64)
        if v.size:
            out[key] = [float(v.mean()), float(v.std(ddof=1)) if v.size > 1 else math.nan]
    return out


def summarize_files(paths, eta_lo=230.0):
    """Per-seed asymptotic values and the per-(n, era) summary from record files."""
    runs = {}
    for path in paths:
        with open(path) as f:
            for line in f:
                r = json.loads(line)
                runs.setdefault((r["n"], r["era"], r["seed"]), []).append(r)
    groups = {}
    for (n, era, seed), recs in sorted(runs.items()):
        recs.sort(key=lambda r: r["eta"])
        lo = eta_lo if n == 1024 else eta_lo * n / 1024.0
        asym = asymptotic(recs, lo, recs[-1]["eta"])
        groups.setdefault((n, era), []).append({"seed": seed, **asym})
    return groups


def table(groups):
    """Markdown rows: era, quantity, mean +- std (and the sqrt(3/2) reading of the slopes)."""
    rows = ["| n | era | quantity | mean ± std over seeds | with L → (2/3) L |", "|---|---|---|---|---|"]
    for (n, era), per_seed in sorted(groups.items()):
        sm = summarize(per_seed)
        name = "radiation" if abs(era - 0.5) < 1e-9 else ("matter" if abs(era - 2.0 / 3.0) < 1e-6 else f"m={era}")
        for key in SUMMARY_KEYS:
            if key not in sm:
                continue
            m, sd = sm[key]
            # the reading changes only the separations taken from the winding length (xi_L comes
            # from the Lagrangian and the tension, not from a counted length)
            alt = f"{m * MANHATTAN:.4g} ± {sd * MANHATTAN:.2g}" if key in WINDING_SLOPES else ""
            rows.append(f"| {n} | {name} ({sm['seeds']} seeds) | {key} | {m:.4g} ± {sd:.2g} | {alt} |")
    return "\n".join(rows)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--era", type=float, default=0.5)
    ap.add_argument("--m-damp", type=float, default=0.9)
    ap.add_argument("--seeds", type=int, nargs="+", default=[1])
    ap.add_argument("--eta-lo", type=float, default=230.0)
    ap.add_argument("--records", type=str, default=None,
                    help="append the records of each run's averaging window here (JSON lines)")
    ap.add_argument("--autotune-cache", type=str, default=None,
                    help="file of stored autotuner choices (mts_autotune_cached)")
    ap.add_argument("--summarize", type=str, nargs="+", default=None,
                    help="record files to summarise (no runs)")
    a = ap.parse_args(argv)
    if a.summarize:
        groups = summarize_files(a.summarize, a.eta_lo)
        for (n, era), per_seed in sorted(groups.items()):
            for ps in per_seed:
                print(json.dumps({"n": n, "era": era, **ps}), flush=True)
            print(json.dumps({"summary": {"n": n, "era": era, **summarize(per_seed)}}), flush=True)
        print(table(groups), flush=True)
        return
    per_seed = []
    rec_file = open(a.records, "a") if a.records else None
    for seed in a.seeds:
        eta_lo = a.eta_lo if a.n == 1024 else a.eta_lo * a.n / 1024.0
        records, asym = run(a.n, a.era, seed, m_damp=a.m_damp, eta_lo=eta_lo, tune_cache=a.autotune_cache)
        if rec_file:
            for r in records:
                if r["eta"] >= eta_lo:
                    rec_file.write(json.dumps({"n": a.n, "era": a.era, "m_damp": a.m_damp, "seed": seed, **r}) + "\n")
            rec_file.flush()
        line = {"n": a.n, "era": a.era, "m_damp": a.m_damp, "seed": seed, **asym}
        print(json.dumps(line), flush=True)
        per_seed.append(asym)
    print(json.dumps({"summary": {"n": a.n, "era": a.era, **summarize(per_seed)}}), flush=True)


if __name__ == "__main__":
    main()
