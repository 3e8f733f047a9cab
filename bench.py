"""Benchmark of the U(1)xU(1) lattice update on one MI355X.

Workload (one step = one leapfrog step of the whole box, both sectors, with
the fused diagnostics every 10th step): 512^3 periodic box, dx = 0.5,
dt = 0.1, radiation era (m = 1/2), s = 1, lambda = 2, e = 1, sigma = 1,
kappa = 0.9, seeded random-phase initial conditions, FP32 fields with FP64
reductions, a = 1 at eta = 128.  Warm-up steps run from eta = 1; the timed
steps continue the same run (the default 10 + 1260 steps reach eta = 128).

Printed: one JSON line with site-updates/s (`value`: whole steps, the
diagnostic steps included; `pure_step_value`: from the update kernel's time
alone), the HBM roofline of the update kernel (timed with HIP events around
each launch on the library's stream; `box_ceiling`: this box's rate for a
plain copy and for the update's access pattern without its stencil,
measured by the library's bandwidth probe), an FP64 leg of the same box,
the batched ensemble, and the FP64 CPU oracle timed on a bounded sample of
the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "site-updates/s & % HBM roofline, FP32 vs FP64, 512^3 box and batched ensemble"
HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE = {"fp32": 160, "fp64": 320}   # 20 reals read + 20 written per site-update


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_tile_512.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2208_01525_amd", "csrc", f)
                  for f in ("step_tile.hip", "site.h", "device.h", "kernels.h")]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(n, precision, tile, nt, pf, pp=False, xcd=True):
    """HBM bytes per launch of the update kernel from the committed rocprofv3
    counter summary, if it was taken on this kernel source, tile shape, store
    mode, load pipeline, momentum mode, tile order and workload; else None.
    Returns (bytes, source description) or (None, reason)."""
    rel = os.path.relpath(TRAFFIC_FILE, ROOT)
    if n != 512 or precision != "fp32" or not os.path.exists(TRAFFIC_FILE):
        return None, f"no counter file for {n}^3 {precision}"
    lines = [l.strip() for l in open(TRAFFIC_FILE) if l.strip() and not l.startswith("#")]
    head = dict(l.split("=", 1) for l in lines if " " not in l and "=" in l)
    src = kernel_source_hash()
    if head.get("source_sha256") != src:
        return None, f"{rel} was taken on kernel source {head.get('source_sha256', '?')[:16]}, not {src[:16]}"
    want = f"{tile[0]},{tile[1]},{int(nt)},{int(pf)},{int(pp)},{int(xcd)}"
    for l in lines:
        kv = dict(f.split("=", 1) for f in l.split() if "=" in f)
        if kv.get("config") == want:
            return int(kv["bytes_per_launch"]), f"{rel} (rocprofv3 FETCH_SIZE + WRITE_SIZE, config {want}, " \
                                                 f"kernel source sha256 {src[:16]})"
    return None, f"{rel} has no pass for config {want}"


def run_box(P, torch, n, precision, warmup, steps, diag_every, eta0=1.0, era_m=0.5, s=1.0, eta_ref=128.0, seed=1,
            tile=None, time_blocking=None, tune_cache=None):
    params = P.make_params(n, precision=precision, eta_ref=eta_ref, diag_every=diag_every)
    lat = P.Lattice(params, device="cuda:0")
    tuned = None
    if tile is not None:
        lat.set_tile(*tile[:2])
        if len(tile) > 2:
            lat.set_streaming_stores(bool(tile[2]))
        if len(tile) > 3:
            lat.set_prefetch(bool(tile[3]))
        if len(tile) > 4:
            lat.set_momentum_pingpong(bool(tile[4]))
        if len(tile) > 5:
            lat.set_tile_order(bool(tile[5]))
    else:
        tuned = lat.autotune(4, cache=tune_cache)   # times every tile shape on this machine (unless cached)
    if time_blocking is not None:
        lat.set_time_blocking(*time_blocking)
    ceiling = lat.bandwidth_probe(5)  # this box's copy rate and the update pattern's rate (overwrites)
    lat.init_fields(seed)
    lat.step(warmup, eta0, era_m, s)
    lat.diagnostics()
    torch.cuda.synchronize()
    lat.timing_read()
    lat.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps, eta0 + warmup * params.dt, era_m, s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = lat.timing_read()
    recs = lat.diagnostics()
    lat.timing_enable(False)
    sites = n ** 3
    wall = t1 - t0
    # the dominant update kernel: one step per launch, or two with time blocking
    tblock = lat.get_time_blocking()
    if tm["ms_pair"] > tm["ms_plain"]:
        launch_ms, per_launch, kname = tm["ms_pair"] / tm["n_pair"], 2, "step_pair_kernel"
    else:
        launch_ms, per_launch, kname = tm["ms_plain"] / max(tm["n_plain"], 1), 1, "step_tile_kernel"
    kern_ms = launch_ms / per_launch
    achieved = BYTES_PER_SITE[precision] * sites * per_launch / (launch_ms * 1e-3) / 1e9
    traffic, traffic_src = (measured_traffic(n, precision, lat.get_tile(), lat.get_streaming_stores(),
                                             lat.get_prefetch(), lat.get_momentum_pingpong(), lat.get_tile_order())
                            if per_launch == 1 else (None, "no counter pass for the two-step kernel"))
    eta_first = eta0 + warmup * params.dt
    eta_last = eta0 + (warmup + steps - 1) * params.dt
    out = {
        "value": sites * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "kernel_ms": kern_ms,
        "diag_step_kernel_ms": tm["ms_diag"] / max(tm["n_diag"], 1),
        "diag_post_ms": tm["ms_post"] / max(tm["n_diag"], 1),
        "roofline": {"bound": "hbm", "kernel": kname, "steps_per_launch": per_launch,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_source": traffic_src,
                     "algorithmic_bytes": BYTES_PER_SITE[precision] * sites,
                     "box_ceiling": {**{k: round(v, 1) for k, v in ceiling.items()},
                                     "frac_of_pattern": achieved / ceiling["pattern_GBps"]}},
        "pure_step_value": sites / (kern_ms * 1e-3),
        "eta_timed": [eta_first, eta_last],
        "diag_steps_timed": tm["n_diag"],
        "fused_diagnostics_rows": lat.get_fused_diagnostics(),
        "tile": lat.get_tile(),
        "streaming_stores": lat.get_streaming_stores(),
        "prefetch": lat.get_prefetch(),
        "tile_order": "xcd_runs" if lat.get_tile_order() else "round_robin",
        "momentum_pingpong": lat.get_momentum_pingpong(),
        "time_blocking": {"steps_per_sweep": tblock[0], "tile": list(tblock[1:])},
        "autotune_ms_per_step": tuned[2] if tuned else None,
        "last_record": {k: recs[-1][k] for k in ("eta", "xi_W", "xi_lag", "v2_lag", "f_total", "gauss_rel")}
        if recs else None,
    }
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def run_batch(P, torch, steps, small=48, big=16, tune_steps=3):
    """Ensemble of uneven boxes: `small` boxes of 128^3 and `big` of 256^3; box b has seed
    1000 + b, m = 1/2 (b even) or 2/3 (b odd), s = 0 if b//2 is even else 1; all FP32, dx = 0.5,
    dt = 0.1, kappa = 0.9, diagnostics every 10 steps, `steps` steps from eta = 1 with a = 1 at
    the end, all advanced by one graph launch; tile shape, streaming stores, momentum ping-pong, tile
    order and the persistent launch of the plain steps from the autotuner (both forms' plain-step
    times reported)."""
    nb = small + big
    eta_end = 1.0 + steps * 0.1
    params = [P.make_params(128 if b < small else 256, precision="fp32", eta_ref=eta_end, diag_every=10)
              for b in range(nb)]
    bt = P.Batch(params)
    ty, tz, tune_ms = bt.autotune(tune_steps)
    bt.init_fields([1000 + b for b in range(nb)])
    era = [0.5 if b % 2 == 0 else 2.0 / 3.0 for b in range(nb)]
    sv = [0.0 if (b // 2) % 2 == 0 else 1.0 for b in range(nb)]
    torch.cuda.synchronize()
    bt.timing_read()
    t0 = time.perf_counter()
    bt.step(steps, [1.0] * nb, era, sv)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = bt.timing_read()
    sites = sum(p.nx * p.ny * p.nz for p in params)
    nrec = [len(bt.diagnostics(b)) for b in range(nb)]
    achieved = BYTES_PER_SITE["fp32"] * sites * steps / (tm["ms"] * 1e-3) / 1e9
    out = {"value": sites * steps / wall, "unit": "site-updates/s", "boxes": f"{small}x128^3 + {big}x256^3",
           "sites": sites, "steps": steps, "ms_per_step": 1e3 * wall / steps, "graph_ms": tm["ms"],
           "tile": [ty, tz], "streaming_stores": bt.get_streaming_stores(),
           "momentum_pingpong": bt.get_momentum_pingpong(),
           "tile_order": "xcd_runs" if bt.get_tile_order() else "round_robin", "autotune_ms_per_step": tune_ms,
           "persistent": bt.get_persistent(), "autotune_plain_ms_per_step": bt.autotune_times(),
           "records_per_box": min(nrec),
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "note": "whole graph time, diagnostic kernels included"}}
    bt.close()
    del bt
    torch.cuda.empty_cache()
    return out


def cpu_baseline(full_steps=3):
    """The FP64 oracle on bounded samples of the workload, on all host threads OpenMP gives
    it: the 512^3 box itself (same schedule: radiation era, s = 1, a = 1 at eta = 128, random
    phases of seed 1) for `full_steps` plain steps from eta = 1 (about 35 s of CPU work and
    32 GB of host memory for three steps; an oracle diagnostic step at this size would hold
    about 80 GB); a 128^3 box for 80 steps with the diagnostics every 10th step; and a 64^3
    box on one thread."""
    import oracle as O

    threads = O.num_threads()
    out = {"unit": "site-updates/s", "cores": threads, "kind": "oracle"}
    if full_steps:
        n = 512
        m = O.model(n, eta_ref=128.0)
        st = O.init_random_phase(m, 1)
        t0 = time.perf_counter()
        O.run(m, st, full_steps, 1.0, 0.5, 1.0, diag_every=0)
        dt = time.perf_counter() - t0
        del st
        out.update(value=n ** 3 * full_steps / dt,
                   sample=f"{n}^3 box, {full_steps} plain steps from eta=1 (m=1/2, s=1), FP64, {dt:.1f} s on "
                          f"{threads} threads")
    n, steps = 128, 80
    m = O.model(n, eta_ref=128.0)
    st = O.init_random_phase(m, 1)
    t0 = time.perf_counter()
    O.run(m, st, steps, 1.0, 0.5, 1.0, diag_every=10)
    dt = time.perf_counter() - t0
    small = {"value": n ** 3 * steps / dt, "unit": "site-updates/s", "cores": threads,
             "sample": f"{n}^3 box, {steps} steps from eta=1 (m=1/2, s=1, diagnostics every 10), FP64, {dt:.1f} s"}
    if "value" not in out:
        out.update(value=small["value"], sample=small["sample"])
    else:
        out["sample_128"] = small
    # the same on one thread, on a smaller sample (about 3 s)
    n1, steps1 = 64, 10
    m1 = O.model(n1, eta_ref=128.0)
    st1 = O.init_random_phase(m1, 1)
    O.set_num_threads(1)
    t1 = time.perf_counter()
    O.run(m1, st1, steps1, 1.0, 0.5, 1.0, diag_every=10)
    dt1 = time.perf_counter() - t1
    O.set_num_threads(threads)
    out["single_thread"] = {"value": n1 ** 3 * steps1 / dt1, "unit": "site-updates/s", "cores": 1,
                            "sample": f"{n1}^3 box, {steps1} steps from eta=1 (same schedule), FP64, {dt1:.1f} s"}
    return out


def leg_summary(r, precision, n, steps, workload):
    return {"workload": workload, "precision": precision, "sites": n ** 3, "steps": steps, "value": r["value"],
            "unit": "site-updates/s", "ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
            "diag_step_kernel_ms": r["diag_step_kernel_ms"], "diag_post_ms": r["diag_post_ms"],
            "eta_timed": r["eta_timed"], "tile": r["tile"], "fused_diagnostics_rows": r["fused_diagnostics_rows"],
            "roofline": {k: r["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                       "algorithmic_bytes", "box_ceiling")}}


def copy_probe(torch, gib=2, reps=5):
    """A plain device-to-device copy of known size (`gib` GiB per copy), the
    calibration for the HBM byte counters of the profiler."""
    n = gib * (1 << 30)
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "reps": reps,
                      "GB_per_s": 2 * n / dt / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1260)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=400)
    ap.add_argument("--copy-probe", action="store_true", help="only time a plain copy (counter calibration)")
    ap.add_argument("--source-hash", action="store_true", help="print the update kernel's source hash")
    ap.add_argument("--tile", type=str, default=None,
                    help="ty,tz[,nt[,pf[,pp[,xcd]]]] of the update kernel (0,1: per-site kernel; nt 1/0: streaming "
                         "or plain stores; pf 1/0: deeper load pipeline or not; pp 1/0: momentum ping-pong; xcd "
                         "1/0: tiles in contiguous runs per XCD or round-robin)")
    ap.add_argument("--time-blocking", type=str, default=None,
                    help="steps,ty,tz: steps per sweep (1, or 2: the two-step kernel with 64 x ty x tz tiles), FP32 leg")
    ap.add_argument("--cpu-full-steps", type=int, default=3,
                    help="steps of the oracle's 512^3 sample in cpu_baseline (0: only the smaller samples)")
    ap.add_argument("--legs", type=str, default="",
                    help="comma list of extra legs: 1024 (1024^3 matter era, s=0, FP32 then FP64, no diagnostics) "
                         "and/or 1280 (1280^3 radiation era, s=1, FP32, diagnostics every 50)")
    ap.add_argument("--leg-steps", type=int, default=20)
    ap.add_argument("--autotune-cache", type=str, default=None,
                    help="file of stored autotuner choices (mts_autotune_cached); default: tune afresh")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print("bench.py: this implementation runs on one GPU only (the lattice is not sharded); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2208_01525_amd as P

    if args.copy_probe:
        copy_probe(torch)
        return

    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    tblock = tuple(int(v) for v in args.time_blocking.split(",")) if args.time_blocking else None
    fp32 = run_box(P, torch, args.n, "fp32", args.warmup, args.steps, diag_every=10, tile=tile, time_blocking=tblock,
                   tune_cache=args.autotune_cache)
    print(f"fp32: {fp32['value']:.4g} site-updates/s, kernel {fp32['kernel_ms']:.3f} ms, "
          f"{fp32['roofline']['frac']:.3f} of HBM peak", file=sys.stderr, flush=True)
    fp64 = (run_box(P, torch, args.n, "fp64", args.warmup, args.fp64_steps, diag_every=10,
                    tune_cache=args.autotune_cache) if args.fp64_steps else None)
    if fp64:
        print(f"fp64: {fp64['value']:.4g} site-updates/s, kernel {fp64['kernel_ms']:.3f} ms, "
              f"{fp64['roofline']['frac']:.3f} of HBM peak", file=sys.stderr, flush=True)
    batch = run_batch(P, torch, args.batch_steps) if args.batch_steps else None
    if batch:
        print(f"batch: {batch['value']:.4g} site-updates/s, {batch['roofline']['frac']:.3f} of HBM peak, "
              f"tile {batch['tile']}", file=sys.stderr, flush=True)
    legs = {}
    for leg in [v for v in args.legs.split(",") if v]:
        if leg == "1024":
            # 1024^3, matter era (m = 2/3), core growth s = 0 (the switch to s = 1 at eta = 32 lies beyond
            # these steps), a = 1 at eta = 256, FP32 then FP64, no diagnostics (the configuration has none)
            wl = "1024^3, matter era (m=2/3), s=0, a=1 at eta=256, no diagnostics"
            for prec in ("fp32", "fp64"):
                r = run_box(P, torch, 1024, prec, 5, args.leg_steps, diag_every=0, era_m=2.0 / 3.0, s=0.0,
                            eta_ref=256.0, tune_cache=args.autotune_cache)
                legs[f"1024_{prec}"] = leg_summary(r, prec, 1024, args.leg_steps, wl)
                print(f"leg 1024 {prec}: kernel {r['kernel_ms']:.2f} ms, {r['roofline']['frac']:.3f} of HBM peak",
                      file=sys.stderr, flush=True)
        elif leg == "1280":
            wl = "1280^3, radiation era (m=1/2), s=1, a=1 at eta=201, diagnostics every 50"
            r = run_box(P, torch, 1280, "fp32", 5, args.leg_steps, diag_every=50, eta_ref=201.0,
                        tune_cache=args.autotune_cache)
            legs["1280_fp32"] = leg_summary(r, "fp32", 1280, args.leg_steps, wl)
            print(f"leg 1280 fp32: kernel {r['kernel_ms']:.2f} ms, {r['roofline']['frac']:.3f} of HBM peak",
                  file=sys.stderr, flush=True)
        else:
            raise SystemExit(f"bench.py: unknown leg {leg!r} (1024 or 1280)")
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_full_steps)

    line = {
        "metric": METRIC,
        "value": fp32["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.n}^3 periodic box, radiation era (m=1/2), s=1, a=1 at eta=128, dx=0.5, "
                               "dt=0.1, lambda=2, e=1, sigma=1, kappa=0.9, random-phase ICs (seed 1), FP32 fields + "
                               f"FP64 reductions, diagnostics every 10 steps; timed {args.steps} steps from eta="
                               f"{fp32['eta_timed'][0]:.1f} to {fp32['eta_timed'][1]:.1f} after {args.warmup} "
                               "warm-up steps from eta=1 (the full configuration runs 1270 steps to eta=128)",
                   "sites": args.n ** 3},
        "roofline": fp32["roofline"],
        "cpu_baseline": cpu,
        "kernel_ms": fp32["kernel_ms"],
        "pure_step_value": fp32["pure_step_value"],
        "tile": fp32["tile"],
        "streaming_stores": fp32["streaming_stores"],
        "prefetch": fp32["prefetch"],
        "momentum_pingpong": fp32["momentum_pingpong"],
        "tile_order": fp32["tile_order"],
        "time_blocking": fp32["time_blocking"],
        "diag_step_kernel_ms": fp32["diag_step_kernel_ms"],
        "diag_post_ms": fp32["diag_post_ms"],
        "diag_steps_timed": fp32["diag_steps_timed"],
        "fused_diagnostics_rows": fp32["fused_diagnostics_rows"],
        "fp64": {"value": fp64["value"], "unit": "site-updates/s", "steps": args.fp64_steps,
                 "ms_per_step": fp64["ms_per_step"], "kernel_ms": fp64["kernel_ms"], "tile": fp64["tile"],
                 "streaming_stores": fp64["streaming_stores"], "tile_order": fp64["tile_order"],
                 "roofline": fp64["roofline"]} if fp64 else None,
        "batch": batch,
        "legs": legs or None,
        "last_record": fp32["last_record"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
