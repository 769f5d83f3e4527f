#!/usr/bin/env python3
"""Throughput benchmark of the MI355X FSLBM step; prints ONE JSON line.

Workload (default): the cylindrical dam break, 512 x 512 x 96 cells (~25M),
liquid cylinder r = 64, h = 80 at the centre, D3Q19 TRT omega = 1.9,
g = 2e-5 along -z, walls on all sides, EQ refilling, FP32 shifted-PDF
storage with FP64 mass / fill level.  Synthetic, seeded geometry (no dataset).

value      MLUPS_fluid = (liquid + interface cells) x steps / time, whole job,
           state resident in HBM, steps replayed as HIP graphs.
roofline   the bulk stream-collide kernel: algorithmic bytes per launch (per
           liquid cell 19 PDFs read and written plus its flag byte; per
           interface cell its flag byte and its 4-byte list entry) / its
           average duration, measured live with HIP events that every bulk
           launch stamps, in a second context run through the same warm-up
           and the same steps (the same part of the run).  `traffic` is the HBM bytes per
           launch that rocprofv3 FETCH_SIZE + WRITE_SIZE counted, scaled by
           the same counters' reading for a device copy of known size
           (--calibrate-copy), when such a measurement of the current kernel
           source is on record.
event_timed_windows  the same steps in four equal windows of the second
           context (launched one by one with the bulk kernel's events): per
           window its steps, fluid and interface cells, step time, MLUPS_fluid and
           bulk-kernel time, so that the run's phases (the column's collapse)
           show.
cpu_baseline  the FP64 CPU oracle (single thread) on a bounded sample of the
           same workload.
standing_wave_cpu  the 64 x 128 standing wave (SRT omega = 1.8, g = 1e-5, EQ,
           FP64), 1000 steps: the oracle's CPU seconds (single thread) next to
           the GPU's seconds for the same 1000 steps, and how far the two
           final states differ.
variants   other storage types, the dense pool-wave case (83% fluid), and the
           reduced-precision error against the FP64 run.
wave_frequency  the Sec. 4.1 gravity wave at L = 400 in every storage type.
storage_speedup  per workload, FP32, FP16 and BF16 storage against FP64 and
           FP32 (whole step and bulk kernel), each beside its error against the
           FP64 run (fill level, interface height, wave half-periods).
gravity_wave_schemes  (--gravity-wave-schemes) the same wave at L = 800 (FP64)
           with each refilling scheme, next to the per-scheme series the paper prints.
dam_break  rectangular dam break 256 x 128 x 64 (FP32), each refilling scheme,
           20000 steps: front position, residual height, stability, mass drift.
paper_dam_break  the rectangular dam break as the paper sets it up (Sec. 4.2):
           15W x 2H, H = 2W, W = 50, SRT omega = 1.9995, Smagorinsky C_S = 0.1,
           free-slip walls, each refilling scheme: w*(t*), h*(t*), stability.
drop_impact  drop impact 256^3 with surface tension, every storage type, 8000
           steps: centre-column height, cavity depth, mass drift, and the
           fill-level / flag differences against the FP64 run.
adjoint    the reverse mode at full size (64 domains of the 128 x 256 standing
           wave, 4000 steps, sqrt(T) checkpoints): forward and backward wall
           time and cell updates per second.
bubbles    eight enclosed bubbles rising in a 128 x 64 x 192 box (FP32): step
           time with and without the bubble model, pressure range, and the
           total gas amount sum p V over the run.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
METRIC = "FSLBM MLUPS + HBM GB/s (% peak); FP16/FP32-store vs FP64 at stated error"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bulk_kernel_hbm_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2207_14496_amd", "csrc", "step_kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bulk_bytes(n_liquid, n_if, storage_bytes):
    """Algorithmic HBM bytes of one bulk stream-collide launch: every liquid cell
    reads and writes its 19 PDFs and reads its flag; every interface cell has its
    flag read and is written to the interface list."""
    return n_liquid * (38 * storage_bytes + 1) + n_if * (1 + 4)


def kernel_src_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload, storage_name):
    """HBM bytes per bulk launch from committed rocprofv3 PMC summaries, or None
    if absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    want = kernel_src_hash()
    for line in open(TRAFFIC_FILE):
        if not line.startswith("traffic "):
            continue
        kv = dict(tok.split("=", 1) for tok in line.split()[1:])
        if kv.get("workload") == workload and kv.get("storage") == storage_name:
            if kv.get("kernel_src") != want:
                return None
            return float(kv["bytes_per_launch"])
    return None


def run_case(fslbm, setup, storage, steps, warmup, use_graphs=True, windows=1):
    """`steps` timed steps after `warmup` (graph replay), then the bulk
    kernel's own duration over the same part of the run: a second context from
    the same setup goes through the same warm-up and the same steps with every
    bulk launch stamped by HIP events of its own dispatch, in `windows` equal
    calls, each reported on its own (its steps, fluid cells, step and bulk-kernel
    time; these steps are launched one by one with their events, not replayed)."""
    import torch
    sim = fslbm.from_setup(setup, storage=storage)
    sim.use_graphs(use_graphs)
    sim.step(warmup)
    torch.cuda.synchronize()
    d0 = sim.diagnostics()[0]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d1 = sim.diagnostics()[0]
    fluid = 0.5 * ((d0["n_liquid"] + d0["n_interface"]) + (d1["n_liquid"] + d1["n_interface"]))
    n_if = 0.5 * (d0["n_interface"] + d1["n_interface"])
    n_liq = 0.5 * (d0["n_liquid"] + d1["n_liquid"])
    twin = fslbm.from_setup(setup, storage=storage)
    twin.use_graphs(use_graphs)
    twin.step(warmup)
    bulk_ms, win, t = 0.0, [], warmup
    for w in range(windows):
        k = steps // windows + (steps % windows if w == windows - 1 else 0)
        da = twin.diagnostics()[0]
        b, tot = twin.step_timed(k)
        db = twin.diagnostics()[0]
        bulk_ms += b
        fl = 0.5 * ((da["n_liquid"] + da["n_interface"]) + (db["n_liquid"] + db["n_interface"]))
        win.append({"steps": [t, t + k], "fluid_cells_avg": int(fl),
                    "interface_cells_avg": int(0.5 * (da["n_interface"] + db["n_interface"])),
                    "ms_per_step": round(tot / k, 5), "mlups_fluid": round(fl * k / (tot * 1e-3) / 1e6, 1),
                    "bulk_kernel_ms": round(b / k, 5)})
        t += k
    twin.close()
    out = dict(sim=sim, ms=ms, fluid=fluid, n_if=n_if, n_liq=n_liq, d0=d0, d1=d1,
               bulk_ms_avg=bulk_ms / steps, windows=win)
    return out


def roofline(setup, storage_bytes, r, traffic):
    nbytes = bulk_bytes(r["n_liq"], r["n_if"], storage_bytes)
    achieved = nbytes / (r["bulk_ms_avg"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": int(nbytes),
            "kernel_avg_ms": round(r["bulk_ms_avg"], 5)}


def cpu_baseline(setup, target_s=20.0):
    """The oracle as it stands, single-threaded, on whole steps of the same
    initial state, stopping after ~target_s seconds of CPU work."""
    sys.path.insert(0, ROOT)
    import oracle
    p = oracle.Params(setup.nx, setup.ny, setup.nz, tuple(setup.periodic), setup.collision,
                      setup.refill, setup.omega, setup.trt_lambda, tuple(setup.g), setup.sigma,
                      setup.p_volume, setup.eps_phi)
    st = oracle.init_state(p, setup.flags, setup.phi, setup.rho, setup.u)
    fluid = setup.fluid_cells()
    oracle.step(p, st, 1)   # builds the neighbour table, warms caches
    steps, t0 = 0, time.perf_counter()
    while True:
        oracle.step(p, st, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el > target_s or steps >= 50:
            break
    return {"value": round(fluid * steps / el / 1e6, 3), "unit": "MLUPS (fluid cells)",
            "cores": 1, "kind": "oracle",
            "sample": f"{steps} whole steps of the same {setup.nx}x{setup.ny}x{setup.nz} "
                      f"initial state after 1 untimed step ({el:.1f} s, FP64, single thread, "
                      f"host nproc={os.cpu_count()})"}


def standing_wave_cpu(fslbm, setups, torch, steps=1000):
    """The 64 x 128 standing wave (FP64, SRT, EQ) for `steps` steps: the oracle
    as it stands (single thread, CPU seconds) and the GPU for the same steps
    (one call, graph replay), and the difference of the two final states."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import oracle
    s = setups.config("standing-wave-64")
    p = oracle.Params(s.nx, s.ny, s.nz, tuple(s.periodic), s.collision, s.refill, s.omega,
                      s.trt_lambda, tuple(s.g), s.sigma, s.p_volume, s.eps_phi)
    st = oracle.init_state(p, s.flags, s.phi, s.rho, s.u)
    t0 = time.perf_counter()
    oracle.step(p, st, steps)
    cpu_s = time.perf_counter() - t0
    sim = fslbm.from_setup(s, storage=fslbm.F64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    got = {k: v.cpu().numpy()[0] for k, v in sim.read(("flags", "pdf", "mass", "phi")).items()}
    sim.close()
    fluid = st.flags != 4
    rec = {"workload": f"standing wave {s.nx}x{s.ny}x{s.nz} SRT omega={s.omega} g={abs(s.g[1]):g} "
                       f"EQ, FP64", "steps": steps, "cells": s.N,
           "cpu_seconds": round(cpu_s, 3), "cpu_cores": 1, "cpu_kind": "oracle",
           "host_nproc": os.cpu_count(), "gpu_seconds": round(gpu_s, 4),
           "flags_equal": bool(np.array_equal(got["flags"], st.flags)),
           "max_abs_pdf_diff": float(np.abs(got["pdf"][:, fluid] - st.f[:, fluid]).max()),
           "max_abs_phi_diff": float(np.abs(got["phi"] - st.phi).max())}
    log(f"standing wave {steps} steps: oracle {cpu_s:.2f} s (1 thread), GPU {gpu_s * 1e3:.1f} ms")
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--workload", default="cyl-dam-break",
                    choices=["cyl-dam-break", "pool-wave", "rect-dam-break", "drop-impact"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variant-steps", type=int, default=300)
    ap.add_argument("--no-reports", action="store_true",
                    help="skip the configuration reports (dam breaks, drop impact, adjoint)")
    ap.add_argument("--dam-break-steps", type=int, default=20000)
    ap.add_argument("--gravity-wave-schemes", action="store_true",
                    help="also run the L = 800 gravity wave with every refilling scheme (about 3 min)")
    ap.add_argument("--drop-steps", type=int, default=8000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB elementwise copy kernel 5 times (HBM counter calibration)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the reverse-mode report (64 x 128x256, 4000 steps) and print it")
    ap.add_argument("--bubbles-only", action="store_true",
                    help="only run the bubble-model report and print it")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this library runs on exactly one GPU (the path has no multi-GPU "
              "sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    sys.path.insert(0, ROOT)
    import torch
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 2.0, out=dst)   # one elementwise kernel: reads and writes 1 GiB
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": 1 << 30, "dispatches": 5}), flush=True)
        return
    if args.adjoint_only:
        from paper_2207_14496_amd import fslbm, setups
        print(json.dumps({"adjoint": adjoint_report(fslbm, setups, torch)}), flush=True)
        return
    if args.bubbles_only:
        from paper_2207_14496_amd import fslbm, setups
        print(json.dumps({"bubbles": bubble_report(fslbm, setups, torch)}), flush=True)
        return
    from paper_2207_14496_amd import fslbm, setups

    storage = {"f64": fslbm.F64, "f32": fslbm.F32, "f16": fslbm.F16, "bf16": fslbm.BF16}[args.storage]
    sb = fslbm.STORAGE_BYTES[storage]
    log(f"building workload {args.workload}")
    setup = setups.config(args.workload)
    log(f"{setup.nx}x{setup.ny}x{setup.nz}: {setup.fluid_cells()} fluid cells; warmup "
        f"{args.warmup}, timed {args.steps} steps, storage {args.storage}")
    r = run_case(fslbm, setup, storage, args.steps, args.warmup, windows=4 if args.steps >= 4 else 1)
    ms_step = r["ms"] / args.steps
    value = r["fluid"] * args.steps / (r["ms"] * 1e-3) / 1e6
    mlups_domain = setup.N * args.steps / (r["ms"] * 1e-3) / 1e6
    log(f"{value:.1f} MLUPS_fluid, {mlups_domain:.1f} MLUPS_domain, {ms_step * 1e3:.1f} us/step, "
        f"bulk kernel {r['bulk_ms_avg'] * 1e3:.1f} us")
    traffic = measured_traffic(args.workload, args.storage)
    rl = roofline(setup, sb, r, traffic)
    mass_drift = (r["d1"]["total_mass"] - r["d0"]["total_mass"]) / r["d0"]["total_mass"]
    r["sim"].close()
    del r["sim"]
    torch.cuda.empty_cache()

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "MLUPS (fluid-cell updates/s)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": f"{args.workload} {setup.nx}x{setup.ny}x{setup.nz} D3Q19 "
                               f"{'TRT' if setup.collision else 'SRT'} omega={setup.omega} "
                               f"g={abs(sum(setup.g)):g} EQ refill, {args.storage} shifted PDFs, "
                               f"f64 mass/fill level",
                   "cells": setup.N, "fluid_cells_avg": int(r["fluid"]),
                   "interface_cells_avg": int(r["n_if"]),
                   "mlups_domain": round(mlups_domain, 1), "mass_drift_rel": mass_drift,
                   "graphs": True, "parallelism": "single GPU"},
        "roofline": rl,
        "event_timed_windows": r["windows"],
    }

    if not args.no_variants:
        result["variants"] = variants(fslbm, setups, torch, args)
        result["wave_frequency"] = wave_frequency(fslbm)
        result["storage_speedup"] = storage_speedup(result["variants"], result["wave_frequency"])
    if args.gravity_wave_schemes:
        result["gravity_wave_schemes"] = gravity_wave_schemes(fslbm)
    if not args.no_reports:
        result["dam_break"] = dam_break_report(fslbm, setups, torch, args.dam_break_steps)
        result["paper_dam_break"] = paper_dam_break_report(fslbm, setups, torch)
        result["drop_impact"] = drop_impact_report(fslbm, setups, torch, args.drop_steps)
        result["adjoint"] = adjoint_report(fslbm, setups, torch)
        result["bubbles"] = bubble_report(fslbm, setups, torch)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        result["cpu_baseline"] = cpu_baseline(setup)
        result["standing_wave_cpu"] = standing_wave_cpu(fslbm, setups, torch)
    print(json.dumps(result), flush=True)


def storage_speedup(variants, wave):
    """Each reduced-precision storage type against FP32 and FP64 storage on the
    same workload (per step and per bulk launch), beside its measured error
    against the FP64 run: the 300-step variants' fill-level and interface-height
    differences, and the gravity wave's half-period error."""
    wave_err = {w["storage"]: w.get("rel_err_vs_f64") for w in wave}
    out = {}
    for wl in sorted({v["workload"] for v in variants}):
        rows = {v["storage"]: v for v in variants if v["workload"] == wl}
        if "f32" not in rows or "f64" not in rows:
            continue
        rec = {}
        for name in ("f32", "f16", "bf16"):
            if name not in rows:
                continue
            v = rows[name]
            rec[name] = {
                "step_over_f64": round(rows["f64"]["ms_per_step"] / v["ms_per_step"], 3),
                "step_over_f32": round(rows["f32"]["ms_per_step"] / v["ms_per_step"], 3),
                "bulk_over_f64": round(rows["f64"]["bulk_kernel_ms"] / v["bulk_kernel_ms"], 3),
                "bulk_over_f32": round(rows["f32"]["bulk_kernel_ms"] / v["bulk_kernel_ms"], 3),
                "error_vs_f64": dict(v.get("vs_f64", {}), wave_half_period_rel=wave_err.get(name)),
            }
        out[wl] = rec
    return out


def wave_frequency(fslbm, L=400, t_star_end=10.0):
    """Sec. 4.1 gravity wave at L = 400 in every storage type: the first two
    half-periods T*/2 and their error against the FP64 run and against the
    analytic pi."""
    import math
    from paper_2207_14496_amd import waves
    out, ref = [], None
    for name, st in (("f64", fslbm.F64), ("f32", fslbm.F32), ("f16", fslbm.F16), ("bf16", fslbm.BF16)):
        t, a, s, _ = waves.run(L, st, t_star_end=t_star_end, every=20)
        hp = [float(v) for v in waves.half_periods(t, a)[:2]]
        rec = {"storage": name, "L": L, "half_periods": [round(v, 5) for v in hp],
               "rel_err_vs_pi": [round(v / math.pi - 1, 5) for v in hp]}
        if ref is None:
            ref = hp
        else:
            rec["rel_err_vs_f64"] = [round(v / r - 1, 6) for v, r in zip(hp, ref)]
        out.append(rec)
        log(f"  gravity wave L={L} {name}: T*/2 = {rec['half_periods']}")
    return out


def gravity_wave_schemes(fslbm, L=800, t_star_end=15.0):
    """Sec. 4.1 gravity wave at the paper's resolution L = 800 (FP64) with each
    refilling scheme: the first four half-periods T*/2 and the first two
    logarithmic decrements, next to the series the paper prints for the same
    scheme (tests/golden/gravity_wave_sec41.json)."""
    from paper_2207_14496_amd import waves
    with open(os.path.join(ROOT, "tests", "golden", "gravity_wave_sec41.json")) as fh:
        paper = json.load(fh)["schemes_L800"]
    out = []
    for scheme, name in enumerate(("EQ", "EQ+NEQ", "GEQ", "EXT", "AVG")):
        t0 = time.perf_counter()
        t, a, _, diag = waves.run(L, fslbm.F64, t_star_end=t_star_end, every=80, refill=scheme)
        hp = [float(v) for v in waves.half_periods(t, a)[:4]]
        ld = waves.log_decrements(t, a)[:2]
        ref = paper[name]
        rec = {"scheme": name, "L": L, "half_periods": [round(v, 4) for v in hp],
               "paper_half_periods": [round(v, 4) for v in ref["half_period"][:len(hp)]],
               "rel_diff_vs_paper": [round(v / r - 1, 4) for v, r in zip(hp, ref["half_period"])],
               "log_decrement": [[round(x, 3), round(dl, 4)] for x, dl in ld],
               "paper_log_decrement": [[round(x, 3), round(dl, 4)] for x, dl in ref.get("log_decrement", [])[:2]],
               "stable": bool(diag["finite"]), "wall_s": round(time.perf_counter() - t0, 1)}
        out.append(rec)
        log(f"  gravity wave L={L} {name}: T*/2 {rec['half_periods']} (paper {rec['paper_half_periods']}), "
            f"delta {rec['log_decrement']} (paper {rec['paper_log_decrement']})")
    return out


def dam_break_report(fslbm, setups, torch, steps, every=1000, omega=1.95, smagorinsky_cs=0.0,
                     free_slip=0):
    """Rectangular dam break 256x128x64 (FP32 storage), each refilling scheme:
    front position and residual height every `every` steps in cells and in the
    paper's dimensionless form (w* = front / W, h* = height / H, t* = t sqrt(2 g / W),
    Sec. 4.2), the first check at which the run was unstable, and the mass drift.
    omega / smagorinsky_cs / free_slip: the relaxation rate, the turbulence
    model and the wall condition."""
    import math
    from paper_2207_14496_amd import observe
    out = []
    for scheme, name in enumerate(("EQ", "EQ+NEQ", "GEQ", "EXT", "AVG")):
        s = setups.rect_dam_break(refill=scheme, omega=omega)
        W, H, g = s.meta["width"], s.meta["height"], abs(s.g[2])
        sim = fslbm.from_setup(s, storage=fslbm.F32, smagorinsky_cs=smagorinsky_cs, free_slip=free_slip)
        m0 = sim.diagnostics()[0]["total_mass"]
        series, unstable_at, done, t0 = [], None, 0, time.perf_counter()
        while done < steps:
            k = min(every, steps - done)
            sim.step(k)
            done += k
            d = sim.diagnostics()[0]
            if not d["stable"]:
                unstable_at = done
                break
            fl = sim.read(("flags",))["flags"][0]
            xf = observe.front_position(fl, s.nx, s.ny, s.nz)
            hz = observe.residual_height(fl, s.nx, s.ny, s.nz)
            series.append([done, round(done * math.sqrt(2 * g / W), 4), xf, round(xf / W, 4), hz,
                           round(hz / H, 4)])
        el = time.perf_counter() - t0
        rec = {"scheme": name, "steps_run": done, "first_unstable_check": unstable_at,
               "mass_drift_rel": (d["total_mass"] - m0) / m0 if unstable_at is None else None,
               "series": series, "series_columns": ["step", "t*", "front_cells", "w*",
                                                     "height_cells", "h*"],
               "wall_s": round(el, 2)}
        sim.close()
        torch.cuda.empty_cache()
        out.append(rec)
        last = series[-1] if series else None
        log(f"  dam break {name} (omega {omega}, C_S {smagorinsky_cs}): {done} steps, "
            f"unstable at {unstable_at}, last {last}")
    return {"workload": f"rect-dam-break 256x128x64 D3Q19 TRT omega={omega} g=2e-5, f32 shifted PDFs"
                        + (f", Smagorinsky C_S={smagorinsky_cs}" if smagorinsky_cs else "")
                        + (", free-slip walls" if free_slip else ", no-slip walls"),
            "schemes": out}


def paper_dam_break_report(fslbm, setups, torch, W=50, t_star_end=8.0, dt_star=0.25):
    """The rectangular dam break as the paper sets it up (Sec. 4.2): 15W x 2H,
    H = 2W, W = 50, SRT omega = 1.9995 with the Smagorinsky model (C_S = 0.1),
    free-slip walls, FP64; each refilling scheme until the front reaches 14 W
    (w* >= 14) or t* = t_star_end: w*(t*) and h*(t*) every dt_star, and whether
    the run stayed stable."""
    import math
    from paper_2207_14496_amd import observe
    out = []
    for scheme, name in enumerate(("EQ", "EQ+NEQ", "GEQ", "EXT", "AVG")):
        s = setups.paper_dam_break(W=W, refill=scheme)
        H, g = s.meta["height"], s.meta["g"]
        sim = fslbm.from_setup(s, storage=fslbm.F64, smagorinsky_cs=0.1, free_slip=1)
        m0 = sim.diagnostics()[0]["total_mass"]
        unit = math.sqrt(2.0 * g / W)               # t* per step
        every = max(1, int(round(dt_star / unit)))
        series, done, unstable_at, t0 = [], 0, None, time.perf_counter()
        while done * unit < t_star_end:
            sim.step(every)
            done += every
            d = sim.diagnostics()[0]
            if not d["stable"]:
                unstable_at = round(done * unit, 3)
                break
            fl = sim.read(("flags",))["flags"][0]
            wst = observe.front_position(fl, s.nx, s.ny, s.nz) / W
            hst = observe.residual_height(fl, s.nx, s.ny, s.nz) / H
            series.append([round(done * unit, 3), round(wst, 3), round(hst, 4)])
            if wst >= 14.0:
                break
        rec = {"scheme": name, "steps_run": done, "unstable_at_t_star": unstable_at,
               "mass_drift_rel": (d["total_mass"] - m0) / m0 if unstable_at is None else None,
               "series": series, "series_columns": ["t*", "w*", "h*"],
               "wall_s": round(time.perf_counter() - t0, 2)}
        sim.close()
        torch.cuda.empty_cache()
        out.append(rec)
        log(f"  paper dam break W={W} {name}: {done} steps, unstable at t* {unstable_at}, "
            f"last {series[-1] if series else None}")
    return {"workload": f"paper-dam-break {15 * W}x1x{4 * W}, W={W}, H=2W, D3Q19 SRT omega=1.9995, "
                        f"Smagorinsky C_S=0.1, free-slip walls, Ga=1.83e9, f64", "schemes": out}


def adjoint_report(fslbm, setups, torch, T=4000, B=64, x_probe=32):
    """Reverse mode at its full configuration: the 128 x 256 standing wave
    (FP64, SRT, EQ refilling), B seeded domains in one launch, a loss window of
    T steps with ceil(sqrt(T)) checkpoints.  Wall time of the checkpointed
    forward (T steps, records, heights) and of the backward (each segment
    recomputed from its record, then the reverse steps), the cell updates per
    second of each, and the workspace size.  The target only changes the loss
    value, not the work, so h* = 0 is used."""
    import numpy as np
    from paper_2207_14496_amd import adjoint
    nx, ny, depth, a0v, om, gv = 128, 256, 128.0, 1.28, 1.8, 1e-5
    pert = [setups.target_perturbation(s) for s in range(B)]
    a0 = torch.tensor([a0v * (1 + p[2]) for p in pert], dtype=torch.float64, device="cuda")
    flags, pdf0, mass0, phi0 = adjoint.standing_wave_state(a0, nx, ny, depth)
    params = fslbm.Params(nx, ny, 1, B, (1, 0, 1), fslbm.SRT, fslbm.F64, fslbm.REFILL_EQ, om,
                          omega_b=[om * (1 + p[0]) for p in pert],
                          gravity_b=[(0.0, -gv * (1 + p[1]), 0.0) for p in pert])
    sim = fslbm.Simulation(params, flags, phi0, pdf=pdf0, mass=mass0)
    target = np.zeros((B, T))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, _ = sim.adjoint_forward(target, T, x_probe)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = sim.adjoint_backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ws = int(sim._adj[3])
    finite = bool(np.all(np.isfinite(loss)) and np.all(np.isfinite(g["omega"]))
                  and np.all(np.isfinite(g["gravity"])) and bool(torch.isfinite(g["phi"]).all()))
    sim.close()
    del g
    torch.cuda.empty_cache()
    updates = float(B) * nx * ny * T
    fwd, bwd = t1 - t0, t2 - t1
    log(f"  adjoint {B} x {nx}x{ny}, T={T}: forward {fwd:.2f} s, backward {bwd:.2f} s "
        f"({updates / fwd / 1e6:.0f} / {updates / bwd / 1e6:.0f} MLUPS), workspace {ws / 1e9:.1f} GB")
    return {"workload": f"adjoint standing wave {nx}x{ny}, {B} domains, T={T}, "
                        f"ceil(sqrt(T)) checkpoints, FP64 SRT EQ",
            "forward_s": round(fwd, 3), "backward_s": round(bwd, 3),
            "backward_over_forward": round(bwd / fwd, 2),
            "mlups_forward": round(updates / fwd / 1e6, 1), "mlups_backward": round(updates / bwd / 1e6, 1),
            "workspace_gb": round(ws / 1e9, 2), "finite": finite}


def bubble_report(fslbm, setups, torch, steps=200, warmup=10):
    """The bubble model (Sec. 2.2, volume pressure of enclosed gas): eight
    bubbles of radius 10 rising in a 128 x 64 x 192 liquid box (periodic x, y),
    FP32 storage.  Step time with the model and without it (the labels and the
    per-bubble sums are its cost), the bubble pressure
    range at the end, and the total gas amount sum_k p_k V_k at the start and
    the end (every bubble is enclosed, so the amount is conserved but for the
    gas of cells that fill)."""
    centres = [(32.0 + 64.0 * i, 16.0 + 32.0 * j, 24.0 + 24.0 * k + 6.0 * i)
               for i in range(2) for j in range(2) for k in range(2)]
    s = setups.rising_bubbles(nx=128, ny=64, nz=192, centres=centres, radius=10.0, g=2e-5)
    out = {"workload": "rising-bubbles 128x64x192, 8 bubbles of radius 10, TRT omega=1.7 g=2e-5, "
                       "f32 shifted PDFs"}

    def amount(sim):
        f = sim.read(("phi", "bubble_pressure"))
        gas = torch.clamp(1.0 - f["phi"][0], min=0.0)
        return float((f["bubble_pressure"][0] * gas).sum()), f

    for bm in (1, 0):
        sim = fslbm.from_setup(s, storage=fslbm.F32, bubble_model=bm)
        if bm:
            a0, _ = amount(sim)
        sim.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        key = "with_model" if bm else "without_model"
        out[key] = {"ms_per_step": round(dt * 1e3, 4), "mlups_domain": round(s.N / dt / 1e6, 1)}
        if bm:
            a1, f = amount(sim)
            liq = sim.read(("flags",))["flags"][0] == 1
            pb = f["bubble_pressure"][0][~liq]
            out["pressure_range"] = [round(float(pb.min()), 6), round(float(pb.max()), 6)]
            out["amount_start_end"] = [round(a0, 6), round(a1, 6)]
            out["amount_drift_rel"] = (a1 - a0) / a0
        sim.close()
        torch.cuda.empty_cache()
    log(f"  bubbles: {out['with_model']['ms_per_step']} ms/step with the model, "
        f"{out['without_model']['ms_per_step']} without; pressures {out['pressure_range']}, "
        f"amount drift {out['amount_drift_rel']:.2e}")
    return out


def drop_impact_report(fslbm, setups, torch, steps, every=1000):
    """Drop impact 256^3 with surface tension (sigma = 1e-4), EQ refilling, in
    every storage type: centre-column liquid height and cavity depth below the
    initial surface every `every` steps, mass drift, and the fill-level and
    flag differences against the FP64 run at the end."""
    from paper_2207_14496_amd import observe
    s = setups.drop_impact()
    n, depth = s.nx, s.meta["pool_depth"]
    c = n // 2
    out, ref = [], None
    for name, st in (("f64", fslbm.F64), ("f32", fslbm.F32), ("f16", fslbm.F16), ("bf16", fslbm.BF16)):
        sim = fslbm.from_setup(s, storage=st)
        m0 = sim.diagnostics()[0]["total_mass"]
        series, done, unstable_at = [], 0, None
        t0 = time.perf_counter()
        while done < steps:
            k = min(every, steps - done)
            sim.step(k)
            done += k
            d = sim.diagnostics()[0]
            if not d["stable"]:
                unstable_at = done
                break
            phi = sim.read(("phi",))["phi"][0]
            series.append([done, round(observe.column_height(phi, n, n, n, c, c), 4),
                           round(observe.cavity_depth(phi, n, n, n, c, c, depth), 2)])
        el = time.perf_counter() - t0
        rec = {"storage": name, "steps_run": done, "first_unstable_check": unstable_at,
               "ms_per_step": round(el * 1e3 / max(done, 1), 4),
               "mass_drift_rel": (d["total_mass"] - m0) / m0,
               "series": series, "series_columns": ["step", "centre_column_height", "cavity_depth"]}
        f = sim.read(("phi", "flags"))
        if ref is None:
            ref = {"phi": f["phi"][0].clone(), "flags": f["flags"][0].clone(), "series": series}
        else:
            dphi = (f["phi"][0] - ref["phi"]).abs()
            rec["vs_f64"] = {"l1_phi": float(dphi.mean()), "max_abs_phi": float(dphi.max()),
                             "flag_mismatch_cells": int((f["flags"][0] != ref["flags"]).sum()),
                             "max_abs_centre_height": max((abs(a[1] - b[1]) for a, b in
                                                           zip(series, ref["series"])), default=None)}
        sim.close()
        del f
        torch.cuda.empty_cache()
        out.append(rec)
        log(f"  drop impact {name}: {done} steps, {rec['ms_per_step']} ms/step, "
            f"last {series[-1] if series else None}, vs f64 {rec.get('vs_f64')}")
    return {"workload": "drop-impact 256^3 D3Q19 TRT omega=1.989 sigma=1e-4 g=1e-6 EQ refill",
            "runs": out}


def variants(fslbm, setups, torch, args):
    """Other storage types on the same workload, the dense pool case, and the
    reduced-precision error against the FP64 run after the same steps."""
    out = []
    ks = args.variant_steps
    for wl in ("cyl-dam-break", "pool-wave"):
        log(f"variants on {wl}")
        setup = setups.config(wl)
        ref = None
        for name, st in (("f64", fslbm.F64), ("f32", fslbm.F32), ("f16", fslbm.F16),
                         ("bf16", fslbm.BF16)):
            r = run_case(fslbm, setup, st, ks, 20)
            sb = fslbm.STORAGE_BYTES[st]
            rl = roofline(setup, sb, r, measured_traffic(wl, name))
            rec = {"workload": wl, "storage": name, "steps": ks,
                   "mlups_fluid": round(r["fluid"] * ks / (r["ms"] * 1e-3) / 1e6, 1),
                   "mlups_domain": round(setup.N * ks / (r["ms"] * 1e-3) / 1e6, 1),
                   "ms_per_step": round(r["ms"] / ks, 5), "bulk_gbs": rl["achieved"],
                   "bulk_frac": rl["frac"], "bulk_kernel_ms": rl["kernel_avg_ms"],
                   "bulk_algorithmic_bytes": rl["algorithmic_bytes_per_launch"],
                   "bulk_traffic_bytes": rl["traffic"]}
            f = r["sim"].read(("phi", "flags"))
            phi = f["phi"][0]
            d = r["d1"]
            rec["mass_drift_rel"] = (d["total_mass"] - r["d0"]["total_mass"]) / r["d0"]["total_mass"]
            if ref is None:
                ref = {"phi": phi.clone(), "flags": f["flags"][0].clone()}
            else:
                dphi = (phi - ref["phi"]).abs()
                nz, ny, nx = setup.nz, setup.ny, setup.nx
                h = phi.reshape(nz, ny, nx).clamp(0, 1).sum(0)
                h_ref = ref["phi"].reshape(nz, ny, nx).clamp(0, 1).sum(0)
                rec["vs_f64"] = {"max_abs_phi": float(dphi.max()),
                                 "mean_abs_phi": float(dphi.mean()),
                                 "max_abs_column_height": float((h - h_ref).abs().max()),
                                 "flag_mismatch_cells": int((f["flags"][0] != ref["flags"]).sum())}
            r["sim"].close()
            del r["sim"], f
            torch.cuda.empty_cache()
            out.append(rec)
            log(f"  {wl} {name}: {rec['mlups_fluid']} MLUPS_fluid, bulk {rec['bulk_gbs']} GB/s "
                f"({rec['bulk_frac'] * 100:.1f}%)")
    return out


if __name__ == "__main__":
    main()
