#!/usr/bin/env python3
"""Benchmark of the boosted-frame PIC hot path on one MI355X.

One step = gather, push, current deposition (all particles), ion current,
Yee FDTD, window shift and plasma injection, on the 128x128x512 workload
(gamma_R = 20, 4,194,304-particle beam plus 2 ppc cold plasma with immobile
ions).  Prints one JSON line: whole-job particle-steps/s, FDTD
cell-updates/s, the roofline fraction of the dominant (particle) kernel
measured with HIP events on the library's stream, and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s and FDTD cell-updates/s; FP32 vs FP64 speedup at stated error"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(precision: int, n_particles: float, n_cells: int) -> dict:
    """Bytes the particle phase must move per step: each particle's state read
    and written once, the fields it gathers read once, the current written once."""
    if precision == 1:  # FP32 split: cell int32 + 3 offsets + 3 momenta + weight read; all but weight written
        per_p, per_c = 32 + 28, 24 + 24  # E,B float read; J int64 written
    else:  # FP64 plain: 7 doubles read, 6 written; E,B double read, J double written
        per_p, per_c = 56 + 48, 48 + 24
    return {"per_particle": per_p, "per_cell": per_c, "total": per_p * n_particles + per_c * n_cells}


COUNTERS = os.path.join(ROOT, "profiles", "k_split_step_128x128x512_hbm_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2411_04703_amd", "csrc", "k_split32.hip")


def measured_traffic(tile):
    """HBM bytes per launch of the particle kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter runs (calibrated against a plain copy), or None when the
    kernel source or the tile changed since they were taken."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch: ", "kernel_source_sha256: ", "tile: ")))
    if len(vals) != 3 or [int(v) for v in vals["tile"].split()] != list(tile):
        return None
    if hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest() != vals["kernel_source_sha256"].strip():
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(seconds_budget: float = 20.0) -> dict:
    """The oracle, single-threaded FP64, on 1/64 of the workload's volume (same densities)."""
    import numpy as np  # noqa: F401
    import picinputs as pin
    from oracle import build as ob
    from oracle import pyoracle as po

    if not os.path.exists(os.path.join(ROOT, "oracle", "liborc.so")):
        ob.build()
    w = pin.scaled(pin.workload(1), nx=32, ny=32, nz=128, n_beam=4_194_304 // 64, sigma=(4, 4, 8))
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    s = po.Sim(w, nrm)
    i = s.info()
    npart = i.n_beam + i.n_plasma
    t0 = time.perf_counter()
    steps = 0
    while True:
        s.step(1)
        steps += 1
        if time.perf_counter() - t0 > seconds_budget / 2 or steps >= 20:
            break
    dt = time.perf_counter() - t0
    return {"value": npart * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"32x32x128 cells (1/64 of the workload volume), {i.n_beam} beam + {i.n_plasma} plasma "
                      f"particles, {steps} steps, single-threaded FP64 C",
            "host_cpu": host_cpu_model(), "host_cores": len(os.sched_getaffinity(0)),
            "host_cores_online": os.cpu_count()}


def host_cpu_model() -> str:
    import platform
    try:
        return next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        return platform.processor() or "unknown"


def cpu_table():
    """The oracle (one host core, FP64) beside the GPU paths on the small
    workloads it can run: the 32x32x64 undulator workload in full (100 steps)
    and the 16x16x64 adjoint case (100 steps forward, and forward + adjoint).
    Prints one JSON line; the host's CPU model and core count are included."""
    import math

    import torch

    import picinputs as pin
    from oracle import build as ob
    from oracle import pyoracle as po
    from paper_2411_04703_amd import abi
    from paper_2411_04703_amd.autograd import bunching_grad
    from paper_2411_04703_amd.sim import Sim

    if not os.path.exists(os.path.join(ROOT, "oracle", "liborc.so")):
        ob.build()
    model = host_cpu_model()
    rows = []

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def gpu_forward(w, nrm, prec, nsteps):
        s = Sim(w, nrm, precision=prec, **({} if prec else {"max_steps": 64}))
        s.step(2)
        s.sync()
        d = s.diag()
        dt = timed(lambda: (s.step(nsteps), s.sync()))
        return (d["n_beam"] + d["n_plasma"]) * nsteps / dt

    for name, w, nsteps in (("32x32x64 undulator beam, 16384 particles", pin.workload(0), 100),
                            ("16x16x64 adjoint case (beam, undulator, plasma, ions)", pin.adjoint_subcase(), 100)):
        nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
        o = po.Sim(w, nrm)
        i = o.info()
        npart = i.n_beam + i.n_plasma
        t0 = time.perf_counter()
        o.step(nsteps)
        orc = npart * nsteps / (time.perf_counter() - t0)
        ww = pin.scaled(w)
        ww["frame"]["window_beta"] = i.bw
        row = {"workload": name, "steps": nsteps, "oracle_particle_steps_per_s": orc,
               "oracle_cell_updates_per_s": orc / npart * o.nc,
               "gpu_fp64_particle_steps_per_s": gpu_forward(ww, nrm, abi.PIC_FP64_PLAIN, nsteps),
               "gpu_fp32_particle_steps_per_s": gpu_forward(ww, nrm, abi.PIC_FP32_SPLIT, nsteps)}
        if "checkpoint_every" in w:
            kb = 2 * math.pi / 20.0
            t0 = time.perf_counter()
            po.grad_bunching(w, nrm, nsteps, kb)
            row["oracle_forward_adjoint_s"] = time.perf_counter() - t0
            for key, prec in (("gpu_fp64_forward_adjoint_s", abi.PIC_FP64_PLAIN),
                              ("gpu_fp32_mode_forward_adjoint_s", abi.PIC_FP32_SPLIT)):
                row[key] = timed(lambda: bunching_grad(ww, nrm, nsteps, every=10, precision=prec))
        rows.append(row)
    print(json.dumps({"host_cpu": model, "host_cores": os.cpu_count(), "oracle_threads": 1, "rows": rows}),
          flush=True)


def atomic_calibration(mega: int):
    """64-bit integer atomic adds to distinct device addresses in random order
    (torch index_add_): a reference rate, and a reference reading of the L2
    atomic counters, for the particle kernel's current flush."""
    import torch
    n = mega * (1 << 20)
    dst = torch.zeros(n, dtype=torch.int64, device="cuda")
    idx = torch.randperm(n, device="cuda")
    src = torch.ones(n, dtype=torch.int64, device="cuda")
    for _ in range(2):
        dst.index_add_(0, idx, src)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.index_add_(0, idx, src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"atomics": n, "ms": dt * 1e3, "atomics_per_s": n / dt}), flush=True)


def copy_calibration(mib: int):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings calibrate
    the HBM-traffic counters of the particle kernel."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out = {"copy_mib": mib, "bytes_read": 4 * n, "bytes_written": 4 * n,
           "ms": dt * 1e3, "GBps_read_plus_write": 8 * n / dt / 1e9}
    del a, b
    torch.cuda.empty_cache()
    return out


def describe(w: dict) -> str:
    """The workload named by what it is, with its sizes."""
    g, b, p, u = w["grid"], w["beam"], w["plasma"], w["undulator"]
    text = (f"{g['nx']}x{g['ny']}x{g['nz']} cells, gamma_R={w['frame']['gamma_boost']:g}, beam {b['n_macro']:,} "
            f"macroparticles (sigma {b['sigma_cells'][0]:g}x{b['sigma_cells'][1]:g}x{b['sigma_cells'][2]:g} cells, "
            f"lab gamma {b['gamma_lab']:g})")
    if p["n0_lab_cm3"] > 0:
        ppc = p["ppc"][0] * p["ppc"][1] * p["ppc"][2]
        shape = "uniform" if p["length_lab_m"] <= 0 else \
            f"{p['length_lab_m'] * 100:g} cm channel with a {p['ramp_up_lab_m'] * 100:g} cm up-ramp"
        ions = {0: "no ions", 1: "immobile ions", 2: "mobile ions"}[p["ions"]]
        text += f" + cold plasma {p['n0_lab_cm3']:g} cm^-3 ({shape}) at {ppc} ppc with {ions}"
    if u["kind"]:
        text += f" in a {'helical' if u['kind'] == 1 else 'planar'} undulator, K={u['K']:g}"
    cfl = g["cfl"]
    return text + (", c dt = dx/2" if abs(cfl - 0.8660254037844386) < 1e-12 else f", CFL {cfl:g}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", type=int, default=1, choices=(1, 2, 4, 5),
                    help="1: 128x128x512 (the metric's configuration, default); 2: 256x256x1024 plasma channel; "
                         "4: 512x512x2048 undulator + plasma; 5: 2048x1x4096 x-z grid")
    ap.add_argument("--steps", type=int, default=1000, help="timed steps (default: the workload's full 1000-step run)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip timing the FP64 path (speedup and error)")
    ap.add_argument("--variant", type=int, default=0, help="FP32 current-deposit variant (0, 1 or 2)")
    ap.add_argument("--tile", default="0,0,0", help="FP32 cell tile nx,ny,nz (0,0,0: the library's choice)")
    ap.add_argument("--wg-per-cu", type=int, default=0, help="FP32 particle-kernel workgroups per CU (0 = max)")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only time the oracle beside the GPU paths on the small workloads and exit")
    ap.add_argument("--atomic-calibration", type=int, default=0, metavar="M",
                    help="only time M x 2^20 int64 atomic adds to distinct addresses and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only time a plain device-to-device copy of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.cpu_table:
        cpu_table()
        return
    if args.copy_calibration:
        print(json.dumps(copy_calibration(args.copy_calibration)), flush=True)
        return
    if args.atomic_calibration:
        atomic_calibration(args.atomic_calibration)
        return
    tile = tuple(int(v) for v in args.tile.split(","))
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import picinputs as pin
    from paper_2411_04703_amd import abi
    from paper_2411_04703_amd.sim import Sim

    w = pin.workload(args.workload)
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    g = w["grid"]
    n_cells = g["nx"] * g["ny"] * g["nz"]
    if args.workload != 1:  # the FP64 comparison and the oracle sample are defined on the metric's workload
        args.no_fp64 = True
        args.no_cpu_baseline = True
    copy = copy_calibration(1024)  # the HBM bandwidth a plain copy reaches, beside the vendor peak

    def run(precision, instrument):
        """warm-up, then K timed steps; instrument: HIP events around every phase of every step
        (kernel times per phase; the events themselves add gaps to the stream's timeline)"""
        opts = dict(precision=precision)
        if precision == abi.PIC_FP32_SPLIT:
            opts.update(variant=args.variant, tile=tile, wg_per_cu=args.wg_per_cu)
        if precision == abi.PIC_FP64_PLAIN:
            opts["max_steps"] = 64
        sim = Sim(w, nrm, **opts)
        sim.step(args.warmup)
        d0 = sim.diag(abi.PIC_DIAG_MOMENTS)
        sim.timing(instrument)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.steps)
        sim.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, launches = sim.timing_read() if instrument else (None, None)
        sim.timing(False)
        d1 = sim.diag(abi.PIC_DIAG_MOMENTS | abi.PIC_DIAG_BUNCHING)
        n_active = 0.5 * ((d0["n_beam"] + d0["n_plasma"]) + (d1["n_beam"] + d1["n_plasma"]))
        del sim
        torch.cuda.empty_cache()
        return wall, ms, launches, n_active, d1

    prec = abi.PIC_FP32_SPLIT if args.precision == "fp32" else abi.PIC_FP64_PLAIN
    from paper_2411_04703_amd.sim import derive
    tile_used = derive(w, precision=abi.PIC_FP32_SPLIT, tile=tile)["tile"] if prec == abi.PIC_FP32_SPLIT else None
    # the throughput from K uninstrumented steps; the phase times and the roofline from the same run
    # repeated from a fresh context with the phase events on (the FP32 path is deterministic: both
    # passes compute the same states, checked on the end moments)
    wall, _, _, n_active, dlast = run(prec, instrument=False)
    print(f"bench: {args.precision} run done, {wall / args.steps * 1e3:.3f} ms per step", file=sys.stderr, flush=True)
    wall_i, ms, launches, _, dlast_i = run(prec, instrument=True)
    print(f"bench: {args.precision} instrumented run done, {wall_i / args.steps * 1e3:.3f} ms per step",
          file=sys.stderr, flush=True)
    steps = args.steps
    ps = n_active * steps / wall
    fdtd_ms = ms[1] / steps
    part_ms = ms[0] / steps
    ab = algorithmic_bytes(prec, n_active, n_cells)
    achieved = ab["total"] / (part_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": ps,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "ms_per_step_instrumented": wall_i / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == abi.PIC_FP32_SPLIT else "f64",
        "data": "synthetic",
        "config": {"workload": describe(w),
                   "particles_active": n_active, "cells": n_cells,
                   "precision": "fp32_split_fixed_point" if prec == abi.PIC_FP32_SPLIT else "fp64_plain",
                   "deposit_variant": args.variant, "tile": tile_used, "wg_per_cu": args.wg_per_cu},
        "fdtd_cell_updates_per_s": n_cells / (fdtd_ms * 1e-3) if fdtd_ms > 0 else None,
        "cell_updates_per_s_whole_step": n_cells * steps / wall,
        "phase_ms_per_step": {"particles": part_ms, "fdtd": fdtd_ms, "window_ion_inject_sort": ms[2] / steps,
                              "step_events": ms[3] / steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(tile_used) if (prec == abi.PIC_FP32_SPLIT and tile == (0, 0, 0)
                                                       and args.variant == 0 and args.workload == 1) else None,
                     "measured_copy_GBps": copy["GBps_read_plus_write"],
                     "frac_of_measured_copy": achieved / copy["GBps_read_plus_write"],
                     "kernel": "fused particle kernel(s): gather, push, deposit",
                     "bytes_per_step": ab["total"], "bytes_per_particle": ab["per_particle"],
                     "bytes_per_cell": ab["per_cell"], "avg_ms_per_step": part_ms,
                     "launches": launches[0]},
        "beam_end": {"sigma": dlast["sigma"], "b1_abs": dlast["b1_abs"], "emit": dlast["emit"]},
        "timing": "value and ms_per_step: K steps without instrumentation; phase_ms_per_step and roofline: the "
                  "same run repeated with HIP events around each phase (ms_per_step_instrumented)",
        # the passes' states are the same particles and fields bit for bit; the order of the particles in
        # their bins (atomic slot reservation) is not, so the end moments' FP64 sums agree to rounding
        "passes_max_rel_diff": max(abs(a - b) / max(abs(b), 1e-300) for k in ("mean", "sigma", "usigma", "emit")
                                   for a, b in zip(dlast[k], dlast_i[k])),
    }
    if not args.no_fp64 and prec != abi.PIC_FP64_PLAIN:
        w64, _, _, na64, d64 = run(abi.PIC_FP64_PLAIN, instrument=False)
        print(f"bench: fp64 run done, {w64 / steps * 1e3:.3f} ms per step", file=sys.stderr, flush=True)
        ps64 = na64 * steps / w64
        out["fp64_particle_steps_per_s"] = ps64
        out["fp64_ms_per_step"] = w64 / steps * 1e3
        out["fp32_vs_fp64_speedup"] = ps / ps64
        # error of the FP32 path at the same step, against the FP64 GPU path
        rel = {}
        for k in ("mean", "sigma", "usigma", "emit"):
            a, b = dlast[k], d64[k]
            rel[k] = max(abs(x - y) / max(abs(y), 1e-300) for x, y in zip(a, b))
        rel["b1_abs_abs"] = abs(dlast["b1_abs"] - d64["b1_abs"])
        out["fp32_vs_fp64_error"] = rel
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
