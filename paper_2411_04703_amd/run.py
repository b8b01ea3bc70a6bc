"""Run one of the synthetic workloads on the GPU and print diagnostics.

    python -m paper_2411_04703_amd.run --workload 2 --steps 5000 --every 500

Prints one JSON line per report: step, window origin, particle counts, beam
moments and normalised emittances, bunching factors |b| at the bunching
wavenumber and its second harmonic, field and kinetic energies, the Gauss-law
residual (FP64) and its drift since the previous report, and the time per step
of the interval (HIP events on the library's stream).
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", type=int, default=1, help="synthetic workload 0-5")
    ap.add_argument("--steps", type=int, default=None, help="steps (default: the workload's)")
    ap.add_argument("--every", type=int, default=100, help="report interval in steps")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--device-draws", action="store_true",
                    help="draw the beam's normals on the device from --seed (Philox4x32-10 + Box-Muller; no host "
                         "array, no upload) instead of the host draws the tests and the benchmark use")
    ap.add_argument("--no-gauss", action="store_true", help="skip the FP64 Gauss-law residual (a full-grid pass)")
    ap.add_argument("--init-fields", action="store_true", help="start from the beam's self-field (else zero fields)")
    ap.add_argument("--mobile-ions", type=float, default=None, metavar="MASS",
                    help="plasma ions as particles of this mass in electron masses (0: the proton's); "
                         "default: immobile ions")
    ap.add_argument("--track-window", type=int, default=0, metavar="N",
                    help="adjust the window speed every N steps so that the beam keeps its place in the window "
                         "(0: the speed stays the beam's mean velocity at t' = 0)")
    a = ap.parse_args(argv)

    import torch

    import picinputs as pin
    from . import abi
    from .sim import Sim, WindowTracker

    w = pin.workload(a.workload)
    if a.mobile_ions is not None and w["plasma"]["n0_lab_cm3"] > 0:
        w["plasma"].update(ions=2, ion_mass=a.mobile_ions)
    steps = a.steps if a.steps is not None else w["steps"]
    prec = abi.PIC_FP32_SPLIT if a.precision == "fp32" else abi.PIC_FP64_PLAIN
    opts = {} if prec == abi.PIC_FP32_SPLIT else {"max_steps": max(64, a.every)}
    if a.init_fields:
        opts["init_fields"] = 1
    t0 = time.perf_counter()
    if a.device_draws:
        sim = Sim(w, None, precision=prec, seed=a.seed, **opts)
    else:
        sim = Sim(w, pin.beam_normals(w["beam"]["n_macro"], a.seed), precision=prec, **opts)
    sim.sync()
    init_s = time.perf_counter() - t0
    mask = abi.PIC_DIAG_MOMENTS | abi.PIC_DIAG_BUNCHING | abi.PIC_DIAG_ENERGY
    if not a.no_gauss:
        mask |= abi.PIC_DIAG_GAUSS
    period = w.get("bunch_period_cells", 20.0)

    def report(ms_per_step):
        d = sim.diag(mask, period)
        keep = ("step", "t", "k0", "window_x", "window_beta", "n_beam", "n_plasma", "beam_lost", "mean", "sigma",
                "umean", "usigma", "emit", "b1_abs", "b2_abs", "field_energy", "kin_beam", "kin_plasma", "gauss_max",
                "gauss_drift", "rho_max")
        out = {k: d[k] for k in keep if k in d}
        out["ms_per_step"] = ms_per_step
        out["particle_steps_per_s"] = (d["n_beam"] + d["n_plasma"]) / (ms_per_step * 1e-3) if ms_per_step else None
        print(json.dumps(out), flush=True)

    print(json.dumps({"workload": a.workload, "grid": w["grid"], "n_beam": w["beam"]["n_macro"], "steps": steps,
                      "precision": a.precision, "init_s": init_s,
                      "arena_GB": sim.layout.arena_bytes / 1e9}), flush=True)
    report(None)
    tracker = WindowTracker(sim, a.track_window) if a.track_window > 0 else None
    done = 0
    while done < steps:
        k = min(a.every, steps - done)
        if tracker:
            k = min(k, a.track_window - done % a.track_window)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.step(k)
        sim.sync()
        dt = time.perf_counter() - t1
        done += k
        if tracker and done % a.track_window == 0:
            tracker.update()
        if done % a.every == 0 or done == steps:
            report(dt / k * 1e3)
    return 0


if __name__ == "__main__":
    sys.exit(main())
