"""Writes adjoint_subcase_500.json: the oracle's loss L = |b(2 pi / 20 cells)| after 500 steps of
the 16x16x64 reduction of the adjoint workload (beam seed 0), its stored-state discrete adjoint
(K dL/dK, n0 dL/dn0), and the complex-step derivatives of the oracle's forward run (an imaginary 1e-30 K,
then 1e-30 n0, added), which pin the adjoint independently of its code.  Calls only oracle/.

    python tests/golden/make_adjoint_subcase_500.py
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import picinputs as pin  # noqa: E402
from oracle import build as ob  # noqa: E402
from oracle import pyoracle as po  # noqa: E402

NSTEPS = 500
SEED = 0


def main():
    ob.build()
    w = pin.adjoint_subcase()
    nrm = pin.beam_normals(w["beam"]["n_macro"], SEED)
    kb = 2 * math.pi / w["bunch_period_cells"]
    bw = po.Sim(w, nrm).info().bw
    t0 = time.time()
    L, gK, gn = po.grad_bunching(w, nrm, NSTEPS, kb)
    t_adj = time.time() - t0
    H = 1e-30
    K, n0 = w["undulator"]["K"], w["plasma"]["n0_lab_cm3"]
    csK = po.loss_bunching(w, nrm, NSTEPS, kb, complex_step=True, hK=H * K)[1] / H  # K dL/dK
    csn = po.loss_bunching(w, nrm, NSTEPS, kb, complex_step=True, hn0=H * n0)[1] / H  # n0 dL/dn0
    out = {
        "_about": "oracle only (plain FP64 C); written by make_adjoint_subcase_500.py",
        "workload": "picinputs.adjoint_subcase(), beam normals seed 0",
        "nsteps": NSTEPS, "seed": SEED, "bunch_period_cells": w["bunch_period_cells"],
        "window_beta": bw,
        "L": L, "K_dL_dK": gK, "n0_dL_dn0": gn,
        "complex_step_K_dL_dK": csK, "complex_step_n0_dL_dn0": csn,
        "oracle_adjoint_seconds": t_adj,
    }
    with open(os.path.join(HERE, "adjoint_subcase_500.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
