"""Window speed following the beam (section 3: in an undulator the beam's mean
longitudinal velocity drops and, in a window that keeps its speed, it drifts to
the back; the window's speed is adjusted to the beam's).

Policy (the same one paper_2411_04703_amd.sim.WindowTracker applies to the GPU
runs, restated here on the oracle's own diagnostics): every N steps the window
speed becomes the centroid's mean velocity over the interval just ended plus
the centroid's offset from its place in the window divided by the interval's
duration.  Pinned: without it the beam falls back by several cells once it is
in the undulator (its boosted velocity drops from 0.923 to 0.852 at
gamma_R = 40, K = 1); with it the centroid stays within half a cell of its place;
the window's position stays continuous and its origin is that position's
floor."""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

pytestmark = pytest.mark.usefixtures("oracle_built")

N_EVERY = 20


def _case():
    w = pin.scaled(pin.workload(4), nx=16, ny=16, nz=128, n_beam=4096, sigma=(2, 2, 8))
    w["plasma"]["n0_lab_cm3"] = 0.0
    w["plasma"]["ions"] = 0
    g, dx = w["frame"]["gamma_boost"], w["grid"]["dx_m"]
    w["undulator"]["z_start_lab_m"] = g * (3 * 8 + 20) * dx  # one lab period ahead of the beam head
    return w


def _offsets(sim, place, nsteps, track):
    dt = sim.info().dt
    z_prev = sim.diag(1.0)["mean"][2]
    out = []
    for _ in range(nsteps // N_EVERY):
        sim.step(N_EVERY)
        i = sim.info()
        assert i.k0 <= i.window_x < i.k0 + 2  # the origin follows the position, one shift per step at most
        z = sim.diag(1.0)["mean"][2]
        off = z - i.window_x - place
        out.append(off)
        if track:
            dur = N_EVERY * dt
            sim.set_window_beta(min(max((z - z_prev) / dur + off / dur, 1e-6), 1.0))
        z_prev = z
    return np.array(out)


def test_window_speed_follows_the_beam_through_the_undulator():
    w = _case()
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    fixed, tracked = po.Sim(w, nrm), po.Sim(w, nrm)
    i0 = fixed.info()
    place = fixed.diag(1.0)["mean"][2] - i0.window_x
    assert abs(place - w["beam"]["z_center_cells"]) < 0.5 and i0.window_x == 0.0  # sample mean of 4096
    nsteps = 400
    off_fixed = _offsets(fixed, place, nsteps, track=False)
    off_tracked = _offsets(tracked, place, nsteps, track=True)
    # the beam has entered the undulator: it slows down (boosted beta_z 0.923 -> 0.852)
    assert off_fixed[-1] < -10.0, off_fixed
    assert np.all(np.abs(off_tracked) < 0.5), off_tracked
    assert tracked.info().bw < 0.9 < fixed.info().bw
    # both windows shifted one cell at a time: the tracked one less far
    assert tracked.info().k0 < fixed.info().k0
