"""The moving window's front face holds the tangential E at zero, which would
reflect what reaches it, where the paper says fields are absorbed (section 1;
a Mur condition at a face that jumps forward every one or two steps is
unstable once plasma streams in).  Its effect on the results is measured
here: the same beam in a window that reaches 32 cells further ahead (same
particles, same distance from the back face) gives the same beam diagnostics
to 1e-8 and better -- the face's field never acts back on the beam."""
import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

pytestmark = pytest.mark.usefixtures("oracle_built")


def _longer(w, extra):
    w2 = pin.scaled(w, nz=w["grid"]["nz"] + extra)
    w2["beam"]["z_center_cells"] = w["beam"]["z_center_cells"]
    return w2


def _compare(w, nsteps, normals):
    # the draws are clipped at 3 sigma so that no particle starts outside either window's band
    nrm = np.clip(normals, -3.0, 3.0)
    a = po.Sim(w, nrm)
    b = po.Sim(_longer(w, 32), nrm)
    assert a.info().bw == b.info().bw
    a.step(nsteps)
    b.step(nsteps)
    kb = 2 * np.pi / w["bunch_period_cells"]
    da, db = a.diag(kb), b.diag(kb)
    assert da["n_beam_alive"] == db["n_beam_alive"] > 0
    rel = {k: max(abs(x - y) / abs(y) for x, y in zip(np.atleast_1d(da[k]), np.atleast_1d(db[k])))
           for k in ("mean", "sigma", "usigma", "emit", "kin_beam")}
    rel["b1_abs"] = abs(da["b1_abs"] - db["b1_abs"])
    return rel


def test_front_face_changes_no_result_undulator_workload():
    """Workload 0 (32x32x64, helical undulator, window at 0.995 c) over its 100 steps; the
    tangential E a few planes behind the face reaches ~1 % of the field's peak, yet the beam
    moments differ by < 1e-9 (momentum spread < 1e-7)."""
    w = pin.workload(0)
    rel = _compare(w, w["steps"], pin.beam_normals(w["beam"]["n_macro"], 0))
    assert max(rel["mean"], rel["sigma"], rel["emit"], rel["kin_beam"], rel["b1_abs"]) < 1e-8, rel
    assert rel["usigma"] < 1e-6, rel


def test_front_face_changes_no_result_with_plasma():
    """A 16x16x64 beam + plasma + ions case in a window at 0.98 c, 60 steps: < 1e-10."""
    w = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=4096, sigma=(2, 2, 6))
    w["beam"]["charge_C"] = 3e-9
    rel = _compare(w, 60, pin.beam_normals(w["beam"]["n_macro"], 0))
    assert max(rel.values()) < 1e-10, rel
