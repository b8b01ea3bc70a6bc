"""GPU parity of the FP64 plain path against the CPU oracle (through the C-ABI).

Bar: 1e-12 relative (L2 per array) per step from identical inputs; the two
sides differ only in the order of floating-point sums (FP64 atomics on the
GPU), so agreement is at round-off.  Where plasma electrons and ions are
present the net current, and hence the field, is the small residual of two
gross currents of size n' beta_R per cell that cancel; rounding is relative
to the gross terms, so a field's error is measured against
max(|field|, dt |gross current|), and a momentum component's against the
momentum magnitude.  Cases span several tiles of the grid, a
moving window with shifts, plasma inflow/outflow, the undulator entrance and
a plasma up-ramp entering the window."""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]

FIELDS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
PKEYS = ("x", "y", "z", "ux", "uy", "uz", "w")


def _case(name):
    if name == "undulator_beam":
        return pin.workload(0)
    if name == "beam_plasma_ions":
        return pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=8192, sigma=(2, 2, 8))
    if name == "adjoint_sub":
        w = pin.adjoint_subcase()
        w["undulator"]["z_start_lab_m"] = w["frame"]["gamma_boost"] * 20 * w["grid"]["dx_m"]
        return w
    if name == "ramp_channel":
        w = pin.scaled(pin.workload(2), nx=16, ny=16, nz=64, n_beam=4096, sigma=(2, 2, 8))
        dx, g = w["grid"]["dx_m"], w["frame"]["gamma_boost"]
        w["plasma"].update(z_start_lab_m=g * (64 - 32 - 6) * dx, length_lab_m=g * 40 * dx, ramp_up_lab_m=g * 6 * dx)
        w["beam"]["charge_C"] = 3e-9
        return w
    # degenerate cases of the method
    if name == "plasma_only":  # no beam: the window speed is given
        w = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=0)
        w["frame"]["window_beta"] = 0.98
        return w
    if name == "beam_only":  # no plasma, no ions: most tiles empty
        w = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=4096, sigma=(2, 2, 8))
        w["plasma"]["n0_lab_cm3"] = 0.0
        w["beam"]["charge_C"] = 3e-9
        return w
    if name == "static_window":  # window at rest: Mur at both faces, plasma still streaming through
        w = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=4096, sigma=(2, 2, 8))
        w["frame"]["window_beta"] = 0.0
        w["beam"]["charge_C"] = 3e-9
        return w
    if name == "no_boost":  # gamma_R -> 1: the lab frame
        w = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=4096, sigma=(2, 2, 8))
        w["frame"]["gamma_boost"] = 1.0001
        w["beam"]["charge_C"] = 3e-9
        return w
    if name == "planar_undulator":  # planar lab field (0, B0 sin phi, 0) instead of the helical one
        w = pin.workload(0)
        w["undulator"]["kind"] = 2
        return w
    if name == "plane_2d":  # two-dimensional x-z grid (ny = 1), as the paper's runs: beam, plasma, ions
        w = pin.scaled(pin.workload(1), nx=32, ny=1, nz=64, n_beam=2048, sigma=(2, 1, 8))
        w["beam"]["charge_C"] = 3e-10
        return w
    if name == "planar_2d":  # planar undulator on the x-z grid
        w = pin.scaled(pin.workload(0), ny=1, n_beam=4096)
        w["undulator"]["kind"] = 2
        w["beam"]["charge_C"] = 3e-10
        return w
    if name == "mobile_ions":  # ions as particles (protons), pushed and deposited like the electrons
        w = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=8192, sigma=(2, 2, 8))
        w["plasma"].update(ions=2, ion_mass=0.0)
        w["beam"]["charge_C"] = 3e-9
        return w
    if name == "light_ions":  # mass 4 ions: a strong ion response within a few steps
        w = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=4096, sigma=(2, 2, 8))
        w["plasma"].update(ions=2, ion_mass=4.0)
        w["beam"]["charge_C"] = 3e-9
        return w
    if name == "ions_2d":  # mobile ions (M = 4) on the x-z grid
        w = _case("plane_2d")
        w["plasma"].update(ions=2, ion_mass=4.0)
        return w
    if name == "ragged":  # non-power-of-two grid of 3 x 5 x 4 tiles (8 x 8 x 16), beam count not a multiple of 64
        w = pin.scaled(pin.workload(1), nx=24, ny=40, nz=64, n_beam=4099, sigma=(2, 3, 8))
        w["beam"]["charge_C"] = 3e-9
        return w
    raise KeyError(name)


CASES = ["undulator_beam", "beam_plasma_ions", "adjoint_sub", "ramp_channel", "plasma_only", "beam_only",
         "static_window", "no_boost", "ragged", "planar_undulator", "plane_2d", "planar_2d", "mobile_ions",
         "light_ions", "ions_2d"]


def _pair(w, seed=0, **opts):
    from paper_2411_04703_amd.sim import Sim
    nrm = pin.beam_normals(w["beam"]["n_macro"], seed)
    ref = po.Sim(w, nrm)
    w = pin.scaled(w)
    w["frame"]["window_beta"] = ref.info().bw  # same window schedule on both sides
    gpu = Sim(w, nrm, precision=0, max_steps=opts.pop("max_steps", 200), **opts)
    return ref, gpu


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _gross_field_scale(ref):
    """dt times the L2 norm of the plasma electrons' gross drift current (zero without plasma)."""
    i = ref.info()
    if i.n0n == 0:
        return 0.0
    return i.dt * i.gR * i.n0n * i.bR * math.sqrt(ref.nc)


def _compare(ref, gpu, tol, what=""):
    gross = _gross_field_scale(ref)
    for f in FIELDS:
        a, b = gpu.field(f), ref.field(f)
        scale = max(np.linalg.norm(b), gross, 1e-30)
        assert np.linalg.norm(a - b) <= tol * scale + 1e-300, (what, f, _rel(a, b))
    pairs = [(gpu.particles(0), ref.particles(0)), (gpu.particles(1), ref.particles(1))]
    if ref.info().n_ions:
        # mobile ions share the GPU's plasma slots (after the electrons of each sheet), weight negated
        g = pairs[1][0]
        ion = g["w"] < 0
        gi = {k: v[ion] for k, v in g.items()}
        gi["w"] = -gi["w"]
        pairs = [pairs[0], ({k: v[~ion] for k, v in g.items()}, pairs[1][1]), (gi, ref.particles(2))]
    for sp, (g, o) in enumerate(pairs):
        ag, ao = g["alive"] == 1, o["alive"] == 1
        assert ag.sum() == ao.sum(), (what, sp, ag.sum(), ao.sum())
        if ao.sum() == 0:
            continue
        umag = np.sqrt(o["ux"][ao] ** 2 + o["uy"][ao] ** 2 + o["uz"][ao] ** 2)
        for k in PKEYS:
            a, b = g[k][ag], o[k][ao]
            # a momentum component is measured against the particles' momentum magnitude:
            # transverse plasma momenta are round-off-sized responses to cancelling fields
            scale = max(np.linalg.norm(b), np.linalg.norm(umag) if k.startswith("u") else 0.0, 1e-300)
            assert np.linalg.norm(a - b) <= tol * scale, (what, sp, k, np.linalg.norm(a - b) / scale)


@pytest.mark.parametrize("case", CASES)
def test_init_parity(case):
    ref, gpu = _pair(_case(case))
    _compare(ref, gpu, 1e-13, "init")  # u_z' = gR (u_z - bR gamma) cancels ~20x
    assert gpu.diag()["window_beta"] == ref.info().bw


@pytest.mark.parametrize("case", CASES)
def test_step_parity(case):
    ref, gpu = _pair(_case(case))
    for n in (1, 4, 10, 20):
        k = n - ref.info().step
        ref.step(k)
        gpu.step(k)
        _compare(ref, gpu, 1e-12 * max(1, n / 4), f"step {n}")
    i = ref.info()
    d = gpu.diag()
    assert d["k0"] == i.k0 and d["step"] == i.step


def test_full_run_workload0():
    """The whole 100-step FP64 parity run of the undulator workload."""
    w = pin.workload(0)
    ref, gpu = _pair(w)
    ref.step(w["steps"])
    gpu.step(w["steps"])
    _compare(ref, gpu, 1e-10, "100 steps")
    dg, do = gpu.diag(), ref.diag(2 * math.pi / 20)
    for k in ("b1_abs", "b2_abs", "field_energy", "kin_beam"):
        assert dg[k] == pytest.approx(do[k], rel=1e-10), k
    for k in ("mean", "sigma", "umean", "usigma", "emit"):
        np.testing.assert_allclose(dg[k], do[k], rtol=1e-10, err_msg=k)


def test_gauss_residual_fp64_stays_at_roundoff():
    from paper_2411_04703_amd import abi
    w = _case("beam_plasma_ions")
    w["beam"]["charge_C"] = 3e-9
    _, gpu = _pair(w)
    d0 = gpu.diag(abi.PIC_DIAG_GAUSS)
    drift = []
    for _ in range(8):
        gpu.step(3)
        d = gpu.diag(abi.PIC_DIAG_GAUSS)
        drift.append(d["gauss_drift"])
    assert max(drift) < 1e-12 * d0["rho_max"], (drift, d0["rho_max"])
    assert gpu.diag(abi.PIC_DIAG_ENERGY)["field_energy"] > 0


def test_checkpoint_resume_matches_straight_run():
    from paper_2411_04703_amd.sim import Sim
    w = _case("beam_plasma_ions")
    nrm = pin.beam_normals(w["beam"]["n_macro"], 3)
    a = Sim(w, nrm, precision=0, max_steps=100)
    a.step(7)
    st = a.get_state()
    a.step(9)
    b = Sim(w, nrm, precision=0, max_steps=100)
    b.set_state(st)
    b.step(9)
    ref = po.Sim(pin.scaled(w, n_beam=16), pin.beam_normals(16))
    gross = _gross_field_scale(ref)
    for f in FIELDS:
        x, y = a.field(f), b.field(f)
        assert np.linalg.norm(x - y) < 1e-13 * max(np.linalg.norm(y), gross), f
    da, db = a.diag(), b.diag()
    assert da["step"] == db["step"] == 16 and da["k0"] == db["k0"]
    assert da["b1_abs"] == pytest.approx(db["b1_abs"], rel=1e-13)


def test_compaction_keeps_particle_order():
    """Forward mode compacts dead plasma slots; the alive sequence is unchanged."""
    w = _case("beam_plasma_ions")
    ref, gpu = _pair(w, check_every=4)
    ref.step(13)
    gpu.step(13)
    _compare(ref, gpu, 1e-12, "compacted")
    assert len(gpu.particles(1)["alive"]) < len(ref.particles(1)["alive"])


@pytest.mark.parametrize("case,nsteps", [("adjoint_sub", 12), ("beam_plasma_ions", 10)])
def test_adjoint_gradient_matches_oracle(case, nsteps):
    from paper_2411_04703_amd.autograd import bunching_grad
    w = _case(case)
    if w["undulator"]["kind"] == 0:
        w = pin.scaled(w)
        w["undulator"] = dict(pin.workload(3)["undulator"])
        w["undulator"]["z_start_lab_m"] = w["frame"]["gamma_boost"] * 20 * w["grid"]["dx_m"]
    w["beam"]["charge_C"] = 3e-9
    nrm = pin.beam_normals(w["beam"]["n_macro"], 2)
    ref = po.Sim(w, nrm)
    w["frame"]["window_beta"] = ref.info().bw
    L, gK, gn = po.grad_bunching(w, nrm, nsteps, 2 * math.pi / 20)
    Lg, gKg, gng = bunching_grad(w, nrm, nsteps, every=5)
    assert Lg == pytest.approx(L, rel=1e-12)
    assert gKg == pytest.approx(gK, rel=1e-9, abs=1e-15), (gKg, gK)
    assert gng == pytest.approx(gn, rel=1e-9, abs=1e-15), (gng, gn)
    assert abs(gK) > 1e-10 and abs(gn) > 1e-10


def test_window_tracking_matches_oracle():
    """The window speed adjusted every 20 steps (sim.WindowTracker on the GPU, the same policy
    restated on the oracle's diagnostics): 400 steps of a gamma_R = 40 beam entering a helical
    undulator, FP64 path against the oracle (window speeds to 1e-10, window positions to round-off,
    fields to 1e-9 after the run); the
    FP32 path's window keeps the beam within half a cell of its place too."""
    from test_oracle_window_tracking import N_EVERY, _case
    from paper_2411_04703_amd.sim import Sim, WindowTracker
    w = _case()
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    ref = po.Sim(w, nrm)
    w2 = pin.scaled(w)
    w2["frame"]["window_beta"] = ref.info().bw
    gpu = Sim(w2, nrm, precision=0, max_steps=64)
    s32 = Sim(w2, nrm, precision=1)
    trk, trk32 = WindowTracker(gpu, N_EVERY), WindowTracker(s32, N_EVERY)
    dt = ref.info().dt
    z_prev = ref.diag(1.0)["mean"][2]
    place = z_prev - ref.info().window_x
    for _ in range(400 // N_EVERY):
        ref.step(N_EVERY)
        gpu.step(N_EVERY)
        s32.step(N_EVERY)
        i = ref.info()
        z = ref.diag(1.0)["mean"][2]
        dur = N_EVERY * dt
        ref.set_window_beta(min(max((z - z_prev) / dur + (z - i.window_x - place) / dur, 1e-6), 1.0))
        z_prev = z
        b64, b32 = trk.update(), trk32.update()
        d, d32 = gpu.diag(), s32.diag()
        assert d["k0"] == i.k0 and abs(d["window_x"] - i.window_x) <= 1e-12 * i.window_x
        assert abs(b64 - ref.info().bw) <= 1e-10, (b64, ref.info().bw)
        assert abs(d32["mean"][2] - d32["window_x"] - place) < 0.5
    for f in FIELDS:  # 400 steps of round-off (the 100-step workload-0 run agrees to 1e-10)
        assert _rel(gpu.field(f), ref.field(f)) <= 1e-9, f
    assert ref.info().bw < 0.9
