"""GPU checks at the full 128x128x512 size (gamma_R = 20, 4,194,304-particle
beam plus 2 ppc plasma with immobile ions), in the launch configuration
bench.py times (FP32 split path, library-chosen tile, default deposit).

At this size the oracle cannot run the whole step, so it checks sampled
outputs one by one and properties that hold at any size:
* sampled beam and plasma particles: the oracle gathers (FP64) from the GPU's
  own field arrays, pushes and moves them; the GPU's next state must hold a
  particle there (nearest-neighbour match, positions far closer than the
  inter-particle spacing);
* charge conservation: the Gauss residual moves only at FP32 round-off;
* particle bookkeeping and beam moments against the FP64 GPU path, whose
  per-step agreement with the oracle is established at small sizes."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import picinputs as pin
from oracle import pyoracle as po

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]

W = pin.workload(1)
FIELDS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


def _gpu(precision=1, w=W, **kw):
    from paper_2411_04703_amd.sim import Sim
    return Sim(w, pin.beam_normals(w["beam"]["n_macro"], 0), precision=precision, **kw)


def _oracle_grid():
    """A particle-free oracle grid of the same size, frame and time step."""
    w = pin.scaled(W, n_beam=16)
    w["plasma"]["n0_lab_cm3"] = 0.0
    return po.Sim(w, pin.beam_normals(16, 0))


def _predict(ref, p, idx, dt, pusher, qm=-1.0):
    """Oracle gather (at B^n), push and move of particles idx of state p (charge-to-mass ratio qm)."""
    X = np.stack([p["x"][idx], p["y"][idx], p["z"][idx]], axis=1)
    U = np.stack([p["ux"][idx], p["uy"][idx], p["uz"][idx]], axis=1)
    X1 = np.empty_like(X)
    U1 = np.empty_like(U)
    for k in range(len(idx)):
        E, B = ref.gather(X[k])
        u1 = po.push(pusher, qm, dt, U[k], E, B)
        X1[k] = X[k] + dt * u1 / math.sqrt(1.0 + u1 @ u1)
        U1[k] = u1
    return X1, U1


def _match(pred_x, pred_u, after):
    """Nearest particle of the next state to each prediction (candidates near them only)."""
    A = np.stack([after["x"], after["y"], after["z"]], axis=1)
    lo, hi = pred_x.min(axis=0) - 1.0, pred_x.max(axis=0) + 1.0
    m = np.all((A >= lo) & (A <= hi), axis=1)
    cand = np.nonzero(m)[0]
    d, k = cKDTree(A[cand]).query(pred_x)
    j = cand[k]
    U = np.stack([after["ux"][j], after["uy"][j], after["uz"][j]], axis=1)
    return d, np.abs(U - pred_u).max(axis=1) / np.maximum(1.0, np.abs(pred_u).max(axis=1))


def test_workload1_sampled_particles_follow_the_oracle_push():
    from paper_2411_04703_amd import abi
    gpu = _gpu()
    gpu.step(3)  # E^3 and B^(5/2) nonzero everywhere the beam has been
    ref = _oracle_grid()
    for f in FIELDS:
        ref.field(f)[:] = gpu.field(f)
    ref.b_half()  # B^n, as the GPU forms it for the gather
    i = ref.info()
    # the oracle grid's window origin is 0: shift the GPU's absolute z into its frame
    k0 = int(gpu.diag()["k0"])
    rng = np.random.default_rng(11)
    before = [gpu.particles(0), gpu.particles(1)]
    gpu.step(1)
    after = [gpu.particles(0), gpu.particles(1)]
    assert np.abs(np.concatenate([ref.field(f).ravel() for f in ("Ex", "Bx")])).max() > 0
    for sp, n in ((0, 1500), (1, 1500)):
        p = dict(before[sp])
        p["z"] = p["z"] - k0
        if sp == 0:
            idx = rng.choice(len(p["x"]), n, replace=False)
        else:  # plasma inside the beam's column, where the fields are strong
            near = np.nonzero((np.abs(p["x"] - 64) < 6) & (np.abs(p["y"] - 64) < 6) &
                              (np.abs(p["z"] - W["beam"]["z_center_cells"]) < 60))[0]
            idx = rng.choice(near, n, replace=False)
        X1, U1 = _predict(ref, p, idx, i.dt, abi.PIC_BORIS)
        X1[:, 2] += k0
        d, du = _match(X1, U1, after[sp])
        # FP32 offsets and FP32 fields: ~1e-6 cells; neighbours are >= 0.05 cells apart
        assert np.quantile(d, 0.999) < 2e-5 and d.max() < 1e-4, (sp, np.sort(d)[-5:])
        assert du.max() < 1e-5, (sp, np.sort(du)[-5:])


def test_workload1_mobile_ions_follow_the_oracle_push():
    """Mobile ions of mass 4 at full size: sampled ions near the beam are pushed
    by the oracle (q/m = +1/4) from the GPU's fields and found among the GPU's
    ions (negative weights) of the next state, to the bars of the electrons."""
    from paper_2411_04703_amd import abi
    w = pin.scaled(W)
    w["plasma"].update(ions=2, ion_mass=4.0)
    gpu = _gpu(w=w)
    gpu.step(3)
    ref = _oracle_grid()
    for f in FIELDS:
        ref.field(f)[:] = gpu.field(f)
    ref.b_half()
    i = ref.info()
    k0 = int(gpu.diag()["k0"])
    rng = np.random.default_rng(12)
    before = gpu.particles(1)
    gpu.step(1)
    pa = gpu.particles(1)
    after = {k: v[pa["w"] < 0] for k, v in pa.items()}
    ion = before["w"] < 0
    p = {k: v[ion] for k, v in before.items()}
    p["z"] = p["z"] - k0
    near = np.nonzero((np.abs(p["x"] - 64) < 6) & (np.abs(p["y"] - 64) < 6) &
                      (np.abs(p["z"] - W["beam"]["z_center_cells"]) < 60))[0]
    idx = rng.choice(near, 1500, replace=False)
    X1, U1 = _predict(ref, p, idx, i.dt, abi.PIC_BORIS, qm=0.25)
    X1[:, 2] += k0
    d, du = _match(X1, U1, after)
    assert np.quantile(d, 0.999) < 2e-5 and d.max() < 1e-4, np.sort(d)[-5:]
    assert du.max() < 1e-5, np.sort(du)[-5:]
    # the ions did respond to the beam's field (the push is not the identity)
    assert np.abs(U1[:, :2]).max() > 1e-7


def test_workload1_charge_conservation_and_counts():
    from paper_2411_04703_amd import abi
    gpu = _gpu()
    d0 = gpu.diag(abi.PIC_DIAG_GAUSS | abi.PIC_DIAG_MOMENTS)
    assert d0["n_beam"] == W["beam"]["n_macro"]
    assert d0["n_plasma"] == 128 * 128 * (512 - 7) * 2
    drift = []
    for _ in range(4):
        gpu.step(5)
        drift.append(gpu.diag(abi.PIC_DIAG_GAUSS)["gauss_drift"])
    # plasma electrons and ions carry opposite gross charge densities gamma_R n0 that cancel;
    # FP32 rounds the deposit relative to that gross density (~6e-8 of it per step)
    from paper_2411_04703_amd.sim import derive
    dv = derive(W)
    gross = dv["gamma_R"] * dv["n0_norm"]
    assert max(drift) < 1e-6 * gross, (drift, gross, d0["rho_max"])
    assert gpu.diag()["n_beam"] == W["beam"]["n_macro"]


def test_workload1_fp32_tracks_fp64_at_full_size():
    a, b = _gpu(1), _gpu(0, max_steps=64)
    a.step(12)
    b.step(12)
    da, db = a.diag(), b.diag()
    assert da["n_beam"] == db["n_beam"] and da["n_plasma"] == db["n_plasma"]
    for k in ("mean", "sigma", "usigma", "emit"):
        np.testing.assert_allclose(da[k], db[k], rtol=1e-4, err_msg=k)
    assert abs(da["b1_abs"] - db["b1_abs"]) < 1e-5
    # FP32 rounds each step's field change relative to the gross (cancelling) plasma and
    # ion currents, gamma_R n0 beta_R per cell -- 2e4 times the beam's current here
    from paper_2411_04703_amd.sim import derive
    dv = derive(W)
    gross = dv["dt"] * dv["gamma_R"] * dv["n0_norm"] * dv["beta_R"] * math.sqrt(128 * 128 * 512)
    total = math.sqrt(sum(np.linalg.norm(b.field(f)) ** 2 for f in FIELDS))
    for f in FIELDS:
        err = np.linalg.norm(a.field(f) - b.field(f))
        assert err <= 1e-4 * max(total, gross), (f, err, total, gross)


def _ulp_perturbed(sim, rng):
    """Every coordinate of every live particle of an FP64 state moved by one FP32 ulp, up or down
    at random: positions by the ulp of their in-cell offset (how the FP32 path stores them),
    momenta by the ulp of their FP32 value."""
    from paper_2411_04703_amd import abi
    for which, alive in ((abi.PIC_A_BEAM, abi.PIC_A_BEAM_ALIVE), (abi.PIC_A_PLASMA, abi.PIC_A_PLASMA_ALIVE)):
        a = sim.read(which).cpu().numpy()
        live = sim.read(alive).cpu().numpy() == 1
        n = int(live.sum())
        if n == 0:
            continue
        for r in range(3):
            off = a[r, live] - np.floor(a[r, live])
            a[r, live] += rng.choice((-1.0, 1.0), n) * np.spacing(off.astype(np.float32)).astype(np.float64)
        for r in range(3, 6):
            u = np.abs(a[r, live]).astype(np.float32)
            a[r, live] += rng.choice((-1.0, 1.0), n) * np.spacing(u).astype(np.float64)
        sim.write(which, a)


@pytest.mark.timeout(900)
def test_workload1_full_run_fp32_within_stated_tolerance(progress):
    """After the workload's full 1000 steps the FP32 path's beam moments agree with the FP64
    path's (which follows the oracle to 1e-12 per step at small sizes) within the tolerance stated
    before the measurement: per quantity, max(1e-3 relative, 3x the spread of four FP64 runs
    whose initial particles -- beam and plasma -- are each moved by one FP32 ulp per coordinate,
    independently and at random).  The spread measures how far the discretised system itself
    carries such rounding-sized differences in 1000 steps; the FP32 run makes them at every
    step.  The bunching factor, at noise level here, absolutely within max(1e-6, 3x its
    spread)."""
    from paper_2411_04703_amd.sim import Sim
    nsteps = W["steps"]
    nrm = pin.beam_normals(W["beam"]["n_macro"], 0)
    s = Sim(W, nrm, precision=1)
    s.step(nsteps)
    d32 = s.diag()
    del s
    d64p = []
    for seed in range(5):  # seed 0: unperturbed
        s = Sim(W, nrm, precision=0, max_steps=64)
        if seed:
            _ulp_perturbed(s, np.random.default_rng(seed))
        s.step(nsteps)
        d64p.append(s.diag())
        del s
        progress("full-run tolerance: fp64 run", seed, "of 0-4 done")
    d64 = d64p[0]
    assert d32["n_beam"] == d64["n_beam"] and d32["n_plasma"] == d64["n_plasma"]
    report = {}
    for k in ("mean", "sigma", "usigma", "emit"):
        b = np.asarray(d64[k], dtype=float)
        scale = np.maximum(np.abs(b), 1e-300)
        err = np.abs(np.asarray(d32[k], dtype=float) - b) / scale
        spread = np.max([np.abs(np.asarray(d[k], dtype=float) - b) / scale for d in d64p[1:]], axis=0)
        tol = np.maximum(1e-3, 3.0 * spread)
        report[k] = (err.tolist(), spread.tolist(), tol.tolist())
    print("full-run tolerance report (error, spread, tolerance)", report, flush=True)
    eb = abs(d32["b1_abs"] - d64["b1_abs"])
    sb = max(abs(d["b1_abs"] - d64["b1_abs"]) for d in d64p[1:])
    print("b1_abs", eb, sb, max(1e-6, 3.0 * sb), flush=True)
    for k, (err, _, tol) in report.items():
        assert np.all(np.asarray(err) <= np.asarray(tol)), (k, err, tol)
    assert eb <= max(1e-6, 3.0 * sb), (eb, sb)


def test_workload1_stays_stable_over_two_and_a_half_runs():
    """2500 steps of the FP32 path (2.5x the workload's length): the wake's field
    energy peaks near step 1000 and then decays; no growing mode (the moving
    window's front face keeps its tangential E, see the Mur treatment; the
    half-cell time step keeps the drifting plasma's numerical Cherenkov growth
    down)."""
    from paper_2411_04703_amd import abi
    s = _gpu()
    fe = []
    for _ in range(25):
        s.step(100)
        d = s.diag(abi.PIC_DIAG_ENERGY | abi.PIC_DIAG_MOMENTS)
        assert math.isfinite(d["field_energy"]) and d["error_flags"] == 0
        fe.append(d["field_energy"])
    peak = max(fe[:12])
    # after the peak the energy decays; the only excursions are short transients at the back
    # face (a few steps, every 800 steps, when the lattice sheets' phase against the grid
    # leaves a sheet hovering at the removal plane), well below a growing mode
    assert float(np.median(fe[12:])) < peak and max(fe[12:]) <= 1.5 * peak, fe
    assert fe[-1] < 0.8 * peak, fe
    # the beam is still there (a percent of its tail has left the window by now)
    assert s.diag()["n_beam"] > 0.98 * W["beam"]["n_macro"]


@pytest.mark.timeout(900)
def test_workload1_front_face_changes_no_result(progress):
    """The moving window's front face holds the tangential E at zero.  Over the workload's 1000
    steps, sampled every 100, the tangential E of the five planes behind the face stays below 1e-6
    of the field's peak in both paths (measured: 3e-14 in FP64, 0 in FP32), and the FP64 path in a
    window that reaches 64 cells further ahead (same particles, same distance from the back face)
    ends with the same beam moments to 1e-6 relative and |b| to 1e-9 absolute (measured: 4e-9 and
    8e-13).  What the face changes starts in the planes next to it and is carried back with the
    inflowing plasma; two FP32 runs that differ anywhere by an ulp end 1e-5 to 4e-4 apart in these
    moments after this beam-plasma run (the spread of the full-run tolerance test), so comparing
    the FP32 path's two windows would measure that amplification of an ulp, not the face."""
    import copy
    nsteps = W["steps"]
    w2 = copy.deepcopy(W)
    w2["grid"]["nz"] = W["grid"]["nz"] + 64
    diags = []
    for w, precs in ((W, (0, 1)), (w2, (0,))):
        nz = w["grid"]["nz"]
        for prec in precs:
            s = _gpu(prec, w=w, **({"max_steps": 64} if prec == 0 else {}))
            worst = 0.0
            for _ in range(10):
                s.step(nsteps // 10)
                E = [s.field(f) for f in ("Ex", "Ey", "Ez")]
                peak = max(float(np.abs(e).max()) for e in E)
                near = max(float(np.abs(e[nz - 6:nz - 1]).max()) for e in E[:2])
                assert near <= 1e-6 * peak, (prec, nz, near, peak)
                worst = max(worst, near / peak)
            if prec == 0:
                diags.append(s.diag())
            del s
            progress("front face: precision", prec, "nz", nz, "tangential E near the face / peak", worst)
    a, b = diags
    assert a["n_beam"] == b["n_beam"] == W["beam"]["n_macro"]
    for k in ("mean", "sigma", "usigma", "emit"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-6, atol=1e-12, err_msg=k)
    assert abs(a["b1_abs"] - b["b1_abs"]) < 1e-9
