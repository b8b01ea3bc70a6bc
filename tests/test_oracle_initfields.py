"""Pins of the oracle's initial beam self-field (the relativistic Poisson
problem of the boosted frame, section 1 field transformation).

* brute force: the FFT + tridiagonal solver equals a dense linear solve of the
  same discrete operator, written out node by node, on a tiny grid;
* Gauss: the oracle's own divergence (C code) of the field equals the charge;
* closed form: far from a point charge moving at beta, the field is the
  relativistic Coulomb field, gamma q / (4 pi r^2) across the motion and
  q / (4 pi gamma^2 r^2) along it (gamma^3 between the two);
* quasi-statics: one Yee step of the oracle from this field moves the pattern
  with the beam, so E after one step equals the initial field of the moved
  beam (a wrong sign or time level of B would launch a transient instead);
* time level: B at t' = -dt/2 makes one leap-frog step from the initial field
  third-order accurate in dt (residual / 8 per halving), where B at t' = 0 or
  +dt/2 gives second order (residual / 4).
"""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

pytestmark = pytest.mark.usefixtures("oracle_built")


def _dense_solve(rho, g2):
    """(D_xx + D_yy + g2 D_zz) phi = -rho, periodic x, y, phi = 0 beyond the z faces: one row per node."""
    nz, ny, nx = rho.shape
    n = rho.size
    A = np.zeros((n, n))

    def idx(i, j, l):
        return (l * ny + j % ny) * nx + i % nx

    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(i, j, l)
                A[r, idx(i + 1, j, l)] += 1.0
                A[r, idx(i - 1, j, l)] += 1.0
                A[r, idx(i, j + 1, l)] += 1.0
                A[r, idx(i, j - 1, l)] += 1.0
                A[r, r] -= 4.0 + 2.0 * g2
                if l + 1 < nz:
                    A[r, idx(i, j, l + 1)] += g2
                if l > 0:
                    A[r, idx(i, j, l - 1)] += g2
    return np.linalg.solve(A, -rho.ravel()).reshape(rho.shape)


@pytest.mark.parametrize("gamma", [1.0, 3.7])
def test_poisson_equals_dense_solve(gamma):
    rng = np.random.default_rng(5)
    rho = rng.standard_normal((7, 5, 6))
    beta = math.sqrt(1.0 - 1.0 / gamma**2)
    phi, _, _ = po.relativistic_poisson(rho, gamma, beta, 0.5)
    ref = _dense_solve(rho, 1.0 / gamma**2)
    assert np.abs(phi - ref).max() <= 1e-12 * np.abs(ref).max()


def _beam_only(nx=32, ny=32, nz=64, n=4096, sigma=(2, 2, 6)):
    w = pin.scaled(pin.workload(1), nx=nx, ny=ny, nz=nz, n_beam=n, sigma=sigma)
    w["plasma"]["n0_lab_cm3"] = 0.0
    w["plasma"]["ions"] = 0
    w["beam"]["charge_C"] = 3e-9
    return w


def test_initial_field_satisfies_gauss_law():
    w = _beam_only()
    s = po.Sim(w, pin.beam_normals(w["beam"]["n_macro"], 1))
    beta, gamma = po.init_beam_fields(s)
    assert 0.9 < beta < 1.0 and gamma > 2.0
    r = s.gauss()[1:]  # the oracle's divergence leaves out E_z below plane 0
    rho = s.rho(1)
    assert np.abs(rho).max() > 0
    assert np.abs(r).max() <= 1e-12 * np.abs(rho).max()
    # the field is not trivial: transverse and longitudinal parts of the expected size
    assert np.abs(s.field("Ex")).max() > 1e-3 * np.abs(rho).max()


def test_point_charge_far_field_is_relativistic_coulomb():
    nx = ny = 192
    nz = 128
    gamma = 2.0
    beta = math.sqrt(1.0 - 1.0 / gamma**2)
    rho = np.zeros((nz, ny, nx))
    c0 = (nz // 2, ny // 2, nx // 2)
    s1 = {-1: 0.125, 0: 0.75, 1: 0.125}  # quadratic shape of a charge sitting on a node
    for a, wa in s1.items():
        for b, wb in s1.items():
            for c, wc in s1.items():
                rho[c0[0] + c, c0[1] + b, c0[2] + a] = wa * wb * wc
    _, (Ex, Ey, Ez), _ = po.relativistic_poisson(rho, gamma, beta, 0.5)
    # at 7-9 cells the grid (a few % at r ~ 5, falling as 1/r^2), the periodic transverse images and
    # the zero-potential z faces each shift the field by about 1 %; a missing or extra factor of gamma
    # would be off by 100 % or more
    for d in (7, 9):
        r = d + 0.5  # E_x[i] sits at x = i + 1/2, E_z[l] at z = l + 1/2
        ex = Ex[c0[0], c0[1], c0[2] + d]
        ez = Ez[c0[0] + d, c0[1], c0[2]]
        assert ex == pytest.approx(gamma / (4 * math.pi * r * r), rel=0.04), d
        assert ez == pytest.approx(1.0 / (4 * math.pi * gamma**2 * r * r), rel=0.04), d
        assert ex / ez == pytest.approx(gamma**3, rel=0.04), d


def test_initial_field_moves_with_the_beam():
    """E and B after one oracle step from the initial field = initial field of
    the moved beam.  The residual is the grid-scale part of a grainy charge
    density moving 0.54 cells (it falls as the particle count grows); leaving
    B out, or flipping its sign, gives errors of 100-200 % in B and E_z."""
    w = _beam_only(n=65536, sigma=(3, 3, 8))
    w["beam"]["charge_C"] = 3e-12  # self-fields must not change the orbits over the step
    w["beam"]["rel_energy_spread_rms"] = 0.0
    w["beam"]["emit_n_m"] = [1e-9, 1e-9]
    nrm = pin.beam_normals(w["beam"]["n_macro"], 2)
    a = po.Sim(w, nrm)
    po.init_beam_fields(a)
    a.step(1)
    b = po.Sim(w, nrm)
    b.step(1)
    assert np.abs(a.particles(0)["z"] - b.particles(0)["z"]).max() < 1e-6
    po.init_beam_fields(b)  # E^1 and B^(1/2) of the moved beam
    for f, tol in (("Ex", 0.04), ("Ey", 0.04), ("Ez", 0.1), ("Bx", 0.03), ("By", 0.03)):
        ea, eb = a.field(f), b.field(f)
        scale = np.abs(eb).max()
        assert scale > 0
        assert np.abs(ea - eb).max() <= tol * scale, (f, np.abs(ea - eb).max() / scale)


def _set_beam_fields(sim, shift_dt):
    """The beam's self-field with B taken at t' = -shift_dt / 2 (shift_dt = dt: the library's reading)."""
    beta = po.beam_mean_beta(sim)
    gamma = 1.0 / math.sqrt((1.0 - beta) * (1.0 + beta))
    _, E, B = po.relativistic_poisson(np.real(sim.rho(1)), gamma, beta, shift_dt)
    for name, v in zip(po.FIELD_NAMES, E + B):
        sim.field(name)[:] = v


def _one_step_residual(w, nrm, dt, shift):
    """max |E after one step of dt - E after 32 steps of dt/32| / max |E|, both started from the
    beam's self-field with B at t' = -shift * (own step) / 2."""
    coarse = po.Sim(w, nrm, dt_override=dt)
    _set_beam_fields(coarse, shift * dt)
    coarse.step(1)
    fine = po.Sim(w, nrm, dt_override=dt / 32)
    _set_beam_fields(fine, shift * dt / 32)
    fine.step(32)
    num = max(np.abs(coarse.field(n) - fine.field(n)).max() for n in ("Ex", "Ey", "Ez"))
    return num / max(np.abs(fine.field(n)).max() for n in ("Ex", "Ey", "Ez"))


def test_initial_b_time_level_converges_at_third_order():
    """The state between steps is (E^n, B^(n-1/2)), so the initial B must be
    the moving pattern's B half a step earlier.  Taken so, B^(-1/2) is off by
    O(dt^2) and one leap-frog step from it is off by O(dt^3) from the same
    start resolved with 32 small steps: halving dt divides the residual by 8.
    B taken at t' = 0, or half a step late, is off by O(dt) and the residual
    falls only as dt^2 (ratio 4), and is 50x larger at the smaller step."""
    w = _beam_only(nx=16, ny=16, nz=48, n=16384, sigma=(3, 3, 6))
    w["beam"]["charge_C"] = 3e-12  # the orbits stay straight over the step
    w["beam"]["rel_energy_spread_rms"] = 0.0
    w["beam"]["emit_n_m"] = [1e-12, 1e-12]
    w["frame"]["window_beta"] = 0.0
    nrm = pin.beam_normals(w["beam"]["n_macro"], 2)
    res = {shift: [_one_step_residual(w, nrm, dt, shift) for dt in (0.1, 0.05)] for shift in (1, 0, -1)}
    assert 7.0 < res[1][0] / res[1][1] < 9.0, res
    for wrong in (0, -1):
        assert 3.9 < res[wrong][0] / res[wrong][1] < 4.1, res
        assert res[wrong][1] > 30 * res[1][1], res


def _fade_case():
    w = _beam_only(nx=32, ny=32, nz=64, n=16384, sigma=(3, 3, 6))
    return w, pin.beam_normals(w["beam"]["n_macro"], 1)


FADE_CELLS = 10.0  # fade time in cells / c


def _fade_seconds(w):
    return FADE_CELLS * w["grid"]["dx_m"] / 299792458.0


def test_neutraliser_fades_with_gauss_law_kept():
    """Section 3's artificial ions: a charge opposite to the beam's at t' = 0, faded linearly to
    zero over T and carried off by the current -E_b f'(t) (E_b its electrostatic field, the
    charge E_b's divergence).  div E - rho keeps its value at t' = 0 on every interior node, to
    round-off, through the fade and after it, as the window moves (the residual is compared plane
    by plane in the boosted frame).  That value is zero except on the window's top plane at
    t' = 0, where E_b leaves out the components the front face holds at zero: 5e-3 of the peak
    charge at most.  Leaving the faded charge out of rho shows what was carried: the residual
    then differs by f(t) times the charge."""
    w, nrm = _fade_case()
    s = po.Sim(w, nrm)
    arrs = po.init_neutraliser(s, _fade_seconds(w))
    rho_n = arrs[0].reshape(s.rho(1).shape)
    nz = rho_n.shape[0]
    scale = np.abs(np.real(s.rho(1))).max()
    r0 = np.real(s.gauss())  # (plane 0: the back face, which the divergence sees only in part)
    assert np.abs(r0[1:-1]).max() <= 1e-12 * scale and 0 < np.abs(r0[-1]).max() <= 5e-3 * scale
    dt = s.info().dt
    seen = []
    for n in range(0, 40, 4):
        t = s.info().step * dt
        k0 = s.info().k0
        r = np.real(s.gauss())
        # plane l of the window is plane k0 + l of the window at t' = 0
        drift = r[8:nz - 8 - k0] - r0[8 + k0:nz - 8] if k0 < nz - 16 else np.zeros(1)
        assert np.abs(drift).max() <= 1e-12 * scale, (n, np.abs(drift).max() / scale)
        f = max(0.0, 1.0 - t / FADE_CELLS)
        carried = np.real(s.rho(8))  # the faded charge's part of rho now
        expect = np.zeros_like(rho_n)
        expect[: nz - k0] = -f * rho_n[k0:]
        assert np.abs(carried - expect).max() <= 1e-14 * scale, n
        seen.append((f, k0))
        s.step(4)
    assert seen[-1][0] == 0.0 and seen[-1][1] > 0 and 0.0 < seen[2][0] < 1.0


def test_neutraliser_field_nears_the_beams_own():
    """After the fade the beam carries (close to) its self-consistent field -- the moving beam's
    relativistic field -- where from a frozen neutralising background it starts without one and
    is still far from it: transverse E within 25 % of it after the fade against 80 % off."""
    w = _beam_only(nx=32, ny=32, nz=96, n=32768, sigma=(3, 3, 6))
    w["beam"]["charge_C"] = 3e-12
    w["beam"]["rel_energy_spread_rms"] = 0.0
    w["beam"]["emit_n_m"] = [1e-9, 1e-9]
    nrm = pin.beam_normals(w["beam"]["n_macro"], 1)
    off = []
    for fade in (False, True):
        s = po.Sim(w, nrm)
        if fade:
            po.init_neutraliser(s, _fade_seconds(w))
        s.step(int((FADE_CELLS + 20.0) / s.info().dt))
        beta = po.beam_mean_beta(s)
        gamma = 1.0 / math.sqrt((1.0 - beta) * (1.0 + beta))
        _, E, _ = po.relativistic_poisson(np.real(s.rho(1)), gamma, beta, s.info().dt)
        sc = max(np.abs(e[8:-8]).max() for e in E[:2])
        off.append(max(np.abs(s.field(f)[8:-8] - e[8:-8]).max() / sc for f, e in zip(("Ex", "Ey"), E[:2])))
    assert off[0] > 0.8 and off[1] < 0.25, off
