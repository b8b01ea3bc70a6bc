"""Oracle pins of mobile plasma ions (ions = 2): a species of its own, charge +e
and mass M electron masses, loaded on the electrons' lattice with the same
shape and weight (sec. 1: ion current computed directly, one weighting for
both plasma populations).

* two-species cold plasma frequency: the uniform transverse mode of electrons
  against ions oscillates at omega^2 = omega_p^2 (1 + 1/M), for the leap-frog
  orbit sin(theta/2) = omega dt / 2, in every frame (a wrong ion charge sign,
  a missing ion current or a wrong mass scaling moves it: M = 1 doubles
  omega^2);
* heavy-ion limit: mobile ions of mass 1e10 reproduce the rigid lattice of
  immobile ions (whose 1D sheet current is pinned against a brute-force
  lattice deposit elsewhere);
* charge conservation with light ions and a beam: div E - rho keeps its
  value to round-off;
* loading: neutral, and the plasma's kinetic energy is (1 + M) times the
  electrons' (gamma_R - 1) sum w.
"""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po
from test_oracle_particles import _aligned_residuals

pytestmark = pytest.mark.usefixtures("oracle_built")


def _plasma_box(nx, ny, nz, gR, M, ions=2, bc_z=1, ppc=(1, 1, 2)):
    w = pin.scaled(pin.workload(0), nx=nx, ny=ny, nz=nz, n_beam=0)
    w["frame"]["gamma_boost"] = gR
    w["undulator"]["kind"] = 0
    w["plasma"].update(n0_lab_cm3=1e16, ppc=list(ppc), ions=ions, ion_mass=M)
    return po.Sim(w, pin.beam_normals(0), bc_z=bc_z)


@pytest.mark.parametrize("M", [1.0, 4.0, 1836.15267343])
@pytest.mark.parametrize("gR", [1.0001, 20.0])
def test_two_species_plasma_frequency(M, gR):
    s = _plasma_box(2, 2, 8, gR, M)
    i = s.info()
    assert i.n_ions == i.n_plasma > 0 and i.ion_mass == M
    e, ion = s.particles(1, view=True), s.particles(2, view=True)
    A = 1e-6
    e["ux"][:] = A
    d = []
    for _ in range(12):
        d.append(e["ux"].mean() - ion["ux"].mean())
        s.step(1)
    d = np.array(d)
    cos_th = (d[2:] + d[:-2]) / (2 * d[1:-1])
    w2 = i.n0n * (1.0 + 1.0 / M)
    np.testing.assert_allclose(cos_th, 1 - 2 * (math.sqrt(w2) * i.dt / 2) ** 2, atol=1e-9)
    # the centre of momentum of the pair stays where it was
    cm = e["ux"].mean() + M * ion["ux"].mean()
    assert cm == pytest.approx(A, rel=1e-9)


def _window_case(ions, M=0.0, n=2048):
    w = pin.scaled(pin.workload(3), nx=8, ny=8, nz=48, n_beam=n, sigma=(2, 2, 6))
    w["beam"]["charge_C"] = 3e-9  # strong self fields
    w["plasma"].update(ions=ions, ion_mass=M)
    return po.Sim(w, pin.beam_normals(n, 1))


def test_heavy_ions_reproduce_immobile_ions():
    a = _window_case(1)
    b = _window_case(2, 1e10)
    for n in (5, 30):
        a.step(n - a.info().step)
        b.step(n - b.info().step)
        ia, ib = a.info(), b.info()
        assert ia.k0 == ib.k0 and ia.n_plasma == ib.n_plasma == ib.n_ions
        gross = ia.dt * ia.gR * ia.n0n * ia.bR * math.sqrt(a.nc)
        for f in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            fa, fb = a.field(f), b.field(f)
            scale = max(np.linalg.norm(fa), gross)
            assert np.linalg.norm(fa - fb) <= 1e-9 * scale, (n, f, np.linalg.norm(fa - fb) / scale)
        for sp in (0, 1):
            pa, pb = a.particles(sp), b.particles(sp)
            assert (pa["alive"] == pb["alive"]).all()
            for k in ("x", "y", "z", "ux", "uy", "uz"):
                assert np.abs(pa[k] - pb[k]).max() <= 1e-9 * max(1.0, np.abs(pa[k]).max()), (n, sp, k)
        # the ions ride the lattice: alive exactly where the electrons' sheets are
        pi = b.particles(2)
        assert (pi["alive"] == b.particles(1)["alive"]).all()
        assert np.abs(pi["ux"]).max() < 1e-9 and np.abs(pi["uy"]).max() < 1e-9


def test_light_ions_conserve_charge():
    s = _window_case(2, 25.0)
    rho_scale = np.abs(s.rho(2)).max() + np.abs(s.rho(1)).max()
    res = _aligned_residuals(s, 30)
    assert max(res) < 1e-12 * rho_scale, res
    ion = s.particles(2)
    al = ion["alive"] == 1
    assert np.abs(ion["ux"][al]).max() > 1e-9  # the ions did respond to the beam


def test_mobile_ion_loading_is_neutral_and_heavy():
    M = 1836.15267343
    s = _plasma_box(4, 4, 48, 20.0, M, bc_z=0)
    i = s.info()
    e = s.particles(1)
    assert i.n_ions == i.n_plasma
    ion = s.particles(2)
    for k in ("x", "y", "z", "ux", "uy", "uz", "w"):
        assert (ion[k] == e[k]).all(), k
    re_, ri = s.rho(2), s.rho(4)
    assert np.abs(re_ + ri).max() <= 1e-14 * np.abs(re_).max()
    d = s.diag(1.0)
    ke = (e["w"] * (math.sqrt(1 + i.uR**2) - 1)).sum()
    assert d["kin_plasma"] == pytest.approx((1 + M) * ke, rel=1e-12)
    # the default mass is the proton's
    assert _plasma_box(2, 2, 8, 5.0, 0.0).info().ion_mass == M
