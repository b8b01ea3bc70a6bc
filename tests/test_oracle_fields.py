"""Oracle pins for the Yee field solver [sec. 1, Eq. Max1, Max2] and the absorbing z faces."""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

pytestmark = pytest.mark.usefixtures("oracle_built")


def _empty(nx, ny, nz, **kw):
    w = pin.scaled(pin.workload(0), nx=nx, ny=ny, nz=nz, n_beam=0)
    w["undulator"]["kind"] = 0
    w["frame"]["window_beta"] = 0.0
    return po.Sim(w, pin.beam_normals(0), **kw)


def _theta(dt, ks):
    return 2 * math.asin(dt * math.sqrt(sum(math.sin(k / 2) ** 2 for k in ks)))


@pytest.mark.parametrize("comp,ka,kb", [("Ez", (2, 1, 0), None), ("Ey", (1, 0, 2), None), ("Ex", (0, 2, 1), None)])
def test_yee_single_mode_dispersion(comp, ka, kb):
    """A transverse Fourier mode with B^{-1/2} = 0 evolves as
    E^n = E^0 cos((n + 1/2) theta) / cos(theta / 2), sin^2(theta/2) = dt^2 sum_d sin^2(k_d/2)."""
    nx, ny, nz = 16, 8, 12
    s = _empty(nx, ny, nz, bc_z=1)
    k = (2 * math.pi * ka[0] / nx, 2 * math.pi * ka[1] / ny, 2 * math.pi * ka[2] / nz)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    # the chosen component is uniform along its own axis -> discretely divergence free
    E0 = np.cos(k[0] * ii + k[1] * jj + k[2] * kk)
    s.field(comp)[:] = E0
    dt = s.info().dt
    th = _theta(dt, k)
    N = 37
    s.step(N)
    expect = E0 * math.cos((N + 0.5) * th) / math.cos(th / 2)
    np.testing.assert_allclose(s.field(comp), expect, atol=1e-12)
    for other in ("Ex", "Ey", "Ez"):
        if other != comp:
            assert np.abs(s.field(other)).max() < 1e-13


def test_div_b_stays_zero():
    nx, ny, nz = 8, 8, 8
    s = _empty(nx, ny, nz, bc_z=1)
    rng = np.random.default_rng(0)
    for c in ("Ex", "Ey", "Ez"):
        s.field(c)[:] = rng.normal(size=(nz, ny, nx))
    s.step(25)
    Bx, By, Bz = s.field("Bx"), s.field("By"), s.field("Bz")
    div = (np.roll(Bx, -1, 2) - Bx) + (np.roll(By, -1, 1) - By) + (np.roll(Bz, -1, 0) - Bz)
    assert np.abs(div).max() < 1e-12 * max(1.0, np.abs(Bx).max())


@pytest.mark.parametrize("direction", [-1, +1])
def test_mur_exact_absorption_1d_magic_step(direction):
    """With no transverse variation and c dt = dx, Yee is an exact shift and the
    first-order Mur face (coefficient (dt-1)/(dt+1) = 0) absorbs exactly."""
    nz = 64
    s = _empty(1, 1, nz, dt_override=1.0)
    z = np.arange(nz, dtype=float)
    f = lambda x: np.exp(-((x - (40 if direction < 0 else 20)) / 3.0) ** 2)  # noqa: E731
    s.field("Ex")[:, 0, 0] = f(z)
    # By at k + 1/2, time -1/2: -f(k) for a wave toward -z, f(k + 1) toward +z
    s.field("By")[:, 0, 0] = -f(z) if direction < 0 else f(z + 1)
    s.field("By")[nz - 1, 0, 0] = 0.0
    shift = 10
    s.step(shift)  # exact translation while the pulse is inside
    np.testing.assert_allclose(s.field("Ex")[5:nz - 5, 0, 0], f(z[5:nz - 5] - direction * shift), atol=1e-13)
    s.step(60)
    assert np.abs(s.field("Ex")).max() < 1e-12
    assert np.abs(s.field("By")).max() < 1e-12


def test_mur_3d_normal_incidence_reflection_small():
    nx, ny, nz = 4, 4, 96
    s = _empty(nx, ny, nz)
    dt = s.info().dt
    z = np.arange(nz, dtype=float)
    f = np.exp(-((z - 60) / 6.0) ** 2)
    s.field("Ex")[:] = f[:, None, None]
    # approximate -z travelling wave: By(k+1/2, -dt/2) = -f(k + 1/2 - dt/2)
    s.field("By")[:] = -np.exp(-((z + 0.5 - 0.5 * dt - 60) / 6.0) ** 2)[:, None, None]
    e0 = (s.field("Ex") ** 2).sum()
    s.step(int(100 / dt))
    e1 = (s.field("Ex") ** 2).sum()
    assert e1 < 1e-3 * e0


def test_moving_window_with_plasma_is_stable():
    """A small random field seeded into a cold plasma streaming through a window
    that moves at nearly c must not grow.  (A static-face Mur condition applied
    at the moving front face made a face mode grow ~1e5-fold per 20 steps.)"""
    w = pin.scaled(pin.adjoint_subcase(), nx=8, ny=8, nz=64, n_beam=16)
    w["beam"]["charge_C"] = 1e-30
    s = po.Sim(w, pin.beam_normals(16))
    assert s.info().bw > 0.99
    rng = np.random.default_rng(3)
    for f in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        s.field(f)[:] = 1e-12 * rng.standard_normal(s.field(f).shape)
    e = []
    for _ in range(8):
        s.step(20)
        e.append(s.diag(1.0)["field_energy"])
    assert max(e) < 1e-19, e


def test_field_energy_of_three_modes_closed_form():
    """The diagnostics' field energy 1/2 sum(E^2 + B^2) of three superposed
    Fourier modes of different polarisation.  A mode with E^0 = A cos(k.x) and
    B^(-1/2) = 0 has, by the Yee recurrence, E^n = A cos((n + 1/2) theta) /
    cos(theta/2) and a B^(n-1/2) field of amplitude A sin(n theta) /
    cos(theta/2) in units where its grid sum of squares is nc/2 like E's, so
    field_energy(n) = sum_modes nc A^2 (cos^2((n + 1/2) theta) + sin^2(n theta))
    / (4 cos^2(theta/2)); the modes are orthogonal, so no cross terms.  A
    missing factor 1/2, a missing component or a B at the wrong time level
    fails."""
    nx, ny, nz = 16, 8, 12
    s = _empty(nx, ny, nz, bc_z=1)
    dt = s.info().dt
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    modes = [("Ez", (2, 1, 0), 1.3), ("Ey", (1, 0, 2), 0.7), ("Ex", (0, 2, 1), 2.1)]
    thetas = []
    for comp, ka, amp in modes:
        k = (2 * math.pi * ka[0] / nx, 2 * math.pi * ka[1] / ny, 2 * math.pi * ka[2] / nz)
        s.field(comp)[:] = amp * np.cos(k[0] * ii + k[1] * jj + k[2] * kk)
        thetas.append(_theta(dt, k))
    nc = nx * ny * nz

    def expect(n):
        return sum(nc * amp**2 * (math.cos((n + 0.5) * th) ** 2 + math.sin(n * th) ** 2) / (4 * math.cos(th / 2) ** 2)
                   for (_, _, amp), th in zip(modes, thetas))

    done = 0
    for n in (0, 1, 5, 17, 40):
        s.step(n - done)
        done = n
        fe = s.diag(1.0)["field_energy"]
        assert fe == pytest.approx(expect(n), rel=1e-12), n
    # B carries a sizeable share of the energy at n = 40
    assert any(abs(math.sin(40 * th)) > 0.3 for th in thetas)


def test_yee_discrete_energy_invariant():
    """In a periodic vacuum box the Yee update keeps W^n = |E^n|^2 +
    B^(n-1/2) . B^(n+1/2) exactly (the scheme's discrete energy), whatever the
    initial fields; held to round-off over 60 steps from random fields."""
    nx, ny, nz = 8, 6, 10
    s = _empty(nx, ny, nz, bc_z=1)
    rng = np.random.default_rng(11)
    for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        s.field(c)[:] = rng.standard_normal((nz, ny, nx))

    def fields():
        return [s.field(c).copy() for c in ("Ex", "Ey", "Ez")], [s.field(c).copy() for c in ("Bx", "By", "Bz")]

    E, B = fields()
    ex0 = E[0].copy()
    W = []
    for _ in range(60):
        s.step(1)
        E1, B1 = fields()
        W.append(sum((e * e).sum() for e in E) + sum((b0 * b1).sum() for b0, b1 in zip(B, B1)))
        E, B = E1, B1
    W = np.array(W)
    assert np.abs(W - W[0]).max() <= 1e-12 * abs(W[0])
    # the fields did evolve: the invariant is not met trivially
    assert np.abs(E[0] - ex0).max() > 0.1 * np.abs(ex0).max()
