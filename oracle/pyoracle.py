"""ctypes wrapper of the CPU oracle.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It maps a workload dictionary (see ``picinputs``) onto the
oracle's C configuration and exposes its arrays as numpy views.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc_z", C.c_int32),
        ("dx_m", C.c_double), ("cfl", C.c_double), ("dt_override", C.c_double),
        ("gamma_boost", C.c_double), ("window_beta", C.c_double),
        ("n_beam", C.c_int64),
        ("charge_C", C.c_double), ("gamma_lab", C.c_double), ("espread", C.c_double),
        ("sigma", C.c_double * 3), ("emit", C.c_double * 2), ("zc_cells", C.c_double),
        ("n0_cm3", C.c_double), ("pl_z0_m", C.c_double), ("pl_len_m", C.c_double), ("pl_ramp_m", C.c_double),
        ("ppc", C.c_int32 * 3), ("ions", C.c_int32),
        ("und_kind", C.c_int32), ("pusher", C.c_int32),
        ("K", C.c_double), ("lu_m", C.c_double), ("und_z0_m", C.c_double), ("und_len_m", C.c_double),
        ("und_ramp_periods", C.c_double),
        ("hK", C.c_double), ("hn0", C.c_double),
        ("ion_mass", C.c_double),
    ]


class Info(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("dt", "gR", "bR", "uR", "bw", "nref_m3", "wbeam", "ku", "B0", "n0n", "zoff", "F_elong", "sig_zlab")] + \
               [(n, C.c_int64) for n in
                ("k0", "step", "n_beam", "n_plasma", "sheet_lo", "sheet_hi", "beam_lost", "plasma_removed",
                 "n_ions")] + [("ion_mass", C.c_double), ("window_x", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("n_beam_alive", C.c_double), ("wsum", C.c_double),
                ("mean", C.c_double * 3), ("sigma", C.c_double * 3), ("umean", C.c_double * 3),
                ("usigma", C.c_double * 3), ("emit", C.c_double * 2),
                ("b1_re", C.c_double), ("b1_im", C.c_double), ("b2_re", C.c_double), ("b2_im", C.c_double),
                ("b1_abs", C.c_double), ("b2_abs", C.c_double),
                ("field_energy", C.c_double), ("kin_beam", C.c_double), ("kin_plasma", C.c_double)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else float(v)
        return out


_LIBS = {}


def lib(complex_step: bool = False):
    key = bool(complex_step)
    if key not in _LIBS:
        path = os.path.join(HERE, "liborc_cs.so" if key else "liborc.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (oracle/build.py)
            _b.build()
        L = C.CDLL(path)
        R = C.c_void_p
        L.orc_new.restype = R
        L.orc_new.argtypes = [C.POINTER(Config), C.c_void_p]
        L.orc_free.argtypes = [R]
        L.orc_step.argtypes = [R, C.c_int32]
        L.orc_set_window_beta.argtypes = [R, C.c_double]
        L.orc_set_fading_charge.argtypes = [R, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]
        L.orc_info.argtypes = [R, C.POINTER(Info)]
        L.orc_diag.argtypes = [R, C.c_double, C.POINTER(Diag)]
        L.orc_field.restype = C.c_void_p
        L.orc_field.argtypes = [R, C.c_int32]
        L.orc_particles.restype = C.c_void_p
        L.orc_particles.argtypes = [R, C.c_int32, C.c_int32]
        L.orc_alive.restype = C.c_void_p
        L.orc_alive.argtypes = [R, C.c_int32]
        L.orc_rho.argtypes = [R, C.c_int32, C.c_void_p]
        L.orc_gauss.argtypes = [R, C.c_void_p]
        L.orc_zero_J.argtypes = [R]
        L.orc_b_half.argtypes = [R]
        L.orc_e_update.argtypes = [R]
        L.orc_deposit.argtypes = [R, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_ion_current.argtypes = [R, C.c_double, C.c_double, C.c_int32]
        L.orc_gather.argtypes = [R, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_push.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        for f in ("orc_beta",):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double]
        for f in ("orc_elongation", "orc_doppler"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double, C.c_double]
        L.orc_fel_wavelength.restype = C.c_double
        L.orc_fel_wavelength.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_lab_to_boosted.argtypes = [C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_state_len.restype = C.c_int64
        L.orc_state_len.argtypes = [R]
        L.orc_get_state.argtypes = [R, C.c_void_p]
        L.orc_set_state.argtypes = [R, C.c_void_p]
        L.orc_adjoint_step.argtypes = [R, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_grad_bunching.argtypes = [C.POINTER(Config), C.c_void_p, C.c_int32, C.c_double, C.c_void_p]
        L.orc_loss_bunching.argtypes = [C.POINTER(Config), C.c_void_p, C.c_int32, C.c_double, C.c_void_p]
        if not key:
            L.orc_shape.restype = C.c_double
            L.orc_shape.argtypes = [C.c_double]
            L.orc_dshape.restype = C.c_double
            L.orc_dshape.argtypes = [C.c_double]
        _LIBS[key] = L
    return _LIBS[key]


def make_config(w: dict, *, pusher: int | None = None, bc_z: int = 0, dt_override: float = 0.0,
                hK: float = 0.0, hn0: float = 0.0) -> Config:
    g, fr, b, p, u = w["grid"], w["frame"], w["beam"], w["plasma"], w["undulator"]
    c = Config()
    c.nx, c.ny, c.nz, c.bc_z = g["nx"], g["ny"], g["nz"], bc_z
    c.dx_m, c.cfl, c.dt_override = g["dx_m"], g["cfl"], dt_override
    c.gamma_boost, c.window_beta = fr["gamma_boost"], fr["window_beta"]
    c.n_beam = b["n_macro"]
    c.charge_C, c.gamma_lab, c.espread = b["charge_C"], b["gamma_lab"], b["rel_energy_spread_rms"]
    c.sigma[:] = b["sigma_cells"]
    c.emit[:] = b["emit_n_m"]
    c.zc_cells = b["z_center_cells"]
    c.n0_cm3, c.pl_z0_m, c.pl_len_m, c.pl_ramp_m = p["n0_lab_cm3"], p["z_start_lab_m"], p["length_lab_m"], p["ramp_up_lab_m"]
    c.ppc[:] = p["ppc"]
    c.ions = p["ions"]
    c.ion_mass = p.get("ion_mass", 0.0)
    c.und_kind = u["kind"]
    c.K, c.lu_m, c.und_z0_m, c.und_len_m, c.und_ramp_periods = (u["K"], u["period_lab_m"], u["z_start_lab_m"],
                                                               u["length_lab_m"], u["entrance_ramp_periods"])
    c.pusher = (1 if u["kind"] != 0 else 0) if pusher is None else pusher
    c.hK, c.hn0 = hK, hn0
    return c


FIELD_NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz")


class Sim:
    """One oracle simulation.  ``complex_step`` selects the complex build."""

    def __init__(self, w: dict, normals: np.ndarray, *, complex_step: bool = False, **cfg_kw):
        self.L = lib(complex_step)
        self.cs = complex_step
        self.dtype = np.complex128 if complex_step else np.float64
        self.w = w
        self.cfg = make_config(w, **cfg_kw)
        self.normals = np.ascontiguousarray(normals, dtype=np.float64)
        assert self.normals.shape == (6, w["beam"]["n_macro"])
        self.h = self.L.orc_new(C.byref(self.cfg), self.normals.ctypes.data)
        if not self.h:
            raise RuntimeError("orc_new failed")

    def close(self):
        if self.h:
            self.L.orc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        self.L.orc_step(self.h, int(n))

    def set_window_beta(self, beta: float):
        """The window moves at beta (units of c) from the current step on."""
        self.L.orc_set_window_beta(self.h, float(beta))

    def info(self) -> Info:
        i = Info()
        self.L.orc_info(self.h, C.byref(i))
        return i

    def diag(self, kb: float) -> dict:
        d = Diag()
        self.L.orc_diag(self.h, float(kb), C.byref(d))
        return d.as_dict()

    @property
    def nc(self):
        return self.cfg.nx * self.cfg.ny * self.cfg.nz

    def _view(self, ptr, n, dtype):
        """Writable view of n elements at ptr; valid only while this simulation lives."""
        if n == 0:
            return np.zeros(0, dtype)
        buf = (C.c_char * (n * np.dtype(dtype).itemsize)).from_address(ptr)
        return np.frombuffer(buf, dtype=dtype, count=n)

    def field(self, name) -> np.ndarray:
        """Writable view (nz, ny, nx) of a field in logical window order (valid while the simulation lives)."""
        k = FIELD_NAMES.index(name) if isinstance(name, str) else int(name)
        v = self._view(self.L.orc_field(self.h, k), self.nc, self.dtype)
        return v.reshape(self.cfg.nz, self.cfg.ny, self.cfg.nx)

    def gather(self, X) -> tuple:
        """E, B at absolute boosted position X (cells) from the current field arrays."""
        X = np.ascontiguousarray(X, self.dtype)
        E = np.zeros(3, self.dtype)
        B = np.zeros(3, self.dtype)
        self.L.orc_gather(self.h, X.ctypes.data, E.ctypes.data, B.ctypes.data)
        return E, B

    def b_half(self):
        """One half step of the Yee B update on the current fields."""
        self.L.orc_b_half(self.h)

    def particles(self, species: int, view: bool = False) -> dict:
        """Particle arrays of a species (0 beam, 1 plasma electrons, 2 mobile
        ions): copies, or writable views valid while the simulation lives when
        ``view`` is set."""
        i = self.info()
        n = (i.n_beam, i.n_plasma, i.n_ions)[species]
        out = {}
        for k, name in enumerate(("x", "y", "z", "ux", "uy", "uz", "w")):
            out[name] = self._view(self.L.orc_particles(self.h, species, k), n, self.dtype)
        out["alive"] = self._view(self.L.orc_alive(self.h, species), n, np.int32)
        return out if view else {k: v.copy() for k, v in out.items()}

    def rho(self, mask: int = 7) -> np.ndarray:
        r = np.zeros(self.nc, self.dtype)
        self.L.orc_rho(self.h, mask, r.ctypes.data)
        return r.reshape(self.cfg.nz, self.cfg.ny, self.cfg.nx)

    def gauss(self) -> np.ndarray:
        r = np.zeros(self.nc, self.dtype)
        self.L.orc_gauss(self.h, r.ctypes.data)
        return r.reshape(self.cfg.nz, self.cfg.ny, self.cfg.nx)

    def _no_mobile_ions(self):
        if self.cfg.ions == 2:
            raise NotImplementedError("the oracle's adjoint does not model mobile ions")

    def state(self) -> np.ndarray:
        self._no_mobile_ions()
        v = np.zeros(self.L.orc_state_len(self.h), self.dtype)
        self.L.orc_get_state(self.h, v.ctypes.data)
        return v

    def set_state(self, v: np.ndarray):
        self._no_mobile_ions()
        v = np.ascontiguousarray(v, dtype=self.dtype)
        assert v.size == self.L.orc_state_len(self.h)
        self.L.orc_set_state(self.h, v.ctypes.data)

    def adjoint_step(self, lam_in: np.ndarray, n_out: int):
        self._no_mobile_ions()
        lam_in = np.ascontiguousarray(lam_in, dtype=self.dtype)
        out = np.zeros(n_out, self.dtype)
        gK = np.zeros(1, self.dtype)
        gn = np.zeros(1, self.dtype)
        self.L.orc_adjoint_step(self.h, lam_in.ctypes.data, out.ctypes.data, gK.ctypes.data, gn.ctypes.data)
        return out, gK[0], gn[0]


def grad_bunching(w: dict, normals: np.ndarray, nsteps: int, kb: float, **cfg_kw):
    """(L, K dL/dK, n0 dL/dn0) from the oracle's stored-state adjoint."""
    L = lib(False)
    cfg = make_config(w, **cfg_kw)
    if cfg.ions == 2:
        raise NotImplementedError("the oracle's adjoint does not model mobile ions")
    nrm = np.ascontiguousarray(normals, dtype=np.float64)
    out = np.zeros(3)
    L.orc_grad_bunching(C.byref(cfg), nrm.ctypes.data, int(nsteps), float(kb), out.ctypes.data)
    return out


def loss_bunching(w: dict, normals: np.ndarray, nsteps: int, kb: float, *, complex_step=False, **cfg_kw):
    L = lib(complex_step)
    cfg = make_config(w, **cfg_kw)
    nrm = np.ascontiguousarray(normals, dtype=np.float64)
    out = np.zeros(2)
    L.orc_loss_bunching(C.byref(cfg), nrm.ctypes.data, int(nsteps), float(kb), out.ctypes.data)
    return out


def push(pusher: int, qm: float, dt: float, u, E, B):
    L = lib(False)
    u = np.ascontiguousarray(u, np.float64)
    E = np.ascontiguousarray(E, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    out = np.zeros(3)
    L.orc_push(pusher, qm, dt, u.ctypes.data, E.ctypes.data, B.ctypes.data, out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Initial self-field of the beam (boosted frame, t' = 0).
#
# Section 1 transforms fields between frames.  The beam moves along z at
# beta_b in the boosted frame; in its own rest frame its field is
# electrostatic, E_r = -grad phi_r with lap phi_r = -rho_r.  Transforming with
# z_r = gamma_b z', rho' = gamma_b rho_r, phi' = gamma_b phi_r gives, on the
# boosted grid,
#     (d_xx + d_yy + d_zz / gamma_b^2) phi' = -rho',
#     E'_perp = -grad_perp phi',  E'_z = -d_z phi' / gamma_b^2,  B' = beta_b z x E'.
# Discretisation (the Yee grid of the step): phi and rho on nodes, E on edges,
# B on faces; second differences D+D-; periodic in x and y like the field
# solver, phi = 0 one plane beyond each z face.  Then div E = rho holds node
# by node.  The state between steps is (E^n, B^(n-1/2)): the pattern moves at
# beta_b, so B is taken at t' = -dt/2, i.e. beta_b z x E displaced by
# beta_b dt / 2 along z (linear interpolation between the planes).
def relativistic_poisson(rho: np.ndarray, gamma_b: float, beta_b: float, dt: float, open_top: bool = False):
    """phi, (Ex, Ey, Ez), (Bx, By, Bz) for node charge rho of shape (nz, ny, nx).

    The transverse operator is diagonalised with a 2D FFT (library primitive);
    each (kx, ky) column is then a tridiagonal system in z, solved by plain
    forward elimination and back substitution.  phi = 0 one plane below the
    back face, and one plane above the top face -- or, with open_top, equal
    there to the top plane's (no field through the top face)."""
    rho = np.asarray(rho, dtype=np.float64)
    nz, ny, nx = rho.shape
    g2 = 1.0 / (gamma_b * gamma_b)
    R = np.fft.fft2(rho, axes=(1, 2))
    lam = (-4.0 * np.sin(np.pi * np.arange(ny) / ny) ** 2)[:, None] + \
          (-4.0 * np.sin(np.pi * np.arange(nx) / nx) ** 2)[None, :]
    # rows: g2 phi[l-1] + (lam - 2 g2) phi[l] + g2 phi[l+1] = -R[l], phi[-1] = phi[nz] = 0
    diag = lam - 2.0 * g2
    cp = np.empty((nz, ny, nx))
    dp = np.empty((nz, ny, nx), dtype=complex)
    cp[0] = g2 / diag
    dp[0] = -R[0] / diag
    for l in range(1, nz):
        m = (diag + g2 if open_top and l == nz - 1 else diag) - g2 * cp[l - 1]
        cp[l] = g2 / m
        dp[l] = (-R[l] - g2 * dp[l - 1]) / m
    ph = np.empty_like(dp)
    ph[nz - 1] = dp[nz - 1]
    for l in range(nz - 2, -1, -1):
        ph[l] = dp[l] - cp[l] * ph[l + 1]
    phi = np.real(np.fft.ifft2(ph, axes=(1, 2)))
    above = phi[-1:] if open_top else np.zeros((1, ny, nx))
    up = np.concatenate([phi[1:], above], axis=0)  # phi one plane up
    Ex = -(np.roll(phi, -1, axis=2) - phi)
    Ey = -(np.roll(phi, -1, axis=1) - phi)
    Ez = -(up - phi) * g2
    w = 0.5 + 0.5 * beta_b * dt  # weight of the upper plane at z = l + 1/2 + beta_b dt / 2
    zero = np.zeros((1, ny, nx))
    Exu = np.concatenate([Ex[1:], zero], axis=0)
    Eyu = np.concatenate([Ey[1:], zero], axis=0)
    Bx = -beta_b * ((1.0 - w) * Ey + w * Eyu)
    By = beta_b * ((1.0 - w) * Ex + w * Exu)
    Bz = np.zeros_like(phi)
    return phi, (Ex, Ey, Ez), (Bx, By, Bz)


def init_neutraliser(sim: "Sim", fade_s: float):
    """Section 3's neutralising ions: a charge equal and opposite to the beam's at t' = 0, faded
    linearly to zero over fade_s seconds (boosted frame) while the fields start from zero; its
    field is the beam charge's electrostatic field (the relativistic Poisson problem at rest)
    with no field through the top face and none on the top plane, which the front face holds
    at zero."""
    _, E, _ = relativistic_poisson(np.real(sim.rho(1)), 1.0, 0.0, sim.info().dt, open_top=True)
    Ex, Ey, Ez = (e.copy() for e in E)
    Ex[-1] = 0.0  # the front face keeps its tangential E at zero: none of the field may sit there
    Ey[-1] = 0.0
    # the charge is the field's divergence on the nodes (x, y periodic, E_z below plane 0 left
    # out, as the oracle's Gauss residual does): the beam's, except on the top plane
    rho = (Ex - np.roll(Ex, 1, axis=2)) + (Ey - np.roll(Ey, 1, axis=1)) + Ez
    rho[1:] -= Ez[:-1]
    arrs = [np.ascontiguousarray(a, dtype=sim.dtype) for a in (rho, Ex, Ey, Ez)]
    sim.L.orc_set_fading_charge(sim.h, *[a.ctypes.data for a in arrs], float(fade_s))
    return arrs


def beam_mean_beta(sim: "Sim") -> float:
    """Mean boosted beta_z of the live beam particles (equal weights)."""
    p = sim.particles(0)
    al = p["alive"] == 1
    ux, uy, uz = (np.real(p[k][al]) for k in ("ux", "uy", "uz"))
    return float(np.mean(uz / np.sqrt(1.0 + ux * ux + uy * uy + uz * uz)))


def init_beam_fields(sim: "Sim"):
    """Overwrite the simulation's (zero) initial fields with the beam's self-field."""
    beta = beam_mean_beta(sim)
    gamma = 1.0 / np.sqrt((1.0 - beta) * (1.0 + beta))
    _, E, B = relativistic_poisson(np.real(sim.rho(1)), gamma, beta, sim.info().dt)
    for name, v in zip(FIELD_NAMES, E + B):
        sim.field(name)[:] = v
    return beta, gamma


# ---------------------------------------------------------------------------
# The beam in the lab frame at one boosted instant (section 2; the inverse
# Lorentz transform of each particle's event and four-velocity, Eq. Lor1 and
# Lor2 read backwards): lab time gR (t' + bR (z' - z0)), lab position
# gR (z' - z0 + bR t'), transverse coordinates unchanged,
# u_z,lab = gR (u'_z + bR gamma'), gamma_lab = gR (gamma' + bR u'_z).
def lab_beam(sim: "Sim") -> dict:
    """Per beam slot: x, y, z_lab, t_lab, ux, uy, uz_lab, gamma_lab, alive."""
    i = sim.info()
    gR, bR, zc = i.gR, i.bR, i.zoff
    t = i.step * i.dt
    p = sim.particles(0)
    x, y, z, ux, uy, uz = (np.real(p[k]) for k in ("x", "y", "z", "ux", "uy", "uz"))
    g = np.sqrt(1.0 + ux * ux + uy * uy + uz * uz)
    return {"x": x, "y": y, "z": gR * (z - zc + bR * t), "t": gR * (t + bR * (z - zc)), "ux": ux, "uy": uy,
            "uz": gR * (uz + bR * g), "gamma": gR * (g + bR * uz), "alive": p["alive"],
            "w": np.real(p["w"]), "z_boost": z, "uz_boost": uz}


# Groups of the beam by slices of boosted z' and u'_z (section 2, Eq. DT: a
# slice dz' of the beam at one boosted instant spans lab times gR bR dz').
LAB_GROUP_FIELDS = ("count", "w", "w_t", "t_min", "t_max", "w_z", "w_zz", "w_x", "w_xx", "w_y", "w_yy", "w_ux",
                    "w_uxux", "w_uy", "w_uyuy", "w_gamma")


def lab_groups(sim: "Sim", z_lo: float, dz: float, nz: int, u_lo: float = -1e300, du: float = 1e308,
               nu: int = 1) -> np.ndarray:
    """(nz * nu, 16) table, group iz * nu + iu holding the live beam particles with
    floor((z' - z_lo) / dz) = iz and floor((u'_z - u_lo) / du) = iu; columns
    LAB_GROUP_FIELDS (min/max +inf/-inf for an empty group)."""
    L = lab_beam(sim)
    iz = np.floor((L["z_boost"] - z_lo) / dz)
    iu = np.floor((L["uz_boost"] - u_lo) / du)
    out = np.zeros((nz * nu, 16))
    out[:, 3], out[:, 4] = np.inf, -np.inf
    for a in range(nz):
        for b in range(nu):
            m = (L["alive"] == 1) & (iz == a) & (iu == b)
            w = L["w"][m]
            row = out[a * nu + b]
            row[0] = m.sum()
            row[1] = w.sum()
            row[2] = (w * L["t"][m]).sum()
            if m.any():
                row[3], row[4] = L["t"][m].min(), L["t"][m].max()
            for c, k in zip((5, 7, 9, 11, 13), ("z", "x", "y", "ux", "uy")):
                row[c] = (w * L[k][m]).sum()
                row[c + 1] = (w * L[k][m] ** 2).sum()
            row[15] = (w * L["gamma"][m]).sum()
    return out


# Lab-frame probe (section 2: relating the boosted frame's data to the lab).
# A particle at boosted position z' and time t' is at lab time
# t = gR (t' + bR (z' - z0)) and lab position z_lab = gR (z' - z0 + bR t'),
# z0 being the boosted-grid offset of the beam centre (lab origin at the beam
# centre at lab time 0).  Over a step a particle moves on a straight line, so
# the instant its lab time passes T is found on that line and its lab
# position taken there.  Every beam particle is sampled once.
def lab_probe(sim: "Sim", nsteps: int, t_lab: float, k_lab: float) -> dict:
    """Advance nsteps steps; return the sums over sampled beam particles of w,
    w cos(k z_lab), w sin(k z_lab), w z_lab, w z_lab^2, and per beam slot the
    sampled lab x, z (NaN where not sampled)."""
    i = sim.info()
    gR, bR, dt, z0c = i.gR, i.bR, i.dt, i.zoff
    p = sim.particles(0)
    n = len(p["z"])
    xs = np.full(n, np.nan)
    zs = np.full(n, np.nan)
    for _ in range(nsteps):
        t0 = sim.info().step * dt
        x0, z0, a0 = np.real(p["x"]), np.real(p["z"]), p["alive"] == 1
        sim.step(1)
        p = sim.particles(0)
        x1, z1, a1 = np.real(p["x"]), np.real(p["z"]), p["alive"] == 1
        t1 = t0 + dt
        tl0 = gR * (t0 + bR * (z0 - z0c))
        tl1 = gR * (t1 + bR * (z1 - z0c))
        m = a0 & a1 & np.isnan(zs) & (tl0 <= t_lab) & (t_lab < tl1)
        f = (t_lab - tl0[m]) / (tl1[m] - tl0[m])
        zc = z0[m] + f * (z1[m] - z0[m])
        tc = t0 + f * dt
        zs[m] = gR * (zc - z0c + bR * tc)
        xs[m] = x0[m] + f * (x1[m] - x0[m])
    w = np.real(sim.particles(0)["w"])
    s = ~np.isnan(zs)
    ws, zz = w[s], zs[s]
    return {"w": ws.sum(), "c": (ws * np.cos(k_lab * zz)).sum(), "s": (ws * np.sin(k_lab * zz)).sum(),
            "z": (ws * zz).sum(), "zz": (ws * zz * zz).sum(), "x_lab": xs, "z_lab": zs}
