"""Python handle on one simulation context.

PyTorch provides the device memory (one uint8 arena tensor, borrowed by the
library) and the stream; every step of the method runs in the HIP library
through the C-ABI.  There is no CPU fallback: without the built library or a
HIP device the constructor raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import abi

_ARRAYS = {"Ex": abi.PIC_A_EX, "Ey": abi.PIC_A_EY, "Ez": abi.PIC_A_EZ,
           "Bx": abi.PIC_A_BX, "By": abi.PIC_A_BY, "Bz": abi.PIC_A_BZ}


def _check(L, ctx, status, what):
    if status != abi.PIC_OK:
        msg = L.pic_last_error(ctx).decode() if ctx else ""
        raise abi.PicError(status, f"{what}: {msg}")


def query_layout(w: dict, **opts) -> abi.pic_layout:
    L = abi.load()
    s = abi.structs_from_workload(w, **opts)
    out = abi.pic_layout()
    st = L.pic_query_layout(*[C.byref(x) for x in s], C.byref(out))
    _check(L, None, st, "pic_query_layout")
    return out


def derive(w: dict, **opts) -> dict:
    L = abi.load()
    s = abi.structs_from_workload(w, **opts)
    out = abi.pic_derived()
    st = L.pic_derive(*[C.byref(x) for x in s], C.byref(out))
    _check(L, None, st, "pic_derive")
    return {n: (list(getattr(out, n)) if n == "tile" else getattr(out, n)) for n, _ in out._fields_}


class Sim:
    """A simulation on the current HIP device.

    precision: abi.PIC_FP64_PLAIN or abi.PIC_FP32_SPLIT.  normals: (6, n_macro)
    float64 standard normals the beam is sampled from (host array), or None: the
    library draws them on the device from seed (an integer option; see pic_beam).
    """

    def __init__(self, w: dict, normals: np.ndarray | None, *, device="cuda", stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the simulation runs only on the GPU")
        self.L = abi.load()
        self.w = w
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if normals is None:
            if "seed" not in opts:
                raise ValueError("Sim: give either the beam's normals or a seed to draw them on the device")
            self.normals = None
        else:
            self.normals = np.ascontiguousarray(normals, dtype=np.float64)
            assert self.normals.shape == (6, w["beam"]["n_macro"])
        structs = abi.structs_from_workload(w, stream=self.stream.cuda_stream, normals=self.normals, **opts)
        self.structs = structs
        lay = abi.pic_layout()
        _check(self.L, None, self.L.pic_query_layout(*[C.byref(x) for x in structs], C.byref(lay)),
               "pic_query_layout")
        self.layout = lay
        with torch.cuda.device(self.device):
            self.arena = torch.empty(int(lay.arena_bytes), dtype=torch.uint8, device=self.device)
        self.ctx = C.c_void_p()
        st = self.L.pic_init(*[C.byref(x) for x in structs], C.c_void_p(self.arena.data_ptr()),
                             C.c_uint64(self.arena.numel()), C.byref(self.ctx))
        _check(self.L, None, st, "pic_init")

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.L.pic_free(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(self.L, self.ctx, self.L.pic_step(self.ctx, int(n)), "pic_step")

    def timing(self, enable: bool):
        _check(self.L, self.ctx, self.L.pic_timing(self.ctx, int(bool(enable))), "pic_timing")

    def timing_read(self):
        ms = (C.c_double * 4)()
        n = (C.c_int64 * 4)()
        _check(self.L, self.ctx, self.L.pic_timing_read(self.ctx, ms, n), "pic_timing_read")
        return list(ms), list(n)

    def set_window_beta(self, beta: float):
        """Window speed (units of c) from the current step on."""
        _check(self.L, self.ctx, self.L.pic_set_window_beta(self.ctx, float(beta)), "pic_set_window_beta")

    def sync(self):
        _check(self.L, self.ctx, self.L.pic_sync(self.ctx), "pic_sync")

    def diag(self, mask=abi.PIC_DIAG_MOMENTS | abi.PIC_DIAG_BUNCHING | abi.PIC_DIAG_ENERGY, bunch_period=20.0,
             static=False) -> dict:
        """Diagnostics; static=True takes the allocation-free entry point (pic_diag_static)."""
        out = abi.pic_diag_out()
        f = self.L.pic_diag_static if static else self.L.pic_diag
        _check(self.L, self.ctx, f(self.ctx, mask, float(bunch_period), C.byref(out)),
               "pic_diag_static" if static else "pic_diag")
        return out.as_dict()

    def read(self, which) -> torch.Tensor:
        k = _ARRAYS.get(which, which)
        n = C.c_int64()
        _check(self.L, self.ctx, self.L.pic_read(self.ctx, k, None, C.byref(n)), "pic_read")
        alive = k in (abi.PIC_A_BEAM_ALIVE, abi.PIC_A_PLASMA_ALIVE)
        if k in (abi.PIC_A_BEAM, abi.PIC_A_PLASMA, abi.PIC_A_BEAM_LAB):
            t = torch.empty((8 if k == abi.PIC_A_BEAM_LAB else 7, max(n.value, 0)), dtype=torch.float64,
                            device=self.device)
        else:
            t = torch.empty(max(n.value, 0), dtype=torch.int32 if alive else torch.float64, device=self.device)
        if n.value:
            _check(self.L, self.ctx, self.L.pic_read(self.ctx, k, C.c_void_p(t.data_ptr()), C.byref(n)), "pic_read")
        return t

    def field(self, name) -> np.ndarray:
        g = self.w["grid"]
        return self.read(name).cpu().numpy().reshape(g["nz"], g["ny"], g["nx"])

    def particles(self, species: int) -> dict:
        a = self.read(abi.PIC_A_PLASMA if species else abi.PIC_A_BEAM).cpu().numpy()
        al = self.read(abi.PIC_A_PLASMA_ALIVE if species else abi.PIC_A_BEAM_ALIVE).cpu().numpy()
        out = {k: a[i] for i, k in enumerate(("x", "y", "z", "ux", "uy", "uz", "w"))}
        out["alive"] = al
        return out

    def write(self, which, arr: np.ndarray):
        k = _ARRAYS.get(which, which)
        t = torch.as_tensor(np.ascontiguousarray(arr, dtype=np.float64), device=self.device)
        n = t.shape[-1] if k in (abi.PIC_A_BEAM, abi.PIC_A_PLASMA) else t.numel()
        _check(self.L, self.ctx, self.L.pic_write(self.ctx, k, C.c_void_p(t.data_ptr()), n), "pic_write")

    def new_state_buffer(self) -> torch.Tensor:
        return torch.empty(int(self.layout.state_bytes), dtype=torch.uint8, device=self.device)

    def get_state(self, buf: torch.Tensor | None = None) -> torch.Tensor:
        buf = self.new_state_buffer() if buf is None else buf
        _check(self.L, self.ctx, self.L.pic_get_state(self.ctx, C.c_void_p(buf.data_ptr())), "pic_get_state")
        return buf

    def set_state(self, buf: torch.Tensor):
        _check(self.L, self.ctx, self.L.pic_set_state(self.ctx, C.c_void_p(buf.data_ptr())), "pic_set_state")

    def export_to(self, fp64: "Sim"):
        """Write this FP32 record-mode state into an FP64 record-mode simulation of the same workload."""
        _check(self.L, fp64.ctx, self.L.pic_state_to_fp64(self.ctx, fp64.ctx), "pic_state_to_fp64")

    def lab_probe(self, t_lab: float, k_lab: float):
        """Arm the lab-frame probe (lab time t_lab, wavenumber k_lab; NaN disarms) and clear its sums."""
        _check(self.L, self.ctx, self.L.pic_lab_probe(self.ctx, float(t_lab), float(k_lab)), "pic_lab_probe")

    def lab_probe_read(self) -> dict:
        """Sums over the sampled beam particles: w, w cos(k z_lab), w sin(k z_lab), w z_lab, w z_lab^2."""
        out = (C.c_double * 5)()
        _check(self.L, self.ctx, self.L.pic_lab_probe_read(self.ctx, out), "pic_lab_probe_read")
        return dict(zip(("w", "c", "s", "z", "zz"), list(out)))

    def beam_lab(self) -> dict:
        """The beam's lab-frame phase space at the current boosted time, each particle at its own lab time."""
        a = self.read(abi.PIC_A_BEAM_LAB).cpu().numpy()
        out = {k: a[i] for i, k in enumerate(("x", "y", "z", "t", "ux", "uy", "uz", "gamma"))}
        out["alive"] = self.read(abi.PIC_A_BEAM_ALIVE).cpu().numpy()
        return out

    def lab_groups(self, z_lo, dz, nz, u_lo=-1e300, du=1e308, nu=1) -> np.ndarray:
        """Lab-frame sums of the beam grouped by boosted z and u_z slices: (nz * nu, 16) array."""
        spec = abi.pic_lab_groups_spec(float(z_lo), float(dz), float(u_lo), float(du), int(nz), int(nu))
        out = torch.empty((nz * nu, abi.PIC_LAB_GROUP_VALUES), dtype=torch.float64, device=self.device)
        _check(self.L, self.ctx, self.L.pic_lab_groups(self.ctx, C.byref(spec), C.c_void_p(out.data_ptr())),
               "pic_lab_groups")
        return out.cpu().numpy()

    def lambda_len(self) -> int:
        return int(self.L.pic_lambda_len(self.ctx))

    def adjoint_seed(self, lam: torch.Tensor, bunch_period=20.0) -> float:
        loss = C.c_double()
        _check(self.L, self.ctx, self.L.pic_adjoint_seed_bunching(self.ctx, float(bunch_period),
                                                                  C.c_void_p(lam.data_ptr()), C.byref(loss)),
               "pic_adjoint_seed_bunching")
        return loss.value

    def adjoint_step(self, lam: torch.Tensor, grad: np.ndarray):
        g = (C.c_double * 2)(*grad)
        _check(self.L, self.ctx, self.L.pic_adjoint_step(self.ctx, C.c_void_p(lam.data_ptr()), g), "pic_adjoint_step")
        grad[0], grad[1] = g[0], g[1]


class WindowTracker:
    """Keeps the beam's centroid at its place in the moving window (section 3: a beam
    that slows down, e.g. in an undulator, drifts to the back of a window that keeps
    its speed; the window's speed is adjusted to the beam's).

    Call update() every ``every`` steps.  It sets the window speed to the centroid's
    mean velocity over the interval just ended plus the centroid's offset from its
    place in the window divided by the interval's duration, so the next interval takes
    the offset up; the place is where the centroid sat, relative to the window, when
    the tracker was made."""

    def __init__(self, sim: Sim, every: int):
        if every < 1:
            raise ValueError("every must be >= 1")
        d = sim.diag(abi.PIC_DIAG_MOMENTS)
        self.sim, self.every = sim, int(every)
        self.duration = every * derive(sim.w)["dt"]
        self.z_prev = d["mean"][2]
        self.place = d["mean"][2] - d["window_x"]

    def update(self) -> float:
        d = self.sim.diag(abi.PIC_DIAG_MOMENTS)
        z = d["mean"][2]
        velocity = (z - self.z_prev) / self.duration
        offset = z - d["window_x"] - self.place
        beta = min(max(velocity + offset / self.duration, 1e-6), 1.0)
        self.sim.set_window_beta(beta)
        self.z_prev = z
        return beta
