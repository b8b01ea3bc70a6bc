"""Gradient of the final bunching factor w.r.t. undulator K and plasma density.

``bunching_loss(K, n0, ...)`` is a ``torch.autograd.Function``.  The forward
pass runs the simulation and keeps a full-state checkpoint every ``every``
steps; the backward pass walks the segments in reverse, restores each
checkpoint, recomputes and keeps the segment's states, then applies the
hand-written adjoint step (``pic_adjoint_step``) once per step.  The library
returns K dL/dK and n0 dL/dn0 (both parameters enter linearly: the external
field is proportional to K, every plasma weight to n0).

precision = PIC_FP64_PLAIN: FP64 forward in record mode, adjoint on it.
precision = PIC_FP32_SPLIT: FP32 forward (particles carry their FP64 record
slot); its recomputation is bitwise identical to the forward, and every
recomputed state is handed to an FP64 record context (``pic_state_to_fp64``),
where the adjoint step linearises about the FP32 trajectory.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import abi
from .sim import Sim


class BunchingLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, K, n0, w, normals, nsteps, every, bunch_period, precision, init_hook=None):
        w2 = copy.deepcopy(w)
        w2["undulator"]["K"] = float(K)
        w2["plasma"]["n0_lab_cm3"] = float(n0)
        nsteps = int(nsteps)
        fp64 = Sim(w2, normals, precision=abi.PIC_FP64_PLAIN, record=1, max_steps=nsteps + 2)
        sim = fp64 if precision == abi.PIC_FP64_PLAIN else Sim(w2, normals, precision=abi.PIC_FP32_SPLIT, record=1,
                                                                  max_steps=nsteps + 2)
        if init_hook is not None:
            init_hook(sim)
        ckpts = []
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append(sim.get_state())
            sim.step(1)
        if sim is not fp64:
            sim.export_to(fp64)
        lam = torch.zeros(fp64.lambda_len(), dtype=torch.float64, device=fp64.device)
        L = fp64.adjoint_seed(lam, bunch_period)
        ctx.sim, ctx.fp64, ctx.ckpts, ctx.lam = sim, fp64, ckpts, lam
        ctx.nsteps, ctx.every = nsteps, int(every)
        ctx.K, ctx.n0 = float(K), float(n0)
        return torch.tensor(L, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gL):
        sim, fp64, lam = ctx.sim, ctx.fp64, ctx.lam
        grad = np.zeros(2)
        buf = [sim.new_state_buffer() for _ in range(ctx.every)]
        for seg in reversed(range(len(ctx.ckpts))):
            a = seg * ctx.every
            b = min(a + ctx.every, ctx.nsteps)
            sim.set_state(ctx.ckpts[seg])
            for n in range(a, b):  # recompute the segment's states
                sim.get_state(buf[n - a])
                if n + 1 < b:
                    sim.step(1)
            for n in reversed(range(a, b)):
                sim.set_state(buf[n - a])
                if sim is not fp64:
                    sim.export_to(fp64)
                fp64.adjoint_step(lam, grad)
        g = float(gL)
        dK = grad[0] / ctx.K * g if ctx.K != 0 else 0.0
        dn = grad[1] / ctx.n0 * g if ctx.n0 != 0 else 0.0
        ctx.log_grads = grad.copy()
        return (torch.tensor(dK, dtype=torch.float64), torch.tensor(dn, dtype=torch.float64),
                None, None, None, None, None, None, None)


def bunching_loss(K, n0, w, normals, nsteps, every=50, bunch_period=20.0, precision=abi.PIC_FP64_PLAIN,
                  init_hook=None):
    """L = |b(2 pi / bunch_period)| after nsteps; differentiable in K and n0 (torch scalars).
    init_hook(sim), if given, is applied to the forward simulation before its first step (to
    perturb its initial particles, say); the gradient is the perturbed run's."""
    return BunchingLoss.apply(K, n0, w, normals, nsteps, every, bunch_period, precision, init_hook)


def bunching_grad(w, normals, nsteps, every=50, bunch_period=20.0, precision=abi.PIC_FP64_PLAIN, init_hook=None):
    """(L, K dL/dK, n0 dL/dn0) for the workload's own K and n0."""
    K = torch.tensor(w["undulator"]["K"], dtype=torch.float64, requires_grad=True)
    n0 = torch.tensor(w["plasma"]["n0_lab_cm3"], dtype=torch.float64, requires_grad=True)
    L = bunching_loss(K, n0, w, normals, nsteps, every, bunch_period, precision, init_hook)
    L.backward()
    return float(L.detach()), float(K.grad) * w["undulator"]["K"], float(n0.grad) * w["plasma"]["n0_lab_cm3"]
