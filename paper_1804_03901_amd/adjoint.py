"""Gradients of the time-integrated field energy through the VHS step.

J = sum_{n=1..N} sum_i (E_i^n)^2 dx dt, the rectangle rule for the time
integral of |E|^2 over the run.  ``FieldEnergy`` is a torch.autograd.Function
of the marker weights f_l: its forward runs the simulation on the GPU and its
backward returns dJ/df_l from the library's hand-written adjoint (reverse
gather, push, reconstruction, moments and spectral solve, with a checkpoint
every ``every`` steps).  The parameters of the initial distribution enter
only through f_l = f0(x_l, v_l; theta) (markers are placed independently of
theta), so writing f0 in torch makes torch carry dJ/df_l on to theta.
"""
from __future__ import annotations

import math
from typing import Optional

from . import avl, inputs


def f0_torch(w: "inputs.Workload", x, v, amplitudes=None, beam_drift=None):
    """The bump-on-tail f0 of ``w`` at markers (x, v) as a torch expression of
    the mode amplitudes (one per mode number) and the beam drift; values equal
    ``inputs.f0`` at the workload's own parameters."""
    import torch
    dt = torch.float64
    x = torch.as_tensor(x, dtype=dt)
    v = torch.as_tensor(v, dtype=dt).reshape(-1)
    k1 = 2.0 * math.pi / w.L
    phases = torch.as_tensor(inputs.mode_phases(w), dtype=dt, device=x.device)
    if amplitudes is None:
        amplitudes = torch.full((len(w.mode_numbers),), w.mode_amplitude, dtype=dt, device=x.device)
    dens = torch.ones_like(x)
    for k, mnum in enumerate(w.mode_numbers):
        dens = dens + amplitudes[k] * torch.cos(k1 * mnum * x + phases[k])
    g = torch.zeros_like(x)
    for p_i, p in enumerate(w.populations):
        u = p.drift[0]
        if p_i == 1 and beam_drift is not None:
            u = beam_drift
        s = p.vth[0]
        g = g + p.density * torch.exp(-((v - u) ** 2) / (2.0 * s * s)) / (s * math.sqrt(2.0 * math.pi))
    return dens * g


def _function():
    import torch

    class FieldEnergyFn(torch.autograd.Function):
        """J(f) for a fixed initial marker placement (x, v): forward runs the
        simulation; backward returns gJ * dJ/df from the adjoint sweep."""

        @staticmethod
        def forward(ctx, f, sim, x, v, nsteps, every):
            J, grad = energy_and_gradient(sim, x, v, f.detach(), nsteps, every, want_grad=f.requires_grad)
            ctx.save_for_backward(grad if grad is not None else torch.zeros_like(f))
            return J

        @staticmethod
        def backward(ctx, gJ):
            (grad,) = ctx.saved_tensors
            return gJ * grad, None, None, None, None, None

    return FieldEnergyFn


_FN = None


def field_energy(f, sim: "avl.Simulation", x, v, nsteps: int, every: int = 50):
    """J as a differentiable function of the marker weights f (torch, FP64)."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(f, sim, x, v, int(nsteps), int(every))


def energy_and_gradient(sim: "avl.Simulation", x, v, f, nsteps: int, every: int = 50, want_grad: bool = True):
    """J of a run from markers (x, v, f) (FP64, caller order) on the geometry
    of ``sim``, and dJ/df (same order) when ``want_grad`` (else None)."""
    import torch
    dev = sim.device
    x = torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous()
    v = torch.as_tensor(v, dtype=torch.float64, device=dev).reshape(-1).contiguous()
    f = torch.as_tensor(f, dtype=torch.float64, device=dev).contiguous()
    w = sim.w
    if not want_grad:
        fresh = avl.Simulation(w, x, v, f, precision=sim.precision, device=str(dev))
        try:
            d = fresh.step(nsteps).detach().cpu()
        finally:
            fresh.close()
        return torch.as_tensor(2.0 * w.c_p * w.dt * float(d[:, 0].sum()), dtype=torch.float64, device=dev), None
    nbytes = avl.avl_adjoint_workspace_bytes(sim.cfg, nsteps, every)
    if nbytes == 0:
        raise avl.AvlError(-6, "avl_adjoint_workspace_bytes")
    rec = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-rec.data_ptr()) % 256
    rec = rec[off:off + nbytes]
    J = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.empty_like(f)
    avl.avl_adjoint(sim.h, x, v, f, nsteps, every, rec, J, grad)
    return J[0], grad
