"""Differentiable hydro steps: a torch.autograd.Function whose forward runs K
steps of the HIP path keeping what each step's adjoint needs (the step's
sweep inputs, or a checkpoint of the state before it), and whose backward
runs the hand-written adjoint of each step (HIP kernels, dt of every step
frozen at its forward value) from the last step to the first."""
from __future__ import annotations

import torch

GHOST = 3


def active_mask(mesh) -> torch.Tensor:
    g, N, M = GHOST, mesh.N, mesh.M
    m = torch.zeros((M, M, M), dtype=torch.bool, device=mesh.device)
    m[g:g + N, g:g + N, g:g + N] = True
    return m


class HydroSteps(torch.autograd.Function):
    """U_K = step_{K-1}(... step_0(U_0)); gradients flow to U_0's active cells.

    record=True keeps, for every step, its refreshed input and the inputs of
    its second and third sweeps (three states per step, no copies: the
    forward writes them as it goes) and the step's floor-reset count; the
    backward then recomputes nothing.  record=False keeps one checkpoint per
    step and recomputes the refresh and the first two sweeps in the backward.
    Ghost cells of the returned state are unspecified with record=True."""

    @staticmethod
    def forward(ctx, U0, mesh, steps: int, start: int = 0, record: bool = True):
        U = U0.detach().clone()
        saved, dts = [], []
        for k in range(start, start + steps):
            dt = mesh.dt_tensor()
            if record:
                S1, S2, Uo = (torch.empty_like(U) for _ in range(3))
                floors = torch.empty(1, dtype=torch.int64, device=U.device)
                mesh.step_record(U, dt, S1, S2, Uo, floors, k)
                saved.append((U, S1, S2, floors))
                U = Uo
            else:
                saved.append(U.clone())
                mesh.step(U, dt, k)
            dts.append(dt)
        ctx.mesh, ctx.saved, ctx.dts, ctx.start, ctx.record = mesh, saved, dts, start, record
        return U

    @staticmethod
    def backward(ctx, gU):
        mesh = ctx.mesh
        # ghost values of U_K influence nothing
        lam = torch.where(active_mask(mesh), gU.detach(), torch.zeros((), dtype=gU.dtype, device=gU.device))
        if ctx.record:
            scratch = mesh.adjoint_face_scratch()
            # every step's floor-reset count in one read: each sweep transpose
            # then launches only the kernel variant its step needs
            counts = torch.cat([s[3] for s in ctx.saved]).cpu().tolist()
            for i in range(len(ctx.saved) - 1, -1, -1):
                S0, S1, S2, floors = ctx.saved[i]
                mesh.step_adjoint_recorded(S0, S1, S2, ctx.dts[i], floors, lam, scratch, ctx.start + i,
                                           floors_host=int(counts[i]))
        else:
            scratch = mesh.adjoint_scratch()
            for i in range(len(ctx.saved) - 1, -1, -1):
                mesh.step_adjoint(ctx.saved[i], ctx.dts[i], lam, scratch, ctx.start + i)
        return lam, None, None, None, None


def run_steps(U0: torch.Tensor, mesh, steps: int, start: int = 0, record: bool = True) -> torch.Tensor:
    return HydroSteps.apply(U0, mesh, steps, start, record)


class ComovingSteps(torch.autograd.Function):
    """Comoving steps with given (dt, a, H) per step (dt a float64 device
    tensor of one element, a and H at the step's mid time), all frozen in the
    backward; every step keeps its refreshed input, its second and third
    sweeps' inputs, its state before the expansion sources and its floor
    count (four states per step)."""

    @staticmethod
    def forward(ctx, U0, mesh, schedule, start: int = 0):
        U = U0.detach().clone()
        saved = []
        for i, (dt, a, hubble) in enumerate(schedule):
            S1, S2, Up, Uo = (torch.empty_like(U) for _ in range(4))
            floors = torch.empty(1, dtype=torch.int64, device=U.device)
            mesh.step_comoving_record(U, dt, a, hubble, S1, S2, Up, Uo, floors, start + i)
            saved.append((U, S1, S2, Up, floors))
            U = Uo
        ctx.mesh, ctx.saved, ctx.schedule, ctx.start = mesh, saved, list(schedule), start
        return U

    @staticmethod
    def backward(ctx, gU):
        mesh = ctx.mesh
        lam = torch.where(active_mask(mesh), gU.detach(), torch.zeros((), dtype=gU.dtype, device=gU.device))
        scratch = mesh.adjoint_face_scratch()
        counts = torch.cat([s[4] for s in ctx.saved]).cpu().tolist()
        for i in range(len(ctx.saved) - 1, -1, -1):
            S0, S1, S2, Up, floors = ctx.saved[i]
            dt, a, hubble = ctx.schedule[i]
            mesh.step_comoving_adjoint_recorded(S0, S1, S2, Up, dt, a, hubble, floors, lam, scratch, ctx.start + i,
                                                floors_host=int(counts[i]))
        return lam, None, None, None


def run_comoving_steps(U0: torch.Tensor, mesh, schedule, start: int = 0) -> torch.Tensor:
    """schedule: one (dt device tensor, a, H) per step."""
    return ComovingSteps.apply(U0, mesh, schedule, start)


class DensityMisfit(torch.autograd.Function):
    """L = sum over leaf cells of w (rho - rho_target)^2; its backward writes
    dL/dU (2 w (rho - rho_target) on the active densities, zero elsewhere,
    ghosts included) in one pass instead of autograd's chain of slices."""

    @staticmethod
    def forward(ctx, U, w, target_rho):
        g = GHOST
        N = target_rho.shape[-1]
        d = U[:, 0, g:g + N, g:g + N, g:g + N] - target_rho
        ctx.save_for_backward(d, w)
        ctx.shape = U.shape
        return (w * d * d).sum()

    @staticmethod
    def backward(ctx, gL):
        d, w = ctx.saved_tensors
        g, N = GHOST, d.shape[-1]
        gU = torch.zeros(ctx.shape, dtype=d.dtype, device=d.device)
        gU[:, 0, g:g + N, g:g + N, g:g + N] = (2.0 * gL) * (w * d)
        return gU, None, None


def density_misfit(mesh, U: torch.Tensor, target_rho: torch.Tensor) -> torch.Tensor:
    """sum over leaf cells of (V_c / V_root) (rho_c - rho_target_c)^2."""
    lev = torch.as_tensor(mesh.keys[:, 0], device=U.device, dtype=torch.float64)
    w = torch.pow(0.125, lev)[:, None, None, None]
    return DensityMisfit.apply(U, w, target_rho)


class WithDensity(torch.autograd.Function):
    """A copy of the state U with the active densities replaced by rho; the
    gradient flows to rho only (U is data), without materialising a gradient
    for the rest of the state."""

    @staticmethod
    def forward(ctx, U, rho):
        g, N = GHOST, rho.shape[-1]
        out = U.detach().clone()
        out[:, 0, g:g + N, g:g + N, g:g + N] = rho
        return out

    @staticmethod
    def backward(ctx, gU):
        g = GHOST
        N = gU.shape[-1] - 2 * g
        return None, gU[:, 0, g:g + N, g:g + N, g:g + N].contiguous()


def with_density(U: torch.Tensor, rho: torch.Tensor) -> torch.Tensor:
    return WithDensity.apply(U, rho)
