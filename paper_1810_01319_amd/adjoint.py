"""Differentiable hydro steps: a torch.autograd.Function whose forward runs K
steps of the HIP path keeping a checkpoint of the state before every step,
and whose backward runs the hand-written adjoint of each step (HIP kernels,
dt of every step frozen at its forward value) from the last step to the
first."""
from __future__ import annotations

import torch

GHOST = 3


def active_mask(mesh) -> torch.Tensor:
    g, N, M = GHOST, mesh.N, mesh.M
    m = torch.zeros((M, M, M), dtype=torch.bool, device=mesh.device)
    m[g:g + N, g:g + N, g:g + N] = True
    return m


class HydroSteps(torch.autograd.Function):
    """U_K = step_{K-1}(... step_0(U_0)); gradients flow to U_0's active cells."""

    @staticmethod
    def forward(ctx, U0, mesh, steps: int, start: int = 0):
        U = U0.detach().clone()
        ckpts, dts = [], []
        for k in range(start, start + steps):
            ckpts.append(U.clone())
            dt = mesh.dt_tensor()
            mesh.step(U, dt, k)
            dts.append(dt)
        ctx.mesh, ctx.ckpts, ctx.dts, ctx.start = mesh, ckpts, dts, start
        return U

    @staticmethod
    def backward(ctx, gU):
        mesh = ctx.mesh
        lam = gU.detach().clone().contiguous()
        lam[:, :, ~active_mask(mesh)] = 0.0  # ghost values of U_K influence nothing
        scratch = mesh.adjoint_scratch()
        for i in range(len(ctx.ckpts) - 1, -1, -1):
            mesh.step_adjoint(ctx.ckpts[i], ctx.dts[i], lam, scratch, ctx.start + i)
        return lam, None, None, None


def run_steps(U0: torch.Tensor, mesh, steps: int, start: int = 0) -> torch.Tensor:
    return HydroSteps.apply(U0, mesh, steps, start)


def density_misfit(mesh, U: torch.Tensor, target_rho: torch.Tensor) -> torch.Tensor:
    """sum over leaf cells of (V_c / V_root) (rho_c - rho_target_c)^2."""
    g, N = GHOST, mesh.N
    rho = U[:, 0, g:g + N, g:g + N, g:g + N]
    lev = torch.as_tensor(mesh.keys[:, 0], device=U.device, dtype=torch.float64)
    w = torch.pow(0.125, lev)[:, None, None, None]
    return (w * (rho - target_rho) ** 2).sum()
