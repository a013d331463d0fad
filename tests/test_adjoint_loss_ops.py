"""The differentiable helpers around the adjoint (the density misfit and the
substitution of the active densities into a state) give the gradients of
their plain autograd expressions, on the CPU."""
import torch

from paper_1810_01319_amd import adjoint as A

G = A.GHOST


def test_density_misfit_and_with_density_match_autograd():
    gen = torch.Generator().manual_seed(3)
    nleaf, N = 3, 4
    M = N + 2 * G
    base = torch.randn((nleaf, 5, M, M, M), generator=gen, dtype=torch.float64)
    rho = torch.randn((nleaf, N, N, N), generator=gen, dtype=torch.float64)
    target = torch.randn((nleaf, N, N, N), generator=gen, dtype=torch.float64)
    w = torch.tensor([1.0, 0.125, 0.015625], dtype=torch.float64)[:, None, None, None]
    scale = torch.randn((nleaf, 5, M, M, M), generator=gen, dtype=torch.float64)

    def plain(r):
        U = base.clone()
        U[:, 0, G:G + N, G:G + N, G:G + N] = r
        V = U * scale  # stands in for the steps between the two helpers
        return (w * (V[:, 0, G:G + N, G:G + N, G:G + N] - target) ** 2).sum()

    def fused(r):
        V = A.with_density(base, r) * scale
        return A.DensityMisfit.apply(V, w, target)

    ra = rho.clone().requires_grad_(True)
    rb = rho.clone().requires_grad_(True)
    La, Lb = plain(ra), fused(rb)
    La.backward()
    Lb.backward()
    assert torch.allclose(La, Lb, rtol=1e-15, atol=0)
    assert torch.allclose(ra.grad, rb.grad, rtol=1e-14, atol=1e-300)
    # the substituted state carries the densities and nothing else changes
    S = A.with_density(base, rho)
    assert torch.equal(S[:, 0, G:G + N, G:G + N, G:G + N], rho)
    S[:, 0, G:G + N, G:G + N, G:G + N] = base[:, 0, G:G + N, G:G + N, G:G + N]
    assert torch.equal(S, base)
