"""GPU parity of the mg0 Poisson solver with the oracle, through the C ABI:
uniform periodic meshes of several shapes (power-of-two and not, so that the
coarsest level ranges from 2^3 to 6 x 4 x 2 cells), random right-hand sides
and initial guesses, V(2,2) and V(1,3) cycles.  Bar: phi within 1e-12 of the
oracle relative to max |phi| (the solver's means and norms are fixed-order
two-stage sums, the oracle's sequential ones, so the last bits may differ);
residual histories within 1e-10 of the initial residual.  Also: a discrete
eigenmode solved to round-off on the GPU alone, bitwise repeatability, and
the refusals (batch, outflow; refined meshes take mg0 on the octree,
test_gpu_mgc.py)."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd._lib import AmrError
from paper_1810_01319_amd.mesh import Mesh

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-mg] {msg}", file=sys.stderr, flush=True)


def to_global(m, blocks):
    """[n_leaves, N, N, N] (z, y, x) block arrays -> [nz, ny, nx] grid."""
    N = m.N
    R = m.params["root"]
    g = np.empty((R[2] * N, R[1] * N, R[0] * N))
    for s, (l, i, j, k) in enumerate(m.keys):
        g[k * N:(k + 1) * N, j * N:(j + 1) * N, i * N:(i + 1) * N] = blocks[s]
    return g


def to_blocks(m, g):
    N = m.N
    out = np.empty((m.nleaf, N, N, N))
    for s, (l, i, j, k) in enumerate(m.keys):
        out[s] = g[k * N:(k + 1) * N, j * N:(j + 1) * N, i * N:(i + 1) * N]
    return out


def solve_gpu(m, f, phi0, ncycles, nu1, nu2):
    fb = torch.from_numpy(to_blocks(m, f)).to(m.device)
    pb = torch.from_numpy(to_blocks(m, phi0)).to(m.device)
    r = m.poisson_solve(fb, pb, ncycles, nu1, nu2)
    torch.cuda.synchronize()
    return to_global(m, pb.cpu().numpy()), r.cpu().numpy()


@pytest.mark.parametrize("root,N,nu", [((2, 2, 2), 8, (2, 2)), ((2, 2, 2), 32, (2, 2)), ((3, 2, 1), 16, (2, 2)),
                                        ((1, 1, 1), 8, (1, 3)), ((4, 2, 2), 16, (1, 3))])
def test_mg_matches_oracle(root, N, nu):
    spec = I.MeshSpec(root=root, block_cells=N)
    m = Mesh(**spec.kwargs())
    shape = (root[2] * N, root[1] * N, root[0] * N)
    say(f"mg root={root} N={N} grid={shape} levels={O.mg_levels(shape)} nu={nu}")
    rng = np.random.default_rng(N + sum(root))
    f = rng.standard_normal(shape)
    phi0 = 0.01 * rng.standard_normal(shape)
    h = spec.dx(0)
    pg, rg = solve_gpu(m, f, phi0, 6, *nu)
    po, ro = O.mg_solve(f, h, 6, *nu, phi0=phi0)
    scale = np.max(np.abs(po))
    err = np.max(np.abs(pg - po)) / scale
    say(f"mg: max rel diff {err:.2e}, bitwise fraction {np.mean(pg == po):.4f}, residual {ro[0]:.3e} -> {ro[-1]:.3e}")
    assert err <= 1e-12
    assert np.max(np.abs(rg - ro)) <= 1e-10 * ro[0]
    assert abs(np.mean(pg)) < 1e-13 * scale


def test_mg_discrete_eigenmode_on_gpu():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=16)
    m = Mesh(**spec.kwargs())
    n = 32
    h = spec.dx(0)
    c = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    kx, ky, kz = 2 * np.pi, 4 * np.pi, 2 * np.pi
    s = np.sin(kx * x) * np.sin(ky * y) * np.cos(kz * z)
    lam = -(4.0 / h ** 2) * (np.sin(0.5 * kx * h) ** 2 + np.sin(0.5 * ky * h) ** 2 + np.sin(0.5 * kz * h) ** 2)
    pg, rg = solve_gpu(m, lam * s, np.zeros_like(s), 25, 2, 2)
    assert np.max(np.abs(pg - s)) < 1e-11
    assert rg[-1] < 1e-11 * rg[0]


def test_mg_is_repeatable_bitwise():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=16)
    m = Mesh(**spec.kwargs())
    f = np.random.default_rng(1).standard_normal((32, 32, 32))
    a, ra = solve_gpu(m, f, np.zeros_like(f), 4, 2, 2)
    b, rb = solve_gpu(m, f, np.zeros_like(f), 4, 2, 2)
    assert np.array_equal(a, b) and np.array_equal(ra, rb)


def test_mg_refusals():
    bad = [I.MeshSpec(root=(2, 2, 2), block_cells=8, bc="outflow")]
    for spec in bad:
        m = Mesh(**spec.kwargs())
        with pytest.raises(AmrError):
            m.poisson_workspace()
    bm = Mesh.batch([I.MeshSpec(root=(2, 2, 2), block_cells=8).kwargs()] * 2)
    with pytest.raises(AmrError):
        bm.poisson_workspace()


def test_mg_full_size_eigenmode():
    """The benchmark's grid (16^3 roots x 32^3 cells = 512^3, 8 levels, the
    XCD row bands in use at every level with ny >= 8): a discrete eigenmode of
    the 7-point operator, built on the GPU in the block layout, is solved to
    round-off, and the mean stays zero."""
    spec = I.MeshSpec(root=(16, 16, 16), block_cells=32)
    m = Mesh(**spec.kwargs())
    N, h = 32, spec.dx(0)
    say(f"mg full size 512^3, {m.nleaf} leaves")
    keys = torch.as_tensor(np.asarray(m.keys), device=m.device)
    r = (torch.arange(N, device=m.device, dtype=torch.float64) + 0.5)
    x = ((keys[:, 1, None] * N).double() + r[None, :]) * h  # [leaf, N] along x
    y = ((keys[:, 2, None] * N).double() + r[None, :]) * h
    z = ((keys[:, 3, None] * N).double() + r[None, :]) * h
    kx, ky, kz = 2 * np.pi, 4 * np.pi, 6 * np.pi
    s = (torch.cos(kz * z)[:, :, None, None] * torch.sin(ky * y)[:, None, :, None]
         * torch.sin(kx * x)[:, None, None, :]).contiguous()
    lam = -(4.0 / h ** 2) * (np.sin(0.5 * kx * h) ** 2 + np.sin(0.5 * ky * h) ** 2 + np.sin(0.5 * kz * h) ** 2)
    f = (lam * s).contiguous()
    phi = torch.zeros_like(s)
    res = m.poisson_solve(f, phi, 20)
    torch.cuda.synchronize()
    err = float((phi - s).abs().max())
    rr = res.cpu().numpy()
    say(f"mg full size: max |phi - s| {err:.2e}, residual {rr[0]:.3e} -> {rr[-1]:.3e}, mean {float(phi.mean()):.1e}")
    assert err < 1e-10
    assert rr[-1] < 1e-9 * rr[0]
    assert abs(float(phi.mean())) < 1e-13
