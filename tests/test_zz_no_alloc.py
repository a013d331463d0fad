"""The Poisson entry point that allocates nothing (amr_poisson_solve_static:
the library's fixed per-GPU buffer as the solver's workspace) against
amr_poisson_solve with a caller workspace, through the C ABI: two calls in a
row on the same GPU, the second on a smaller mesh (the buffer keeps the
first call's contents), bit for bit equal results and residual norms; a grid
whose workspace exceeds the buffer is refused and leaves phi unchanged."""
import sys

import numpy as np
import pytest
import torch

from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd._lib import AmrError
from paper_1810_01319_amd.mesh import Mesh

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-no-alloc] {msg}", file=sys.stderr, flush=True)


def solve_both(root, N, seed, ncycles=3):
    m = Mesh(**I.MeshSpec(root=root, block_cells=N).kwargs(), device="cuda:0")
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    f = torch.randn((m.nleaf, N, N, N), generator=g, dtype=torch.float64, device="cuda:0")
    phi0 = 0.1 * torch.randn((m.nleaf, N, N, N), generator=g, dtype=torch.float64, device="cuda:0")
    pa, pb = phi0.clone(), phi0.clone()
    ra = m.poisson_solve(f, pa, ncycles)
    rb = torch.empty(ncycles + 1, dtype=torch.float64, device="cuda:0")
    m.poisson_solve_static(f, pb, ncycles, resid=rb)
    torch.cuda.synchronize()
    return pa, pb, ra, rb


@pytest.mark.parametrize("first,second", [(((4, 4, 4), 32), ((2, 2, 2), 16))])
def test_static_workspace_solve_equals_the_workspace_solve(first, second):
    for (root, N), seed in ((first, 11), (second, 12)):
        say(f"root={root} N={N} seed={seed}")
        pa, pb, ra, rb = solve_both(root, N, seed)
        assert torch.equal(pa, pb), "potential differs from amr_poisson_solve"
        assert torch.equal(ra, rb), "residual norms differ from amr_poisson_solve"
        r = ra.cpu().numpy()
        assert r[-1] < 1e-2 * r[0]
        assert torch.count_nonzero(pa).item() > 0


def test_static_workspace_refuses_a_grid_above_its_size():
    say("refusal at 256^3")
    m = Mesh(**I.MeshSpec(root=(8, 8, 8), block_cells=32).kwargs(), device="cuda:0")
    f = torch.ones((m.nleaf, 32, 32, 32), dtype=torch.float64, device="cuda:0")
    phi = torch.zeros_like(f)
    with pytest.raises(AmrError, match="fixed buffer"):
        m.poisson_solve_static(f, phi, 1)
    torch.cuda.synchronize()
    assert torch.count_nonzero(phi).item() == 0
