"""GPU tests of the hand-written adjoint.

* refresh transpose: <R v, w> = <v, R^T w> to 1e-12 (the refresh is
  positively homogeneous and piecewise linear, so R v = J_R(v) v exactly);
* one full step: sampled adjoint entries (all fields, interior and block
  edges) against coordinate-wise central differences of the forward step
  with dt fixed, for both sweep orders;
* the differentiation workload (4^3 roots of 32^3 cells, central octant
  refined once, 10 steps, density misfit to a target field): the autograd
  gradient against central differences on 32 random unit directions,
  |g.v - FD| <= 1e-6 |FD|;
* a tiny mesh: gradient entries against central differences of the FP64
  CPU oracle's forward (same dt sequence).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_01319_amd import adjoint as A
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd.mesh import Mesh

pytestmark = pytest.mark.gpu
G = 3


def say(msg):
    print(f"[gpu-adjoint] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU adjoint tests need an MI355X"


def amr_spec(N=8, seed=3):
    root = (2, 2, 2)
    return I.MeshSpec(root=root, block_cells=N, max_level=2, gamma=5 / 3,
                      refine=I.random_refine_list(root, 2, 4, seed))


def test_refresh_adjoint_dot_product():
    for N, seed in ((8, 3), (16, 4)):
        spec = amr_spec(N, seed)
        m = Mesh(**spec.kwargs())
        say(f"refresh dot test N={N} leaves={m.nleaf}")
        rng = np.random.default_rng(seed)
        v = rng.normal(size=(m.nleaf, 5, N, N, N))
        Uv = m.state_from_active(v)
        m.refresh(Uv)
        w = torch.from_numpy(rng.normal(size=tuple(Uv.shape))).to(Uv.device)
        lhs = float((Uv * w).sum())
        lam = w.clone()
        m.refresh_adjoint(Uv, lam)
        act = A.active_mask(m)
        assert float(lam[:, :, ~act].abs().max()) == 0.0
        rhs = float((torch.from_numpy(v).to(Uv.device) * lam[:, :, G:G + N, G:G + N, G:G + N]).sum())
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0), (lhs, rhs)


@pytest.mark.parametrize("k", [0, 1])
def test_step_adjoint_matches_differences(k):
    """Every sampled entry of the one-step adjoint against a coordinate-wise
    central difference, all five fields, interior and block-edge cells (the
    latter reach the ghost refresh and the coarse-fine reflux).  Random
    all-field directions are avoided: on smooth data with u near 0 they
    cross the tracing's wave-direction switches, where the step is not
    differentiable and no difference quotient converges."""
    spec = amr_spec(16, 5)
    m = Mesh(**spec.kwargs())
    N = 16
    U0 = m.state_from_active(I.smooth_state(spec, m.keys, seed=9, amp=0.2, vel=0.4))
    dt = m.dt_tensor()
    m.cfl_dt(U0, dt)
    rng = np.random.default_rng(10 + k)
    act = A.active_mask(m)
    lam0 = torch.zeros_like(U0)
    lam0[:, :, act] = torch.from_numpy(rng.normal(size=(m.nleaf, 5, N ** 3))).to(U0.device)
    lam = lam0.clone()
    m.step_adjoint(U0, dt, lam, m.adjoint_scratch(), k)

    def advance(U):
        W = U.clone()
        m.step_dt(W, dt, k)
        return W

    worst = 0.0
    edge = [0, 1, 2, N - 3, N - 2, N - 1]
    for t in range(40):
        f = t % 5
        s = int(rng.integers(m.nleaf))
        z, y, x = (int(v) for v in rng.integers(N, size=3))
        if t % 2:  # pin one coordinate to a block edge
            c = [z, y, x]
            c[int(rng.integers(3))] = edge[int(rng.integers(len(edge)))]
            z, y, x = c
        z, y, x = z + G, y + G, x + G
        h = 1e-6 * max(1.0, abs(float(U0[s, f, z, y, x])))
        Up, Um = U0.clone(), U0.clone()
        Up[s, f, z, y, x] += h
        Um[s, f, z, y, x] -= h
        # <lam0, S(U+h e) - S(U-h e)> summed cell by cell without cancellation
        fd = float(((advance(Up) - advance(Um)) * lam0).sum()) / (2 * h)
        ad = float(lam[s, f, z, y, x])
        err = abs(fd - ad) / max(1.0, abs(fd))
        worst = max(worst, err)
        assert err <= 1e-6, (k, f, s, z, y, x, ad, fd)
    say(f"step k={k}: 40 adjoint entries, worst relative error {worst:.3e}")


@pytest.mark.parametrize("record", [True, False])
def test_differentiation_workload_gradient_on_random_directions(record):
    spec = I.grf_spec(root=4, block_cells=32)
    m = Mesh(**spec.kwargs())
    assert m.nleaf == 120
    N = spec.block_cells
    say(f"grf workload: {m.nleaf} leaves")
    rho0 = torch.from_numpy(I.grf_density(spec, m.keys, seed=4)).to(m.device)
    target = torch.from_numpy(I.grf_density(spec, m.keys, seed=40)).to(m.device)
    base = m.state_from_active(I.grf_state(spec, m.keys, seed=4))
    steps = 10

    def state(rho):
        U = base.clone()
        U[:, 0, G:G + N, G:G + N, G:G + N] = rho
        return U

    r = rho0.clone().requires_grad_(True)
    UK = A.run_steps(state(r), m, steps, record=record)
    L = A.density_misfit(m, UK, target)
    L.backward()
    g = r.grad.detach()
    say(f"record={record}: loss {float(L.detach()):.6e}, |g| {float(g.norm()):.6e}")
    # frozen dt sequence of the forward
    dts = []
    U = state(rho0)
    for k in range(steps):
        dt = m.dt_tensor()
        m.step(U, dt, k)
        dts.append(dt)
    lev = torch.as_tensor(m.keys[:, 0], device=m.device, dtype=torch.float64)
    w = torch.pow(0.125, lev)[:, None, None, None]

    def run(rho):
        U = state(rho)
        for k in range(steps):
            m.step_dt(U, dts[k], k)
        return U[:, 0, G:G + N, G:G + N, G:G + N]

    rng = np.random.default_rng(41)
    # central differences: truncation O(eps^2) is far below the tolerance
    # at eps = 1e-4, while at 1e-6 the rounding of the ten-step forward
    # (about an ulp per cell, divided by eps) reaches a few 1e-6 relative
    # on directions whose projection onto g is small
    eps = 1e-4
    worst = 0.0
    for t in range(32):
        v = torch.from_numpy(rng.normal(size=tuple(rho0.shape))).to(m.device)
        v /= v.norm()
        rp, rm = run(rho0 + eps * v), run(rho0 - eps * v)
        # L(+) - L(-) summed cell by cell without cancellation
        fd = float((w * (rp - rm) * (rp + rm - 2 * target)).sum()) / (2 * eps)
        gv = float((g * v).sum())
        rel = abs(gv - fd) / max(abs(fd), 1e-30)
        worst = max(worst, rel)
        assert rel <= 1e-6, (t, gv, fd, rel)
    say(f"32 directions: worst relative error {worst:.3e}")


def test_tiny_mesh_gradient_against_oracle_differences():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=1, gamma=5 / 3, refine=[(0, 1, 0, 1)])
    m = Mesh(**spec.kwargs())
    N = 8
    assert m.nleaf == 15
    act0 = I.smooth_state(spec, m.keys, seed=77, amp=0.2, vel=0.3)
    target = torch.from_numpy(I.grf_density(spec, m.keys, seed=78, amplitude=0.05)).to(m.device)
    U0 = m.state_from_active(act0)
    rho0 = U0[:, 0, G:G + N, G:G + N, G:G + N].clone()
    steps = 2

    def state(rho):
        U = U0.clone()
        U[:, 0, G:G + N, G:G + N, G:G + N] = rho
        return U

    r = rho0.clone().requires_grad_(True)
    L = A.density_misfit(m, A.run_steps(state(r), m, steps), target)
    L.backward()
    g = r.grad.detach().cpu().numpy()
    # dt sequence (identical on the oracle: the forward is bitwise equal)
    dts = []
    U = state(rho0)
    for k in range(steps):
        dt = m.dt_tensor()
        m.step(U, dt, k)
        dts.append(float(dt.cpu()[0]))
    om = O.OracleMesh(**spec.kwargs())
    idx = {tuple(k): s for s, k in enumerate(om.keys)}
    perm = np.array([idx[tuple(k)] for k in m.keys])
    lev = m.keys[:, 0]
    w = 0.125 ** lev
    tgt = target.cpu().numpy()

    def oracle_rho(act):
        o = np.empty_like(act)
        o[perm] = act
        om.set_active(o)
        for k in range(steps):
            om.step_dt(k, dts[k])
        return om.active()[perm][:, 0]

    rng = np.random.default_rng(79)
    cells = [(int(rng.integers(m.nleaf)), *map(int, rng.integers(N, size=3))) for _ in range(48)]
    h = 1e-6
    scale = np.abs(g).max()
    worst = 0.0
    for (s, z, y, x) in cells:
        ap, am = act0.copy(), act0.copy()
        ap[s, 0, z, y, x] += h
        am[s, 0, z, y, x] -= h
        rp, rm = oracle_rho(ap), oracle_rho(am)
        fd = float(np.sum(w[:, None, None, None] * (rp - rm) * (rp + rm - 2 * tgt))) / (2 * h)
        err = abs(fd - g[s, z, y, x]) / max(abs(fd), 1e-3 * scale)
        worst = max(worst, err)
        assert err <= 1e-6, ((s, z, y, x), g[s, z, y, x], fd)
    say(f"tiny mesh: 48 oracle difference entries, worst relative error {worst:.3e}")


@pytest.mark.parametrize("case", ["smooth", "floors"])
def test_recorded_adjoint_equals_recomputing_adjoint(case):
    """Adjoint from the recorded sweep inputs against the adjoint that
    recomputes them from a checkpoint (which always handles floors), on a
    smooth AMR state and on a state whose steps reset floors; the recompute
    leaves the mesh's floor-reset count unchanged; the recorded count passed
    from the host selects the same transpose kernels."""
    if case == "smooth":
        spec = amr_spec(16, 6)
        m = Mesh(**spec.kwargs())
        act = I.smooth_state(spec, m.keys, seed=12, amp=0.2, vel=0.4)
    else:
        spec = I.MeshSpec(root=(4, 1, 1), block_cells=8, gamma=1.4, p_floor=1e-3, rho_floor=1e-6)
        m = Mesh(**spec.kwargs())
        x = I.cell_centres(spec, m.keys)[0]
        u = np.where(x < 0.5, -4.0, 4.0)
        act = I.conserved(1.4, np.ones_like(x), u, 0.0, 0.0, np.full(x.shape, 2e-3))
    N = spec.block_cells
    say(f"recorded vs recomputing adjoint: {case}, {m.nleaf} leaves")
    U = m.state_from_active(act)
    rng = np.random.default_rng(13)
    act_mask = A.active_mask(m)
    total = 0
    for k in range(3):
        ck = U.clone()
        dt = m.dt_tensor()
        S1, S2, Uo = (torch.empty_like(U) for _ in range(3))
        floors = torch.empty(1, dtype=torch.int64, device=U.device)
        m.step_record(U, dt, S1, S2, Uo, floors, k)
        total += int(floors.cpu()[0])
        lam0 = torch.zeros_like(U)
        lam0[:, :, act_mask] = torch.from_numpy(rng.normal(size=(m.nleaf, 5, N ** 3))).to(U.device)
        la, lb, lc = lam0.clone(), lam0.clone(), lam0.clone()
        m.step_adjoint_recorded(U, S1, S2, dt, floors, la, m.adjoint_face_scratch(), k)
        # the count read on the host launches only the matching kernels: same result
        m.step_adjoint_recorded(U, S1, S2, dt, floors, lc, m.adjoint_face_scratch(), k,
                                floors_host=int(floors.cpu()[0]))
        before = m.floor_count()
        m.step_adjoint(ck, dt, lb, m.adjoint_scratch(), k)
        assert m.floor_count() == before
        scale = float(lb.abs().max())
        err = float((la - lb).abs().max()) / scale
        say(f"step {k}: floors {int(floors.cpu()[0])}, max |recorded - recomputed| / max {err:.3e}")
        assert err <= 1e-13, (k, err)
        # the refresh transpose adds with atomics: equal up to their order
        assert float((la - lc).abs().max()) <= 1e-15 * scale
        U = Uo
    if case == "floors":
        assert total > 0


def frozen_oracle_gradient(spec, keys_gpu, act0_gpu_order, tgt_gpu_order, steps, eps=1e-5, stride=1, label=""):
    """The oracle's frozen-branch central differences of the density misfit
    (its own dt sequence and branch choices) at every stride-th active
    density, in the GPU's leaf order."""
    om = O.OracleMesh(**spec.kwargs())
    idx = {tuple(k): s for s, k in enumerate(om.keys)}
    perm = np.array([idx[tuple(k)] for k in keys_gpu])  # GPU leaf -> oracle leaf
    act = np.empty_like(act0_gpu_order)
    act[perm] = act0_gpu_order
    tgt = np.empty_like(tgt_gpu_order)
    tgt[perm] = tgt_gpu_order
    om.set_active(act)
    probe = O.OracleMesh(**spec.kwargs())
    probe.set_active(act)
    dts = [probe.step(k) for k in range(steps)]
    N3 = spec.block_cells ** 3
    gpu_flat = np.arange(0, len(keys_gpu) * N3, stride)
    oracle_flat = perm[gpu_flat // N3] * N3 + gpu_flat % N3
    out = np.empty(gpu_flat.size)
    chunk = 1024
    for c0 in range(0, gpu_flat.size, chunk):
        out[c0:c0 + chunk], _ = om.frozen_fd_density_grad(0, dts, tgt, eps, idx=oracle_flat[c0:c0 + chunk])
        say(f"{label} oracle frozen-branch differences {min(c0 + chunk, gpu_flat.size)}/{gpu_flat.size}")
    return gpu_flat, out


@pytest.mark.parametrize("case,stride", [("smooth", 1), ("shocked", 4)])
def test_tiny_mesh_gradient_against_frozen_branch_oracle(case, stride):
    """Every density entry (every fourth on the shocked state) of the
    adjoint gradient on the tiny two-level mesh (2^3 roots of 8^3, one root
    refined, 2 steps) against the oracle's central differences with its dt
    sequence and all discrete choices frozen at the unperturbed run's
    (eps 1e-5; at 1e-6 the rounding of the perturbed runs' whole-mesh
    density differences alone reaches 1e-9 of the gradient's scale): relative
    error <= 1e-6 of max(|difference|, 1e-3 max).  Measured on the smooth
    state: 1.0e-7."""
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=1, gamma=5 / 3, refine=[(0, 1, 0, 1)])
    m = Mesh(**spec.kwargs())
    N, steps = 8, 2
    if case == "smooth":
        act0 = I.smooth_state(spec, m.keys, seed=77, amp=0.2, vel=0.3)
    else:
        x, y, z = I.cell_centres(spec, m.keys)
        rho = np.where(x < 0.5, 1.0, 0.125) * (1 + 0.05 * np.sin(2 * np.pi * y))
        act0 = I.conserved(spec.gamma, rho, 0.1 * np.sin(2 * np.pi * z), 0.0, 0.0, np.where(x < 0.5, 1.0, 0.1))
    tgt = I.grf_density(spec, m.keys, seed=78, amplitude=0.05)
    target = torch.from_numpy(tgt).to(m.device)
    U0 = m.state_from_active(act0)
    r = U0[:, 0, G:G + N, G:G + N, G:G + N].clone().requires_grad_(True)
    U = U0.clone()
    U[:, 0, G:G + N, G:G + N, G:G + N] = r
    A.density_misfit(m, A.run_steps(U, m, steps), target).backward()
    g = r.grad.detach().cpu().numpy().reshape(-1)
    say(f"tiny mesh {case}: adjoint gradient done")
    flat, fd = frozen_oracle_gradient(spec, m.keys, act0, tgt, steps, stride=stride, label=case)
    scale = np.abs(fd).max()
    err = np.abs(g[flat] - fd) / np.maximum(np.abs(fd), 1e-3 * scale)
    say(f"tiny mesh {case}: {flat.size} entries, worst relative error {err.max():.3e}")
    assert err.max() <= 1e-6, (flat[np.argmax(err)], g[flat][np.argmax(err)], fd[np.argmax(err)])
