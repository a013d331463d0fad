"""GPU tests of the comoving step's adjoint (ComovingSteps over
amr_hydro_step_comoving_record / amr_hydro_step_comoving_adjoint_recorded).

* A static universe (a = 1, H = 0): the forward equals the plain step bit
  for bit and the gradient the plain recorded adjoint's to 1e-13 of its
  largest entry (the expansion transpose is then the identity and dt / 1 =
  dt; the refresh transpose adds with FP64 atomics, so two runs of either
  adjoint may differ in the last bits).
* A tiny two-level mesh, two comoving steps with an Einstein-de Sitter
  schedule: 100 sampled gradient entries of every field against central
  differences (eps 1e-5) of the FP64 oracle's comoving steps with the same
  dt, a and H and every discrete choice frozen at the unperturbed run's (the
  oracle's branch tape; plain differences straddle limiter and prolongation
  kinks within 1e-6 of some entries).  Loss: misfits of the final density, x
  momentum and energy, so the last expansion's transpose is reached
  directly; misfits keep the loss small, so that the rounding of the
  oracle's sums stays far below the differences.
* Expansion floors: a cold region whose internal energy the expansion
  lowers below the pressure floor, a warm one it does not; one step with a
  dt of 1e-6 of the CFL dt and c = (dt / 2) H = 0.4, so the expansion acts in
  full while the sweeps barely move the gas (their limiter and Riemann
  branches at the cold-warm jump then weigh nothing in the differences; a
  second step would start from cells sitting exactly at the floor, whose
  sweep floors any perturbation flips); the gradient along seeded directions
  against central differences of the GPU forward.
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
    print(f"[gpu-comoving-adjoint] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def tiny_spec(**kw):
    return I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=1, gamma=5 / 3, refine=[(0, 1, 0, 1)], **kw)


def eds_schedule(m, U, steps, t0, H0=2.0 / 3.0):
    """dt from the comoving CFL at a(t), then a and H at the mid time of an
    Einstein-de Sitter expansion a = (t / t1)^(2/3); returns the schedule
    (device dt, a_mid, H_mid) and the host dts, advancing a copy of U."""
    U = U.clone()
    t = t0
    sched, host = [], []
    for k in range(steps):
        a = (1.5 * H0 * t) ** (2.0 / 3.0)
        dt = m.dt_tensor()
        m.cfl_dt_comoving(U, a, dt)
        d = float(dt.cpu()[0])
        tm = t + 0.5 * d
        am = (1.5 * H0 * tm) ** (2.0 / 3.0)
        hm = 2.0 / (3.0 * tm)
        m.step_comoving(U, dt, k, am, hm)
        sched.append((dt, am, hm))
        host.append((d, am, hm))
        t += d
    return sched, host


def loss_terms(U, N, w, target):
    """sum of w ((rho - rho_t)^2 + 0.2 (m_x - m_t)^2 + 0.3 (E - E_t)^2) over
    active cells; target = (rho_t, m_t, E_t)."""
    g = G
    a = U[:, :, g:g + N, g:g + N, g:g + N]
    dr, dm, de = a[:, 0] - target[0], a[:, 1] - target[1], a[:, 4] - target[2]
    return (w * (dr * dr + 0.2 * (dm * dm) + 0.3 * (de * de))).sum()


def targets(act, seed, device):
    """(rho_t, m_t, E_t): the density, x momentum and energy of `act`,
    perturbed by seeded noise; near the loss's minimum when `act` is the
    final state, so the loss and the rounding of its sums stay small."""
    rng = np.random.default_rng(seed)
    rho_t = act[:, 0] * (1.0 + 0.01 * rng.standard_normal(act[:, 0].shape))
    m_t = act[:, 1] + 0.01 * rng.standard_normal(act[:, 1].shape)
    E_t = act[:, 4] * (1.0 + 0.001 * rng.standard_normal(act[:, 4].shape))
    return tuple(torch.from_numpy(np.ascontiguousarray(t)).to(device) for t in (rho_t, m_t, E_t))


def test_static_universe_gradient_equals_the_plain_adjoint():
    spec = tiny_spec()
    m = Mesh(**spec.kwargs())
    N = 8
    act0 = I.smooth_state(spec, m.keys, seed=81, amp=0.2, vel=0.3)
    U0 = m.state_from_active(act0)
    target = targets(act0, 82, m.device)
    w = torch.pow(0.125, torch.as_tensor(m.keys[:, 0], device=m.device, dtype=torch.float64))[:, None, None, None]
    steps = 3
    # the plain recorded path takes each step's dt from the CFL; a = 1 gives the same dt
    U = U0.clone()
    sched = []
    for k in range(steps):
        dt = m.dt_tensor()
        m.cfl_dt_comoving(U, 1.0, dt)
        m.step_comoving(U, dt, k, 1.0, 0.0)
        sched.append((dt, 1.0, 0.0))
    Ua = U0.clone().requires_grad_(True)
    loss_terms(A.run_steps(Ua, m, steps), N, w, target).backward()
    Ub = U0.clone().requires_grad_(True)
    Uc = A.run_comoving_steps(Ub, m, sched)
    loss_terms(Uc, N, w, target).backward()
    assert torch.equal(Uc.detach()[:, :, G:G + N, G:G + N, G:G + N], U[:, :, G:G + N, G:G + N, G:G + N])
    diff = float((Ua.grad - Ub.grad).abs().max())
    scale = float(Ua.grad.abs().max())
    say(f"static universe: comoving gradient against the plain adjoint, max difference {diff:.3e} of {scale:.3e}")
    assert diff <= 1e-13 * scale


@pytest.mark.parametrize("de", [False, True])
def test_tiny_mesh_gradient_against_oracle_differences(de):
    """With the dual-energy field (eta2 = 0.99, so that rho e keeps its own
    evolution) the loss also takes the misfit of rho e, and the entries
    sampled cover all six fields."""
    spec = tiny_spec(dual_energy=True, eta1=1e-3, eta2=0.99) if de else tiny_spec()
    m = Mesh(**spec.kwargs())
    N, steps = 8, 2
    act0 = I.smooth_state(spec, m.keys, seed=83, amp=0.2, vel=0.3)
    if de:
        act0 = I.with_internal_energy(act0)
        act0[:, 5] *= 1.0 + 0.01 * np.random.default_rng(88).standard_normal(act0[:, 5].shape)
    nf = act0.shape[1]
    U0 = m.state_from_active(act0)
    lev = m.keys[:, 0]
    wn = 0.125 ** lev
    w = torch.from_numpy(wn).to(m.device)[:, None, None, None]
    sched, host = eds_schedule(m, U0, steps, t0=0.9)
    say(f"schedule (dt, a, H): {host}")
    om = O.OracleMesh(**spec.kwargs())
    idx = {tuple(k): s for s, k in enumerate(om.keys)}
    perm = np.array([idx[tuple(k)] for k in m.keys])

    def oracle_final(act):
        o = np.empty_like(act)
        o[perm] = act
        om.set_active(o)
        for k, (d, am, hm) in enumerate(host):
            om.step_comoving(k, d, am, hm)
        return om.active()[perm]

    # targets near the oracle's own final state
    fin = oracle_final(act0)
    target = targets(fin, 84, m.device)
    tgt = [t.cpu().numpy() for t in target]
    ge_t = fin[:, 5] * (1.0 + 0.001 * np.random.default_rng(89).standard_normal(fin[:, 5].shape)) if de else None
    Ug = U0.clone().requires_grad_(True)
    Uc = A.run_comoving_steps(Ug, m, sched)
    L = loss_terms(Uc, N, w, target)
    if de:
        dge = Uc[:, 5, G:G + N, G:G + N, G:G + N] - torch.from_numpy(ge_t).to(m.device)
        L = L + 0.3 * (w * dge * dge).sum()
    L.backward()
    g = Ug.grad.detach().cpu().numpy()[:, :, G:G + N, G:G + N, G:G + N]
    wb = wn[:, None, None, None]

    O.tape_record()
    oracle_final(act0)
    O.tape_stop()

    def oracle_loss(act):
        O.tape_replay()
        a = oracle_final(act)
        O.tape_stop()
        dr, dm, dE = a[:, 0] - tgt[0], a[:, 1] - tgt[1], a[:, 4] - tgt[2]
        v = np.sum(wb * (dr * dr + 0.2 * (dm * dm) + 0.3 * (dE * dE)))
        if de:
            v += 0.3 * np.sum(wb * (a[:, 5] - ge_t) ** 2)
        return float(v)

    rng = np.random.default_rng(85)
    scale = np.abs(g).max()
    worst = 0.0
    for e in range(100):
        s, f = int(rng.integers(m.nleaf)), e % nf
        z, y, x = (int(v) for v in rng.integers(N, size=3))
        h = 1e-5 * max(1.0, abs(act0[s, f, z, y, x]))
        ap, am_ = act0.copy(), act0.copy()
        ap[s, f, z, y, x] += h
        am_[s, f, z, y, x] -= h
        fd = (oracle_loss(ap) - oracle_loss(am_)) / (2 * h)
        err = abs(fd - g[s, f, z, y, x]) / max(abs(fd), 1e-3 * scale)
        worst = max(worst, err)
        assert err <= 1e-6, ((s, f, z, y, x), g[s, f, z, y, x], fd)
    say(f"tiny mesh (dual energy {de}): 100 frozen-branch oracle difference entries over all fields, "
        f"worst relative error {worst:.3e}")


def test_expansion_floors_gradient_on_directions():
    p_floor = 1e-3
    spec = tiny_spec(p_floor=p_floor)
    m = Mesh(**spec.kwargs())
    N, steps = 8, 1
    x, y, z = I.cell_centres(spec, m.keys)
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * y) * np.cos(2 * np.pi * z)
    cold = x < 0.5
    p = np.where(cold, 3e-3, 1.0) * (1.0 + 0.05 * np.sin(2 * np.pi * z))
    act0 = I.conserved(spec.gamma, rho, 0.05 * np.sin(2 * np.pi * z), 0.02, 0.0, p)
    U0 = m.state_from_active(act0)
    w = torch.pow(0.125, torch.as_tensor(m.keys[:, 0], device=m.device, dtype=torch.float64))[:, None, None, None]
    target = targets(act0, 87, m.device)
    # a strong expansion: c = (dt / 2) H = 0.4, so the internal energy falls by
    # fe = 0.2 / 1.8 and the cold cells (p fe < p_floor) are floored
    dt0 = m.dt_tensor()
    m.cfl_dt_comoving(U0, 1.0, dt0)
    dt0 *= 1e-6
    d = float(dt0.cpu()[0])
    sched = [(dt0, 1.0, 0.8 / d)] * steps
    f0 = m.floor_count()
    U = U0.clone()
    for k in range(steps):
        m.step_comoving(U, dt0, k, 1.0, 0.8 / d)
    fired = m.floor_count() - f0
    say(f"expansion floors fired: {fired}")
    assert fired == int(cold.sum())  # every cold cell, nothing else

    def forward(V):
        V = V.clone()
        for k in range(steps):
            m.step_comoving(V, dt0, k, 1.0, 0.8 / d)
        return float(loss_terms(V, N, w, target))

    Ug = U0.clone().requires_grad_(True)
    loss_terms(A.run_comoving_steps(Ug, m, sched), N, w, target).backward()
    g = Ug.grad.detach()
    mask = A.active_mask(m)
    gen = torch.Generator(device="cpu").manual_seed(86)
    worst = 0.0
    for t in range(8):
        v = torch.randn(U0.shape, generator=gen, dtype=torch.float64).to(m.device)
        v = torch.where(mask, v, torch.zeros((), dtype=torch.float64, device=m.device))
        v = v * (1e-2 * U0.abs().clamp(min=1e-2))  # relative perturbation per entry
        eps = 1e-4
        fd = (forward(U0 + eps * v) - forward(U0 - eps * v)) / (2 * eps)
        gv = float((g * v).sum())
        err = abs(gv - fd) / abs(fd)
        worst = max(worst, err)
        assert err <= 1e-6, (t, gv, fd)
    say(f"expansion floors: 8 directions, worst relative error {worst:.3e}")
