"""GPU tests of the adjoint of the step with the dual-energy field rho e
(amr_hydro_step_record / amr_hydro_step_adjoint_recorded on a six-field
mesh, through adjoint.HydroSteps).

On the tiny two-level mesh (2^3 roots of 8^3, one root refined), two steps,
100 sampled gradient entries of all six fields against central differences
(eps 1e-5) of the FP64 oracle's dual-energy steps with the same dt sequence
and every discrete choice frozen at the unperturbed run's (the oracle's
branch tape).  Three regimes of the two thresholds: the defaults (the
pressure from E - ke, rho e resynchronised from E almost everywhere); rho e
carried by its own flux and work term (eta2 = 0.99); and a fast flow whose
pressure comes from rho e (eta1 = 0.5).  Loss: misfits of the final density,
x momentum, energy and rho e to targets near the oracle's final state.

The same check at 32^3 blocks (2 roots, one refined: 9 leaves, one step, 24
entries per regime), where the transposes run in their N = 32 tile shapes.
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
    print(f"[gpu-de-adjoint] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


REGIMES = {
    "defaults": dict(eta1=1e-3, eta2=0.1, vel=0.3),
    "own rho e": dict(eta1=1e-3, eta2=0.99, vel=0.3),
    "pressure from rho e": dict(eta1=0.5, eta2=0.99, vel=2.5),
}


def check_against_frozen_oracle(spec, steps, entries, seed, vel, label):
    m = Mesh(**spec.kwargs())
    N = spec.block_cells
    act5 = I.smooth_state(spec, m.keys, seed=seed, amp=0.2, vel=vel)
    act0 = I.with_internal_energy(act5)
    rng = np.random.default_rng(seed + 1)
    act0[:, 5] *= 1.0 + 0.01 * rng.standard_normal(act0[:, 5].shape)  # rho e near, not at, E - ke
    U0 = m.state_from_active(act0)
    # the dt sequence of the forward (the oracle's is the same: the forward is bitwise equal)
    dts = []
    U = U0.clone()
    for k in range(steps):
        dt = m.dt_tensor()
        m.step(U, dt, k)
        dts.append(float(dt.cpu()[0]))
    om = O.OracleMesh(**spec.kwargs())
    idx = {tuple(k): s for s, k in enumerate(om.keys)}
    perm = np.array([idx[tuple(k)] for k in m.keys])

    def oracle_final(act):
        o = np.empty_like(act)
        o[perm] = act
        om.set_active(o)
        for k in range(steps):
            om.step_dt(k, dts[k])
        return om.active()[perm]

    fin = oracle_final(act0)
    t = [fin[:, 0] * (1 + 0.01 * rng.standard_normal(fin[:, 0].shape)),
         fin[:, 1] + 0.01 * rng.standard_normal(fin[:, 1].shape),
         fin[:, 4] * (1 + 0.001 * rng.standard_normal(fin[:, 4].shape)),
         fin[:, 5] * (1 + 0.001 * rng.standard_normal(fin[:, 5].shape))]
    wn = 0.125 ** m.keys[:, 0]
    wb = wn[:, None, None, None]
    w = torch.from_numpy(wn).to(m.device)[:, None, None, None]
    tg = [torch.from_numpy(np.ascontiguousarray(x)).to(m.device) for x in t]

    Ug = U0.clone().requires_grad_(True)
    a = A.run_steps(Ug, m, steps)[:, :, G:G + N, G:G + N, G:G + N]
    d = [a[:, 0] - tg[0], a[:, 1] - tg[1], a[:, 4] - tg[2], a[:, 5] - tg[3]]
    (w * (d[0] * d[0] + 0.2 * d[1] * d[1] + 0.3 * d[2] * d[2] + 0.3 * d[3] * d[3])).sum().backward()
    g = Ug.grad.detach().cpu().numpy()[:, :, G:G + N, G:G + N, G:G + N]
    say(f"{label}: adjoint gradient done ({m.nleaf} leaves of {N}^3)")

    O.tape_record()
    oracle_final(act0)
    O.tape_stop()

    def oracle_loss(act):
        O.tape_replay()
        a = oracle_final(act)
        O.tape_stop()
        dd = [a[:, 0] - t[0], a[:, 1] - t[1], a[:, 4] - t[2], a[:, 5] - t[3]]
        return float(np.sum(wb * (dd[0] * dd[0] + 0.2 * dd[1] * dd[1] + 0.3 * dd[2] * dd[2] + 0.3 * dd[3] * dd[3])))

    scale = np.abs(g).max()
    worst = 0.0
    for e in range(entries):
        s, f = int(rng.integers(m.nleaf)), e % 6
        z, y, x = (int(v) for v in rng.integers(N, size=3))
        h = 1e-5 * max(1.0, abs(act0[s, f, z, y, x]))
        ap, am = act0.copy(), act0.copy()
        ap[s, f, z, y, x] += h
        am[s, f, z, y, x] -= h
        fd = (oracle_loss(ap) - oracle_loss(am)) / (2 * h)
        err = abs(fd - g[s, f, z, y, x]) / max(abs(fd), 1e-3 * scale)
        worst = max(worst, err)
        assert err <= 1e-6, (label, (s, f, z, y, x), g[s, f, z, y, x], fd)
    say(f"{label}: {entries} frozen-branch oracle difference entries over six fields, "
        f"worst relative error {worst:.3e}")


@pytest.mark.parametrize("regime", list(REGIMES))
def test_tiny_mesh_gradient_against_frozen_branch_oracle(regime):
    r = REGIMES[regime]
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=1, gamma=5 / 3, refine=[(0, 1, 0, 1)],
                      dual_energy=True, eta1=r["eta1"], eta2=r["eta2"])
    check_against_frozen_oracle(spec, steps=2, entries=100, seed=91, vel=r["vel"], label=regime)


@pytest.mark.parametrize("regime", ["own rho e", "pressure from rho e"])
def test_block32_gradient_against_frozen_branch_oracle(regime):
    r = REGIMES[regime]
    spec = I.MeshSpec(root=(2, 1, 1), block_cells=32, max_level=1, gamma=5 / 3, refine=[(0, 1, 0, 0)],
                      dual_energy=True, eta1=r["eta1"], eta2=r["eta2"])
    check_against_frozen_oracle(spec, steps=1, entries=24, seed=93, vel=r["vel"], label=f"N=32 {regime}")
