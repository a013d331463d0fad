"""GPU parity of the comoving step (expansion factor a, H = adot / a) with
the oracle, through the C ABI: Einstein-de Sitter runs on random AMR meshes
(dt from the comoving CFL each step, a and H at the step's mid time), the
Sedov blast, pressure floors raised by the expansion source, batched
instances; and the static universe equals the plain GPU step bit for bit.
Bar: dt bitwise; every active cell within 1e-12 of the oracle (the design
target, and the observed result, is bitwise)."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd.mesh import Mesh

from test_gpu_parity import TOL, compare_active, load, pair

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-comoving] {msg}", file=sys.stderr, flush=True)


def eds(t):
    return t ** (2.0 / 3.0), 2.0 / (3.0 * t)


def run_comoving(name, spec, act, steps, t0=1.0, hubble_scale=1.0):
    say(f"case {name}: root={spec.root} N={spec.block_cells} levels={spec.max_level} steps={steps}")
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, act(spec, gm.keys))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = t0
    worst, bw = 0.0, 1.0
    for k in range(steps):
        a, _ = eds(t)
        gm.cfl_dt_comoving(U, a, dt)
        dtg = float(dt.cpu()[0])
        dto = om.cfl_dt_comoving(a)
        assert dtg == dto, f"{name}: dt differs at step {k}: {dtg!r} vs {dto!r}"
        am, hm = eds(t + 0.5 * dtg)
        hm *= hubble_scale
        gm.step_comoving(U, dt, k, am, hm)
        om.step_comoving(k, dtg, am, hm)
        torch.cuda.synchronize()
        err, bw = compare_active(gm, U, om, perm)
        worst = max(worst, err)
        assert err <= TOL, f"{name}: step {k} rel err {err:.3e}"
        t += dtg
    assert gm.floor_count() == om.floors, f"{name}: floor counts differ"
    say(f"case {name}: worst rel err {worst:.3e}, bitwise fraction {bw:.6f}, floors {om.floors}")
    return gm, om


@pytest.mark.parametrize("N,levels,seed", [(8, 2, 1), (16, 2, 2), (32, 1, 3)])
def test_comoving_amr_steps_match_oracle(N, levels, seed):
    root = (2, 2, 2)
    spec = I.MeshSpec(root=root, block_cells=N, max_level=levels, gamma=5.0 / 3.0,
                      refine=I.random_refine_list(root, levels, 4, seed))
    run_comoving(f"smooth N={N}", spec, lambda s, k: I.smooth_state(s, k, seed=20 + seed), 4)


def test_comoving_sedov_matches_oracle():
    spec = I.sedov_spec(root=2, block_cells=16, levels=2)
    run_comoving("sedov", spec, I.sedov_state, 4)


def test_expansion_floor_triggers_match():
    """Cold gas with a strong expansion rate: the source lowers the internal
    energy below the pressure floor in the same cells on both sides."""
    spec = I.MeshSpec(root=(2, 1, 1), block_cells=8, gamma=5.0 / 3.0, p_floor=1e-3, rho_floor=1e-6)

    def act(s, keys):
        x = I.cell_centres(s, keys)[0]
        p = np.where(x < 0.5, 1.2e-3, 1.0)
        return I.conserved(5.0 / 3.0, np.ones_like(x), 0.1 * np.sin(6.283185307179586 * x), 0.0, 0.0, p)

    gm, om = run_comoving("floors", spec, act, 2, hubble_scale=50.0)
    assert om.floors > 0


def test_static_universe_equals_the_plain_gpu_step():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=16, max_level=2, gamma=5.0 / 3.0,
                      refine=I.random_refine_list((2, 2, 2), 2, 4, 11))
    a = Mesh(**spec.kwargs())
    act = I.smooth_state(spec, a.keys, seed=31)
    Ua, Ub = a.state_from_active(act), a.state_from_active(act)
    dta = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtb = torch.zeros_like(dta)
    for k in range(3):
        a.cfl_dt_comoving(Ua, 1.0, dta)
        a.step_comoving(Ua, dta, k, 1.0, 0.0)
        a.step(Ub, dtb, k)
    torch.cuda.synchronize()
    assert torch.equal(dta, dtb)
    assert np.array_equal(a.active(Ua), a.active(Ub))


def test_comoving_batched_instances_match_oracle():
    specs, cents = zip(*[I.batch_instance(i) for i in range(4)])
    gm = Mesh.batch([s.kwargs() for s in specs])
    say(f"batch of 4: {gm.nleaf} leaves")
    oms, acts = [], []
    for i, (sp, c) in enumerate(zip(specs, cents)):
        keys = gm.keys[gm.first_leaf[i]:gm.first_leaf[i + 1]]
        acts.append(I.batch_state(sp, keys, c))
        om = O.OracleMesh(**sp.kwargs())
        idx = {tuple(k): s for s, k in enumerate(om.keys)}
        perm = np.array([idx[tuple(k)] for k in keys])
        o = np.empty_like(acts[-1])
        o[perm] = acts[-1]
        om.set_active(o)
        oms.append((om, perm))
    U = gm.state_from_active(np.concatenate(acts))
    dt = gm.dt_tensor()
    a, h = 0.5, 0.7
    for k in range(3):
        gm.cfl_dt_comoving(U, a, dt)
        dts = dt.cpu().numpy()
        gm.step_comoving(U, dt, k, a, h)
        torch.cuda.synchronize()
        act = gm.active(U)
        for i, (om, perm) in enumerate(oms):
            assert dts[i] == om.cfl_dt_comoving(a)
            om.step_comoving(k, float(dts[i]), a, h)
            got = act[gm.first_leaf[i]:gm.first_leaf[i + 1]]
            assert np.array_equal(got, om.active()[perm]), f"instance {i} step {k}"


@pytest.mark.parametrize("omega_m,omega_l", [(1.0, 0.0), (0.3, 0.7)])
def test_device_resident_comoving_run_matches_oracle(omega_m, omega_l):
    """amr_hydro_steps_comoving (the expansion history evaluated on the
    device, nothing read back) against the oracle stepping with a and H from
    the closed form on the host at the same times: dt within 1e-14, every
    active cell within 1e-12, and the device's time, a and H after the run."""
    from test_cosmology_background import flat_lcdm

    root = (2, 2, 2)
    spec = I.MeshSpec(root=root, block_cells=16, max_level=2, gamma=5.0 / 3.0,
                      refine=I.random_refine_list(root, 2, 4, 9))
    say(f"device-resident comoving run, omega_m {omega_m}, omega_l {omega_l}")
    orc, gm, perm = pair(spec)
    U = load(orc, gm, perm, I.smooth_state(spec, gm.keys, seed=31, amp=0.2, vel=0.6))
    H0, t0, n = 2.0 / 3.0, 1.0, 6
    cosmo = torch.tensor([t0, 0.0, 0.0, 0.0], dtype=torch.float64, device="cuda")
    dts = torch.zeros(n, dtype=torch.float64, device="cuda")
    gm.steps_comoving(U, dts, n, 0, cosmo, H0, omega_m, omega_l)
    d = dts.cpu().numpy()
    t = t0
    for k in range(n):
        a, _ = flat_lcdm(t, H0, omega_m, omega_l)
        dto = orc.cfl_dt_comoving(a)
        assert abs(d[k] - dto) <= 1e-14 * dto, (k, d[k], dto)
        tm = t + 0.5 * d[k]
        am, hm = flat_lcdm(tm, H0, omega_m, omega_l)
        orc.step_comoving(k, float(d[k]), am, hm)
        t += d[k]
    err, bw = compare_active(gm, U, orc, perm)
    say(f"after {n} steps: rel err {err:.3e}, bitwise fraction {bw:.6f}")
    assert err <= TOL
    c = cosmo.cpu().numpy()
    a_last = flat_lcdm(t - d[-1], H0, omega_m, omega_l)[0]
    assert abs(c[0] - t) <= 1e-14 * t
    assert abs(c[1] - a_last) <= 1e-14 * a_last
    assert abs(c[2] - am) <= 1e-14 * am and abs(c[3] - hm) <= 1e-14 * hm
