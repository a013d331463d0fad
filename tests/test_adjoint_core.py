"""CPU unit tests of the hand-written adjoint of the sweep formulas (a host
build of the same header the gfx950 kernels compile) against central finite
differences of the forward: the two-shock Riemann flux and a whole pencil
update including the reflux face fluxes."""
import ctypes
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(os.path.dirname(HERE), "paper_1810_01319_amd", "libamr_core_host.so")
P = ctypes.c_void_p


@pytest.fixture(scope="module")
def core():
    if not os.path.exists(SO):
        from paper_1810_01319_amd import _build

        _build.build_core_host()
    L = ctypes.CDLL(SO)
    L.core_pencil_update.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
    L.core_pencil_vjp.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
    L.core_riemann.argtypes = [P, ctypes.c_int, P, P, P]
    L.core_riemann_vjp.argtypes = [P, ctypes.c_int, P, P, P, P, P]
    return L


def ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


GAS = np.array([1.4, 1e-20, 1e-20])


def riemann(core, L, R):
    F = np.zeros(5)
    core.core_riemann(ptr(GAS), 5, ptr(np.ascontiguousarray(L)), ptr(np.ascontiguousarray(R)), ptr(F))
    return F


STATES = [
    ([1.0, 0.0, 0.1, -0.2, 1.0], [0.125, 0.0, 0.3, 0.1, 0.1]),     # Sod: rarefaction + shock, star left
    ([1.0, 0.75, 0.0, 0.0, 1.0], [0.125, 0.0, 0.0, 0.0, 0.1]),     # transonic fan
    ([1.0, 2.3, 0.2, 0.0, 1.0], [1.0, -2.0, -0.1, 0.3, 1.0]),      # two shocks, u* > 0 (off the side tie)
    ([0.5, -0.3, 0.1, 0.1, 0.4], [1.2, 0.1, 0.0, 0.2, 2.0]),       # star right
    ([1.0, 3.0, 0.1, 0.0, 1.0], [0.9, 3.1, 0.0, 0.1, 0.9]),        # supersonic: left state
    ([1.0, -0.2, 0.0, 0.0, 1.0], [1.1, 0.4, 0.0, 0.0, 0.7]),       # diverging, weak
]


@pytest.mark.parametrize("k", range(len(STATES)))
def test_riemann_vjp_matches_finite_differences(core, k):
    L0, R0 = (np.array(a, dtype=float) for a in STATES[k])
    rng = np.random.default_rng(k)
    for _ in range(6):
        gF = rng.normal(size=5)
        dL, dR = rng.normal(size=5), rng.normal(size=5)
        gL, gR = np.zeros(5), np.zeros(5)
        core.core_riemann_vjp(ptr(GAS), 5, ptr(L0), ptr(R0), ptr(gF), ptr(gL), ptr(gR))
        eps = 1e-6
        fp = gF @ riemann(core, L0 + eps * dL, R0 + eps * dR)
        fm = gF @ riemann(core, L0 - eps * dL, R0 - eps * dR)
        fd = (fp - fm) / (2 * eps)
        ad = gL @ dL + gR @ dR
        assert abs(ad - fd) <= 2e-7 * max(1.0, abs(fd)), (k, ad, fd)


# states whose Newton iteration reaches an exact fixed point before the last
# step (equal states, tiny and weak jumps, an asymmetric cavitation with a
# floored star pressure; a symmetric one would put u* on the star/fan kink)
FIXED = [
    ([1.0, 0.3, 0.1, 0.0, 1.0], [1.0, 0.3, -0.2, 0.4, 1.0]),
    ([1.0, 0.3, 0.0, 0.0, 1.0], [1.0000001, 0.3000001, 0.0, 0.0, 1.0000002]),
    ([1.0, 0.1, 0.0, 0.0, 1.0], [1.02, 0.08, 0.0, 0.0, 1.03]),
    ([1.0, -4.0, 0.0, 0.0, 0.01], [0.8, 3.0, 0.0, 0.0, 0.012]),
]


@pytest.mark.parametrize("k", range(len(FIXED)))
def test_riemann_vjp_at_a_fixed_point_equals_the_stepwise_transpose(core, k):
    """At an exact Newton fixed point the transpose of the identical remaining
    evaluations is taken in closed form; it must equal reversing them one by
    one (up to rounding) and match finite differences."""
    core.core_riemann_vjp_stepwise.argtypes = core.core_riemann_vjp.argtypes
    L0, R0 = (np.array(a, dtype=float) for a in FIXED[k])
    rng = np.random.default_rng(40 + k)
    for _ in range(6):
        gF = rng.normal(size=5)
        a = [np.zeros(5), np.zeros(5)]
        b = [np.zeros(5), np.zeros(5)]
        core.core_riemann_vjp(ptr(GAS), 5, ptr(L0), ptr(R0), ptr(gF), ptr(a[0]), ptr(a[1]))
        core.core_riemann_vjp_stepwise(ptr(GAS), 5, ptr(L0), ptr(R0), ptr(gF), ptr(b[0]), ptr(b[1]))
        scale = max(1.0, float(np.max(np.abs(np.concatenate(b)))))
        assert np.max(np.abs(np.concatenate(a) - np.concatenate(b))) <= 1e-13 * scale, (k, a, b)
        dL, dR = rng.normal(size=5), rng.normal(size=5)
        eps = 1e-6
        fd = (gF @ riemann(core, L0 + eps * dL, R0 + eps * dR) - gF @ riemann(core, L0 - eps * dL, R0 - eps * dR)) / (2 * eps)
        ad = a[0] @ dL + a[1] @ dR
        assert abs(ad - fd) <= 2e-7 * max(1.0, abs(fd)), (k, ad, fd)


def pencil_state(n, rng, kind):
    x = np.arange(n, dtype=float)
    if kind == "smooth":
        rho = 1 + 0.2 * np.sin(0.4 * x + rng.uniform(0, 6))
        u = 0.5 * np.cos(0.3 * x + rng.uniform(0, 6))
        p = 1 + 0.3 * np.sin(0.5 * x + rng.uniform(0, 6))
    elif kind == "shock":
        rho = np.where(x < n // 2, 2.0, 1.0) + 0.05 * np.sin(x)
        u = np.where(x < n // 2, 0.6, -0.2) + 0.01 * np.sin(1.3 * x)  # generic: no exact dL = 0
        p = np.where(x < n // 2, 3.0, 1.0) + 0.02 * np.cos(x)
    else:  # supersonic flow to the left with waves
        rho = 1 + 0.1 * np.sin(0.6 * x)
        u = -2.5 + 0.2 * np.cos(0.4 * x)
        p = 0.5 + 0.05 * np.sin(0.7 * x)
    v = 0.3 * np.sin(0.2 * x)
    w = -0.2 * np.cos(0.25 * x)
    E = p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)
    return np.array([rho, rho * u, rho * v, rho * w, E])


@pytest.mark.parametrize("kind", ["smooth", "shock", "supersonic"])
# kink-free central differences on smooth pencils are checked separately below
@pytest.mark.parametrize("n,lo,hi", [(22, 3, 19), (38, 3, 35), (14, 3, 11)])
def test_pencil_vjp_matches_finite_differences(core, kind, n, lo, hi):
    rng = np.random.default_rng(n + len(kind))
    U0 = pencil_state(n, rng, kind)
    nu = 0.35 / 3.0
    for _ in range(4):
        lam = rng.normal(size=(5, n))
        gface = rng.normal(size=10)
        dU = rng.normal(size=(5, n)) * np.array([1.0, 0.5, 0.5, 0.5, 2.0])[:, None]

        def phi(U):
            out, faces = np.zeros((5, n)), np.zeros(10)
            core.core_pencil_update(ptr(GAS), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U)), ptr(out), ptr(faces))
            return float(np.sum(lam * out) + gface @ faces)

        adj = np.ascontiguousarray(lam.copy())
        core.core_pencil_vjp(ptr(GAS), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U0)), ptr(adj), ptr(gface))
        ad = float(np.sum(adj * dU))
        # The limiters make the update continuous but only piecewise smooth:
        # the adjoint follows the branch the forward took at U0, so it must
        # equal the one-sided difference on that side of any kink.
        eps = 1e-7
        f0 = phi(U0)
        fp = (phi(U0 + eps * dU) - f0) / eps
        fm = (f0 - phi(U0 - eps * dU)) / eps
        err = min(abs(ad - fp), abs(ad - fm))
        assert err <= 2e-5 * max(1.0, abs(ad)), (kind, ad, fp, fm)


def test_pencil_vjp_central_differences_per_cell(core):
    """Coordinate-wise central differences on smooth sub- and supersonic
    pencils (no limiter kink within the step): every adjoint entry."""
    for kind, seed in (("smooth", 3), ("supersonic", 5)):
        n, lo, hi = 22, 3, 19
        rng = np.random.default_rng(seed)
        U0 = pencil_state(n, rng, kind)
        nu = 0.35 / 3.0
        lam = rng.normal(size=(5, n))
        gface = rng.normal(size=10)

        def phi(U):
            out, faces = np.zeros((5, n)), np.zeros(10)
            core.core_pencil_update(ptr(GAS), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U)), ptr(out), ptr(faces))
            return float(np.sum(lam * out) + gface @ faces)

        adj = np.ascontiguousarray(lam.copy())
        core.core_pencil_vjp(ptr(GAS), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U0)), ptr(adj), ptr(gface))
        for v in range(5):
            for j in range(n):
                e = np.zeros((5, n))
                h = 1e-7 * max(1.0, abs(U0[v, j]))
                e[v, j] = h
                fd = (phi(U0 + e) - phi(U0 - e)) / (2 * h)
                assert abs(fd - adj[v, j]) <= 1e-5 * max(1.0, abs(fd)), (kind, v, j, adj[v, j], fd)


FLOOR_GAS = np.array([1.4, 0.1, 0.05])
FLOOR_CASES = [
    ("none", [1.0, 0.3, -0.2, 0.1, 2.0]),
    ("density", [0.05, 0.02, 0.01, -0.03, 0.5]),
    ("pressure", [1.0, 0.9, 0.4, -0.3, 0.6]),
    ("both", [0.07, 0.2, -0.1, 0.15, 0.3]),
]


@pytest.mark.parametrize("k", range(len(FLOOR_CASES)))
def test_floor_vjp_matches_finite_differences(core, k):
    """Post-update floors of one cell: which floor is active is checked from
    the forward's output, then every adjoint entry against a central
    difference (the cases sit away from the floors' switch points)."""
    name, V0 = FLOOR_CASES[k]
    V0 = np.array(V0)
    core.core_floor.argtypes = [P, P, P]
    core.core_floor_vjp.argtypes = [P, P, P, P]

    def fwd(V):
        out = np.zeros(5)
        core.core_floor(ptr(FLOOR_GAS), ptr(np.ascontiguousarray(V)), ptr(out))
        return out

    out = fwd(V0)
    rfl = out[0] == FLOOR_GAS[1]
    ke = 0.5 * (out[1] ** 2 + out[2] ** 2 + out[3] ** 2) / out[0]
    pfl = abs(0.4 * (out[4] - ke) - FLOOR_GAS[2]) < 1e-14
    assert (rfl, pfl) == {"none": (False, False), "density": (True, False),
                          "pressure": (False, True), "both": (True, True)}[name]
    rng = np.random.default_rng(k)
    g = rng.normal(size=5)
    gV = np.zeros(5)
    core.core_floor_vjp(ptr(FLOOR_GAS), ptr(V0), ptr(g), ptr(gV))
    for v in range(5):
        e = np.zeros(5)
        e[v] = 1e-7
        fd = g @ (fwd(V0 + e) - fwd(V0 - e)) / 2e-7
        assert abs(fd - gV[v]) <= 1e-7 * max(1.0, abs(fd)), (name, v, gV[v], fd)
