"""CPU unit tests of the dual-energy adjoint of the sweep formulas (host
build of the header the gfx950 kernels compile) against differences of the
host forward of the same update: the post-update floors and
resynchronisation of one cell, and whole pencils with the pressure taken
from the rho e field (eta1 large), with rho e resynchronised from the total
energy (eta2 small) or carried by its own flux and work term (eta2 near 1)."""
import ctypes
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(os.path.dirname(HERE), "paper_1810_01319_amd", "libamr_core_host.so")
P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double


@pytest.fixture(scope="module")
def core():
    if not os.path.exists(SO):
        from paper_1810_01319_amd import _build

        _build.build_core_host()
    L = ctypes.CDLL(SO)
    L.core_pencil_update_de.argtypes = [P, I, D, I, I, I, P, P, P]
    L.core_pencil_vjp_de.argtypes = [P, I, D, I, I, I, P, P, P]
    L.core_floor_de.argtypes = [P, P, P]
    L.core_floor_vjp_de.argtypes = [P, P, P, P]
    return L


def ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


GAMMA = 1.4
FLOOR_GAS = np.array([GAMMA, 0.1, 0.05, 1e-3, 0.1])
FLOOR_CASES = [
    # (name, V = rho, m_n, m_t1, m_t2, E, rho e before floors, eta2)
    ("resync", [1.0, 0.3, -0.2, 0.1, 2.0, 4.0], 0.1),
    ("own", [1.0, 0.3, -0.2, 0.1, 2.0, 4.0], 0.99),
    ("rho e floor", [1.0, 0.3, -0.2, 0.1, 2.0, 0.01], 0.99),
    ("pressure floor, resync", [1.0, 0.9, 0.4, -0.3, 0.6, 0.3], 0.01),
    ("density floor, resync", [0.05, 0.02, 0.01, -0.03, 0.5, 1.0], 0.1),
    ("density floor, own", [0.05, 0.02, 0.01, -0.03, 0.5, 1.0], 0.99),
]


@pytest.mark.parametrize("k", range(len(FLOOR_CASES)))
def test_floor_vjp_de_matches_finite_differences(core, k):
    name, V0, eta2 = FLOOR_CASES[k]
    V0 = np.array(V0)
    gas = FLOOR_GAS.copy()
    gas[4] = eta2

    def fwd(V):
        out = np.zeros(6)
        core.core_floor_de(ptr(gas), ptr(np.ascontiguousarray(V)), ptr(out))
        return out

    out = fwd(V0)
    ke = 0.5 * (out[1] ** 2 + out[2] ** 2 + out[3] ** 2) / out[0]
    ie = out[4] - ke
    resync = abs(out[5] - ie) < 1e-14 and name != "rho e floor"
    gfl = abs((GAMMA - 1) * out[5] - gas[2]) < 1e-14 and not resync
    assert resync == ("resync" in name)
    assert gfl == (name == "rho e floor")
    rng = np.random.default_rng(k)
    g = rng.normal(size=6)
    gV = np.zeros(6)
    core.core_floor_vjp_de(ptr(gas), ptr(V0), ptr(g), ptr(gV))
    for v in range(6):
        e = np.zeros(6)
        e[v] = 1e-7
        fd = g @ (fwd(V0 + e) - fwd(V0 - e)) / 2e-7
        assert abs(fd - gV[v]) <= 1e-7 * max(1.0, abs(fd)), (name, v, gV[v], fd)


def pencil_state(n, rng, kind):
    x = np.arange(n, dtype=float)
    if kind == "smooth":
        rho = 1 + 0.2 * np.sin(0.4 * x + rng.uniform(0, 6))
        u = 0.5 * np.cos(0.3 * x + rng.uniform(0, 6))
        p = 1 + 0.3 * np.sin(0.5 * x + rng.uniform(0, 6))
    elif kind == "shock":
        rho = np.where(x < n // 2, 2.0, 1.0) + 0.05 * np.sin(x)
        u = np.where(x < n // 2, 0.6, -0.2) + 0.01 * np.sin(1.3 * x)
        p = np.where(x < n // 2, 3.0, 1.0) + 0.02 * np.cos(x)
    else:  # supersonic flow to the left with waves: E - ke is a small part of E
        rho = 1 + 0.1 * np.sin(0.6 * x)
        u = -2.5 + 0.2 * np.cos(0.4 * x)
        p = 0.5 + 0.05 * np.sin(0.7 * x)
    v = 0.3 * np.sin(0.2 * x)
    w = -0.2 * np.cos(0.25 * x)
    E = p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)
    ge = p / (GAMMA - 1) * (1 + 0.01 * np.sin(0.9 * x + 1.0))  # rho e close to, not equal to, E - ke
    return np.array([rho, rho * u, rho * v, rho * w, E, ge])


ETAS = {"select rho e, resync": (0.5, 0.1), "E - ke, resync": (1e-3, 0.1), "select rho e, own": (0.5, 0.99),
        "E - ke, own": (1e-3, 0.99)}


@pytest.mark.parametrize("kind", ["smooth", "shock", "supersonic"])
@pytest.mark.parametrize("etas", list(ETAS))
def test_pencil_vjp_de_matches_one_sided_differences(core, kind, etas):
    n, lo, hi = 22, 3, 19
    rng = np.random.default_rng(n + len(kind) + len(etas))
    gas = np.array([GAMMA, 1e-20, 1e-20, *ETAS[etas]])
    U0 = pencil_state(n, rng, kind)
    nu = 0.35 / 3.0
    for _ in range(4):
        lam = rng.normal(size=(6, n))
        gface = rng.normal(size=12)
        dU = rng.normal(size=(6, n)) * np.array([1.0, 0.5, 0.5, 0.5, 2.0, 2.0])[:, None]

        def phi(U):
            out, faces = np.zeros((6, n)), np.zeros(12)
            core.core_pencil_update_de(ptr(gas), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U)), ptr(out),
                                       ptr(faces))
            return float(np.sum(lam * out) + gface @ faces)

        adj = np.ascontiguousarray(lam.copy())
        core.core_pencil_vjp_de(ptr(gas), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U0)), ptr(adj), ptr(gface))
        ad = float(np.sum(adj * dU))
        # piecewise smooth (limiters, selections): the adjoint follows the
        # branch the forward took at U0, so it equals the one-sided
        # difference on that side of any kink
        eps = 1e-7
        f0 = phi(U0)
        fp = (phi(U0 + eps * dU) - f0) / eps
        fm = (f0 - phi(U0 - eps * dU)) / eps
        err = min(abs(ad - fp), abs(ad - fm))
        assert err <= 2e-5 * max(1.0, abs(ad)), (kind, etas, ad, fp, fm)


@pytest.mark.parametrize("etas", list(ETAS))
def test_pencil_vjp_de_central_differences_per_cell(core, etas):
    """Coordinate-wise central differences on smooth sub- and supersonic
    pencils: every adjoint entry of all six fields."""
    gas = np.array([GAMMA, 1e-20, 1e-20, *ETAS[etas]])
    for kind, seed in (("smooth", 3), ("supersonic", 5)):
        n, lo, hi = 22, 3, 19
        rng = np.random.default_rng(seed)
        U0 = pencil_state(n, rng, kind)
        nu = 0.35 / 3.0
        lam = rng.normal(size=(6, n))
        gface = rng.normal(size=12)

        def phi(U):
            out, faces = np.zeros((6, n)), np.zeros(12)
            core.core_pencil_update_de(ptr(gas), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U)), ptr(out),
                                       ptr(faces))
            return float(np.sum(lam * out) + gface @ faces)

        adj = np.ascontiguousarray(lam.copy())
        core.core_pencil_vjp_de(ptr(gas), 5, nu, n, lo, hi, ptr(np.ascontiguousarray(U0)), ptr(adj), ptr(gface))
        for v in range(6):
            for j in range(n):
                e = np.zeros((6, n))
                h = 1e-7 * max(1.0, abs(U0[v, j]))
                e[v, j] = h
                fd = (phi(U0 + e) - phi(U0 - e)) / (2 * h)
                assert abs(fd - adj[v, j]) <= 1e-5 * max(1.0, abs(fd)), (kind, etas, v, j, adj[v, j], fd)
