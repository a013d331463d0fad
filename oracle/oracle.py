"""ctypes wrapper of the plain FP64 CPU oracle (``amr_oracle.c``).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke entry point
and the benchmark's CPU-baseline leg may import this module.  It imports
nothing from the product package; inputs reach it as plain numpy arrays and
plain mesh parameters.

The oracle follows the paper's description of one Enzo-P/Cello hydro step on
an array-of-octrees mesh (Sec. II-B: Blocks, ghost refresh of a given width,
Restrict/Prolong; Sec. II-C: the PPM Method), with every arithmetic detail a
written reading given in ``amr_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amr_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "mg_oracle.c")]
_SO = os.path.join(_HERE, "libamr_oracle.so")
_INC = os.path.join(_HERE, "ppm_pencil.inc")  # the pencil, included by amr_oracle.c and opcount.cpp
_COUNT_SRC = os.path.join(_HERE, "opcount.cpp")
_COUNT_SO = os.path.join(_HERE, "liborc_opcount.so")
GHOST = 3
NFIELD = 5
BC = {"periodic": 0, "outflow": 1}

# Flags that make the arithmetic exactly the written one: no contraction into
# fused multiply-add, no value-changing optimisation, SSE2 doubles.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libamr_oracle.so`` and its
    operation counter with g++ into ``oracle/liborc_opcount.so``."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _SO)
    if force or not os.path.exists(_COUNT_SO):
        tmp = _COUNT_SO + ".tmp"
        subprocess.check_call(["g++", "-std=c++20", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                               "-o", tmp, _COUNT_SRC])
        os.replace(tmp, _COUNT_SO)
    return _SO


class _Desc(ctypes.Structure):
    _fields_ = [
        ("root", ctypes.c_int32 * 3),
        ("block_cells", ctypes.c_int32),
        ("max_level", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("rho_floor", ctypes.c_double),
        ("p_floor", ctypes.c_double),
        ("riemann_iters", ctypes.c_int32),
        ("n_refine", ctypes.c_int32),
        ("refine", ctypes.POINTER(ctypes.c_int32)),
        ("dual_energy", ctypes.c_int32),
        ("eta1", ctypes.c_double),
        ("eta2", ctypes.c_double),
    ]


def build_sanitized(path: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (abort on the first report) into `path`, for the CPU suite's sanitizer
    run; loaded in place of the plain build when AMR_ORACLE_LIBRARY names it."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", *CFLAGS[1:], "-o", path, *_SRCS, "-lm"])
    return path


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        so = os.environ.get("AMR_ORACLE_LIBRARY", "")
        if not so:
            so = _SO
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(f) for f in _SRCS + [_INC]):
                build()
        L = ctypes.CDLL(so)
        P, D, I64, I32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int
        L.orc_create.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(P)]
        L.orc_create.restype = I32
        L.orc_create_from_leaves.argtypes = [ctypes.POINTER(_Desc), I64, P, ctypes.POINTER(P)]
        L.orc_create_from_leaves.restype = I32
        L.orc_destroy.argtypes = [P]
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_nleaf.argtypes = [P]
        L.orc_nleaf.restype = I64
        L.orc_leaf_keys.argtypes = [P, P]
        L.orc_state.argtypes = [P]
        L.orc_state.restype = ctypes.POINTER(ctypes.c_double)
        L.orc_floor_count.argtypes = [P]
        L.orc_floor_count.restype = I64
        L.orc_nfields.argtypes = [P]
        L.orc_nfields.restype = I32
        L.orc_refresh.argtypes = [P]
        L.orc_cfl_dt.argtypes = [P]
        L.orc_cfl_dt.restype = D
        L.orc_step.argtypes = [P, I64]
        L.orc_step.restype = D
        L.orc_step_dt.argtypes = [P, I64, D]
        L.orc_frozen_fd_density_grad.argtypes = [P, I64, I32, P, P, D, P, I64, P, P]
        L.orc_frozen_fd_density_grad.restype = I32
        L.orc_tape_stop.restype = I32
        L.orc_cfl_dt_comoving.argtypes = [P, D]
        L.orc_cfl_dt_comoving.restype = D
        L.orc_step_comoving.argtypes = [P, I64, D, D, D]
        L.orc_riemann.argtypes = [P, I32, P, P, P, P, P, P]
        L.orc_pencil_flux.argtypes = [P, I32, D, I32, P, P]
        L.orc_set_debug.argtypes = [I32]
        L.orc_num_threads.restype = I32
        if hasattr(L, "orc_remesh"):
            L.orc_remesh.argtypes = [P, D, D, I64, ctypes.POINTER(P), P]
            L.orc_remesh.restype = I32
            L.orc_indicator.argtypes = [P, P]
        L.orc_locate.argtypes = [P, P]
        L.orc_locate.restype = I64
        L.orc_tracers_drift.argtypes = [P, D, I64, P, P, P, P]
        L.orc_tracers_drift.restype = I64
        L.orc_step_tracers.argtypes = [P, I64, I64, P, P, P, P]
        L.orc_step_tracers.restype = D
        L.orc_step_gravity.argtypes = [P, I64, D, P, I32, I32, I32, I32]
        L.orc_step_gravity.restype = D
        L.orc_step_gravity_comoving.argtypes = [P, I64, D, D, D, D, D, D, P, I32, I32, I32, I32]
        L.orc_step_gravity_comoving.restype = I32
        L.orc_mg_set_debug.argtypes = [I32]
        L.orc_mg_prolong_add.argtypes = [I32, I32, I32, P, P]
        L.orc_mg_restrict_residual.argtypes = [I32, I32, I32, D, P, P, P]
        L.orc_mg_levels.argtypes = [I32, I32, I32]
        L.orc_mg_levels.restype = I32
        L.orc_mg_solve.argtypes = [I32, I32, I32, D, P, P, I32, I32, I32, P]
        L.orc_step_gravity_amr.argtypes = [P, I64, D, P, I32, I32, I32, I32]
        L.orc_step_gravity_amr.restype = D
        L.orc_mgc_set_debug.argtypes = [I32]
        L.orc_mgc_apply.argtypes = [P, P, P]
        L.orc_mgc_apply.restype = I32
        L.orc_mgc_solve.argtypes = [P, P, P, I32, I32, I32, P]
        L.orc_mgc_solve.restype = I32
        L.orc_mg_solve.restype = I32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_desc(root, block_cells, max_level=0, bc="periodic", gamma=1.4, cfl=0.4,
              rho_floor=1e-20, p_floor=1e-20, riemann_iters=5, refine=(), dual_energy=False,
              eta1=1e-3, eta2=0.1):
    d = _Desc()
    d.root[:] = [int(r) for r in root]
    d.block_cells = int(block_cells)
    d.max_level = int(max_level)
    bcs = [bc] * 3 if isinstance(bc, str) else list(bc)
    d.bc[:] = [BC[b] if isinstance(b, str) else int(b) for b in bcs]
    d.gamma, d.cfl, d.rho_floor, d.p_floor = float(gamma), float(cfl), float(rho_floor), float(p_floor)
    d.riemann_iters = int(riemann_iters)
    d.dual_energy = 1 if dual_energy else 0
    d.eta1, d.eta2 = float(eta1), float(eta2)
    ref = np.ascontiguousarray(np.asarray(refine, dtype=np.int32).reshape(-1, 4))
    d.n_refine = ref.shape[0]
    d.refine = ref.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if ref.size else None
    return d, ref


class OracleMesh:
    """One mesh of the oracle with its padded FP64 state."""

    def __init__(self, root, block_cells, max_level=0, bc="periodic", gamma=1.4, cfl=0.4,
                 rho_floor=1e-20, p_floor=1e-20, riemann_iters=5, refine=(), leaves=None,
                 dual_energy=False, eta1=1e-3, eta2=0.1, _handle=None):
        self._kw = dict(root=root, block_cells=block_cells, max_level=max_level, bc=bc, gamma=gamma,
                        cfl=cfl, rho_floor=rho_floor, p_floor=p_floor, riemann_iters=riemann_iters,
                        dual_energy=dual_energy, eta1=eta1, eta2=eta2)
        L = lib()
        h = ctypes.c_void_p()
        if _handle is not None:
            h = _handle
        else:
            d, keep = make_desc(refine=refine, **self._kw)
            if leaves is not None:
                lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
                rc = L.orc_create_from_leaves(ctypes.byref(d), lv.shape[0], _ptr(lv), ctypes.byref(h))
            else:
                rc = L.orc_create(ctypes.byref(d), ctypes.byref(h))
            if rc != 0:
                raise ValueError("oracle mesh: " + L.orc_last_error().decode())
        self._h = h
        self.N = int(block_cells)
        self.M = self.N + 2 * GHOST
        self.nleaf = int(L.orc_nleaf(h))
        keys = np.zeros((self.nleaf, 4), dtype=np.int32)
        L.orc_leaf_keys(h, _ptr(keys))
        self.keys = keys
        self.nf = int(L.orc_nfields(h))  # 5, or 6 with the dual-energy field rho e
        n = self.nleaf * self.nf * self.M ** 3
        buf = np.ctypeslib.as_array(L.orc_state(h), shape=(n,))
        self.U = buf.reshape(self.nleaf, self.nf, self.M, self.M, self.M)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # state access -----------------------------------------------------
    def set_active(self, act: np.ndarray) -> None:
        g, N = GHOST, self.N
        self.U[...] = 0.0
        self.U[:, :, g:g + N, g:g + N, g:g + N] = act

    def active(self) -> np.ndarray:
        g, N = GHOST, self.N
        return np.array(self.U[:, :, g:g + N, g:g + N, g:g + N])

    @property
    def floors(self) -> int:
        return int(lib().orc_floor_count(self._h))

    # method -----------------------------------------------------------
    def refresh(self) -> None:
        lib().orc_refresh(self._h)

    def cfl_dt(self) -> float:
        return float(lib().orc_cfl_dt(self._h))

    def step(self, k: int) -> float:
        return float(lib().orc_step(self._h, int(k)))

    def step_dt(self, k: int, dt: float) -> None:
        lib().orc_step_dt(self._h, int(k), float(dt))

    def frozen_fd_density_grad(self, first_step: int, dts, target: np.ndarray, eps: float, idx=None):
        """Central differences of the density misfit after len(dts) steps
        from this mesh's state (left unchanged), with the dt sequence and
        every discrete choice of the scheme frozen at the unperturbed run's:
        returns (gradient at the flat density indices idx, default all
        active cells, leaf * N^3 + (z N + y) N + x; the unperturbed loss)."""
        dts = np.ascontiguousarray(dts, dtype=np.float64)
        target = np.ascontiguousarray(target, dtype=np.float64).reshape(self.nleaf, -1)
        if target.shape[1] != self.N ** 3:
            raise ValueError("target must hold N^3 densities per leaf")
        if idx is None:
            idx = np.arange(self.nleaf * self.N ** 3, dtype=np.int64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        grad = np.zeros(idx.size)
        loss = ctypes.c_double()
        rc = lib().orc_frozen_fd_density_grad(self._h, int(first_step), int(dts.size), _ptr(dts), _ptr(target),
                                              float(eps), _ptr(idx), int(idx.size), _ptr(grad), ctypes.byref(loss))
        if rc != 0:
            raise ValueError("oracle frozen-branch differences: " + lib().orc_last_error().decode())
        return grad, float(loss.value)

    def cfl_dt_comoving(self, a: float) -> float:
        """CFL dt in comoving coordinates with expansion factor a."""
        return float(lib().orc_cfl_dt_comoving(self._h, float(a)))

    def step_comoving(self, k: int, dt: float, a: float, hubble: float) -> None:
        """One comoving step: the plain step with dt / a, then the expansion
        sources over dt with H = hubble (a and H at the step's mid time)."""
        lib().orc_step_comoving(self._h, int(k), float(dt), float(a), float(hubble))

    def step_gravity(self, k: int, four_pi_G: float, phi: np.ndarray, phi_current: bool, ncycles: int = 2,
                     nu1: int = 2, nu2: int = 2) -> float:
        """Self-gravity step (uniform periodic mesh): kick-drift-kick with the
        mg0 potential; phi is the global [nz, ny, nx] grid, updated in place."""
        assert phi.dtype == np.float64 and phi.flags.c_contiguous
        dt = float(lib().orc_step_gravity(self._h, int(k), float(four_pi_G), _ptr(phi), int(bool(phi_current)),
                                          int(ncycles), int(nu1), int(nu2)))
        if dt < 0:
            raise ValueError("oracle gravity: " + lib().orc_last_error().decode())
        return dt

    def step_gravity_amr(self, k: int, four_pi_G: float, phi: np.ndarray, phi_current: bool, ncycles: int = 2,
                         nu1: int = 2, nu2: int = 2) -> float:
        """Self-gravity step on any periodic mesh, phi [n_leaves, N, N, N]
        (updated in place) from mg0 on the octree; returns dt."""
        if phi.dtype != np.float64 or not phi.flags.c_contiguous or phi.shape != (self.nleaf,) + (self.N,) * 3:
            raise ValueError("phi must be a contiguous float64 [n_leaves, N, N, N] array")
        dt = lib().orc_step_gravity_amr(self._h, int(k), float(four_pi_G), _ptr(phi), int(bool(phi_current)),
                                        int(ncycles), int(nu1), int(nu2))
        if dt < 0:
            raise ValueError("oracle gravity step: " + lib().orc_last_error().decode())
        return dt

    def step_gravity_comoving(self, k: int, dt: float, a0: float, a_mid: float, a1: float, hubble: float,
                              four_pi_G: float, phi: np.ndarray, phi_current: bool, ncycles: int = 2, nu1: int = 2,
                              nu2: int = 2) -> None:
        """Comoving self-gravity step with the given dt, a at the step's start,
        middle and end, and H at its middle."""
        assert phi.dtype == np.float64 and phi.flags.c_contiguous
        rc = lib().orc_step_gravity_comoving(self._h, int(k), float(dt), float(a0), float(a_mid), float(a1),
                                             float(hubble), float(four_pi_G), _ptr(phi), int(bool(phi_current)),
                                             int(ncycles), int(nu1), int(nu2))
        if rc != 0:
            raise ValueError("oracle gravity: " + lib().orc_last_error().decode())

    def indicator(self) -> np.ndarray:
        out = np.zeros(self.nleaf)
        lib().orc_indicator(self._h, _ptr(out))
        return out

    # tracer particles (positions in level-0 cell units) ----------------
    def locate(self, P: np.ndarray) -> np.ndarray:
        """Leaf index holding each position P[n, 3] (-1 outside)."""
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1, 3)
        out = np.empty(P.shape[0], dtype=np.int64)
        for i in range(P.shape[0]):
            out[i] = lib().orc_locate(self._h, _ptr(P[i]))
        return out

    def tracers_drift(self, dt: float, tr: "Tracers") -> int:
        """One drift of the alive tracers (ghosts must be refreshed)."""
        return int(lib().orc_tracers_drift(self._h, float(dt), tr.n, _ptr(tr.X), _ptr(tr.Y), _ptr(tr.Z),
                                            _ptr(tr.alive)))

    def step_tracers(self, k: int, tr: "Tracers") -> float:
        """dt from CFL, refresh, tracer drift, hydro step; returns dt."""
        return float(lib().orc_step_tracers(self._h, int(k), tr.n, _ptr(tr.X), _ptr(tr.Y), _ptr(tr.Z),
                                            _ptr(tr.alive)))

    def remesh(self, refine_slope, coarsen_slope, max_blocks):
        """Returns (new OracleMesh, stats[refined, coarsened, refused])."""
        L = lib()
        h = ctypes.c_void_p()
        stats = np.zeros(3, dtype=np.int64)
        rc = L.orc_remesh(self._h, float(refine_slope), float(coarsen_slope), int(max_blocks),
                          ctypes.byref(h), _ptr(stats))
        if rc != 0:
            raise ValueError("oracle remesh: " + L.orc_last_error().decode())
        return OracleMesh(_handle=h, **self._kw), stats


class Tracers:
    """Flat particle arrays of the oracle: positions in level-0 cell units,
    ids, alive flags."""

    def __init__(self, X, Y, Z, ids):
        self.X = np.ascontiguousarray(X, dtype=np.float64).copy()
        self.Y = np.ascontiguousarray(Y, dtype=np.float64).copy()
        self.Z = np.ascontiguousarray(Z, dtype=np.float64).copy()
        self.ids = np.ascontiguousarray(ids, dtype=np.int64).copy()
        self.alive = np.ones(self.X.size, dtype=np.int32)
        self.n = int(self.X.size)

    def positions(self) -> np.ndarray:
        return np.stack([self.X, self.Y, self.Z], axis=1)


DEBUG_SKIP_REFLUX = 1
DEBUG_DE_PDV_SIGN = 2
DEBUG_DE_ENTHALPY = 4
DEBUG_DE_ETA1_FLIP = 8
DEBUG_GRAVITY_SIGN = 16
DEBUG_GRAVITY_NO_A = 32
DEBUG_FLOOR_E_NO_KE = 64
DEBUG_FLOOR_KEEP_VEL = 128
DEBUG_DE_FLOOR_NO_IG = 256
DEBUG_EDGE_NO_FLOOR = 512
DEBUG_CFL_SUM = 1024
DEBUG_EXP_FLOOR_NO_IG = 2048
DEBUG_FLOOR_NO_COUNT = 4096


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_debug(flags: int) -> None:
    """Plant a known mistake in the oracle (tests of the pins' power only)."""
    lib().orc_set_debug(int(flags))


def tape_record() -> None:
    """Record the discrete choices of the oracle calls that follow (this
    thread), until tape_stop(); loops over blocks run serially meanwhile."""
    lib().orc_tape_record()


def tape_replay() -> None:
    """Make the oracle calls that follow take the recorded choices."""
    lib().orc_tape_replay()


def tape_stop() -> None:
    if lib().orc_tape_stop() != 0:
        raise RuntimeError(lib().orc_last_error().decode())


def riemann(WL, WR, gamma=1.4, p_floor=1e-20, iters=5):
    """Two-shock Riemann solve at one interface: (state, flux, p*, u*)."""
    gas = np.array([gamma, p_floor])
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    st, fl = np.zeros(5), np.zeros(5)
    ps, us = ctypes.c_double(), ctypes.c_double()
    lib().orc_riemann(_ptr(gas), int(iters), _ptr(WL), _ptr(WR), _ptr(st), _ptr(fl),
                      ctypes.byref(ps), ctypes.byref(us))
    return st, fl, ps.value, us.value


def pencil_flux(U, nu, gamma=1.4, rho_floor=1e-20, p_floor=1e-20, iters=5):
    """Fluxes of a pencil U[5, n] at interfaces j+1/2, j = 2..n-4."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = U.shape[1]
    out = np.zeros((5, n - 5))
    gas = np.array([gamma, rho_floor, p_floor])
    lib().orc_pencil_flux(_ptr(gas), int(iters), float(nu), int(n), _ptr(U), _ptr(out))
    return out


_count_lib = None


def _counter() -> ctypes.CDLL:
    global _count_lib
    if _count_lib is None:
        if not os.path.exists(_COUNT_SO) or os.path.getmtime(_COUNT_SO) < max(
                os.path.getmtime(f) for f in (_COUNT_SRC, _INC)):
            build()
        L = ctypes.CDLL(_COUNT_SO)
        P, D, I32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
        L.orc_count_sweep_ops.argtypes = [P, I32, D, I32, P, P]
        L.orc_count_sweep_ops.restype = I32
        L.orc_count_riemann_ops.argtypes = [P, I32, P, P, P, P]
        L.orc_count_block_ops.argtypes = [I32, P, D, P, P]
        L.orc_count_block_ops.restype = I32
        _count_lib = L
    return _count_lib


OPS = ("add", "sub", "mul", "div", "sqrt")


def count_sweep_ops(U, nu, gamma=1.4, rho_floor=1e-20, p_floor=1e-20, iters=5):
    """FP64 operations the oracle executes for one sweep of the pencil U[5, n]
    (fluxes at the n - 5 interfaces, then the update and floors of the n - 6
    cells between the ghost layers): dict of add, sub, mul, div, sqrt and
    their total, plus the floor resets."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = U.shape[1]
    gas = np.array([gamma, rho_floor, p_floor])
    c = np.zeros(5, dtype=np.int64)
    nfl = _counter().orc_count_sweep_ops(_ptr(gas), int(iters), float(nu), int(n), _ptr(U), _ptr(c))
    if nfl < 0:
        raise ValueError("a pencil needs at least 7 cells")
    out = dict(zip(OPS, map(int, c)))
    out["total"] = int(c.sum())
    out["floors"] = int(nfl)
    return out


def count_riemann_ops(WL, WR, gamma=1.4, p_floor=1e-20, iters=5):
    """FP64 operations of one two-shock Riemann solve (dict as above, with
    the flux the counting build computed under "flux")."""
    gas = np.array([gamma, p_floor])
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    c = np.zeros(5, dtype=np.int64)
    fl = np.zeros(5)
    _counter().orc_count_riemann_ops(_ptr(gas), int(iters), _ptr(WL), _ptr(WR), _ptr(c), _ptr(fl))
    out = dict(zip(OPS, map(int, c)))
    out["total"] = int(c.sum())
    out["flux"] = fl
    return out


BLOCKS = {"primitives": 0, "slope": 1, "parabola": 2, "trace": 3, "update": 4}


def count_block_ops(block, values, nu=0.0, gamma=1.4, rho_floor=1e-20, p_floor=1e-20):
    """FP64 operations of one building block of the oracle's sweep (see
    ``orc_count_block_ops`` for the layout of ``values``)."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    gas = np.array([gamma, rho_floor, p_floor])
    c = np.zeros(5, dtype=np.int64)
    if _counter().orc_count_block_ops(BLOCKS[block], _ptr(gas), float(nu), _ptr(v), _ptr(c)) != 0:
        raise ValueError(block)
    out = dict(zip(OPS, map(int, c)))
    out["total"] = int(c.sum())
    return out


def mg_levels(shape) -> int:
    """Number of mg0 levels of a grid of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    return int(lib().orc_mg_levels(nx, ny, nz))


def mg_solve(f, h, ncycles, nu1=2, nu2=2, phi0=None):
    """mg0 solve of lap(phi) = f on a periodic grid f[nz, ny, nx] of spacing
    h: returns (phi, residual norms before and after each cycle)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    phi = np.zeros_like(f) if phi0 is None else np.ascontiguousarray(phi0, dtype=np.float64).copy()
    res = np.zeros(ncycles + 1)
    nl = lib().orc_mg_solve(nx, ny, nz, float(h), _ptr(f), _ptr(phi), int(ncycles), int(nu1), int(nu2), _ptr(res))
    if nl < 0:
        raise ValueError("mg0 needs even sizes >= 2 and h > 0")
    return phi, res


MG_DEBUG_INJECT = 1
MG_DEBUG_RESTRICT_SUM = 2
MG_DEBUG_SMOOTH_SIGN = 4
MGC_DEBUG_NO_MATCH = 1
MGC_DEBUG_FLAT = 2


def mgc_set_debug(flags: int) -> None:
    """Plant a known mistake in the composite mg0 oracle (tests of the pins' power only)."""
    lib().orc_mgc_set_debug(int(flags))


def _blocks(om, a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (om.nleaf, om.N, om.N, om.N):
        raise ValueError("expected [n_leaves, N, N, N] (x fastest)")
    return a


def mgc_apply(om, phi):
    """The composite-grid Laplacian of phi ([n_leaves, N, N, N], om's leaf
    order) on om's leaves."""
    phi = _blocks(om, phi)
    out = np.zeros_like(phi)
    if lib().orc_mgc_apply(om._h, _ptr(phi), _ptr(out)) != 0:
        raise ValueError("composite mg0: " + lib().orc_last_error().decode())
    return out


def mgc_solve(om, f, ncycles, nu1=2, nu2=2, phi0=None):
    """mg0 on the octree: ncycles composite V(nu1, nu2) cycles for
    L phi = f on om's leaves; returns (phi, residual norms)."""
    f = _blocks(om, f)
    phi = np.zeros_like(f) if phi0 is None else _blocks(om, phi0).copy()
    res = np.zeros(ncycles + 1)
    if lib().orc_mgc_solve(om._h, _ptr(f), _ptr(phi), int(ncycles), int(nu1), int(nu2), _ptr(res)) < 0:
        raise ValueError("composite mg0: " + lib().orc_last_error().decode())
    return phi, res


def mg_set_debug(flags: int) -> None:
    """Plant a known mistake in the mg0 oracle (tests of the pins' power only)."""
    lib().orc_mg_set_debug(int(flags))


def mg_prolong(coarse):
    """The mg0 prolongation of a coarse grid [nz, ny, nx] onto the doubled grid."""
    c = np.ascontiguousarray(coarse, dtype=np.float64)
    nz, ny, nx = c.shape
    fine = np.zeros((2 * nz, 2 * ny, 2 * nx))
    lib().orc_mg_prolong_add(nx, ny, nz, _ptr(c), _ptr(fine))
    return fine


def mg_restrict_residual(f, phi, h):
    """The mg0 restriction of the residual f - lap(phi) (grid [nz, ny, nx], spacing h)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.zeros((nz // 2, ny // 2, nx // 2))
    lib().orc_mg_restrict_residual(nx, ny, nz, float(h), _ptr(f), _ptr(phi), _ptr(out))
    return out
