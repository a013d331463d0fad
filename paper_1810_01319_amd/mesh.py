"""Python face of one mesh: the C-ABI calls with torch tensors for device
memory and the current HIP stream.  Every step of the path runs in the HIP
library; this module only allocates and passes pointers."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

GHOST = 3


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def arith_selftest(n: int, seed: int = 0, device="cuda") -> tuple[int, int]:
    """Numbers of operands (of n, from seed) on which the kernels' reciprocal
    and square root of positive operands differ from IEEE 1/x and sqrt(x)."""
    counts = torch.zeros(2, dtype=torch.int64, device=device)
    check(lib().amr_arith_selftest(ctypes.c_uint64(seed), n, _ptr(counts), _stream()))
    c = counts.cpu()
    return int(c[0]), int(c[1])


class Mesh:
    """An array-of-octrees mesh with its uploaded tables on one GPU."""

    def __init__(self, root, block_cells, max_level=0, bc="periodic", gamma=1.4, cfl=0.4,
                 rho_floor=1e-20, p_floor=1e-20, riemann_iters=5, refine=(), leaves=None,
                 dual_energy=False, eta1=1e-3, eta2=0.1, device="cuda", _handle=None):
        self.params = dict(root=tuple(root), block_cells=block_cells, max_level=max_level, bc=bc,
                           gamma=gamma, cfl=cfl, rho_floor=rho_floor, p_floor=p_floor,
                           riemann_iters=riemann_iters, dual_energy=dual_energy, eta1=eta1, eta2=eta2)
        L = lib()
        h = ctypes.c_void_p()
        batch = isinstance(root, (list, tuple)) and len(root) > 0 and isinstance(root[0], dict)
        if not batch and _handle is None:
            d, keep = _lib.make_desc(refine=refine, **self.params)
        if _handle is not None:
            h = _handle
        elif batch:
            # a batch: root is a list of per-instance parameter dicts
            descs = (_lib.MeshDesc * len(root))()
            keeps = []
            for i, kw in enumerate(root):
                di, ki = _lib.make_desc(**kw)
                descs[i] = di
                keeps.append(ki)
            check(L.amr_batch_create(descs, len(root), ctypes.byref(h)))
            self.params = None
        elif leaves is not None:
            lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
            check(L.amr_mesh_create_from_leaves(ctypes.byref(d), lv.shape[0],
                                                lv.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        else:
            check(L.amr_mesh_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        info = _lib.MeshInfo()
        check(L.amr_mesh_info(h, ctypes.byref(info)))
        self.info = info
        self.nleaf = int(info.n_leaves)
        self.N = int(info.block_cells)
        self.M = int(info.padded)
        self.nf = int(info.n_fields)  # 5, or 6 with the dual-energy field rho e
        keys = np.zeros((self.nleaf, 4), dtype=np.int32)
        check(L.amr_mesh_blocks(h, keys.ctypes.data_as(ctypes.c_void_p), self.nleaf))
        self.keys = keys
        self.n_instances = int(info.n_instances)
        off = np.zeros(self.n_instances + 1, dtype=np.int64)
        check(L.amr_mesh_instance_offsets(h, off.ctypes.data_as(ctypes.c_void_p), off.size))
        self.first_leaf = off
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=self.device)
        check(L.amr_mesh_upload(h, _ptr(self.workspace), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib._lib is not None:
            _lib._lib.amr_mesh_destroy(h)
            self._h = None

    # storage ----------------------------------------------------------
    def alloc_state(self) -> torch.Tensor:
        return torch.zeros((self.nleaf, self.nf, self.M, self.M, self.M), dtype=torch.float64,
                           device=self.device)

    def state_from_active(self, act: np.ndarray) -> torch.Tensor:
        U = torch.zeros((self.nleaf, self.nf, self.M, self.M, self.M), dtype=torch.float64)
        g, N = GHOST, self.N
        U[:, :, g:g + N, g:g + N, g:g + N] = torch.from_numpy(np.ascontiguousarray(act))
        return U.to(self.device)

    def state_from_blocks(self, fn, chunk: int = 512, out: torch.Tensor = None) -> torch.Tensor:
        """Device state filled chunk by chunk from fn(keys) -> active cells
        [n, nf, N, N, N] (host numpy), for states too large to stage at once;
        placed at the start of the flat buffer `out` if given."""
        shape = (self.nleaf, self.nf, self.M, self.M, self.M)
        if out is not None:
            U = out[:self.nleaf * self.nf * self.M ** 3].view(shape)
        else:
            U = torch.empty(shape, dtype=torch.float64, device=self.device)
        g, N = GHOST, self.N
        for a in range(0, self.nleaf, chunk):
            b = min(self.nleaf, a + chunk)
            act = torch.from_numpy(np.ascontiguousarray(fn(self.keys[a:b])))
            U[a:b, :, g:g + N, g:g + N, g:g + N] = act.to(self.device)
        return U

    def active(self, U: torch.Tensor) -> np.ndarray:
        g, N = GHOST, self.N
        return U[:, :, g:g + N, g:g + N, g:g + N].cpu().numpy()

    def _check_state(self, U: torch.Tensor) -> None:
        if U.dtype != torch.float64 or not U.is_contiguous() or U.device != self.device:
            raise ValueError("state must be a contiguous float64 tensor on the mesh's device")
        if U.numel() * 8 != self.info.field_bytes:
            raise ValueError("state has the wrong size for this mesh")

    # method -----------------------------------------------------------
    def refresh(self, U: torch.Tensor) -> None:
        self._check_state(U)
        check(lib().amr_refresh_ghosts(self._h, _ptr(U), _stream()))

    def cfl_dt(self, U: torch.Tensor, dt: torch.Tensor) -> None:
        self._check_state(U)
        check(lib().amr_cfl_dt(self._h, _ptr(U), _ptr(dt), _stream()))

    def step(self, U: torch.Tensor, dt: torch.Tensor, k: int) -> None:
        """One hydro step; dt (n_instances doubles on the device) receives the
        CFL dt of each instance.  A batch steps through amr_batch_step."""
        self._check_state(U)
        if dt.numel() < self.n_instances:
            raise ValueError("dt needs one double per instance")
        fn = lib().amr_batch_step if self.n_instances > 1 else lib().amr_hydro_step
        check(fn(self._h, _ptr(U), _ptr(dt), int(k), _stream()))

    def steps(self, U: torch.Tensor, dt: torch.Tensor, n: int, first: int = 0, ghosts_fresh: bool = False) -> None:
        """n consecutive steps in one call (the same results as n step calls);
        dt holds n * n_instances doubles, step i's in row i.  Each step's CFL
        reduction is fused into its predecessor.  ghosts_fresh: U's ghosts
        are current (no active cell changed since the last refresh, or since
        a remesh that changed nothing), so the first step skips its refresh."""
        self._check_state(U)
        if dt.numel() < n * self.n_instances:
            raise ValueError("dt holds fewer than n * n_instances values")
        fn = lib().amr_hydro_steps_fresh if ghosts_fresh else lib().amr_hydro_steps
        check(fn(self._h, _ptr(U), _ptr(dt), int(n), int(first), _stream()))

    def step_dt(self, U: torch.Tensor, dt: torch.Tensor, k: int) -> None:
        self._check_state(U)
        check(lib().amr_hydro_step_dt(self._h, _ptr(U), _ptr(dt), int(k), _stream()))

    def cfl_dt_comoving(self, U: torch.Tensor, a: float, dt: torch.Tensor) -> None:
        """CFL dt in comoving coordinates with expansion factor a."""
        self._check_state(U)
        check(lib().amr_cfl_dt_comoving(self._h, _ptr(U), ctypes.c_double(a), _ptr(dt), _stream()))

    def step_comoving(self, U: torch.Tensor, dt: torch.Tensor, k: int, a: float, hubble: float) -> None:
        """One comoving step with the given dt (device): fluxes with dt / a,
        then the expansion sources with H = hubble (a, H at the mid time)."""
        self._check_state(U)
        check(lib().amr_hydro_step_comoving(self._h, _ptr(U), _ptr(dt), int(k), ctypes.c_double(a),
                                            ctypes.c_double(hubble), _stream()))

    def steps_comoving(self, U: torch.Tensor, dts: torch.Tensor, n: int, first: int, cosmo: torch.Tensor,
                       H0: float, omega_m: float = 1.0, omega_l: float = 0.0) -> None:
        """n comoving steps with the expansion history of a flat matter +
        Lambda background evaluated on the device: cosmo is a float64 device
        tensor of 4 ([0] the time t in and out; [1] a(t) at the last step's
        start; [2], [3] a and H at its mid time), dts receives the n dts."""
        self._check_state(U)
        if dts.dtype != torch.float64 or dts.device != U.device or dts.numel() < n or not dts.is_contiguous():
            raise ValueError("dts must be a contiguous float64 device tensor of at least n entries")
        if cosmo.dtype != torch.float64 or cosmo.device != U.device or cosmo.numel() != 4:
            raise ValueError("cosmo must be a float64 device tensor of 4 entries")
        check(lib().amr_hydro_steps_comoving(self._h, _ptr(U), _ptr(dts), int(n), int(first), ctypes.c_double(H0),
                                             ctypes.c_double(omega_m), ctypes.c_double(omega_l), _ptr(cosmo),
                                             _stream()))

    def floor_count(self) -> int:
        out = ctypes.c_int64()
        check(lib().amr_floor_count(self._h, ctypes.byref(out), _stream()))
        return int(out.value)

    @classmethod
    def batch(cls, specs, device="cuda"):
        """Many independent meshes (list of parameter dicts, each with its own
        `refine` list) in one flat worklist; dt tensors hold one double per
        instance."""
        return cls(root=list(specs), block_cells=specs[0]["block_cells"], device=device)

    def dt_tensor(self) -> torch.Tensor:
        return torch.zeros(self.n_instances, dtype=torch.float64, device=self.device)

    def graph(self, U: torch.Tensor, dt: torch.Tensor, first_step: int = 0) -> "Graph":
        """Capture two consecutive steps into a HIP graph (on the current
        stream, which must not be the null stream)."""
        self._check_state(U)
        g = ctypes.c_void_p()
        check(lib().amr_graph_create(self._h, _ptr(U), _ptr(dt), int(first_step), _stream(), ctypes.byref(g)))
        return Graph(g, self, U, dt)

    # adjoint ----------------------------------------------------------
    def adjoint_scratch(self) -> torch.Tensor:
        n = (int(self.info.adjoint_scratch_bytes) + 7) // 8
        return torch.empty(n, dtype=torch.float64, device=self.device)

    def adjoint_face_scratch(self) -> torch.Tensor:
        n = (int(self.info.adjoint_face_bytes) + 7) // 8
        return torch.empty(max(n, 1), dtype=torch.float64, device=self.device)

    @staticmethod
    def _check_scratch(scratch: torch.Tensor, nbytes: int) -> None:
        if scratch.dtype != torch.float64 or not scratch.is_contiguous() or scratch.numel() * 8 < nbytes:
            raise ValueError("adjoint scratch too small or of the wrong type")

    def step_adjoint(self, U_in: torch.Tensor, dt: torch.Tensor, lam: torch.Tensor, scratch: torch.Tensor,
                     k: int) -> None:
        """lam <- (d step_k / d U_in)^T lam, dt frozen, U_in the checkpoint."""
        self._check_state(U_in)
        self._check_state(lam)
        self._check_scratch(scratch, int(self.info.adjoint_scratch_bytes))
        check(lib().amr_hydro_step_adjoint(self._h, _ptr(U_in), _ptr(dt), _ptr(lam), _ptr(scratch), int(k),
                                           _stream()))

    def step_record(self, U: torch.Tensor, dt: torch.Tensor, S1: torch.Tensor, S2: torch.Tensor,
                    U_out: torch.Tensor, floors: torch.Tensor, k: int) -> None:
        """Step k from U (ghosts refreshed in place, otherwise unchanged) into
        U_out, keeping the second and third sweeps' inputs in S1, S2 and the
        step's floor-reset count in floors (one int64 on the device)."""
        for X in (U, S1, S2, U_out):
            self._check_state(X)
        if floors.dtype != torch.int64 or floors.numel() < 1 or floors.device != self.device:
            raise ValueError("floors must be an int64 device tensor")
        check(lib().amr_hydro_step_record(self._h, _ptr(U), _ptr(dt), _ptr(S1), _ptr(S2), _ptr(U_out),
                                          _ptr(floors), int(k), _stream()))

    def step_adjoint_recorded(self, S0: torch.Tensor, S1: torch.Tensor, S2: torch.Tensor, dt: torch.Tensor,
                              floors: torch.Tensor, lam: torch.Tensor, scratch: torch.Tensor, k: int,
                              floors_host: int = -1) -> None:
        """lam <- (d step_k / d U)^T lam from what step_record kept;
        floors_host: the recorded floor-reset count if already read on the
        host (only the matching transpose kernels run), else -1."""
        for X in (S0, S1, S2, lam):
            self._check_state(X)
        self._check_scratch(scratch, int(self.info.adjoint_face_bytes))
        check(lib().amr_hydro_step_adjoint_recorded(self._h, _ptr(S0), _ptr(S1), _ptr(S2), _ptr(dt),
                                                    _ptr(floors), int(floors_host), _ptr(lam), _ptr(scratch),
                                                    int(k), _stream()))

    def step_comoving_record(self, U: torch.Tensor, dt: torch.Tensor, a: float, hubble: float, S1: torch.Tensor,
                             S2: torch.Tensor, U_pre: torch.Tensor, U_out: torch.Tensor, floors: torch.Tensor,
                             k: int) -> None:
        """Comoving step k (dt given on the device; a, H at the mid time) from
        U into U_out as step_record does, keeping also the state before the
        expansion sources in U_pre."""
        for X in (U, S1, S2, U_pre, U_out):
            self._check_state(X)
        if floors.dtype != torch.int64 or floors.numel() < 1 or floors.device != self.device:
            raise ValueError("floors must be an int64 device tensor")
        check(lib().amr_hydro_step_comoving_record(self._h, _ptr(U), _ptr(dt), ctypes.c_double(a),
                                                   ctypes.c_double(hubble), _ptr(S1), _ptr(S2), _ptr(U_pre),
                                                   _ptr(U_out), _ptr(floors), int(k), _stream()))

    def step_comoving_adjoint_recorded(self, S0: torch.Tensor, S1: torch.Tensor, S2: torch.Tensor,
                                       U_pre: torch.Tensor, dt: torch.Tensor, a: float, hubble: float,
                                       floors: torch.Tensor, lam: torch.Tensor, scratch: torch.Tensor, k: int,
                                       floors_host: int = -1) -> None:
        """lam <- (d comoving step_k / d U)^T lam from what
        step_comoving_record kept."""
        for X in (S0, S1, S2, U_pre, lam):
            self._check_state(X)
        self._check_scratch(scratch, int(self.info.adjoint_face_bytes))
        check(lib().amr_hydro_step_comoving_adjoint_recorded(
            self._h, _ptr(S0), _ptr(S1), _ptr(S2), _ptr(U_pre), _ptr(dt), ctypes.c_double(a),
            ctypes.c_double(hubble), _ptr(floors), int(floors_host), _ptr(lam), _ptr(scratch), int(k), _stream()))

    def refresh_adjoint(self, U_ref: torch.Tensor, lam: torch.Tensor) -> None:
        self._check_state(U_ref)
        self._check_state(lam)
        check(lib().amr_refresh_ghosts_adjoint(self._h, _ptr(U_ref), _ptr(lam), _stream()))

    # mg0 Poisson solver ---------------------------------------------
    def poisson_workspace(self) -> torch.Tensor:
        """Device workspace of poisson_solve (the level arrays)."""
        n = ctypes.c_int64()
        check(lib().amr_poisson_workspace_bytes(self._h, ctypes.byref(n)))
        return torch.empty((int(n.value) + 7) // 8, dtype=torch.float64, device=self.device)

    def poisson_solve(self, f: torch.Tensor, phi: torch.Tensor, ncycles: int, nu1: int = 2, nu2: int = 2,
                      work: torch.Tensor = None, resid: bool = True):
        """ncycles mg0 V(nu1, nu2) cycles on lap(phi) = f (uniform periodic mesh);
        f and phi are [n_leaves, N, N, N] float64 device tensors (phi: initial
        guess in, mean-free result out).  Returns the residual norms (device
        tensor of ncycles + 1) or None."""
        shape = (self.nleaf, self.N, self.N, self.N)
        for t in (f, phi):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device or tuple(t.shape) != shape:
                raise ValueError("f and phi must be contiguous float64 [n_leaves, N, N, N] tensors on the device")
        if work is None:
            work = self.poisson_workspace()
        r = torch.empty(ncycles + 1, dtype=torch.float64, device=self.device) if resid else None
        check(lib().amr_poisson_solve(self._h, _ptr(f), _ptr(phi), int(ncycles), int(nu1), int(nu2),
                                      _ptr(r) if r is not None else None, _ptr(work), _stream()))
        return r

    def poisson_solve_static(self, f: torch.Tensor, phi: torch.Tensor, ncycles: int, nu1: int = 2, nu2: int = 2,
                             resid: torch.Tensor = None) -> None:
        """poisson_solve with the library's fixed device buffer as workspace
        (the entry point that allocates nothing; grids up to 128^3).  resid:
        None or a caller-allocated float64 device tensor of ncycles + 1."""
        shape = (self.nleaf, self.N, self.N, self.N)
        for t in (f, phi):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device or tuple(t.shape) != shape:
                raise ValueError("f and phi must be contiguous float64 [n_leaves, N, N, N] tensors on the device")
        if resid is not None and (resid.dtype != torch.float64 or resid.numel() < ncycles + 1
                                  or resid.device != self.device):
            raise ValueError("resid must be a float64 device tensor of ncycles + 1 entries")
        check(lib().amr_poisson_solve_static(self._h, _ptr(f), _ptr(phi), int(ncycles), int(nu1), int(nu2),
                                             _ptr(resid) if resid is not None else None, _stream()))

    def step_gravity(self, U: torch.Tensor, dt: torch.Tensor, k: int, four_pi_G: float, phi: torch.Tensor,
                     phi_current: bool, ncycles: int = 2, nu1: int = 2, nu2: int = 2,
                     work: torch.Tensor = None) -> None:
        """Self-gravity step (kick-drift-kick with the mg0 potential of
        four_pi_G (rho - mean rho)); phi: [n_leaves, N, N, N] mean-free
        potential, current for U's density if phi_current, updated to the new
        density."""
        self._check_state(U)
        if phi.dtype != torch.float64 or not phi.is_contiguous() or phi.numel() != self.nleaf * self.N ** 3:
            raise ValueError("phi must be a contiguous float64 [n_leaves, N, N, N] tensor")
        if work is None:
            work = self.poisson_workspace()
        check(lib().amr_hydro_step_gravity(self._h, _ptr(U), _ptr(dt), int(k), ctypes.c_double(four_pi_G),
                                           _ptr(phi), int(bool(phi_current)), int(ncycles), int(nu1), int(nu2),
                                           _ptr(work), _stream()))

    def step_gravity_comoving(self, U: torch.Tensor, dt: torch.Tensor, k: int, a0: float, a_mid: float, a1: float,
                              hubble: float, four_pi_G: float, phi: torch.Tensor, phi_current: bool,
                              ncycles: int = 2, nu1: int = 2, nu2: int = 2, work: torch.Tensor = None) -> None:
        """Comoving self-gravity step with the given dt (device): kicks
        (dt/2)/a^2 at the start (a0) and end (a1) with the a-free potential
        of four_pi_G (rho - mean rho), expansion sources over dt/2 on both
        sides of the hydro step, which runs with dt / a_mid; H = hubble at
        the mid time."""
        self._check_state(U)
        if phi.dtype != torch.float64 or not phi.is_contiguous() or phi.numel() != self.nleaf * self.N ** 3:
            raise ValueError("phi must be a contiguous float64 [n_leaves, N, N, N] tensor")
        if work is None:
            work = self.poisson_workspace()
        d = ctypes.c_double
        check(lib().amr_hydro_step_gravity_comoving(self._h, _ptr(U), _ptr(dt), int(k), d(a0), d(a_mid), d(a1),
                                                    d(hubble), d(four_pi_G), _ptr(phi), int(bool(phi_current)),
                                                    int(ncycles), int(nu1), int(nu2), _ptr(work), _stream()))

    # remesh -----------------------------------------------------------
    def indicator(self, U: torch.Tensor) -> torch.Tensor:
        """Per-leaf density-slope indicator (ghosts of U must be refreshed)."""
        self._check_state(U)
        out = torch.empty(self.nleaf, dtype=torch.float64, device=self.device)
        check(lib().amr_indicator(self._h, _ptr(U), _ptr(out), _stream()))
        return out

    def remesh(self, U: torch.Tensor, refine_slope: float, coarsen_slope: float, max_blocks: int,
               out: torch.Tensor = None):
        """Returns (new Mesh, new state, stats dict).  Refreshes U's ghosts.
        `out`, if given, is a flat float64 device buffer of at least
        max_blocks blocks that receives the new state (no allocation).  When
        nothing is refined or coarsened the leaf set and its order are
        unchanged: this mesh and U itself are returned (no migration)."""
        self._check_state(U)
        prm = _lib.RemeshParams(float(refine_slope), float(coarsen_slope), int(max_blocks))
        st = _lib.RemeshStats()
        h = ctypes.c_void_p()
        check(lib().amr_remesh_plan(self._h, _ptr(U), ctypes.byref(prm), ctypes.byref(h), ctypes.byref(st),
                                    _stream()))
        stats = {"refined": int(st.refined), "coarsened": int(st.coarsened), "refused": int(st.refused),
                 "n_leaves": int(st.n_leaves)}
        if not h.value:  # nothing refined or coarsened: no new mesh
            return self, U, stats
        new = Mesh(device=self.device, _handle=h, **self.params)
        new.set_launch(**self.get_launch())
        # ghosts are scratch that the next refresh fills; migration writes
        # every active cell.  Cached free blocks are released first so that
        # a state near the capacity limit finds contiguous memory.
        shape = (new.nleaf, new.nf, new.M, new.M, new.M)
        if out is not None:
            n = new.nleaf * new.nf * new.M ** 3
            if out.dtype != torch.float64 or out.numel() < n or out.device != self.device:
                raise ValueError("out buffer too small or of the wrong type")
            if out.data_ptr() == U.data_ptr():
                raise ValueError("out must not alias the old state")
            Un = out[:n].view(shape)
        else:
            torch.cuda.empty_cache()
            Un = torch.empty(shape, dtype=torch.float64, device=self.device)
        check(lib().amr_remesh_apply(new._h, _ptr(U), _ptr(Un), _stream()))
        return new, Un, stats

    # launch shapes ----------------------------------------------------
    def get_launch(self) -> dict:
        c = _lib.LaunchCfg()
        check(lib().amr_mesh_get_launch(self._h, ctypes.byref(c)))
        return {"sweep_mode": list(c.sweep_mode), "sweep_block": c.sweep_block,
                "refresh_block": c.refresh_block, "reflux_block": c.reflux_block}

    def set_launch(self, **kw) -> None:
        cur = self.get_launch()
        cur.update(kw)
        c = _lib.LaunchCfg()
        c.sweep_mode[:] = [int(v) for v in cur["sweep_mode"]]
        c.sweep_block = int(cur["sweep_block"])
        c.refresh_block = int(cur["refresh_block"])
        c.reflux_block = int(cur["reflux_block"])
        check(lib().amr_mesh_set_launch(self._h, ctypes.byref(c)))

    # profiling --------------------------------------------------------
    def profile(self, on: bool) -> None:
        check(lib().amr_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """Summed kernel ms and launch counts per phase since profile(True)."""
        ms = np.zeros(len(_lib.PHASES))
        n = np.zeros(len(_lib.PHASES), dtype=np.int64)
        check(lib().amr_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                     n.ctypes.data_as(ctypes.c_void_p)))
        return {p: (float(ms[i]), int(n[i])) for i, p in enumerate(_lib.PHASES)}


class Graph:
    """Two captured steps; launch() advances the bound state by two steps."""

    def __init__(self, handle, mesh, U, dt):
        self._h, self._keep = handle, (mesh, U, dt)

    def launch(self) -> None:
        check(lib().amr_graph_launch(self._h, _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib._lib is not None:
            _lib._lib.amr_graph_destroy(h)
            self._h = None
