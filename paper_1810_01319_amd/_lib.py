"""ctypes declarations of the C ABI in include/amr.h (argument marshalling only).

The HIP library must have been built (``python -m paper_1810_01319_amd._build``);
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libamr.so")

AMR_OK = 0
STATUS = {-1: "AMR_E_INVALID", -2: "AMR_E_BALANCE", -3: "AMR_E_NOMEM", -4: "AMR_E_HIP",
          -5: "AMR_E_CAPACITY", -6: "AMR_E_STATE"}
BC = {"periodic": 0, "outflow": 1}
PHASES = ["cfl", "refresh1", "refresh2", "sweep_x", "sweep_y", "sweep_z", "reflux",
          "adj_recompute", "adj_reflux", "adj_sweep_x", "adj_sweep_y", "adj_sweep_z", "adj_refresh", "tracers",
          "expansion", "poisson"]


class AmrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("root", ctypes.c_int32 * 3),
        ("block_cells", ctypes.c_int32),
        ("ghost", ctypes.c_int32),
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


class TracerSet(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("id", ctypes.c_void_p), ("count", ctypes.c_void_p)]


class MeshInfo(ctypes.Structure):
    _fields_ = [
        ("n_leaves", ctypes.c_int64),
        ("block_cells", ctypes.c_int32),
        ("padded", ctypes.c_int32),
        ("block_stride", ctypes.c_int64),
        ("field_stride", ctypes.c_int64),
        ("field_bytes", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("n_cf_faces", ctypes.c_int64),
        ("levels", ctypes.c_int32 * 8),
        ("n_instances", ctypes.c_int64),
        ("adjoint_scratch_bytes", ctypes.c_int64),
        ("adjoint_face_bytes", ctypes.c_int64),
        ("n_fields", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
    ]


class LaunchCfg(ctypes.Structure):
    _fields_ = [
        ("sweep_mode", ctypes.c_int32 * 3),
        ("sweep_block", ctypes.c_int32),
        ("refresh_block", ctypes.c_int32),
        ("reflux_block", ctypes.c_int32),
    ]


class RemeshParams(ctypes.Structure):
    _fields_ = [("refine_slope", ctypes.c_double), ("coarsen_slope", ctypes.c_double),
                ("max_blocks", ctypes.c_int64)]


class RemeshStats(ctypes.Structure):
    _fields_ = [("refined", ctypes.c_int64), ("coarsened", ctypes.c_int64), ("refused", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64)]


# every entry point declared in include/amr.h: name -> (restype, argtypes)
_P, _I64, _I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
SIGNATURES = {
    "amr_mesh_create": (_I32, [ctypes.POINTER(MeshDesc), ctypes.POINTER(_P)]),
    "amr_mesh_create_from_leaves": (_I32, [ctypes.POINTER(MeshDesc), _I64, _P, ctypes.POINTER(_P)]),
    "amr_batch_create": (_I32, [_P, _I32, ctypes.POINTER(_P)]),
    "amr_mesh_instance_offsets": (_I32, [_P, _P, _I64]),
    "amr_graph_create": (_I32, [_P, _P, _P, _I64, _P, ctypes.POINTER(_P)]),
    "amr_graph_launch": (_I32, [_P, _P]),
    "amr_graph_destroy": (_I32, [_P]),
    "amr_mesh_destroy": (_I32, [_P]),
    "amr_mesh_info": (_I32, [_P, ctypes.POINTER(MeshInfo)]),
    "amr_mesh_blocks": (_I32, [_P, _P, _I64]),
    "amr_mesh_upload": (_I32, [_P, _P, _P]),
    "amr_refresh_ghosts": (_I32, [_P, _P, _P]),
    "amr_cfl_dt": (_I32, [_P, _P, _P, _P]),
    "amr_hydro_step": (_I32, [_P, _P, _P, _I64, _P]),
    "amr_batch_step": (_I32, [_P, _P, _P, _I64, _P]),
    "amr_hydro_step_dt": (_I32, [_P, _P, _P, _I64, _P]),
    "amr_hydro_step_adjoint": (_I32, [_P, _P, _P, _P, _P, _I64, _P]),
    "amr_hydro_step_record": (_I32, [_P, _P, _P, _P, _P, _P, _P, _I64, _P]),
    "amr_tracer_scratch_bytes": (_I32, [_P, _I64, _P]),
    "amr_tracers_advance": (_I32, [_P, _P, _P, _P, _P, _I64, _P, _P]),
    "amr_hydro_step_tracers": (_I32, [_P, _P, _P, _P, _P, _I64, _P, _I64, _P]),
    "amr_tracer_counters": (_I32, [_P, _P, _I64, _P, _I32, _P]),
    "amr_tracers_remesh": (_I32, [_P, _I64, _P, _P, _I64, _P, _P]),
    "amr_hydro_steps_comoving": (_I32, [_P, _P, _P, _I64, _I64] + [ctypes.c_double] * 3 + [_P, _P]),
    "amr_hydro_step_adjoint_recorded": (_I32, [_P, _P, _P, _P, _P, _P, _I64, _P, _P, _I64, _P]),
    "amr_refresh_ghosts_adjoint": (_I32, [_P, _P, _P, _P]),
    "amr_floor_count": (_I32, [_P, ctypes.POINTER(_I64), _P]),
    "amr_remesh_plan": (_I32, [_P, _P, ctypes.POINTER(RemeshParams), ctypes.POINTER(_P),
                               ctypes.POINTER(RemeshStats), _P]),
    "amr_remesh_plan_host": (_I32, [_P, _P, ctypes.POINTER(RemeshParams), ctypes.POINTER(_P),
                                    ctypes.POINTER(RemeshStats)]),
    "amr_remesh_apply": (_I32, [_P, _P, _P, _P]),
    "amr_indicator": (_I32, [_P, _P, _P, _P]),
    "amr_mesh_set_launch": (_I32, [_P, ctypes.POINTER(LaunchCfg)]),
    "amr_mesh_get_launch": (_I32, [_P, ctypes.POINTER(LaunchCfg)]),
    "amr_profile_enable": (_I32, [_P, _I32]),
    "amr_profile_read": (_I32, [_P, _P, _P]),
    "amr_arith_selftest": (_I32, [ctypes.c_uint64, _I64, _P, _P]),
    "amr_poisson_workspace_bytes": (_I32, [_P, ctypes.POINTER(_I64)]),
    "amr_poisson_solve": (_I32, [_P, _P, _P, _I32, _I32, _I32, _P, _P, _P]),
    "amr_poisson_solve_static": (_I32, [_P, _P, _P, _I32, _I32, _I32, _P, _P]),
    "amr_hydro_step_gravity": (_I32, [_P, _P, _P, _I64, ctypes.c_double, _P, _I32, _I32, _I32, _I32, _P, _P]),
    "amr_hydro_step_gravity_comoving": (_I32, [_P, _P, _P, _I64] + [ctypes.c_double] * 5
                                        + [_P, _I32, _I32, _I32, _I32, _P, _P]),
    "amr_cfl_dt_comoving": (_I32, [_P, _P, ctypes.c_double, _P, _P]),
    "amr_hydro_steps": (_I32, [_P, _P, _P, _I64, _I64, _P]),
    "amr_hydro_steps_fresh": (_I32, [_P, _P, _P, _I64, _I64, _P]),
    "amr_hydro_step_comoving": (_I32, [_P, _P, _P, _I64, ctypes.c_double, ctypes.c_double, _P]),
    "amr_hydro_step_comoving_record": (_I32, [_P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P,
                                              _I64, _P]),
    "amr_hydro_step_comoving_adjoint_recorded": (_I32, [_P, _P, _P, _P, _P, _P, ctypes.c_double, ctypes.c_double,
                                                        _P, _I64, _P, _P, _I64, _P]),
    "amr_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The HIP library; AMR_LIBRARY may name another build of the same
    sources (the sanitizer build of the CPU suite)."""
    global _lib
    if _lib is None:
        so = os.environ.get("AMR_LIBRARY", "") or SO
        if not os.path.exists(so):
            raise ImportError(f"HIP library {so} is not built; run python -m paper_1810_01319_amd._build")
        L = ctypes.CDLL(so)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != AMR_OK:
        raise AmrError(rc, lib().amr_last_error().decode())


def make_desc(root, block_cells, max_level=0, bc="periodic", gamma=1.4, cfl=0.4, rho_floor=1e-20,
              p_floor=1e-20, riemann_iters=5, refine=(), ghost=3, dual_energy=False, eta1=1e-3, eta2=0.1):
    import numpy as np

    d = MeshDesc()
    d.root[:] = [int(r) for r in root]
    d.block_cells = int(block_cells)
    d.ghost = int(ghost)
    d.max_level = int(max_level)
    bcs = [bc] * 3 if isinstance(bc, str) else list(bc)
    d.bc[:] = [BC[b] if isinstance(b, str) else int(b) for b in bcs]
    d.gamma, d.cfl = float(gamma), float(cfl)
    d.rho_floor, d.p_floor = float(rho_floor), float(p_floor)
    d.riemann_iters = int(riemann_iters)
    d.dual_energy = int(dual_energy)
    d.eta1, d.eta2 = float(eta1), float(eta2)
    ref = np.ascontiguousarray(np.asarray(refine, dtype=np.int32).reshape(-1, 4))
    d.n_refine = ref.shape[0]
    d.refine = ref.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if ref.size else None
    return d, ref
