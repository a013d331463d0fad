"""Tracer particles of a mesh on the GPU (the C ABI's amr_tracer_set_t):
two sets of per-leaf slots, the step writing the one it does not read, and
the persistent scratch of the tracer calls.  Positions are in level-0 cell
units (X in [0, root[0] N) etc.)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .mesh import _ptr, _stream

BATCH = 256


class Tracers:
    def __init__(self, mesh, capacity: int):
        if capacity <= 0 or capacity % BATCH:
            raise ValueError("capacity must be a positive multiple of 256")
        self.mesh, self.cap = mesh, int(capacity)
        dev, n = mesh.device, mesh.nleaf
        self.sets = [(torch.zeros((3, n, self.cap), dtype=torch.float64, device=dev),
                      torch.zeros((n, self.cap), dtype=torch.int64, device=dev),
                      torch.zeros(n, dtype=torch.int32, device=dev)) for _ in range(2)]
        self.cur = 0
        nb = ctypes.c_int64()
        check(lib().amr_tracer_scratch_bytes(mesh._h, self.cap, ctypes.byref(nb)))
        self.scratch = torch.zeros(int(nb.value), dtype=torch.uint8, device=dev)

    @classmethod
    def from_positions(cls, mesh, pos: np.ndarray, ids: np.ndarray, capacity: int = None) -> "Tracers":
        """pos[leaf, n, 3], ids[leaf, n] (host) in the mesh's storage order."""
        n = pos.shape[1]
        if capacity is None:
            capacity = ((2 * n + BATCH - 1) // BATCH) * BATCH
        t = cls(mesh, capacity)
        if n > t.cap:
            raise ValueError("more particles per leaf than the capacity")
        P, I, C = t.sets[0]
        P[:, :, :n] = torch.from_numpy(np.ascontiguousarray(np.moveaxis(pos, 2, 0))).to(mesh.device)
        I[:, :n] = torch.from_numpy(np.ascontiguousarray(ids)).to(mesh.device)
        C.fill_(n)
        return t

    def _set(self, i) -> _lib.TracerSet:
        P, I, C = self.sets[i]
        return _lib.TracerSet(P.data_ptr(), I.data_ptr(), C.data_ptr())

    def step(self, U: torch.Tensor, dt: torch.Tensor, k: int) -> None:
        """One hydro step of the mesh that also advances the tracers."""
        self.mesh._check_state(U)
        a, b = self._set(self.cur), self._set(1 - self.cur)
        check(lib().amr_hydro_step_tracers(self.mesh._h, _ptr(U), _ptr(dt), ctypes.byref(a), ctypes.byref(b),
                                           self.cap, _ptr(self.scratch), int(k), _stream()))
        self.cur = 1 - self.cur

    def advance(self, U: torch.Tensor, dt: torch.Tensor) -> None:
        """Advance the tracers alone (U's ghosts must be refreshed)."""
        self.mesh._check_state(U)
        a, b = self._set(self.cur), self._set(1 - self.cur)
        check(lib().amr_tracers_advance(self.mesh._h, _ptr(U), _ptr(dt), ctypes.byref(a), ctypes.byref(b),
                                        self.cap, _ptr(self.scratch), _stream()))
        self.cur = 1 - self.cur

    def remesh(self, new_mesh) -> "Tracers":
        """The tracers moved onto `new_mesh`, the result of this mesh's remesh
        (itself if the remesh kept the mesh)."""
        if new_mesh is self.mesh:
            return self
        t = Tracers(new_mesh, self.cap)
        a, b = self._set(self.cur), t._set(0)
        check(lib().amr_tracers_remesh(new_mesh._h, self.mesh.nleaf, ctypes.byref(a), ctypes.byref(b), self.cap,
                                       _ptr(t.scratch), _stream()))
        return t

    def counters(self, reset: bool = False) -> dict:
        out = np.zeros(3, dtype=np.int64)
        check(lib().amr_tracer_counters(self.mesh._h, _ptr(self.scratch), self.cap,
                                        out.ctypes.data_as(ctypes.c_void_p), int(bool(reset)), _stream()))
        return {"overflow": int(out[0]), "removed": int(out[1]), "lost": int(out[2])}

    def to_host(self):
        """(leaf[n], pos[n, 3], ids[n]) of every particle, host arrays."""
        P, I, C = self.sets[self.cur]
        cnt = C.cpu().numpy()
        Ph, Ih = P.cpu().numpy(), I.cpu().numpy()
        leaf = np.repeat(np.arange(len(cnt)), cnt)
        slot = np.concatenate([np.arange(c) for c in cnt]) if len(cnt) else np.zeros(0, dtype=np.int64)
        pos = np.stack([Ph[a][leaf, slot] for a in range(3)], axis=1)
        return leaf, pos, Ih[leaf, slot]

    @property
    def count(self) -> int:
        return int(self.sets[self.cur][2].sum())
