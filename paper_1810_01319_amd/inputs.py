"""Seeded synthetic inputs: mesh descriptions and initial states.

This module holds no arithmetic of the method (no refresh, no sweep, no
Riemann solve).  It only states the problems: which blocks are refined, and
the initial conserved fields at cell centres.  It is the one module shared by
the HIP path's callers and by the test-suite's oracle runs, so both start from
byte-identical inputs.

The workloads follow the paper's test problems (Sec. III): an array of blast
waves (one per root octree, at seeded random offsets instead of the paper's
letter-shaped sources, for the same purpose of breaking lockstep refinement)
and, as smaller checks, the Sod shock tube and a single Sedov blast.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Sequence, Tuple

import numpy as np

GHOST = 3
NFIELD = 5  # rho, m_x, m_y, m_z, E


@dataclass
class MeshSpec:
    """Plain description of one array-of-octrees mesh and its gas."""

    root: Tuple[int, int, int]
    block_cells: int
    max_level: int = 0
    bc: str = "periodic"            # "periodic" or "outflow" (all axes)
    gamma: float = 1.4
    cfl: float = 0.4
    rho_floor: float = 1e-20
    p_floor: float = 1e-20
    riemann_iters: int = 5
    refine: List[Tuple[int, int, int, int]] = field(default_factory=list)
    dual_energy: bool = False       # sixth field rho e (internal energy density)
    eta1: float = 1e-3              # its pressure-selection threshold
    eta2: float = 0.1               # its resynchronisation threshold

    def kwargs(self) -> dict:
        kw = dict(root=tuple(self.root), block_cells=self.block_cells, max_level=self.max_level,
                  bc=self.bc, gamma=self.gamma, cfl=self.cfl, rho_floor=self.rho_floor,
                  p_floor=self.p_floor, riemann_iters=self.riemann_iters,
                  refine=list(self.refine))
        if self.dual_energy:
            kw.update(dual_energy=True, eta1=self.eta1, eta2=self.eta2)
        return kw

    @property
    def nfields(self) -> int:
        return 6 if self.dual_energy else 5

    def dx(self, level: int) -> float:
        return 1.0 / float(self.root[0] * self.block_cells * (1 << level))


def cell_centres(spec: MeshSpec, keys: np.ndarray):
    """x, y, z cell-centre coordinates of the active cells, each [n, N, N, N]
    (index order z, y, x as in the block storage)."""
    N = spec.block_cells
    keys = np.asarray(keys, dtype=np.int64)
    lev = keys[:, 0]
    dx = np.array([spec.dx(int(l)) for l in lev])
    r = np.arange(N, dtype=np.float64) + 0.5
    out = []
    for ax in range(3):
        origin = keys[:, 1 + ax].astype(np.float64) * N
        c = (origin[:, None] + r[None, :]) * dx[:, None]  # [n, N]
        shape = [len(keys), 1, 1, 1]
        shape[3 - ax] = N
        out.append(np.broadcast_to(c.reshape(shape), (len(keys), N, N, N)))
    return out


def conserved(gamma: float, rho, u, v, w, p) -> np.ndarray:
    """Conserved fields from primitives at cell centres (the initial state is
    defined by point values)."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast_shapes(np.shape(rho), np.shape(u), np.shape(v), np.shape(w), np.shape(p))
    out = np.empty((shape[0], NFIELD) + tuple(shape[1:]), dtype=np.float64)
    rho = np.broadcast_to(rho, shape)
    u, v, w, p = (np.broadcast_to(np.asarray(a, dtype=np.float64), shape) for a in (u, v, w, p))
    out[:, 0] = rho
    out[:, 1] = rho * u
    out[:, 2] = rho * v
    out[:, 3] = rho * w
    out[:, 4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return out


def cold_stream_state(spec: MeshSpec, keys, mach: float, amp: float = 0.2, p0: float = 1.0) -> np.ndarray:
    """A density wave riding a uniform stream along x at Mach `mach` (sound
    speed of the mean density) at uniform pressure p0; six fields, rho e =
    p0 / (gamma - 1) (not E - ke, which has lost the thermal digits)."""
    x, y, z = cell_centres(spec, keys)
    rho = 1.0 + amp * np.sin(2.0 * np.pi * x) * np.cos(2.0 * np.pi * y)
    u0 = mach * np.sqrt(spec.gamma * p0)
    act = conserved(spec.gamma, rho, u0, 0.0, 0.0, np.full(rho.shape, p0))
    ge = np.full(rho.shape, p0 / (spec.gamma - 1.0))
    return np.concatenate([act, ge[:, None]], axis=1)


def with_internal_energy(act: np.ndarray) -> np.ndarray:
    """Append the dual-energy field rho e = E - |m|^2 / (2 rho) to a state of
    five conserved fields (an initial internal energy consistent with E)."""
    act = np.asarray(act, dtype=np.float64)
    rho, m, E = act[:, 0], act[:, 1:4], act[:, 4]
    ge = E - 0.5 * (m[:, 0] ** 2 + m[:, 1] ** 2 + m[:, 2] ** 2) / rho
    return np.concatenate([act, ge[:, None]], axis=1)


# ---------------------------------------------------------------------------
# Sod shock tube along x (uniform level, outflow)
# ---------------------------------------------------------------------------

def sod_spec(root=(4, 4, 4), block_cells=16) -> MeshSpec:
    return MeshSpec(root=tuple(root), block_cells=block_cells, max_level=0, bc="outflow",
                    gamma=1.4, cfl=0.4)


def sod_state(spec: MeshSpec, keys) -> np.ndarray:
    """Left (rho=1, p=1) for x < 0.5, right (rho=0.125, p=0.1); at rest.  The
    jump lies on a cell face, so the initial state is exact."""
    x, _, _ = cell_centres(spec, keys)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return conserved(spec.gamma, rho, 0.0, 0.0, 0.0, p)


# ---------------------------------------------------------------------------
# Sedov blast on a static two-level refinement around the domain centre
# ---------------------------------------------------------------------------

def centre_refine_list(root: int, levels: int) -> List[Tuple[int, int, int, int]]:
    """Refine the 8 blocks touching the domain centre at each level < levels
    (the centre is a vertex shared by 8 blocks when root is even)."""
    assert root % 2 == 0
    out = []
    for l in range(levels):
        h = root * (1 << l) // 2
        for k in (h - 1, h):
            for j in (h - 1, h):
                for i in (h - 1, h):
                    out.append((l, i, j, k))
    return out


def sedov_spec(root=8, block_cells=32, levels=2, gamma=5.0 / 3.0) -> MeshSpec:
    return MeshSpec(root=(root, root, root), block_cells=block_cells, max_level=levels,
                    bc="periodic", gamma=gamma, cfl=0.4, refine=centre_refine_list(root, levels))


def blast_state(spec: MeshSpec, keys, centres, energy=1.0, rho0=1.0, p0=1e-5, radius_cells=2.0,
                level=None) -> np.ndarray:
    """Ambient gas plus, per centre, energy deposited uniformly (as energy
    density) in the cells of level `level` (default: the finest present)
    whose centre lies within radius_cells * dx of the blast centre
    (periodic minimum image).  The deposited total is exactly `energy` per
    blast in exact arithmetic."""
    keys = np.asarray(keys)
    x, y, z = cell_centres(spec, keys)
    lev = keys[:, 0]
    lv = int(lev.max()) if level is None else int(level)
    dx = spec.dx(lv)
    ext = np.array(spec.root, dtype=np.float64) / spec.root[0]
    U = conserved(spec.gamma, np.full(x.shape, rho0), 0.0, 0.0, 0.0, np.full(x.shape, p0))
    on_level = (lev == lv)[:, None, None, None]
    for c in np.atleast_2d(np.asarray(centres, dtype=np.float64)):
        d2 = np.zeros(x.shape)
        for a, X in enumerate((x, y, z)):
            d = X - c[a]
            if spec.bc == "periodic":
                d = d - ext[a] * np.round(d / ext[a])
            d2 = d2 + d * d
        sel = (d2 < (radius_cells * dx) ** 2) & on_level
        n = int(sel.sum())
        if n == 0:
            raise ValueError("blast deposit region is empty")
        U[:, 4][sel] += energy / (n * dx ** 3)
    return U


def sedov_state(spec: MeshSpec, keys) -> np.ndarray:
    ext = np.array(spec.root, dtype=np.float64) / spec.root[0]
    return blast_state(spec, keys, [0.5 * ext], energy=1.0, rho0=1.0, p0=1e-5, radius_cells=2.0)


# ---------------------------------------------------------------------------
# Smooth random fields for parity, conservation and symmetry checks
# ---------------------------------------------------------------------------

def smooth_state(spec: MeshSpec, keys, seed: int, amp=0.2, vel=0.5) -> np.ndarray:
    """A periodic smooth state: a few random low Fourier modes in rho, u, v,
    w, p, evaluated at cell centres (seeded, numpy PCG64)."""
    rng = np.random.default_rng(seed)
    x, y, z = cell_centres(spec, keys)
    ext = np.array(spec.root, dtype=np.float64) / spec.root[0]

    def field_(base, a):
        out = np.full(x.shape, base)
        for _ in range(3):
            k = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            c = rng.uniform(-1, 1)
            out = out + a * c * np.sin(2 * np.pi * (k[0] * x / ext[0] + k[1] * y / ext[1] + k[2] * z / ext[2]) + ph)
        return out

    rho = field_(1.0, amp)
    u = field_(0.0, vel)
    v = field_(0.0, vel)
    w = field_(0.0, vel)
    p = field_(1.0, amp)
    return conserved(spec.gamma, rho, u, v, w, p)


def random_refine_list(root, max_level, n, seed) -> List[Tuple[int, int, int, int]]:
    """n random refinement requests at random levels < max_level."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        l = int(rng.integers(0, max_level))
        e = [int(r) << l for r in root]
        out.append((l, int(rng.integers(0, e[0])), int(rng.integers(0, e[1])), int(rng.integers(0, e[2]))))
    return out


def with_(spec: MeshSpec, **kw) -> MeshSpec:
    return replace(spec, **kw)


# ---------------------------------------------------------------------------
# Array of blasts, one per root octree (the paper's weak-scaling workload)
# ---------------------------------------------------------------------------

def blasts_spec(root=24, block_cells=32, levels=3) -> MeshSpec:
    """Uniform start on root^3 octrees of block_cells^3 cells, refined
    adaptively up to `levels` levels; gamma = 5/3, periodic."""
    return MeshSpec(root=(root, root, root), block_cells=block_cells, max_level=levels, bc="periodic",
                    gamma=5.0 / 3.0, cfl=0.4)


def blast_centres(root: int, seed: int = 5) -> np.ndarray:
    """One blast per root octree at the octree centre plus a uniform random
    offset in [-1/4, 1/4] of the octree width per axis (numpy PCG64, seeded;
    octrees in x-fastest order), standing in for the paper's randomly chosen
    letter-shaped sources that keep the refinement from proceeding in
    lockstep."""
    rng = np.random.default_rng(seed)
    w = 1.0 / root
    out = np.empty((root ** 3, 3))
    n = 0
    for k in range(root):
        for j in range(root):
            for i in range(root):
                out[n] = (np.array([i, j, k]) + 0.5) * w + rng.uniform(-0.25, 0.25, 3) * w
                n += 1
    return out


def blasts_state(spec: MeshSpec, keys, seed: int = 5) -> np.ndarray:
    """rho = 1, p = 1e-5 and E = 1 per blast deposited in the root-level cells
    within 2 dx_0 of its centre.  Each blast lies inside its own octree at
    least N/4 - 2 cells from the octree's faces, so only that octree's root
    block receives it; on a uniform level-0 mesh this is evaluated block by
    block (any subset of the root blocks, in any order)."""
    keys = np.asarray(keys)
    R = spec.root[0]
    centres = blast_centres(R, seed)
    if not np.all(keys[:, 0] == 0) or spec.block_cells < 16:
        return blast_state(spec, keys, centres, energy=1.0, rho0=1.0, p0=1e-5, radius_cells=2.0, level=0)
    N = spec.block_cells
    dx = spec.dx(0)
    x, y, z = cell_centres(spec, keys)
    own = centres[keys[:, 1] + R * (keys[:, 2] + R * keys[:, 3])]  # [n, 3]
    d2 = np.zeros(x.shape)
    for a, X in enumerate((x, y, z)):
        d = X - own[:, a][:, None, None, None]
        d2 = d2 + d * d
    sel = d2 < (2.0 * dx) ** 2
    nsel = sel.reshape(len(keys), -1).sum(axis=1)
    if np.any(nsel == 0):
        raise ValueError("blast deposit region is empty")
    U = conserved(spec.gamma, np.full(x.shape, 1.0), 0.0, 0.0, 0.0, np.full(x.shape, 1e-5))
    add = (1.0 / (nsel * dx ** 3))[:, None, None, None]
    U[:, 4] = np.where(sel, U[:, 4] + add, U[:, 4])
    return U


# ---------------------------------------------------------------------------
# Batched uneven meshes: Gaussian density blobs, one problem per instance
# ---------------------------------------------------------------------------

def batch_instance(i: int, block_cells: int = 16, seed0: int = 3000):
    """Instance i of the batched workload (numpy PCG64 seed seed0 + i): root
    array n^3 with n drawn from {2,4,6,8}, depth L in {0..3}, 1-3 blobs with
    centres uniform in [0,1)^3; rho = 1 + 0.5 sum_b exp(-r_b^2/0.01) (periodic
    minimum image), p = 1, at rest, gamma 5/3, periodic.  Static refinement:
    at each level l < L every block meeting a sphere of radius 0.1 * 2^-l
    around a blob centre.  Returns (MeshSpec, blob centres)."""
    rng = np.random.default_rng(seed0 + i)
    n = int(rng.choice([2, 4, 6, 8]))
    L = int(rng.integers(0, 4))
    nb = int(rng.integers(1, 4))
    centres = rng.uniform(0.0, 1.0, size=(nb, 3))
    refine = []
    for l in range(L):
        e = n << l
        w = 1.0 / e
        rad = 0.1 * 2.0 ** (-l)
        idx = np.arange(e)
        lo = idx * w
        for c in centres:
            # per-axis distance from the centre to each block interval, periodic
            dd = []
            for a in range(3):
                d = np.maximum(0.0, np.maximum(lo - c[a], c[a] - (lo + w)))
                d = np.minimum(d, np.maximum(0.0, np.maximum(lo - (c[a] + 1.0), (c[a] + 1.0) - (lo + w))))
                d = np.minimum(d, np.maximum(0.0, np.maximum(lo - (c[a] - 1.0), (c[a] - 1.0) - (lo + w))))
                dd.append(d)
            d2 = dd[0][None, None, :] ** 2 + dd[1][None, :, None] ** 2 + dd[2][:, None, None] ** 2
            kk, jj, ii = np.nonzero(d2 < rad * rad)
            refine.extend((l, int(a), int(b), int(c_)) for a, b, c_ in zip(ii, jj, kk))
    refine = sorted(set(refine))
    spec = MeshSpec(root=(n, n, n), block_cells=block_cells, max_level=max(L, 0), bc="periodic",
                    gamma=5.0 / 3.0, cfl=0.4, refine=refine)
    return spec, centres


def batch_state(spec: MeshSpec, keys, centres) -> np.ndarray:
    x, y, z = cell_centres(spec, keys)
    rho = np.ones(x.shape)
    for c in centres:
        d2 = np.zeros(x.shape)
        for a, X in enumerate((x, y, z)):
            d = X - c[a]
            d = d - np.round(d)
            d2 = d2 + d * d
        rho = rho + 0.5 * np.exp(-d2 / 0.01)
    return conserved(spec.gamma, rho, 0.0, 0.0, 0.0, np.ones(x.shape))


# ---------------------------------------------------------------------------
# Differentiation workload: density from a power-law Gaussian random field
# ---------------------------------------------------------------------------

def grf_spec(root=4, block_cells=32) -> MeshSpec:
    """root^3 octrees with the central 2x2x2 root blocks refined once."""
    h = root // 2
    refine = [(0, i, j, k) for k in (h - 1, h) for j in (h - 1, h) for i in (h - 1, h)]
    return MeshSpec(root=(root, root, root), block_cells=block_cells, max_level=1, bc="periodic",
                    gamma=5.0 / 3.0, cfl=0.4, refine=refine)


def gaussian_random_field(n: int, seed: int, slope: float = -3.0) -> np.ndarray:
    """Periodic Gaussian random field on an n^3 lattice with power spectrum
    P(k) ~ k^slope (amplitude ~ k^(slope/2)), k = 0 removed, unit RMS
    (numpy PCG64, seeded).  Index order (z, y, x)."""
    rng = np.random.default_rng(seed)
    white = rng.normal(size=(n, n, n))
    fk = np.fft.rfftn(white)
    kx = np.fft.rfftfreq(n) * n
    ky = np.fft.fftfreq(n) * n
    kz = np.fft.fftfreq(n) * n
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)
    f = np.fft.irfftn(fk * amp, s=(n, n, n), axes=(0, 1, 2))
    f -= f.mean()
    return f / np.sqrt(np.mean(f * f))


def grf_density(spec: MeshSpec, keys, seed: int, amplitude: float = 1e-2) -> np.ndarray:
    """rho = 1 + amplitude * field on the finest lattice (level max_level);
    coarser leaves take the mean of the lattice cells they cover."""
    L = spec.max_level
    N = spec.block_cells
    n = spec.root[0] * N << L
    field = 1.0 + amplitude * gaussian_random_field(n, seed)
    keys = np.asarray(keys)
    out = np.empty((len(keys), N, N, N))
    for s, (l, i, j, k) in enumerate(keys):
        r = 1 << (L - l)
        sub = field[k * N * r:(k + 1) * N * r, j * N * r:(j + 1) * N * r, i * N * r:(i + 1) * N * r]
        out[s] = sub.reshape(N, r, N, r, N, r).mean(axis=(1, 3, 5))
    return out


def grf_state(spec: MeshSpec, keys, seed: int = 4) -> np.ndarray:
    rho = grf_density(spec, keys, seed)
    return conserved(spec.gamma, rho, 0.0, 0.0, 0.0, np.ones_like(rho))


# ---------------------------------------------------------------------------
# Tracer particles: positions in level-0 cell units (X in [0, Rx*N) etc.)
# ---------------------------------------------------------------------------

def tracer_positions(spec: MeshSpec, keys, per_axis: int = 1, jitter_seed=None):
    """per_axis^3 particles in every active cell of every leaf, at the centres
    of a per_axis^3 sub-grid of the cell, optionally moved by a seeded uniform
    offset of up to half a sub-cell (numpy PCG64).  Returns (pos, ids):
    pos[leaf, n, 3] and ids[leaf, n] with n = (per_axis * N)^3, ids numbered
    in storage order."""
    keys = np.asarray(keys)
    N = spec.block_cells
    n1 = per_axis * N
    sub = (np.arange(n1) + 0.5) / per_axis  # sub-cell centres in cells
    z, y, x = np.meshgrid(sub, sub, sub, indexing="ij")
    local = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)  # [n, 3] in cells of the leaf's level
    pos = np.empty((len(keys), n1 ** 3, 3))
    rng = np.random.default_rng(jitter_seed) if jitter_seed is not None else None
    for s, (l, i, j, k) in enumerate(keys):
        q = local.copy()
        if rng is not None:
            q += rng.uniform(-0.5, 0.5, size=q.shape) / per_axis
        q += np.array([i, j, k], dtype=np.float64) * N
        pos[s] = q / float(1 << int(l))
    ids = np.arange(len(keys) * n1 ** 3, dtype=np.int64).reshape(len(keys), n1 ** 3)
    return pos, ids
