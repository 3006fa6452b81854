"""FP64 CPU oracle: Python side.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of bench.py import this module.  It shares no code with the GPU library
(paper_2503_07898_amd/) and never imports it.

Contents
  * ctypes binding of lbm_oracle.c (the D3Q19 solver, see that file's header,
    and the same file built for D3Q27);
  * the reference builder of the disaggregated index maps (block ids, Morton
    order per group, neighbour tables, canonical order), written as a direct
    coordinate search (sections "Disaggregation on a Sparse Domain" and
    "Disaggregated Design Method": classify, then map each group with a
    locality order; space-filling-curve managed blocks);
  * small helpers (relative L2 error).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
LIB27_PATH = os.path.join(HERE, "liboracle27.so")
SRC_PATH = os.path.join(HERE, "lbm_oracle.c")
SRC_MR_PATH = os.path.join(HERE, "lbm_oracle_multires.c")
Q = 19

# face ids and boundary kinds of the oracle (its own numbering)
XMIN, XMAX, YMIN, YMAX, ZMIN, ZMAX = range(6)
BB, MOVING, REG_VEL, REG_PRES = range(4)
BGK, REGULARIZED = 0, 1


def build(force: bool = False) -> str:
    """Compile lbm_oracle.c (+ the multires file) with gcc (-O3 -fopenmp) into
    liboracle.so, and lbm_oracle.c with -DORC_D3Q27 into liboracle27.so."""
    newest = max(os.path.getmtime(SRC_PATH), os.path.getmtime(SRC_MR_PATH))
    for path, extra in ((LIB_PATH, [SRC_PATH, SRC_MR_PATH]), (LIB27_PATH, ["-DORC_D3Q27", SRC_PATH])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < newest:
            tmp = path + ".tmp"
            subprocess.check_call(
                ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                 "-Wall", "-Wextra", "-o", tmp] + extra + ["-lm"]
            )
            os.replace(tmp, path)
    return LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("fluid", ctypes.POINTER(ctypes.c_uint8)),
        ("bc_kind", ctypes.c_int32 * 6),
        ("bc_val", (ctypes.c_double * 3) * 6),
        ("tau", ctypes.c_double),
        ("collision", ctypes.c_int32),
    ]


class _MrGrid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("level_map", ctypes.POINTER(ctypes.c_uint8)),
        ("fluid", ctypes.POINTER(ctypes.c_uint8)),
        ("bc_kind", ctypes.c_int32 * 6),
        ("bc_val", (ctypes.c_double * 3) * 6),
        ("tau_coarsest", ctypes.c_double),
        ("collision", ctypes.c_int32),
    ]


_libs = {}


def lib(q: int = 19):
    """The oracle library for lattice q (19 or 27)."""
    if q not in _libs:
        assert q in (19, 27), q
        build()
        L = ctypes.CDLL(LIB_PATH if q == 19 else LIB27_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(_Grid)
        L.orc_step.argtypes = [gp, dp, dp]
        L.orc_run.argtypes = [gp, dp, dp, ctypes.c_int32]
        L.orc_step_voxels.argtypes = [gp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
        L.orc_init_equilibrium.argtypes = [gp, dp, dp, dp]
        L.orc_init_equilibrium.restype = None
        L.orc_macroscopic.argtypes = [gp, dp, dp, dp]
        L.orc_macroscopic.restype = None
        L.orc_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), dp, ctypes.POINTER(ctypes.c_int32)]
        L.orc_lattice.restype = None
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_equilibrium.restype = None
        L.orc_moments.argtypes = [dp, dp, dp]
        L.orc_moments.restype = None
        L.orc_collide_bgk.argtypes = [dp, ctypes.c_double, dp]
        L.orc_collide_bgk.restype = None
        L.orc_collide_regularized.argtypes = [dp, ctypes.c_double, dp]
        L.orc_collide_regularized.restype = None
        L.orc_f1.argtypes = [dp, dp, dp]
        L.orc_f1.restype = None
        if q == 19:
            pp = ctypes.POINTER(ctypes.POINTER(ctypes.c_double))
            L.orc_mr_run.argtypes = [ctypes.POINTER(_MrGrid), pp, pp, pp, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]
            L.orc_mr_mass.argtypes = [ctypes.POINTER(_MrGrid), pp]
            L.orc_mr_mass.restype = ctypes.c_double
        _libs[q] = L
    return _libs[q]


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice(q: int = 19):
    """(c [q,3] int, w [q] float64, opp [q] int) as the oracle defines them."""
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    opp = np.zeros(q, np.int32)
    lib(q).orc_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w),
                       opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return c, w, opp


def equilibrium(rho: float, u, q: int = 19) -> np.ndarray:
    u = np.ascontiguousarray(u, np.float64)
    out = np.zeros(q)
    lib(q).orc_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def moments(f) -> tuple[float, np.ndarray]:
    f = np.ascontiguousarray(f, np.float64)
    r = np.zeros(1)
    u = np.zeros(3)
    lib(f.shape[-1]).orc_moments(_dp(f), _dp(r), _dp(u))
    return float(r[0]), u


def collide_bgk(f, tau: float) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float64)
    out = np.zeros(f.shape[-1])
    lib(f.shape[-1]).orc_collide_bgk(_dp(f), float(tau), _dp(out))
    return out


def collide_regularized(f, tau: float) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float64)
    out = np.zeros(f.shape[-1])
    lib(f.shape[-1]).orc_collide_regularized(_dp(f), float(tau), _dp(out))
    return out


def f1_projection(f, feq) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float64)
    feq = np.ascontiguousarray(feq, np.float64)
    out = np.zeros(f.shape[-1])
    lib(f.shape[-1]).orc_f1(_dp(f), _dp(feq), _dp(out))
    return out


@dataclass
class Grid:
    """A single-resolution voxel box for the oracle.

    fluid: uint8 array shaped (nz, ny, nx) (x fastest in memory) or None.
    bc: per face (XMIN..ZMAX) a (kind, value3) pair; ignored on periodic axes.
    """
    nx: int
    ny: int
    nz: int
    periodic: tuple = (True, True, True)
    fluid: np.ndarray | None = None
    bc: list = field(default_factory=lambda: [(BB, (0.0, 0.0, 0.0))] * 6)
    tau: float = 0.6
    collision: int = BGK
    q: int = 19  # lattice: 19 or 27

    def _struct(self):
        g = _Grid()
        g.nx, g.ny, g.nz = self.nx, self.ny, self.nz
        for a in range(3):
            g.periodic[a] = 1 if self.periodic[a] else 0
        if self.fluid is not None:
            fl = np.ascontiguousarray(self.fluid, np.uint8)
            assert fl.shape == (self.nz, self.ny, self.nx)
            self._fluid_keep = fl
            g.fluid = fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        else:
            g.fluid = ctypes.POINTER(ctypes.c_uint8)()
        for k in range(6):
            kind, val = self.bc[k]
            g.bc_kind[k] = int(kind)
            for a in range(3):
                g.bc_val[k][a] = float(val[a]) if a < len(val) else 0.0
        g.tau = float(self.tau)
        g.collision = int(self.collision)
        return g

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    def fluid_mask(self) -> np.ndarray:
        if self.fluid is None:
            return np.ones((self.nz, self.ny, self.nx), bool)
        return np.asarray(self.fluid, bool)

    def init_equilibrium(self, rho, u) -> np.ndarray:
        """rho (nz,ny,nx), u (nz,ny,nx,3) -> f (nz,ny,nx,q)."""
        rho = np.ascontiguousarray(np.broadcast_to(rho, (self.nz, self.ny, self.nx)), np.float64)
        u = np.ascontiguousarray(np.broadcast_to(u, (self.nz, self.ny, self.nx, 3)), np.float64)
        f = np.zeros((self.nz, self.ny, self.nx, self.q))
        g = self._struct()
        lib(self.q).orc_init_equilibrium(ctypes.byref(g), _dp(rho), _dp(u), _dp(f))
        return f

    def step(self, f: np.ndarray) -> np.ndarray:
        out = np.zeros_like(f)
        g = self._struct()
        r = lib(self.q).orc_step(ctypes.byref(g), _dp(f), _dp(out))
        if r != 0:
            raise ValueError("oracle: a link crosses two regularized faces")
        return out

    def run(self, f: np.ndarray, nsteps: int) -> np.ndarray:
        f = np.array(f, np.float64, order="C", copy=True)
        work = np.zeros_like(f)
        g = self._struct()
        r = lib(self.q).orc_run(ctypes.byref(g), _dp(f), _dp(work), int(nsteps))
        if r != 0:
            raise ValueError("oracle: a link crosses two regularized faces")
        return f

    def step_voxels(self, f: np.ndarray, vox: np.ndarray) -> np.ndarray:
        vox = np.ascontiguousarray(vox, np.int64)
        out = np.zeros((len(vox), self.q))
        g = self._struct()
        r = lib(self.q).orc_step_voxels(ctypes.byref(g), _dp(f),
                                  vox.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  len(vox), _dp(out))
        if r != 0:
            raise ValueError("oracle: a link crosses two regularized faces")
        return out

    def macroscopic(self, f: np.ndarray):
        rho = np.zeros((self.nz, self.ny, self.nx))
        u = np.zeros((self.nz, self.ny, self.nx, 3))
        g = self._struct()
        lib(self.q).orc_macroscopic(ctypes.byref(g), _dp(f), _dp(rho), _dp(u))
        return rho, u


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(a * a)))


# ------------------------------------------------------- index-map builder ---
# Reference builder of the disaggregated block layout, written as a direct
# coordinate search with no hashing.  Conventions (readings of the paper's
# "classify, then map each group with a locality order" and "blocks managed by
# a space-filling curve"):
#   * 4^3-voxel blocks; a block is active if it holds a fluid voxel;
#   * dense grids: the boundary group is every block that touches a
#     non-periodic box face (shell versus interior);
#   * block-sparse grids: the boundary group is every block holding a voxel
#     next to a moving-wall or regularized face (voxels needing the heavy
#     boundary treatment); bounce-back voxels stay in the non-boundary group;
#   * the non-boundary group is split into "masked" blocks (some voxel pulls
#     from a non-fluid source) and "full" blocks (all 18 neighbours active
#     and every voxel of the 3x3x3-block neighbourhood used by D3Q19 is fluid);
#   * group order [boundary | masked | full]; ascending Morton key in each
#     group, key bits interleaved x at 3b, y at 3b+1, z at 3b+2;
#   * voxel-in-block order x + 4y + 16z;
#   * neighbour table in direction order 1..18 of the oracle's lattice, -1 if
#     the neighbour block is inactive or outside a non-periodic box.

def morton_key(bx: int, by: int, bz: int) -> int:
    k = 0
    for b in range(21):
        k |= ((bx >> b) & 1) << (3 * b)
        k |= ((by >> b) & 1) << (3 * b + 1)
        k |= ((bz >> b) & 1) << (3 * b + 2)
    return k


def _face_voxel_kinds(nx, ny, nz, periodic, face_kinds, heavy):
    """Boolean (nz,ny,nx): voxels next to a non-periodic face of a kind in `heavy`."""
    m = np.zeros((nz, ny, nx), bool)
    n = (nx, ny, nz)
    for face in range(6):
        axis, side = face // 2, face % 2
        if periodic[axis] or face_kinds[face] not in heavy:
            continue
        idx = [slice(None)] * 3
        idx[2 - axis] = n[axis] - 1 if side else 0
        m[tuple(idx)] = True
    return m


def build_block_maps(nx, ny, nz, periodic, fluid, face_kinds, dense: bool, grouped: bool = True,
                     q: int = 19, jump=None):
    """Returns a dict with coords [nb,3], nbr [nb,18], fmask [nb] (uint64),
    groups (n_boundary, n_masked, n_full), group [nb] (0 boundary, 1 masked,
    2 full, 3 jump, per storage slot), canon [nb*64] (int64, -1 = not fluid),
    n_fluid, and groups4 (n_jump, n_boundary, n_masked, n_full).  grouped:
    memory-based grouping (jump, boundary, masked, full groups stored one
    after the other, Morton order inside each); otherwise the bitmask-based
    form keeps every block in one Morton order.  q: lattice (19: 18
    face/edge neighbours; 27: 26 with the corners).  jump: optional bool
    (nz,ny,nx) of voxels at distance 0 from a resolution jump (multires
    levels); a block holding one belongs to the jump group, whatever else
    it holds."""
    c, _, _ = lattice(q)
    B = 4
    assert nx % B == 0 and ny % B == 0 and nz % B == 0
    nbx, nby, nbz = nx // B, ny // B, nz // B
    fl = np.ones((nz, ny, nx), bool) if fluid is None else np.asarray(fluid, bool)
    heavy = _face_voxel_kinds(nx, ny, nz, periodic, face_kinds, (MOVING, REG_VEL, REG_PRES))

    def block_view(a, bx, by, bz):
        return a[bz * B:(bz + 1) * B, by * B:(by + 1) * B, bx * B:(bx + 1) * B]

    active = {}
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                if block_view(fl, bx, by, bz).any():
                    active[(bx, by, bz)] = True

    def neighbour(bx, by, bz, d):
        t = [bx + c[d, 0], by + c[d, 1], bz + c[d, 2]]
        nb = (nbx, nby, nbz)
        for a in range(3):
            if t[a] < 0 or t[a] >= nb[a]:
                if not periodic[a]:
                    return None
                t[a] %= nb[a]
        return tuple(t) if tuple(t) in active else None

    jm = None if jump is None else np.asarray(jump, bool)

    def group_of(bx, by, bz):
        if jm is not None and block_view(jm, bx, by, bz).any():
            return 3
        if dense:
            shell = ((not periodic[0] and (bx == 0 or bx == nbx - 1)) or
                     (not periodic[1] and (by == 0 or by == nby - 1)) or
                     (not periodic[2] and (bz == 0 or bz == nbz - 1)))
            if shell:
                return 0
        elif block_view(heavy & fl, bx, by, bz).any():
            return 0
        # full: every source of every voxel in the block is a fluid voxel
        full = block_view(fl, bx, by, bz).all()
        for d in range(1, q):
            nbk = neighbour(bx, by, bz, d)
            if nbk is None or not block_view(fl, *nbk).all():
                full = False
        return 2 if full else 1

    groups = {3: [], 0: [], 1: [], 2: []}
    for key in active:
        groups[group_of(*key)].append(key)
    order = []
    if grouped:
        for gid in (3, 0, 1, 2):
            order += sorted(groups[gid], key=lambda k: morton_key(*k))
    else:
        order = sorted(active, key=lambda k: morton_key(*k))
    gid_of = {k: gid for gid in (3, 0, 1, 2) for k in groups[gid]}
    slot_of = {k: s for s, k in enumerate(order)}
    nb = len(order)
    coords = np.array(order, np.int32).reshape(nb, 3)
    nbr = np.full((nb, q - 1), -1, np.int32)
    fmask = np.zeros(nb, np.uint64)
    for s, (bx, by, bz) in enumerate(order):
        for d in range(1, q):
            nbk = neighbour(bx, by, bz, d)
            if nbk is not None:
                nbr[s, d - 1] = slot_of[nbk]
        bits = 0
        v = block_view(fl, bx, by, bz)
        for lz in range(B):
            for ly in range(B):
                for lx in range(B):
                    if v[lz, ly, lx]:
                        bits |= 1 << (lx + 4 * ly + 16 * lz)
        fmask[s] = np.uint64(bits)
    # canonical order: fluid voxels, x fastest
    lin = -np.ones((nz, ny, nx), np.int64)
    lin[fl] = np.arange(int(fl.sum()), dtype=np.int64)
    canon = -np.ones(nb * 64, np.int64)
    for s, (bx, by, bz) in enumerate(order):
        v = block_view(lin, bx, by, bz)
        for lz in range(B):
            for ly in range(B):
                for lx in range(B):
                    canon[s * 64 + lx + 4 * ly + 16 * lz] = v[lz, ly, lx]
    return dict(coords=coords, nbr=nbr, fmask=fmask,
                groups=tuple(len(groups[g]) for g in (0, 1, 2)),
                groups4=tuple(len(groups[g]) for g in (3, 0, 1, 2)),
                group=np.array([gid_of[k] for k in order], np.int32),
                canon=canon, n_fluid=int(fl.sum()))


def multires_level_masks(nx, ny, nz, levels, periodic, level_map, fluid=None):
    """Active and jump voxels of every level of a multi-resolution box
    ("Disaggregation on a Multi-resolution Domain": the discrete distance
    property P_d, distance 0 meaning immediate proximity to a resolution
    jump).  Readings: a level-l voxel is the cube of 2^l finest cells whose
    level-map entry is l (solids exist on level 0 only); a level-l voxel is
    at distance 0 if one of the voxels it pulls from along a D3Q19 link
    (face or edge neighbour, periodic axes wrapped, sources outside a
    non-periodic face ignored) belongs to another level's territory.
    Direct coordinate search; returns [(active, jump)] with bool arrays
    shaped (nz >> l, ny >> l, nx >> l)."""
    c, _, _ = lattice()
    lm = np.asarray(level_map)
    fl = np.ones((nz, ny, nx), bool) if fluid is None else np.asarray(fluid, bool)
    out = []
    for l in range(levels):
        n = (nx >> l, ny >> l, nz >> l)

        def territory(x, y, z):
            return int(lm[z << l, y << l, x << l])

        act = np.zeros((n[2], n[1], n[0]), bool)
        jmp = np.zeros((n[2], n[1], n[0]), bool)
        for z in range(n[2]):
            for y in range(n[1]):
                for x in range(n[0]):
                    if territory(x, y, z) != l or (l == 0 and not fl[z, y, x]):
                        continue
                    act[z, y, x] = True
                    for i in range(1, 19):
                        src = [x - int(c[i, 0]), y - int(c[i, 1]), z - int(c[i, 2])]
                        inside = True
                        for a in range(3):
                            if src[a] < 0 or src[a] >= n[a]:
                                if not periodic[a]:
                                    inside = False
                                src[a] %= n[a]
                        if inside and territory(*src) != l:
                            jmp[z, y, x] = True
                            break
        out.append((act, jmp))
    return out


def build_multires_maps(nx, ny, nz, levels, periodic, level_map, fluid, face_kinds):
    """Per level, the block maps of build_block_maps on the level's own box
    (voxel mask = the level's active voxels, jump group from
    multires_level_masks)."""
    maps = []
    for l, (act, jmp) in enumerate(multires_level_masks(nx, ny, nz, levels, periodic, level_map, fluid)):
        maps.append(build_block_maps(nx >> l, ny >> l, nz >> l, periodic, act, face_kinds, False, jump=jmp))
    return maps


def brute_force_neighbours(coords, periodic, nblocks_axis):
    """O(n^2) scan: for each block and direction, search every block for the
    one at the offset (used to pin build_block_maps)."""
    c, _, _ = lattice()
    nb = len(coords)
    out = np.full((nb, 18), -1, np.int32)
    for s in range(nb):
        for d in range(1, 19):
            want = []
            ok = True
            for a in range(3):
                q = int(coords[s, a]) + int(c[d, a])
                if q < 0 or q >= nblocks_axis[a]:
                    if not periodic[a]:
                        ok = False
                    q %= nblocks_axis[a]
                want.append(q)
            if not ok:
                continue
            for t in range(nb):
                if list(coords[t]) == want:
                    out[s, d - 1] = t
    return out


# ------------------------------------------------------------- multires ----

@dataclass
class MultiresGrid:
    """Multi-resolution box for the oracle (lbm_oracle_multires.c).

    level_map: uint8 (nz, ny, nx) at the finest resolution, 0 = finest;
    fluid: uint8 (nz, ny, nx) or None (solids only at level 0).
    Per-level state arrays are shaped (nz >> l, ny >> l, nx >> l, 19).
    """
    nx: int
    ny: int
    nz: int
    levels: int
    level_map: np.ndarray
    periodic: tuple = (True, True, True)
    fluid: np.ndarray | None = None
    bc: list = field(default_factory=lambda: [(BB, (0.0, 0.0, 0.0))] * 6)
    tau_coarsest: float = 0.6
    collision: int = BGK

    def _struct(self):
        g = _MrGrid()
        g.nx, g.ny, g.nz, g.levels = self.nx, self.ny, self.nz, self.levels
        for a in range(3):
            g.periodic[a] = 1 if self.periodic[a] else 0
        self._lm = np.ascontiguousarray(self.level_map, np.uint8)
        assert self._lm.shape == (self.nz, self.ny, self.nx)
        g.level_map = self._lm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        if self.fluid is not None:
            self._fl = np.ascontiguousarray(self.fluid, np.uint8)
            g.fluid = self._fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        else:
            g.fluid = ctypes.POINTER(ctypes.c_uint8)()
        for k in range(6):
            kind, val = self.bc[k]
            g.bc_kind[k] = int(kind)
            for a in range(3):
                g.bc_val[k][a] = float(val[a]) if a < len(val) else 0.0
        g.tau_coarsest = float(self.tau_coarsest)
        g.collision = int(self.collision)
        return g

    def shape(self, l):
        return (self.nz >> l, self.ny >> l, self.nx >> l)

    def active(self, l):
        """bool (nz>>l, ny>>l, nx>>l): cells that are fluid voxels of level l."""
        s = 1 << l
        a = self.level_map[::s, ::s, ::s] == l
        if l == 0 and self.fluid is not None:
            a = a & (np.asarray(self.fluid) != 0)
        return a

    def tau(self, l):
        return 0.5 + (self.tau_coarsest - 0.5) * 2 ** (self.levels - 1 - l)

    def init_equilibrium(self, rho, u):
        """rho[l] (shape(l)), u[l] (shape(l)+(3,)) -> list of f[l]."""
        out = []
        for l in range(self.levels):
            nz, ny, nx = self.shape(l)
            g = Grid(nx, ny, nz)
            out.append(g.init_equilibrium(rho[l], u[l]))
        return out

    def run(self, f, nsteps):
        L = self.levels
        bufs = [[np.array(f[l], np.float64, order="C", copy=True) for l in range(L)] for _ in range(3)]
        ptrs = [(ctypes.POINTER(ctypes.c_double) * L)(*[_dp(b[l]) for l in range(L)]) for b in bufs]
        which = (ctypes.c_int32 * L)()
        g = self._struct()
        r = lib().orc_mr_run(ctypes.byref(g), ptrs[0], ptrs[1], ptrs[2], int(nsteps), which)
        if r != 0:
            raise ValueError(f"oracle multires run failed ({r})")
        return [bufs[which[l]][l] for l in range(L)]

    def mass(self, f):
        L = self.levels
        arrs = [np.ascontiguousarray(f[l], np.float64) for l in range(L)]
        ptr = (ctypes.POINTER(ctypes.c_double) * L)(*[_dp(a) for a in arrs])
        g = self._struct()
        return lib().orc_mr_mass(ctypes.byref(g), ptr)

    def macroscopic(self, f):
        out = []
        for l in range(self.levels):
            nz, ny, nx = self.shape(l)
            out.append(Grid(nx, ny, nz).macroscopic(np.ascontiguousarray(f[l])))
        return out
