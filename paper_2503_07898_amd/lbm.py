"""ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the path runs in liblbm's HIP
kernels.  PyTorch supplies device memory (the workspace and the caller's
arrays) and the stream.  There is no fallback: if the library is not built,
loading it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

# enums of include/lbm.h
LBM_OK = 0
DENSE, BLOCK_SPARSE, MULTIRES = 0, 1, 2
F32, F16_SHIFTED, BF16_SHIFTED = 0, 1, 2
BGK, REGULARIZED, MLP = 0, 1, 2
PLAIN_SINGLE_KERNEL, DISAGG, DISAGG_BITMASK, DISAGG_UNIFORM_FUSED = 0, 1, 2, 3
XMIN, XMAX, YMIN, YMAX, ZMIN, ZMAX = range(6)
BC_BOUNCE_BACK, BC_MOVING_WALL, BC_REG_VELOCITY, BC_REG_PRESSURE = range(4)
MAP_GROUPS, MAP_COORDS, MAP_NEIGHBOURS, MAP_FLUIDMASK, MAP_CANONICAL, MAP_BOUNDARY_BITS, MAP_RECORD_IDS = range(7)

STORAGE_BYTES = {F32: 4, F16_SHIFTED: 2, BF16_SHIFTED: 2}


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"liblbm status {status}: {msg}")
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_uint8 * 3),
        ("num_levels", ctypes.c_int32),
        ("fluid_mask", ctypes.c_void_p),
        ("level_map", ctypes.c_void_p),
        ("tau", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("lattice", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2503_07898_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        sigs = {
            "lbm_last_error": ([], ctypes.c_char_p),
            "lbm_grid_create": ([ctypes.POINTER(GridDesc), ctypes.POINTER(vp)], i32),
            "lbm_set_boundary": ([vp, i32, i32, ctypes.POINTER(ctypes.c_double)], i32),
            "lbm_grid_commit": ([vp, ctypes.POINTER(sz)], i32),
            "lbm_grid_bind": ([vp, vp, sz, vp], i32),
            "lbm_num_voxels": ([vp, i32, ctypes.POINTER(i64)], i32),
            "lbm_init_equilibrium": ([vp, i32, vp, vp, vp], i32),
            "lbm_step": ([vp, i32, vp], i32),
            "lbm_read_macroscopic": ([vp, i32, vp, vp, i32, vp], i32),
            "lbm_reduce": ([vp, vp, vp], i32),
            "lbm_reduce_noalloc": ([vp, vp, vp], i32),
            "lbm_read_populations": ([vp, i32, vp, vp], i32),
            "lbm_write_populations": ([vp, i32, vp, vp], i32),
            "lbm_get_index_map": ([vp, i32, i32, vp, ctypes.POINTER(sz)], i32),
            "lbm_step_launches": ([vp, ctypes.POINTER(i64), i32, ctypes.POINTER(i32)], i32),
            "lbm_launch_group": ([vp, i32, vp], i32),
            "lbm_mlp_create": ([ctypes.POINTER(vp), ctypes.POINTER(sz)], i32),
            "lbm_mlp_bind": ([vp, vp, sz, vp], i32),
            "lbm_mlp_set_params": ([vp, vp, vp], i32),
            "lbm_mlp_get_params": ([vp, vp, vp], i32),
            "lbm_mlp_set_standardization": ([vp, vp, vp], i32),
            "lbm_mlp_get_standardization": ([vp, vp, vp], i32),
            "lbm_mlp_fit_standardization": ([vp, vp, i64, vp], i32),
            "lbm_mlp_forward": ([vp, vp, i64, vp, vp], i32),
            "lbm_mlp_gradients": ([vp, vp, vp, i64, vp, vp, vp], i32),
            "lbm_mlp_train_step": ([vp, vp, vp, i64, ctypes.c_float, i32, vp, vp], i32),
            "lbm_mlp_adam": ([vp, vp, ctypes.c_float, i32, vp], i32),
            "lbm_mlp_init_params": ([vp, ctypes.c_uint64, vp], i32),
            "lbm_mlp_set_judge": ([vp, ctypes.c_double], i32),
            "lbm_mlp_fallbacks": ([vp, ctypes.POINTER(ctypes.c_uint64), i32, vp], i32),
            "lbm_mlp_destroy": ([vp], i32),
            "lbm_set_collision": ([vp, i32, vp], i32),
            "lbm_set_merge_limit": ([vp, i64], i32),
            "lbm_set_residency": ([vp, i32], i32),
            "lbm_set_wide_addressing": ([vp, i32], i32),
            "lbm_check": ([vp, vp], i32),
            "lbm_sample_populations": ([vp, i32, ctypes.c_uint64, i64, vp, vp], i32),
            "lbm_grid_destroy": ([vp], i32),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != LBM_OK:
        raise LbmError(status, lib().lbm_last_error().decode())


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


# ------------------------------------------------------ thin C-ABI wrappers --
# Same names as the C functions; each marshals its arguments and checks the
# returned status.

def lbm_grid_create(desc: GridDesc) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(lib().lbm_grid_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def lbm_set_boundary(g, face: int, kind: int, value=(0.0, 0.0, 0.0)) -> None:
    v = (ctypes.c_double * 3)(*[float(x) for x in value])
    check(lib().lbm_set_boundary(g, int(face), int(kind), v))


def lbm_grid_commit(g) -> int:
    n = ctypes.c_size_t()
    check(lib().lbm_grid_commit(g, ctypes.byref(n)))
    return n.value


def lbm_grid_bind(g, ptr: int, nbytes: int, stream=None) -> None:
    check(lib().lbm_grid_bind(g, ctypes.c_void_p(ptr), nbytes, _stream_ptr(stream)))


def lbm_num_voxels(g, level: int = 0) -> int:
    n = ctypes.c_int64()
    check(lib().lbm_num_voxels(g, level, ctypes.byref(n)))
    return n.value


def lbm_init_equilibrium(g, level: int, rho_ptr: int, u_ptr: int, stream=None) -> None:
    check(lib().lbm_init_equilibrium(g, level, rho_ptr, u_ptr, _stream_ptr(stream)))


def lbm_step(g, n: int, stream=None) -> None:
    check(lib().lbm_step(g, int(n), _stream_ptr(stream)))


def lbm_read_macroscopic(g, level: int, rho_ptr: int, u_ptr: int, f64: bool, stream=None) -> None:
    check(lib().lbm_read_macroscopic(g, level, rho_ptr, u_ptr, 1 if f64 else 0, _stream_ptr(stream)))


def lbm_reduce(g, out_ptr: int, stream=None) -> None:
    check(lib().lbm_reduce(g, out_ptr, _stream_ptr(stream)))


def lbm_reduce_noalloc(g, out_ptr: int, stream=None) -> None:
    check(lib().lbm_reduce_noalloc(g, out_ptr, _stream_ptr(stream)))


def lbm_read_populations(g, level: int, f_ptr: int, stream=None) -> None:
    check(lib().lbm_read_populations(g, level, f_ptr, _stream_ptr(stream)))


def lbm_write_populations(g, level: int, f_ptr: int, stream=None) -> None:
    check(lib().lbm_write_populations(g, level, f_ptr, _stream_ptr(stream)))


def lbm_get_index_map(g, level: int, which: int) -> np.ndarray:
    n = ctypes.c_size_t()
    check(lib().lbm_get_index_map(g, level, which, None, ctypes.byref(n)))
    dtype = {MAP_GROUPS: np.int64, MAP_COORDS: np.int32, MAP_NEIGHBOURS: np.int32,
             MAP_FLUIDMASK: np.uint64, MAP_CANONICAL: np.int64, MAP_BOUNDARY_BITS: np.uint32,
             MAP_RECORD_IDS: np.int32}[which]
    out = np.zeros(n.value, dtype)
    check(lib().lbm_get_index_map(g, level, which, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
    return out


def lbm_step_launches(g) -> list[int]:
    n = ctypes.c_int32()
    buf = (ctypes.c_int64 * 256)()
    check(lib().lbm_step_launches(g, buf, 256, ctypes.byref(n)))
    return [int(buf[k]) for k in range(n.value)]


def lbm_launch_group(g, k: int, stream=None) -> None:
    check(lib().lbm_launch_group(g, int(k), _stream_ptr(stream)))


RESIDENCY_AUTO = -1  # lbm_set_residency: per-kernel measured caps
MLP_PARAMS = 6675
MLP_BATCH_MAX = 8192


def lbm_mlp_create():
    h = ctypes.c_void_p()
    n = ctypes.c_size_t()
    check(lib().lbm_mlp_create(ctypes.byref(h), ctypes.byref(n)))
    return h, n.value


def lbm_mlp_bind(m, ptr: int, nbytes: int, stream=None) -> None:
    check(lib().lbm_mlp_bind(m, ctypes.c_void_p(ptr), nbytes, _stream_ptr(stream)))


def lbm_mlp_set_params(m, params: np.ndarray, stream=None) -> None:
    p = np.ascontiguousarray(params, np.float32)
    assert p.size == MLP_PARAMS
    check(lib().lbm_mlp_set_params(m, p.ctypes.data, _stream_ptr(stream)))


def lbm_mlp_get_params(m, stream=None) -> np.ndarray:
    p = np.zeros(MLP_PARAMS, np.float32)
    check(lib().lbm_mlp_get_params(m, p.ctypes.data, _stream_ptr(stream)))
    return p


def lbm_mlp_set_standardization(m, stdz: np.ndarray, stream=None) -> None:
    p = np.ascontiguousarray(stdz, np.float32)
    assert p.size == 128
    check(lib().lbm_mlp_set_standardization(m, p.ctypes.data, _stream_ptr(stream)))


def lbm_mlp_get_standardization(m, stream=None) -> np.ndarray:
    p = np.zeros(128, np.float32)
    check(lib().lbm_mlp_get_standardization(m, p.ctypes.data, _stream_ptr(stream)))
    return p


def lbm_mlp_fit_standardization(m, f_ptr: int, n: int, stream=None) -> None:
    check(lib().lbm_mlp_fit_standardization(m, f_ptr, int(n), _stream_ptr(stream)))


def lbm_mlp_forward(m, f_ptr: int, n: int, y_ptr: int, stream=None) -> None:
    check(lib().lbm_mlp_forward(m, f_ptr, int(n), y_ptr, _stream_ptr(stream)))


def lbm_mlp_gradients(m, f_ptr: int, idx_ptr, n: int, grads_ptr, loss_ptr, stream=None) -> None:
    check(lib().lbm_mlp_gradients(m, f_ptr, idx_ptr, int(n), grads_ptr, loss_ptr, _stream_ptr(stream)))


def lbm_mlp_train_step(m, f_ptr: int, idx_ptr, n: int, lr: float, t: int, loss_ptr=None,
                       stream=None) -> None:
    check(lib().lbm_mlp_train_step(m, f_ptr, idx_ptr, int(n), float(lr), int(t), loss_ptr,
                                   _stream_ptr(stream)))


def lbm_mlp_adam(m, grads_ptr: int, lr: float, t: int, stream=None) -> None:
    check(lib().lbm_mlp_adam(m, grads_ptr, float(lr), int(t), _stream_ptr(stream)))


def lbm_mlp_init_params(m, seed: int, stream=None) -> None:
    check(lib().lbm_mlp_init_params(m, int(seed) & 0xFFFFFFFFFFFFFFFF, _stream_ptr(stream)))


def lbm_mlp_set_judge(m, rel_tol: float) -> None:
    check(lib().lbm_mlp_set_judge(m, ctypes.c_double(rel_tol)))


def lbm_mlp_fallbacks(m, reset: bool = False, stream=None) -> int:
    c = ctypes.c_uint64()
    check(lib().lbm_mlp_fallbacks(m, ctypes.byref(c), 1 if reset else 0, _stream_ptr(stream)))
    return c.value


def lbm_mlp_destroy(m) -> None:
    check(lib().lbm_mlp_destroy(m))


def lbm_set_collision(g, collision: int, mlp=None) -> None:
    check(lib().lbm_set_collision(g, int(collision), mlp))


def lbm_check(g, stream=None) -> None:
    check(lib().lbm_check(g, _stream_ptr(stream)))


def lbm_set_merge_limit(g, max_blocks: int) -> None:
    check(lib().lbm_set_merge_limit(g, int(max_blocks)))


def lbm_set_residency(g, wg_per_cu: int) -> None:
    check(lib().lbm_set_residency(g, int(wg_per_cu)))


def lbm_set_wide_addressing(g, wide: int) -> None:
    check(lib().lbm_set_wide_addressing(g, int(wide)))


def lbm_sample_populations(g, level: int, seed: int, n: int, f_ptr: int, stream=None) -> None:
    check(lib().lbm_sample_populations(g, int(level), ctypes.c_uint64(seed), int(n), f_ptr, _stream_ptr(stream)))


def lbm_grid_destroy(g) -> None:
    check(lib().lbm_grid_destroy(g))


# ------------------------------------------------------------ convenience --

@dataclass
class Grid:
    """One liblbm grid with its device workspace held as a torch tensor.

    fluid: uint8 (nz, ny, nx) or None; faces: {face: (kind, value3)};
    multires grids also take level_map (uint8 (nz, ny, nx), 0 = finest) and
    levels.  Per-level calls take `level` (default 0).
    """
    nx: int
    ny: int
    nz: int
    kind: int = DENSE
    periodic: tuple = (True, True, True)
    fluid: np.ndarray | None = None
    tau: float = 0.6
    storage: int = F32
    collision: int = BGK
    schedule: int = DISAGG
    faces: dict = field(default_factory=dict)
    device: str = "cuda"
    level_map: np.ndarray | None = None
    levels: int = 1
    q: int = 19  # lattice: D3Q19 or D3Q27

    def __post_init__(self):
        d = GridDesc()
        d.kind = self.kind
        d.nx, d.ny, d.nz = self.nx, self.ny, self.nz
        for a in range(3):
            d.periodic[a] = 1 if self.periodic[a] else 0
        d.num_levels = self.levels
        self._lmap = None
        if self.level_map is not None:
            self._lmap = np.ascontiguousarray(self.level_map, np.uint8)
            assert self._lmap.shape == (self.nz, self.ny, self.nx)
            d.level_map = self._lmap.ctypes.data
        self._mask = None
        if self.fluid is not None:
            self._mask = np.ascontiguousarray(self.fluid, np.uint8)
            assert self._mask.shape == (self.nz, self.ny, self.nx)
            d.fluid_mask = self._mask.ctypes.data
        d.tau = float(self.tau)
        d.storage, d.collision, d.schedule = self.storage, self.collision, self.schedule
        d.lattice = self.q
        self.h = lbm_grid_create(d)
        for face, (k, val) in self.faces.items():
            lbm_set_boundary(self.h, face, k, val)
        self.workspace_bytes = lbm_grid_commit(self.h)
        self.ws = None

    def bind(self):
        import torch
        self.ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        lbm_grid_bind(self.h, self.ws.data_ptr(), self.workspace_bytes)
        return self

    @property
    def n(self) -> int:
        return lbm_num_voxels(self.h, 0)

    def n_level(self, level: int) -> int:
        return lbm_num_voxels(self.h, level)

    def init_equilibrium(self, rho, u, level: int = 0):
        """rho [N], u [3][N] canonical order (numpy or torch, converted to FP64 on device)."""
        import torch
        n = self.n_level(level)
        r = torch.as_tensor(np.asarray(rho, np.float64).reshape(-1)).to(self.device)
        v = torch.as_tensor(np.asarray(u, np.float64).reshape(3, -1)).contiguous().to(self.device)
        assert r.numel() == n and v.shape[1] == n
        lbm_init_equilibrium(self.h, level, r.data_ptr(), v.data_ptr())
        torch.cuda.current_stream().synchronize()

    def step(self, n: int = 1):
        lbm_step(self.h, n)

    def macroscopic(self, f64: bool = True, level: int = 0):
        import torch
        dt = torch.float64 if f64 else torch.float32
        n = self.n_level(level)
        rho = torch.empty(n, dtype=dt, device=self.device)
        u = torch.empty(3, n, dtype=dt, device=self.device)
        lbm_read_macroscopic(self.h, level, rho.data_ptr(), u.data_ptr(), f64)
        return rho, u

    def populations(self, level: int = 0):
        import torch
        f = torch.empty(self.q, self.n_level(level), dtype=torch.float64, device=self.device)
        lbm_read_populations(self.h, level, f.data_ptr())
        return f

    def write_populations(self, f, level: int = 0):
        import torch
        n = self.n_level(level)
        t = torch.as_tensor(f, dtype=torch.float64).reshape(self.q, n).contiguous().to(self.device)
        lbm_write_populations(self.h, level, t.data_ptr())
        torch.cuda.current_stream().synchronize()

    def reduce(self):
        import torch
        out = torch.empty(5, dtype=torch.float64, device=self.device)
        lbm_reduce(self.h, out.data_ptr())
        return out

    def reduce_noalloc(self, out=None):
        """lbm_reduce_noalloc into `out` (5 FP64 on the device; allocated here
        when None)."""
        import torch
        if out is None:
            out = torch.empty(5, dtype=torch.float64, device=self.device)
        lbm_reduce_noalloc(self.h, out.data_ptr())
        return out

    def index_map(self, which: int, level: int = 0) -> np.ndarray:
        return lbm_get_index_map(self.h, level, which)

    def launches(self) -> list[int]:
        return lbm_step_launches(self.h)

    def set_collision(self, collision: int, mlp=None) -> None:
        self._mlp_keep = mlp
        lbm_set_collision(self.h, collision, None if mlp is None else mlp.h)

    def check(self) -> None:
        """Raises LbmError (status LBM_ERR_NUMERIC) if any population is NaN or infinite."""
        lbm_check(self.h)

    def set_merge_limit(self, max_blocks: int) -> None:
        lbm_set_merge_limit(self.h, max_blocks)

    def set_residency(self, wg_per_cu: int) -> None:
        """Caps the stepping kernels at wg_per_cu resident workgroups per CU
        (0: no cap, RESIDENCY_AUTO: the measured per-kernel default)."""
        lbm_set_residency(self.h, wg_per_cu)

    def set_wide_addressing(self, wide: bool) -> None:
        """Forces the closure kernel's 64-bit pull addressing (True) or
        restores the automatic 32-bit form for buffers up to 4 GiB (False)."""
        lbm_set_wide_addressing(self.h, 1 if wide else 0)

    def sample(self, seed: int, n: int, level: int = 0):
        import torch
        f = torch.empty(n, 19, dtype=torch.float32, device=self.device)
        lbm_sample_populations(self.h, level, seed, n, f.data_ptr())
        return f

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The learned collision closure with its device buffer (torch tensor)."""

    def __init__(self, device: str = "cuda"):
        import torch
        self.h, self.nbytes = lbm_mlp_create()
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.device = device
        lbm_mlp_bind(self.h, self.buf.data_ptr(), self.nbytes)

    def set_params(self, params) -> None:
        lbm_mlp_set_params(self.h, np.asarray(params, np.float32).reshape(-1))

    def params(self) -> np.ndarray:
        return lbm_mlp_get_params(self.h)

    def set_standardization(self, stdz) -> None:
        lbm_mlp_set_standardization(self.h, np.asarray(stdz, np.float32).reshape(-1))

    def standardization(self) -> np.ndarray:
        return lbm_mlp_get_standardization(self.h)

    def fit_standardization(self, f) -> None:
        lbm_mlp_fit_standardization(self.h, f.data_ptr(), f.shape[0])

    def forward(self, f):
        import torch
        y = torch.empty(f.shape[0], 19, dtype=torch.float32, device=self.device)
        lbm_mlp_forward(self.h, f.data_ptr(), f.shape[0], y.data_ptr())
        return y

    def gradients(self, f):
        import torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        lbm_mlp_gradients(self.h, f.data_ptr(), None, f.shape[0], g.data_ptr(), loss.data_ptr())
        return g, loss

    def train_step(self, f, lr: float, t: int, loss=None, idx=None) -> None:
        """Adam step t on rows idx (int64 device tensor) of f, or on all of f."""
        n = f.shape[0] if idx is None else idx.shape[0]
        lbm_mlp_train_step(self.h, f.data_ptr(), None if idx is None else idx.data_ptr(), n, lr, t,
                           None if loss is None else loss.data_ptr())

    def adam(self, grads, lr: float, t: int) -> None:
        """Adam step t on caller gradients (FP32 device tensor [MLP_PARAMS])."""
        lbm_mlp_adam(self.h, grads.data_ptr(), lr, t)

    def init_params(self, seed: int) -> None:
        """Seeded He-uniform weights and zero biases, drawn on the device."""
        lbm_mlp_init_params(self.h, seed)

    def set_judge(self, rel_tol: float) -> None:
        lbm_mlp_set_judge(self.h, rel_tol)

    def fallbacks(self, reset: bool = False) -> int:
        return lbm_mlp_fallbacks(self.h, reset)

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flatten_params(W) -> np.ndarray:
    """[W1 (19,64), b1, W2 (64,64), b2, W3 (64,19), b3] -> flat LBM_MLP_PARAMS array."""
    return np.concatenate([np.asarray(w, np.float64).reshape(-1) for w in W]).astype(np.float32)


def unflatten_params(p) -> list:
    p = np.asarray(p, np.float64)
    shapes = [(19, 64), (64,), (64, 64), (64,), (64, 19), (19,)]
    out, k = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(p[k:k + n].reshape(s))
        k += n
    return out
