"""ctypes binding of libamr (include/amr.h): argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts
Python/numpy/torch arguments to the C ABI and back.  Importing it loads
``libamr.so`` and raises ImportError when the library has not been built.
Device memory comes from torch's caching allocator through the library's
allocator hook; streams are torch streams.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2508_05020_amd.build`")
# torch ships its own HIP runtime with the same soname as /opt/rocm's.  Loading
# torch first makes the dynamic loader bind libamr to that already-loaded
# runtime, so that one HIP runtime serves the whole process.
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)

MAX_LEVELS = 8
EXEC_PER_PATCH, EXEC_BATCHED = 0, 1
COARSEN_TEXT, COARSEN_LITERAL = 0, 1
SCHEME_WENO, SCHEME_CENTRAL, SCHEME_CHAR = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 32 << 20   # AMR_NOALLOC_SCRATCH_BYTES

STATUS = {0: "AMR_OK", -1: "AMR_E_ARG", -2: "AMR_E_CAPACITY", -3: "AMR_E_HIP",
          -4: "AMR_E_MESH", -5: "AMR_E_NONPHYSICAL", -6: "AMR_E_STATE"}


E_CAPACITY = -2


class AMRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("dim", C.c_int), ("max_levels", C.c_int), ("base_cells", C.c_int),
                ("patch_cells", C.c_int * MAX_LEVELS), ("periodic", C.c_int * 3),
                ("lo", C.c_double), ("hi", C.c_double), ("gamma", C.c_double),
                ("cfl", C.c_double), ("weno_eps", C.c_double), ("tag_theta", C.c_double),
                ("tag_buffer", C.c_int), ("max_patches", C.c_int),
                ("level_capacity", C.c_int * MAX_LEVELS), ("exec_mode", C.c_int),
                ("coarsen_rule", C.c_int), ("scheme", C.c_int)]


class PatchInfo(C.Structure):
    _fields_ = [("pid", C.c_int32), ("level", C.c_int32), ("coord", C.c_int32 * 3),
                ("parent", C.c_int32), ("nchildren", C.c_int32), ("first_child", C.c_int32),
                ("nbr", C.c_int32 * 26)]


class CnnConfig(C.Structure):
    _fields_ = [("patch_cells", C.c_int), ("mean", C.c_float * 5), ("std", C.c_float * 5),
                ("pos_weight", C.c_float), ("max_batch", C.c_int)]


class Allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("ctx", C.c_void_p)]


_H = C.c_void_p
_P = C.POINTER
_sigs = {
    "amr_create_hierarchy": [_P(Config), _P(Allocator), C.c_void_p, _P(_H)],
    "amr_destroy_hierarchy": [_H],
    "amr_num_patches": [_H, _P(C.c_int), _P(C.c_int)],
    "amr_patch_doubles": [_H, C.c_int, _P(C.c_int64)],
    "amr_state_doubles": [_H, _P(C.c_int64)],
    "amr_patch_offset": [_H, C.c_int, _P(C.c_int64)],
    "amr_state_ptr": [_H, C.c_int, _P(C.c_void_p)],
    "amr_get_patch_table": [_H, _P(PatchInfo), C.c_int, _P(C.c_int)],
    "amr_set_state": [_H, C.c_int, C.c_void_p, _P(C.c_int), C.c_int],
    "amr_get_state": [_H, C.c_int, C.c_void_p, _P(C.c_int), C.c_int],
    "amr_set_state_prim": [_H, C.c_int, C.c_void_p, _P(C.c_int), C.c_int],
    "amr_set_state_prim_noalloc": [_H, C.c_int, C.c_void_p, _P(C.c_int), C.c_int],
    "amr_fill_ghosts": [_H, C.c_int],
    "amr_rhs": [_H, C.c_int, C.c_void_p],
    "amr_compute_dt": [_H, C.c_int, C.c_void_p],
    "amr_rk_stage": [_H, C.c_int, C.c_void_p],
    "amr_step": [_H, C.c_void_p],
    "amr_tag": [_H, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
    "amr_regrid": [_H, C.c_void_p, C.c_void_p, _P(C.c_int), _P(C.c_int)],
    "amr_adapt": [_H, _P(C.c_int), _P(C.c_int)],
    "amr_check": [_H, _P(C.c_int)],
    "amr_set_exec_mode": [_H, C.c_int],
    "amr_last_created": [_H, _P(C.c_int), C.c_int, _P(C.c_int)],
    "amr_fill_error": [_H, _P(C.c_int)],
    "amr_leaf_cells": [_H, _P(C.c_int64)],
    "amr_velocity_gradient": [_H, C.c_int, C.c_void_p],
    "amr_profile": [_H, C.c_int],
    "amr_profile_read": [_H, _P(C.c_double), _P(C.c_int), _P(C.c_int64)],
    "amr_cnn_create": [_H, C.c_void_p, _P(_H)],
    "amr_cnn_destroy": [_H],
    "amr_cnn_num_params": [_H, _P(C.c_int)],
    "amr_cnn_set_weights": [_H, C.c_void_p, C.c_int],
    "amr_cnn_get_weights": [_H, C.c_void_p, C.c_int],
    "amr_cnn_gather": [_H, C.c_int, _P(C.c_int), C.c_int, C.c_void_p],
    "amr_cnn_forward": [_H, C.c_void_p, C.c_int, C.c_void_p],
    "amr_cnn_train_step": [_H, C.c_void_p, C.c_void_p, C.c_int, C.c_float, C.c_void_p, C.c_void_p],
    "amr_cnn_predict": [_H, C.c_int, C.c_float, C.c_void_p, C.c_void_p],
    "amr_cnn_mfma_selftest": [_H, C.c_void_p, C.c_void_p, C.c_void_p],
    "amr_judge": [_H, _P(C.c_int)],
    "amr_set_fused_halo": [_H, C.c_int],
    "amr_set_tag_buffer": [_H, C.c_int],
    "amr_set_graph": [_H, C.c_int],
    "amr_graph_records": [_H, _P(C.c_int)],
    "amr_set_tile_variant": [_H, C.c_int],
    "amr_get_tile_variant": [_H, _P(C.c_int), _P(C.c_int), _P(C.c_int), _P(C.c_int), _P(C.c_int)],
    "amr_autotune": [_H, C.c_int, _P(C.c_int), _P(C.c_float)],
    "amr_forest_replay": [_P(Config), _P(C.c_int32), C.c_int, _P(PatchInfo), C.c_int, _P(C.c_int)],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.amr_last_error.argtypes = [_H]
_lib.amr_last_error.restype = C.c_char_p

EXPORTED = tuple(_sigs) + ("amr_last_error",)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libamr needs a GPU (torch.cuda.is_available() is False)")
    return torch


class _TorchPool:
    """Device memory for the library, taken from torch's caching allocator."""

    def __init__(self, device):
        self.torch = _torch()
        self.device = device
        self.live: Dict[int, object] = {}
        self._alloc = Allocator._fields_[0][1](self.alloc)
        self._free = Allocator._fields_[1][1](self.free)
        self.struct = Allocator(self._alloc, self._free, None)

    def alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(int(nbytes) + 256, dtype=self.torch.uint8, device=self.device)
            ptr = t.data_ptr()
            ptr = (ptr + 255) // 256 * 256
            self.live[ptr] = t
            return ptr
        except Exception:  # noqa: BLE001 - must not raise into C
            return None

    def free(self, ptr, ctx):
        self.live.pop(int(ptr), None)

    def tensor(self, ptr: int, nbytes: int, dtype):
        """torch view of nbytes at ptr inside an allocation of this pool."""
        t = self.live[ptr]
        off = ptr - t.data_ptr()
        return t[off:off + nbytes].view(dtype)


def make_config(cfg, exec_mode: int = EXEC_BATCHED, coarsen_rule: int = COARSEN_TEXT,
                scheme: int = SCHEME_WENO, level_capacity: Optional[Sequence[int]] = None) -> Config:
    c = Config()
    c.dim = cfg.dim
    c.max_levels = cfg.max_levels
    c.base_cells = cfg.base_cells
    for l, n in enumerate(cfg.patch_cells):
        c.patch_cells[l] = n
    for j in range(3):
        c.periodic[j] = int(cfg.periodic[j]) if j < cfg.dim else 1
    c.lo, c.hi = cfg.lo, cfg.hi
    c.gamma, c.cfl, c.weno_eps, c.tag_theta = cfg.gamma, cfg.cfl, cfg.weno_eps, cfg.tag_theta
    c.tag_buffer = cfg.tag_buffer
    c.max_patches = cfg.max_patches
    if level_capacity is None:
        level_capacity = getattr(cfg, "level_capacity", ())
    if level_capacity:
        for l, v in enumerate(level_capacity):
            c.level_capacity[l] = v
    c.exec_mode = exec_mode
    c.coarsen_rule = coarsen_rule
    c.scheme = scheme
    return c


class Hierarchy:
    """An AMR hierarchy living in device memory (one per stream)."""

    def __init__(self, cfg, exec_mode: int = EXEC_BATCHED, coarsen_rule: int = COARSEN_TEXT,
                 scheme: int = SCHEME_WENO, device: str = "cuda:0", stream=None,
                 level_capacity: Optional[Sequence[int]] = None):
        torch = _torch()
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.pool = _TorchPool(self.device)
        self._c = make_config(cfg, exec_mode, coarsen_rule, scheme, level_capacity)
        self.h = _H()
        st = _lib.amr_create_hierarchy(C.byref(self._c), C.byref(self.pool.struct),
                                       C.c_void_p(self.stream.cuda_stream), C.byref(self.h))
        if st != 0:
            msg = _lib.amr_last_error(self.h).decode() if self.h else "create failed"
            if self.h:
                _lib.amr_destroy_hierarchy(self.h)
                self.h = _H()
            raise AMRError(st, msg)
        n = C.c_int64()
        self._ok(_lib.amr_state_doubles(self.h, C.byref(n)))
        self.state_doubles = n.value
        self.nvar = cfg.dim + 2
        self._dt = torch.zeros(1, dtype=torch.float64, device=self.device)

    # -- plumbing ------------------------------------------------------------
    def _ok(self, st: int):
        if st != 0:
            raise AMRError(st, _lib.amr_last_error(self.h).decode())

    def close(self):
        if self.h:
            _lib.amr_destroy_hierarchy(self.h)
            self.h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    @staticmethod
    def _ptr(t) -> C.c_void_p:
        if t is None:
            return C.c_void_p(None)
        return C.c_void_p(t.data_ptr())

    # -- queries -------------------------------------------------------------
    def counts(self):
        a, l = C.c_int(), C.c_int()
        self._ok(_lib.amr_num_patches(self.h, C.byref(a), C.byref(l)))
        return a.value, l.value

    def patch_table(self) -> List[dict]:
        n = C.c_int()
        self._ok(_lib.amr_get_patch_table(self.h, None, 0, C.byref(n)))
        arr = (PatchInfo * max(1, n.value))()
        self._ok(_lib.amr_get_patch_table(self.h, arr, n.value, C.byref(n)))
        out = []
        d = self.cfg.dim
        nn = 3 ** d - 1
        for r in arr[:n.value]:
            out.append(dict(pid=r.pid, level=r.level, coord=tuple(r.coord[:d]), parent=r.parent,
                            nchildren=r.nchildren, first_child=r.first_child,
                            nbr=tuple(r.nbr[:nn])))
        return out

    def offset(self, pid: int) -> int:
        o = C.c_int64()
        self._ok(_lib.amr_patch_offset(self.h, pid, C.byref(o)))
        return o.value

    def patch_doubles(self, level: int) -> int:
        n = C.c_int64()
        self._ok(_lib.amr_patch_doubles(self.h, level, C.byref(n)))
        return n.value

    def state_tensor(self, buf: int):
        """Zero-copy float64 view of a whole state buffer."""
        p = C.c_void_p()
        self._ok(_lib.amr_state_ptr(self.h, buf, C.byref(p)))
        return self.pool.tensor(p.value, self.state_doubles * 8, self.torch.float64)

    def new_state_like(self):
        return self.torch.zeros(self.state_doubles, dtype=self.torch.float64, device=self.device)

    def last_created(self) -> List[int]:
        n = C.c_int()
        self._ok(_lib.amr_last_created(self.h, None, 0, C.byref(n)))
        arr = (C.c_int * max(1, n.value))()
        self._ok(_lib.amr_last_created(self.h, arr, n.value, C.byref(n)))
        return list(arr[:n.value])

    # -- state transfer ------------------------------------------------------
    def _pids(self, pids):
        arr = (C.c_int * max(1, len(pids)))(*pids)
        return arr

    def set_state(self, buf: int, patches: Dict[int, np.ndarray]):
        pids = list(patches)
        data = np.ascontiguousarray(np.concatenate([np.asarray(patches[p], np.float64).ravel()
                                                    for p in pids])) if pids else np.zeros(1)
        self._ok(_lib.amr_set_state(self.h, buf, data.ctypes.data_as(C.c_void_p),
                                    self._pids(pids), len(pids)))

    def get_state(self, buf: int, pids: Sequence[int], levels: Dict[int, int]) -> Dict[int, np.ndarray]:
        sizes = [self.patch_doubles(levels[p]) for p in pids]
        data = np.empty(max(1, sum(sizes)))
        self._ok(_lib.amr_get_state(self.h, buf, data.ctypes.data_as(C.c_void_p),
                                    self._pids(list(pids)), len(pids)))
        out, pos = {}, 0
        d = self.cfg.dim
        for p, s in zip(pids, sizes):
            n = self.cfg.patch_cells[levels[p]] + 8
            out[p] = data[pos:pos + s].reshape((self.nvar,) + (n,) * d).copy()
            pos += s
        return out

    def set_state_prim(self, buf: int, prims: Dict[int, np.ndarray]):
        pids = list(prims)
        data = np.ascontiguousarray(np.concatenate([np.asarray(prims[p], np.float64).ravel()
                                                    for p in pids])) if pids else np.zeros(1)
        self._ok(_lib.amr_set_state_prim(self.h, buf, data.ctypes.data_as(C.c_void_p),
                                         self._pids(pids), len(pids)))

    def set_state_prim_noalloc(self, buf: int, prims: Dict[int, np.ndarray]):
        """set_state_prim through the library's fixed per-GPU scratch (no
        device allocation; at most NOALLOC_SCRATCH_BYTES per call)."""
        pids = list(prims)
        data = np.ascontiguousarray(np.concatenate([np.asarray(prims[p], np.float64).ravel()
                                                    for p in pids])) if pids else np.zeros(1)
        self._ok(_lib.amr_set_state_prim_noalloc(self.h, buf, data.ctypes.data_as(C.c_void_p),
                                                 self._pids(pids), len(pids)))

    # -- hot path ------------------------------------------------------------
    def fill_ghosts(self, buf: int):
        self._ok(_lib.amr_fill_ghosts(self.h, buf))

    def rhs(self, buf: int, out=None):
        out = self.new_state_like() if out is None else out
        self._ok(_lib.amr_rhs(self.h, buf, self._ptr(out)))
        return out

    def compute_dt(self, buf: int = 0, out=None):
        out = self._dt if out is None else out
        self._ok(_lib.amr_compute_dt(self.h, buf, self._ptr(out)))
        return out

    def rk_stage(self, stage: int, dt):
        self._ok(_lib.amr_rk_stage(self.h, stage, self._ptr(dt)))

    def step(self, dt_out=None):
        dt_out = self._dt if dt_out is None else dt_out
        self._ok(_lib.amr_step(self.h, self._ptr(dt_out)))
        return dt_out

    def tag(self, buf: int = 0, cell_tags: bool = False):
        t = self.torch
        mp = self.cfg.max_patches
        refine = t.zeros(mp, dtype=t.uint8, device=self.device)
        coarsen = t.zeros(mp, dtype=t.uint8, device=self.device)
        cells = None
        if cell_tags:
            cells = t.zeros(self.state_doubles // self.nvar, dtype=t.uint8, device=self.device)
        self._ok(_lib.amr_tag(self.h, buf, self._ptr(refine), self._ptr(coarsen), self._ptr(cells)))
        return refine, coarsen, cells

    def regrid(self, refine: np.ndarray, coarsen: np.ndarray):
        r = np.ascontiguousarray(refine, dtype=np.uint8)
        c = np.ascontiguousarray(coarsen, dtype=np.uint8)
        nc, nd = C.c_int(), C.c_int()
        self._ok(_lib.amr_regrid(self.h, r.ctypes.data_as(C.c_void_p), c.ctypes.data_as(C.c_void_p),
                                 C.byref(nc), C.byref(nd)))
        return nc.value, nd.value

    def adapt(self):
        nc, nd = C.c_int(), C.c_int()
        self._ok(_lib.amr_adapt(self.h, C.byref(nc), C.byref(nd)))
        return nc.value, nd.value

    def check(self) -> int:
        n = C.c_int()
        st = _lib.amr_check(self.h, C.byref(n))
        if st not in (0, -5):
            self._ok(st)
        return n.value

    def fill_error(self) -> int:
        n = C.c_int()
        self._ok(_lib.amr_fill_error(self.h, C.byref(n)))
        return n.value

    def velocity_gradient(self, buf: int = 0, out=None):
        """Velocity-gradient tensor and density-gradient magnitude at leaf
        interior cells: a device tensor [d*d + 1, state_doubles / nvar] in
        the per-variable cell layout (a new one filled with NaN where nothing
        is written, or ``out``, which is reused as it is)."""
        t = self.torch
        shape = (self.cfg.dim ** 2 + 1, self.state_doubles // self.nvar)
        if out is None:
            out = t.full(shape, float("nan"), dtype=t.float64, device=self.device)
        elif tuple(out.shape) != shape or out.dtype != t.float64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float64 tensor of shape {shape}")
        self._ok(_lib.amr_velocity_gradient(self.h, buf, self._ptr(out)))
        return out

    def leaf_cells(self) -> int:
        n = C.c_int64()
        self._ok(_lib.amr_leaf_cells(self.h, C.byref(n)))
        return n.value

    def profile(self, enable: bool):
        self._ok(_lib.amr_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        ms, n, cells = C.c_double(), C.c_int(), C.c_int64()
        self._ok(_lib.amr_profile_read(self.h, C.byref(ms), C.byref(n), C.byref(cells)))
        return ms.value, n.value, cells.value

    def set_tile_variant(self, v: int):
        self._ok(_lib.amr_set_tile_variant(self.h, v))

    def tile_variant(self):
        v, x, y, z, t = (C.c_int() for _ in range(5))
        self._ok(_lib.amr_get_tile_variant(self.h, C.byref(v), C.byref(x), C.byref(y), C.byref(z),
                                           C.byref(t)))
        return v.value, (x.value, y.value, z.value), t.value

    def autotune(self, reps: int = 5):
        b, ms = C.c_int(), C.c_float()
        self._ok(_lib.amr_autotune(self.h, reps, C.byref(b), C.byref(ms)))
        return b.value, ms.value

    def set_graph(self, enable: bool):
        self._ok(_lib.amr_set_graph(self.h, 1 if enable else 0))

    def graph_records(self) -> int:
        n = C.c_int()
        self._ok(_lib.amr_graph_records(self.h, C.byref(n)))
        return n.value

    def set_fused_halo(self, enable: bool):
        self._ok(_lib.amr_set_fused_halo(self.h, 1 if enable else 0))

    def set_tag_buffer(self, cells: int):
        self._ok(_lib.amr_set_tag_buffer(self.h, int(cells)))

    def judge(self) -> int:
        n = C.c_int()
        self._ok(_lib.amr_judge(self.h, C.byref(n)))
        return n.value

    def set_exec_mode(self, mode: int):
        self._ok(_lib.amr_set_exec_mode(self.h, mode))


class Predictor:
    """The learned refinement predictor of a 2D or 3D hierarchy (device
    weights).  ``mean``/``std`` normalise (rho, u, v, p) in 2D and
    (rho, u, v, w, p) in 3D; a 3D tile has edge ``patch_cells`` = 8."""

    def __init__(self, hier: "Hierarchy", patch_cells: int, mean, std, pos_weight: float = 1.0,
                 max_batch: int = 256):
        self.hier = hier
        self.torch = hier.torch
        self.dim = hier.cfg.dim
        self.n = patch_cells
        self.max_batch = max_batch
        c = CnnConfig()
        c.patch_cells = patch_cells
        nch = self.dim + 2
        if len(mean) != nch or len(std) != nch:
            raise ValueError(f"{nch} normalisation channels expected")
        for k in range(nch):
            c.mean[k] = float(mean[k])
            c.std[k] = float(std[k])
        c.pos_weight = pos_weight
        c.max_batch = max_batch
        self._c = c
        self.h = _H()
        hier._ok(_lib.amr_cnn_create(hier.h, C.byref(c), C.byref(self.h)))
        n = C.c_int()
        hier._ok(_lib.amr_cnn_num_params(self.h, C.byref(n)))
        self.nparams = n.value
        self._loss = self.torch.zeros(1, dtype=self.torch.float32, device=hier.device)

    def close(self):
        if self.h:
            _lib.amr_cnn_destroy(self.h)
            self.h = _H()

    def set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self.hier._ok(_lib.amr_cnn_set_weights(self.h, w.ctypes.data_as(C.c_void_p), w.size))

    def get_weights(self) -> np.ndarray:
        w = np.empty(self.nparams, np.float32)
        self.hier._ok(_lib.amr_cnn_get_weights(self.h, w.ctypes.data_as(C.c_void_p), w.size))
        return w

    def tile_shape(self):
        """(voxels, stored channels) of one input tile."""
        if self.dim == 2:
            return ((self.n + 6) ** 2, 4)
        return ((self.n + 6) ** 3, 8)

    @property
    def tile_cells(self) -> int:
        return self.n ** self.dim

    def gather(self, buf: int, pids):
        t = self.torch
        x = t.empty((len(pids),) + self.tile_shape(), dtype=t.int16, device=self.hier.device)
        arr = (C.c_int * max(1, len(pids)))(*pids)
        self.hier._ok(_lib.amr_cnn_gather(self.h, buf, arr, len(pids), Hierarchy._ptr(x)))
        return x

    def forward(self, x):
        t = self.torch
        z = t.empty((x.shape[0], self.tile_cells), dtype=t.float32, device=self.hier.device)
        self.hier._ok(_lib.amr_cnn_forward(self.h, Hierarchy._ptr(x), x.shape[0], Hierarchy._ptr(z)))
        return z

    def train_step(self, x, labels, lr: float, grads=None):
        self.hier._ok(_lib.amr_cnn_train_step(self.h, Hierarchy._ptr(x), Hierarchy._ptr(labels),
                                              x.shape[0], C.c_float(lr), Hierarchy._ptr(self._loss),
                                              Hierarchy._ptr(grads)))
        return self._loss

    def predict(self, buf: int, tau: float):
        t = self.torch
        mp = self.hier.cfg.max_patches
        r = t.zeros(mp, dtype=t.uint8, device=self.hier.device)
        c = t.zeros(mp, dtype=t.uint8, device=self.hier.device)
        self.hier._ok(_lib.amr_cnn_predict(self.h, buf, C.c_float(tau), Hierarchy._ptr(r),
                                           Hierarchy._ptr(c)))
        return r, c


def mfma_selftest(hier: "Hierarchy", a, b, d):
    hier._ok(_lib.amr_cnn_mfma_selftest(hier.h, Hierarchy._ptr(a), Hierarchy._ptr(b), Hierarchy._ptr(d)))


def forest_replay(cfg, rounds, coarsen_rule: int = COARSEN_TEXT):
    """Host-only mesh adaptation (no GPU): ``rounds`` is a list of
    (refine_keys, coarsen_keys) with keys (level, coord); returns the active
    patches as (level, coord, parent_pid, nchildren, pid) tuples."""
    c = make_config(cfg, coarsen_rule=coarsen_rule)
    recs = []
    for r, (ref, coa) in enumerate(rounds):
        for kind, keys in ((0, ref), (1, coa)):
            for level, coord in keys:
                xyz = list(coord) + [0] * (3 - len(coord))
                recs.append([r, kind, level] + xyz)
    arr = (C.c_int32 * max(1, 6 * len(recs)))(*[v for rec in recs for v in rec])
    n = C.c_int()
    st = _lib.amr_forest_replay(C.byref(c), arr, len(recs), None, 0, C.byref(n))
    if st != 0:
        raise AMRError(st, "forest replay failed")
    out = (PatchInfo * max(1, n.value))()
    st = _lib.amr_forest_replay(C.byref(c), arr, len(recs), out, n.value, C.byref(n))
    if st != 0:
        raise AMRError(st, "forest replay failed")
    d = cfg.dim
    return [(r.level, tuple(r.coord[:d]), r.parent, r.nchildren, r.pid) for r in out[:n.value]]


# ---------------------------------------------------------------------------
# initial hierarchy from a seeded generator (inputs only; all arithmetic of the
# method runs in the library)
# ---------------------------------------------------------------------------


def patch_primitives(cfg, level: int, coord, gen) -> np.ndarray:
    from . import workloads
    pts = workloads.patch_points(cfg, level, coord)
    rho, u, p = gen(pts)
    return np.stack([rho] + list(u) + [p])


def upload_initial(h: Hierarchy, rows, gen, chunk_values: int = 1 << 23):
    """Interior primitives of the given patch-table rows sampled from ``gen``
    and uploaded, a level's patches evaluated together in chunks of about
    ``chunk_values`` cells (the generators take stacked patch grids)."""
    from . import workloads
    cfg = h.cfg
    by_level: Dict[int, list] = {}
    for r in rows:
        by_level.setdefault(r["level"], []).append(r)
    for level, rs in sorted(by_level.items()):
        per = max(1, chunk_values // cfg.patch_cells[level] ** cfg.dim)
        for a in range(0, len(rs), per):
            part = rs[a:a + per]
            pts = workloads.patch_points_batch(cfg, level, [r["coord"] for r in part])
            rho, u, p = gen(pts)
            h.set_state_prim(0, {r["pid"]: np.stack([rho[i]] + [uj[i] for uj in u] + [p[i]])
                                 for i, r in enumerate(part)})


def init_from_ic(h: Hierarchy, gen) -> int:
    """Level-0 data from ``gen``, then max_levels-1 rounds of tag and refine
    with new patches sampled from ``gen``.  Returns the number of rounds."""
    cfg = h.cfg
    upload_initial(h, h.patch_table(), gen)
    rounds = 0
    for _ in range(cfg.max_levels - 1):
        refine, _, _ = h.tag(0)
        r = refine.cpu().numpy()
        if not r.any():
            break
        h.regrid(r, np.zeros_like(r))
        new = set(h.last_created())
        upload_initial(h, [t for t in h.patch_table() if t["pid"] in new], gen)
        rounds += 1
    return rounds
