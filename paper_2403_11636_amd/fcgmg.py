"""Python binding of the fcgmg C-ABI library (include/fcgmg.h).

Argument marshalling only: every step runs in the HIP kernels of libfcgmg.so. PyTorch provides the
device memory (FP64 CUDA/HIP tensors) and the stream. There is no CPU fallback: if the library
is missing or no GPU is visible, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfcgmg.so")

CACHE_INVERSE, CACHE_MATRIX, CACHE_NONE = 0, 1, 2
POLICY_NAMES = {CACHE_INVERSE: "cache_inverse", CACHE_MATRIX: "cache_matrix", CACHE_NONE: "cache_none"}
PREC_FP64, PREC_MIXED = 0, 1
SOLVER_GMG, SOLVER_FGMRES = 0, 1

OK, E_ARG, E_NOMEM, E_HIP, E_SINGULAR, E_NOCONV, E_NAN = 0, -1, -2, -3, -4, -5, -6

EXPORTS = [
    "fcgmg_setup_hierarchy", "fcgmg_num_levels", "fcgmg_num_dofs", "fcgmg_level_stats_get", "fcgmg_rhs",
    "fcgmg_residual", "fcgmg_smooth", "fcgmg_smooth_noalloc", "fcgmg_smooth_multi", "fcgmg_vcycle_multi", "fcgmg_restrict", "fcgmg_prolongate_add", "fcgmg_coarse_solve",
    "fcgmg_vcycle", "fcgmg_vcycle_fp32", "fcgmg_solve", "fcgmg_norm", "fcgmg_device_bytes", "fcgmg_footprint_bytes", "fcgmg_destroy", "fcgmg_last_error",
    "fcgmg_profile_enable", "fcgmg_profile_reset", "fcgmg_profile_read",
    "fcgmg_autotune", "fcgmg_fused_shape", "fcgmg_set_fused_shape", "fcgmg_set_cache_none_assembly",
    "fcgmg_server_create", "fcgmg_server_submit", "fcgmg_server_wait", "fcgmg_server_resident_bytes",
    "fcgmg_server_stats",
    "fcgmg_server_destroy", "fcgmg_batch_create", "fcgmg_batch_vcycle", "fcgmg_batch_solve",
    "fcgmg_batch_destroy", "fcgmg_batch_set_persistent",
]

N_FUSED_SHAPES = 8  # tile shapes of the fused 2D sweep (fcgmg_fused_shape)


def fused_shape(k: int) -> tuple:
    """(tile_x, tile_y, threads, waves_per_simd) of fused-sweep shape k."""
    v = [ctypes.c_int() for _ in range(4)]
    _check(load().fcgmg_fused_shape(int(k), *[ctypes.byref(q) for q in v]))
    return tuple(q.value for q in v)


KERNEL_KINDS = ["residual", "apply_regular", "apply_irregular", "patch_solve", "restrict", "prolong", "coarse",
                "zero", "sweep_fused", "residual_restrict"]


class FcgmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fcgmg error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n_cells", ctypes.c_int), ("n_levels", ctypes.c_int),
        ("quad_depth", ctypes.c_int), ("cache_policy", ctypes.c_int), ("nu_pre", ctypes.c_int),
        ("nu_post", ctypes.c_int), ("force", ctypes.c_int), ("bc", ctypes.c_int * 6),
        ("eta", ctypes.c_double), ("alpha_fict", ctypes.c_double), ("nitsche_beta", ctypes.c_double),
        ("omega", ctypes.c_double), ("ubar", ctypes.c_double), ("precision", ctypes.c_int),
        ("solver", ctypes.c_int), ("krylov_restart", ctypes.c_int), ("immersed_nitsche", ctypes.c_int),
    ]


class ServerParams(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int), ("max_iter", ctypes.c_int), ("hbm_budget", ctypes.c_int64),
                ("continuous_batching", ctypes.c_int)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("policy", ctypes.c_int), ("iters", ctypes.c_int),
                ("cache_hit", ctypes.c_int), ("rel_res", ctypes.c_double), ("t_queue_ms", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("footprint", ctypes.c_int64)]


class LevelStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n_cells_axis", "n_nodes", "n_cut_cells", "n_fict_cells", "n_classes", "n_irregular",
        "irregular_cols", "cached_bytes", "n_stencils")]


_lib = None


def load(path: str = LIB_PATH):
    """Load libfcgmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with paper_2403_11636_amd/build.py")
    # torch bundles its own HIP runtime (SONAME libamdhip64.so.7). Loading torch first makes the
    # library's dependency resolve to that same runtime instead of a second copy from /opt/rocm,
    # which would not see the device context that torch owns.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    L.fcgmg_setup_hierarchy.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.fcgmg_num_levels.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.fcgmg_num_dofs.argtypes = [vp, ctypes.c_int, i64p]
    L.fcgmg_level_stats_get.argtypes = [vp, ctypes.c_int, ctypes.POINTER(LevelStats)]
    L.fcgmg_rhs.argtypes = [vp, ctypes.c_int, vp, vp]
    L.fcgmg_residual.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.fcgmg_smooth.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    L.fcgmg_smooth_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    L.fcgmg_smooth_multi.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    L.fcgmg_vcycle_multi.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    L.fcgmg_restrict.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.fcgmg_prolongate_add.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.fcgmg_coarse_solve.argtypes = [vp, vp, vp, vp]
    L.fcgmg_vcycle.argtypes = [vp, vp, vp, vp]
    L.fcgmg_vcycle_fp32.argtypes = [vp, vp, vp, vp]
    L.fcgmg_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp, dp, vp]
    L.fcgmg_norm.argtypes = [vp, ctypes.c_int, vp, dp, vp]
    L.fcgmg_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.fcgmg_server_create.argtypes = [ctypes.POINTER(ServerParams), ctypes.POINTER(vp)]
    L.fcgmg_server_submit.argtypes = [vp, ctypes.POINTER(Params), dp, ctypes.c_int, ctypes.c_double, vp, i64p]
    L.fcgmg_server_wait.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(RequestResult)]
    L.fcgmg_server_resident_bytes.argtypes = [vp, i64p, ctypes.POINTER(ctypes.c_int)]
    L.fcgmg_server_stats.argtypes = [vp, i64p, i64p, ctypes.POINTER(ctypes.c_int)]
    L.fcgmg_server_destroy.argtypes = [vp]
    L.fcgmg_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp)]
    L.fcgmg_batch_vcycle.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.fcgmg_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), dp, vp]
    L.fcgmg_batch_destroy.argtypes = [vp]
    L.fcgmg_batch_set_persistent.argtypes = [vp, ctypes.c_int]
    L.fcgmg_footprint_bytes.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.fcgmg_destroy.argtypes = [vp]
    L.fcgmg_profile_enable.argtypes = [vp, ctypes.c_int]
    L.fcgmg_profile_reset.argtypes = [vp]
    L.fcgmg_profile_read.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, i64p]
    ip = ctypes.POINTER(ctypes.c_int)
    L.fcgmg_autotune.argtypes = [vp, ctypes.c_int, ip, dp, vp]
    L.fcgmg_fused_shape.argtypes = [ctypes.c_int, ip, ip, ip, ip]
    L.fcgmg_set_fused_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    L.fcgmg_set_cache_none_assembly.argtypes = [vp, ctypes.c_int]
    for name in EXPORTS:
        getattr(L, name).restype = ctypes.c_int
    L.fcgmg_destroy.restype = None
    L.fcgmg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


_device_ready = False


def _init_device():
    """Make torch create the device context (and load its HIP runtime) before the library's first
    HIP call, so that the library and torch share one runtime and one context."""
    global _device_ready
    if not _device_ready:
        import torch
        torch.cuda.init()
        torch.empty(1, device="cuda")
        torch.cuda.synchronize()
        _device_ready = True


def _check(rc: int):
    if rc != OK:
        raise FcgmgError(rc, load().fcgmg_last_error().decode())


def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t, name: str, numel: int):
    """Device pointer of a contiguous FP64 GPU tensor of exactly `numel` values (checked on the host
    so that no kernel is ever handed a buffer shorter than the level it works on)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 GPU tensor")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} values, the level needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def make_params(prob, policy: int = CACHE_INVERSE, precision: int = PREC_FP64, solver: int = SOLVER_GMG,
                krylov_restart: int = 30) -> Params:
    p = Params()
    p.dim = prob.dim
    p.n_cells = prob.n_cells
    p.n_levels = prob.n_levels
    p.quad_depth = prob.quad_depth
    p.cache_policy = policy
    p.nu_pre = prob.nu_pre
    p.nu_post = prob.nu_post
    p.force = prob.force
    for k in range(6):
        p.bc[k] = int(prob.bcs[k])
    p.eta = prob.eta
    p.alpha_fict = prob.alpha_fict
    p.nitsche_beta = prob.nitsche_beta
    p.omega = prob.omega
    p.ubar = prob.ubar
    p.precision = precision
    p.solver = solver
    p.krylov_restart = krylov_restart
    p.immersed_nitsche = int(getattr(prob, "immersed_nitsche", 0))
    return p


def footprint_bytes(prob, policy: int = CACHE_INVERSE, precision: int = PREC_FP64, solver: int = SOLVER_GMG,
                    krylov_restart: int = 30) -> int:
    """Device bytes a Hierarchy of `prob` would hold (fcgmg_footprint_bytes; host-only, no GPU)."""
    L = load()
    prm = make_params(prob, policy, precision, solver, krylov_restart)
    balls = np.ascontiguousarray(np.asarray(prob.balls, dtype=np.float64).reshape(-1, 4))
    bp = balls.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if balls.size else None
    out = ctypes.c_size_t()
    _check(L.fcgmg_footprint_bytes(ctypes.byref(prm), bp, balls.shape[0], ctypes.byref(out)))
    return out.value


class Hierarchy:
    """Device-resident GMG hierarchy of one finite cell Stokes problem (fcgmg_setup_hierarchy)."""

    def __init__(self, prob, policy: int = CACHE_INVERSE, stream=None, precision: int = PREC_FP64,
                 solver: int = SOLVER_GMG, krylov_restart: int = 30):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("fcgmg needs a GPU; none is visible")
        _init_device()
        L = load()
        self.prob = prob
        self.policy = policy
        self.dim = prob.dim
        self.precision = precision
        self.solver = solver
        self._params = make_params(prob, policy, precision, solver, krylov_restart)
        balls = np.ascontiguousarray(np.asarray(prob.balls, dtype=np.float64).reshape(-1, 4))
        self._balls = balls
        h = ctypes.c_void_p()
        bp = balls.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if balls.size else None
        _check(L.fcgmg_setup_hierarchy(ctypes.byref(self._params), bp, balls.shape[0], _stream_ptr(stream),
                                       ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int()
        _check(L.fcgmg_num_levels(self.h, ctypes.byref(n)))
        self.n_levels = n.value
        self.fine = self.n_levels - 1

    def close(self):
        if getattr(self, "h", None):
            load().fcgmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ndofs(self, level: Optional[int] = None) -> int:
        level = self.fine if level is None else level
        n = ctypes.c_int64()
        _check(load().fcgmg_num_dofs(self.h, level, ctypes.byref(n)))
        return n.value

    def stats(self, level: Optional[int] = None) -> dict:
        level = self.fine if level is None else level
        s = LevelStats()
        _check(load().fcgmg_level_stats_get(self.h, level, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in LevelStats._fields_}

    def profile(self, on: bool = True):
        """Enable/disable the library's per-kernel event timers."""
        _check(load().fcgmg_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        _check(load().fcgmg_profile_reset(self.h))

    def profile_read(self) -> dict:
        """{(kind_name, level): (total_ms, launches)} for every kind/level with launches."""
        out = {}
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        for k, name in enumerate(KERNEL_KINDS):
            for lev in range(self.n_levels):
                _check(load().fcgmg_profile_read(self.h, k, lev, ctypes.byref(ms), ctypes.byref(cnt)))
                if cnt.value:
                    out[(name, lev)] = (ms.value, cnt.value)
        return out

    def autotune(self, reps: int = 20, stream=None) -> dict:
        """Time every fused-sweep tile shape per level and keep the fastest (2D cache_inverse).

        Returns {"shape": [index per level, -1 = default], "us": [[us per sweep per shape] per level]}."""
        nl, ns = self.n_levels, N_FUSED_SHAPES
        shapes = (ctypes.c_int * nl)()
        us = (ctypes.c_double * (nl * ns))()
        _check(load().fcgmg_autotune(self.h, int(reps), shapes, us, _stream_ptr(stream)))
        return {"shape": list(shapes), "us": [[us[l * ns + k] for k in range(ns)] for l in range(nl)]}

    def set_fused_shape(self, level: int, k: int, stream=None):
        """Use fused-sweep shape k (-1 = default by size) on `level`, e.g. a stored autotune choice."""
        _check(load().fcgmg_set_fused_shape(self.h, int(level), int(k), _stream_ptr(stream)))

    def tuning_table(self, result: dict) -> dict:
        """The choices of `autotune` keyed by level size: {"<cells per axis>": (tile_x, tile_y, threads,
        waves_per_simd)}, for storing (JSON) and applying to other hierarchies with `apply_tuning`."""
        table = {}
        for lev, k in enumerate(result["shape"]):
            if k >= 0:
                table[str(self.prob.level_cells(lev))] = tuple(fused_shape(k))
        return table

    def apply_tuning(self, table: dict, stream=None) -> list:
        """Give every level whose size appears in `table` the stored shape; returns the shape index per
        level afterwards (-1 where the table has no entry: the default by size)."""
        by_dims = {tuple(fused_shape(k)): k for k in range(N_FUSED_SHAPES)}
        out = []
        for lev in range(self.n_levels):
            dims = table.get(str(self.prob.level_cells(lev)))
            k = by_dims.get(tuple(dims), -1) if dims is not None else -1
            if k >= 0 and lev > 0:
                self.set_fused_shape(lev, k, stream)
            out.append(k if lev > 0 else -1)
        return out

    def set_cache_none_assembly(self, integrate: bool):
        """cache_none: read each block from the operator rows (False, default) or assemble it from the
        window's element integrals with its cut cells integrated on the fly (True)."""
        _check(load().fcgmg_set_cache_none_assembly(self.h, 1 if integrate else 0))

    def device_bytes(self) -> int:
        v = ctypes.c_size_t()
        _check(load().fcgmg_device_bytes(self.h, ctypes.byref(v)))
        return v.value

    def zeros(self, level: Optional[int] = None):
        import torch
        return torch.zeros(self.ndofs(level), dtype=torch.float64, device="cuda")

    def rhs(self, level: Optional[int] = None, out=None, stream=None):
        level = self.fine if level is None else level
        b = self.zeros(level) if out is None else out
        _check(load().fcgmg_rhs(self.h, level, _dptr(b, "b", self.ndofs(level)), _stream_ptr(stream)))
        return b

    def residual(self, x, b, level: Optional[int] = None, out=None, stream=None):
        level = self.fine if level is None else level
        n = self.ndofs(level)
        r = self.zeros(level) if out is None else out
        _check(load().fcgmg_residual(self.h, level, _dptr(x, "x", n), _dptr(b, "b", n), _dptr(r, "r", n),
                                     _stream_ptr(stream)))
        return r

    def smooth(self, x, b, sweeps: int = 1, level: Optional[int] = None, stream=None):
        level = self.fine if level is None else level
        n = self.ndofs(level)
        _check(load().fcgmg_smooth(self.h, level, _dptr(x, "x", n), _dptr(b, "b", n), sweeps, _stream_ptr(stream)))
        return x

    def smooth_noalloc(self, x, b, sweeps: int = 1, level: Optional[int] = None, stream=None):
        """fcgmg_smooth_noalloc: the same sweeps with the library's static scratch (no allocation)."""
        level = self.fine if level is None else level
        n = self.ndofs(level)
        _check(load().fcgmg_smooth_noalloc(self.h, level, _dptr(x, "x", n), _dptr(b, "b", n), sweeps,
                                           _stream_ptr(stream)))
        return x

    def smooth_multi(self, x, b, r, nrhs: int, sweeps: int = 1, level: Optional[int] = None, stream=None):
        """Stacked right-hand sides: x, b, r hold nrhs level vectors one after another (r: scratch)."""
        level = self.fine if level is None else level
        n = self.ndofs(level) * nrhs
        _check(load().fcgmg_smooth_multi(self.h, level, _dptr(x, "x", n), _dptr(b, "b", n), _dptr(r, "r", n), nrhs,
                                         sweeps, _stream_ptr(stream)))
        return x

    def vcycle_multi(self, x, b, nrhs: int, stream=None):
        """One V-cycle for each of nrhs stacked finest-level vectors (x, b: nrhs vectors one after another)."""
        n = self.ndofs() * nrhs
        _check(load().fcgmg_vcycle_multi(self.h, _dptr(x, "x", n), _dptr(b, "b", n), nrhs, _stream_ptr(stream)))
        return x

    def restrict(self, r_fine, fine_level: Optional[int] = None, out=None, stream=None):
        fine_level = self.fine if fine_level is None else fine_level
        bc = self.zeros(fine_level - 1) if out is None else out
        _check(load().fcgmg_restrict(self.h, fine_level, _dptr(r_fine, "r", self.ndofs(fine_level)),
                                     _dptr(bc, "b_coarse", self.ndofs(fine_level - 1)),
                                     _stream_ptr(stream)))
        return bc

    def prolongate_add(self, e_coarse, x_fine, fine_level: Optional[int] = None, stream=None):
        fine_level = self.fine if fine_level is None else fine_level
        _check(load().fcgmg_prolongate_add(self.h, fine_level, _dptr(e_coarse, "e", self.ndofs(fine_level - 1)),
                                           _dptr(x_fine, "x", self.ndofs(fine_level)),
                                           _stream_ptr(stream)))
        return x_fine

    def coarse_solve(self, b, out=None, stream=None):
        x = self.zeros(0) if out is None else out
        n = self.ndofs(0)
        _check(load().fcgmg_coarse_solve(self.h, _dptr(b, "b", n), _dptr(x, "x", n), _stream_ptr(stream)))
        return x

    def vcycle(self, x, b, stream=None):
        n = self.ndofs()
        _check(load().fcgmg_vcycle(self.h, _dptr(x, "x", n), _dptr(b, "b", n), _stream_ptr(stream)))
        return x

    def vcycle_fp32(self, r, out=None, stream=None):
        """e = V(0, r) by one FP32 V-cycle (mixed-precision hierarchies); r, e FP64 finest-level."""
        n = self.ndofs()
        e = self.zeros() if out is None else out
        _check(load().fcgmg_vcycle_fp32(self.h, _dptr(r, "r", n), _dptr(e, "e", n), _stream_ptr(stream)))
        return e

    def norm(self, v, level: Optional[int] = None, stream=None) -> float:
        level = self.fine if level is None else level
        out = ctypes.c_double()
        _check(load().fcgmg_norm(self.h, level, _dptr(v, "v", self.ndofs(level)), ctypes.byref(out),
                                 _stream_ptr(stream)))
        return out.value

    def solve(self, b, x=None, rtol: float = 1e-8, max_iter: int = 100, stream=None, raise_on_noconv=True):
        x = self.zeros() if x is None else x
        it = ctypes.c_int()
        rel = ctypes.c_double()
        hist = np.zeros(max_iter + 1)
        n = self.ndofs()
        rc = load().fcgmg_solve(self.h, _dptr(x, "x", n), _dptr(b, "b", n), rtol, max_iter, ctypes.byref(it),
                                ctypes.byref(rel), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                _stream_ptr(stream))
        if rc != OK and (rc != E_NOCONV or raise_on_noconv):
            _check(rc)
        return x, it.value, rel.value, hist[: it.value + 1], rc


class Server:
    """Solve server (fcgmg_server_*): concurrent solves on device-resident hierarchies, admitted by
    device-memory footprint. submit() queues a problem and returns an id; wait(id) returns the
    solution tensor and the request's result fields."""

    def __init__(self, workers: int = 4, hbm_budget: int = 0, max_iter: int = 200, continuous_batching: int = 1):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("fcgmg needs a GPU; none is visible")
        _init_device()
        L = load()
        sp = ServerParams(workers, max_iter, hbm_budget, continuous_batching)
        h = ctypes.c_void_p()
        _check(L.fcgmg_server_create(ctypes.byref(sp), ctypes.byref(h)))
        self.h = h
        self._out = {}

    def submit(self, prob, policy: int = -1, precision: int = PREC_FP64, rtol: float = 1e-8,
               solver: int = SOLVER_GMG, krylov_restart: int = 30) -> int:
        import torch
        prm = make_params(prob, policy, precision, solver, krylov_restart)
        balls = np.ascontiguousarray(np.asarray(prob.balls, dtype=np.float64).reshape(-1, 4))
        bp = balls.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if balls.size else None
        n = (prob.dim + 1) * (prob.n_cells + 1) ** prob.dim
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        rid = ctypes.c_int64()
        _check(load().fcgmg_server_submit(self.h, ctypes.byref(prm), bp, balls.shape[0], rtol,
                                          ctypes.c_void_p(x.data_ptr()), ctypes.byref(rid)))
        self._out[rid.value] = x
        return rid.value

    def wait(self, rid: int):
        res = RequestResult()
        _check(load().fcgmg_server_wait(self.h, rid, ctypes.byref(res)))
        x = self._out.pop(rid)
        return x, {k: getattr(res, k) for k, _ in RequestResult._fields_}

    def resident(self):
        b = ctypes.c_int64()
        n = ctypes.c_int()
        _check(load().fcgmg_server_resident_bytes(self.h, ctypes.byref(b), ctypes.byref(n)))
        return b.value, n.value

    def stats(self):
        """Continuous batching so far: (batched cycle steps, request-cycles, largest batch)."""
        s = ctypes.c_int64()
        rc = ctypes.c_int64()
        mb = ctypes.c_int()
        _check(load().fcgmg_server_stats(self.h, ctypes.byref(s), ctypes.byref(rc), ctypes.byref(mb)))
        return s.value, rc.value, mb.value

    def close(self):
        if getattr(self, "h", None):
            load().fcgmg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched V-cycles over independent 2D hierarchies (fcgmg_batch_*): one launch per cycle step for
    all problems. The hierarchies stay owned by the caller."""

    def __init__(self, hierarchies):
        L = load()
        self.hs = list(hierarchies)
        arr = (ctypes.c_void_p * len(self.hs))(*[h.h.value for h in self.hs])
        h = ctypes.c_void_p()
        _check(L.fcgmg_batch_create(arr, len(self.hs), ctypes.byref(h)))
        self.h = h

    def _ptrs(self, vecs, name):
        assert len(vecs) == len(self.hs)
        return (ctypes.c_void_p * len(vecs))(*[_dptr(v, name, h.ndofs()).value for v, h in zip(vecs, self.hs)])

    def set_persistent(self, on: bool = True):
        """Fused sweeps as persistent launches (tiles handed out by ticket) or one workgroup per tile."""
        _check(load().fcgmg_batch_set_persistent(self.h, int(on)))

    def vcycle(self, xs, bs, stream=None):
        _check(load().fcgmg_batch_vcycle(self.h, self._ptrs(xs, "x"), self._ptrs(bs, "b"), _stream_ptr(stream)))
        return xs

    def solve(self, bs, xs=None, rtol: float = 1e-8, max_iter: int = 100, stream=None):
        xs = [h.zeros() for h in self.hs] if xs is None else xs
        n = len(self.hs)
        its = (ctypes.c_int * n)()
        rel = np.zeros(n)
        rc = load().fcgmg_batch_solve(self.h, self._ptrs(xs, "x"), self._ptrs(bs, "b"), rtol, max_iter, its,
                                      rel.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(stream))
        return xs, list(its), rel, rc

    def close(self):
        if getattr(self, "h", None):
            load().fcgmg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
