"""ctypes wrapper of the FP64 CPU oracle (oracle/fcm_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by the cpu_baseline
leg of bench.py. The product library never imports, links or runs it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fcm_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

c_long_p = ctypes.POINTER(ctypes.c_long)
c_double_p = ctypes.POINTER(ctypes.c_double)


def build() -> str:
    """Compile the oracle (plain g++, FP64, OpenMP over independent patches)."""
    cmd = ["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c++17", SRC, "-o", LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, c_double_p,
                                 ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_nnodes.restype = ctypes.c_long
        L.orc_nnodes.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_coo.restype = ctypes.c_long
        L.orc_coo.argtypes = [ctypes.c_void_p, ctypes.c_int, c_long_p, c_long_p, c_double_p]
        for name in ("orc_coarse_ok", "orc_bordered"):
            getattr(L, name).argtypes = [ctypes.c_void_p]
        L.orc_patch_dofs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, c_long_p]
        L.orc_patch_matrix.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, c_double_p]
        L.orc_inverse_rows.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, c_double_p]
        L.orc_element_matrix.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, c_double_p]
        L.orc_cell_quadrature.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, c_double_p]
        L.orc_arc_points.restype = ctypes.c_long
        L.orc_arc_points.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, c_double_p, ctypes.c_long]
        L.orc_cell_kinds.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_byte)]
        L.orc_rhs.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p]
        L.orc_matvec.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p]
        L.orc_abs_matvec.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p]
        L.orc_residual.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p, c_double_p]
        L.orc_smooth.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int]
        L.orc_smooth_nodes.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p, ctypes.c_double,
                                       ctypes.c_long, c_long_p, c_double_p]
        L.orc_patch_corrections.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, ctypes.c_long,
                                            c_long_p, c_double_p]
        L.orc_restrict.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p]
        L.orc_prolong_add.argtypes = [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p]
        L.orc_coarse_solve.argtypes = [ctypes.c_void_p, c_double_p, c_double_p]
        L.orc_vcycle.argtypes = [ctypes.c_void_p, c_double_p, c_double_p, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int]
        L.orc_solve.argtypes = [ctypes.c_void_p, c_double_p, c_double_p, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int), c_double_p, c_double_p]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(c_double_p)


def _lp(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(c_long_p)


MODE_LU, MODE_INVERSE = 0, 1


class Oracle:
    """One problem hierarchy held by the oracle. `prob` is an inputs.Problem-like object."""

    def __init__(self, prob):
        L = lib()
        self.prob = prob
        self.d = prob.dim
        balls = np.ascontiguousarray(np.asarray(prob.balls, dtype=np.float64).reshape(-1, 4))
        bc = (ctypes.c_int * 6)(*[int(v) for v in prob.bcs])
        h = L.orc_create(prob.dim, prob.n_cells, prob.n_levels, prob.quad_depth, prob.eta, prob.alpha_fict,
                         prob.nitsche_beta, balls.shape[0], _dp(balls) if balls.size else None, bc,
                         prob.ubar, prob.force, int(getattr(prob, "immersed_nitsche", 0)))
        if not h:
            raise ValueError("oracle: invalid problem")
        self.h = ctypes.c_void_p(h)
        self.nlev = prob.n_levels
        self.fine = prob.n_levels - 1

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # sizes --------------------------------------------------------------------------------
    def nnodes(self, level: int) -> int:
        return int(lib().orc_nnodes(self.h, level))

    def ndofs(self, level: int) -> int:
        return (self.d + 1) * self.nnodes(level)

    def coarse_ok(self) -> bool:
        return bool(lib().orc_coarse_ok(self.h))

    def bordered(self) -> bool:
        return bool(lib().orc_bordered(self.h))

    # operator -----------------------------------------------------------------------------
    def coo(self, level: int):
        L = lib()
        nnz = L.orc_coo(self.h, level, None, None, None)
        rows = np.zeros(nnz, np.int64)
        cols = np.zeros(nnz, np.int64)
        vals = np.zeros(nnz, np.float64)
        L.orc_coo(self.h, level, _lp(rows), _lp(cols), _dp(vals))
        return rows, cols, vals

    def matrix(self, level: int):
        import scipy.sparse as sp
        rows, cols, vals = self.coo(level)
        n = self.ndofs(level)
        return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))

    def element_matrix(self, level: int, cell: int) -> np.ndarray:
        ne = (1 << self.d) * (self.d + 1)
        out = np.zeros(ne * ne)
        lib().orc_element_matrix(self.h, level, cell, _dp(out))
        return out.reshape(ne, ne)

    def cell_quadrature(self, level: int, cell: int) -> np.ndarray:
        out = np.zeros(5)
        lib().orc_cell_quadrature(self.h, level, cell, _dp(out))
        return out

    def arc_points(self, level: int, cell: int) -> np.ndarray:
        """Immersed-boundary quadrature points of one cell: rows [x (d), w, n (d)] (2D: circle arcs,
        3D: sphere pieces)."""
        st = 2 * self.d + 1
        cnt = lib().orc_arc_points(self.h, level, cell, None, 0)
        out = np.zeros(max(cnt, 1) * st)
        lib().orc_arc_points(self.h, level, cell, _dp(out), cnt)
        return out[: cnt * st].reshape(cnt, st)

    def cell_kinds(self, level: int) -> np.ndarray:
        n = self.prob.level_cells(level)
        out = np.zeros(n ** self.d, np.int8)
        lib().orc_cell_kinds(self.h, level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_byte)))
        return out

    def rhs(self, level: int | None = None) -> np.ndarray:
        level = self.fine if level is None else level
        b = np.zeros(self.ndofs(level))
        lib().orc_rhs(self.h, level, _dp(b))
        return b

    def matvec(self, level: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        lib().orc_matvec(self.h, level, _dp(x), _dp(y))
        return y

    def abs_matvec(self, level: int, x: np.ndarray) -> np.ndarray:
        """|L| x with the entrywise absolute value of the level operator."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        lib().orc_abs_matvec(self.h, level, _dp(x), _dp(y))
        return y

    def residual(self, level: int, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        r = np.zeros_like(x)
        lib().orc_residual(self.h, level, _dp(x), _dp(b), _dp(r))
        return r

    # patches ------------------------------------------------------------------------------
    def patch_dofs(self, level: int, node: int) -> np.ndarray:
        L = lib()
        m = L.orc_patch_dofs(self.h, level, node, None)
        out = np.zeros(m, np.int64)
        L.orc_patch_dofs(self.h, level, node, _lp(out))
        return out

    def patch_matrix(self, level: int, node: int) -> np.ndarray:
        m = len(self.patch_dofs(level, node))
        out = np.zeros(m * m)
        lib().orc_patch_matrix(self.h, level, node, _dp(out))
        return out.reshape(m, m)

    def inverse_rows(self, level: int, node: int) -> np.ndarray:
        m = len(self.patch_dofs(level, node))
        out = np.zeros((self.d + 1) * m)
        rc = lib().orc_inverse_rows(self.h, level, node, _dp(out))
        if rc < 0:
            raise np.linalg.LinAlgError("singular patch")
        return out.reshape(self.d + 1, m)

    # smoother, transfers, cycle ------------------------------------------------------------
    def smooth(self, level: int, x: np.ndarray, b: np.ndarray, sweeps: int = 1, omega: float = 0.8,
               mode: int = MODE_LU) -> np.ndarray:
        x = np.array(x, dtype=np.float64, copy=True)
        b = np.ascontiguousarray(b, dtype=np.float64)
        rc = lib().orc_smooth(self.h, level, _dp(x), _dp(b), sweeps, omega, mode)
        if rc == -4:
            raise np.linalg.LinAlgError("singular patch")
        return x

    def smooth_nodes(self, level: int, x: np.ndarray, b: np.ndarray, nodes, omega: float = 0.8) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        out = np.zeros(len(nodes) * (self.d + 1))
        rc = lib().orc_smooth_nodes(self.h, level, _dp(x), _dp(b), omega, len(nodes), _lp(nodes), _dp(out))
        if rc == -4:
            raise np.linalg.LinAlgError("singular patch")
        return out.reshape(len(nodes), self.d + 1)

    def patch_corrections(self, level: int, r: np.ndarray, nodes) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        out = np.zeros(len(nodes) * (self.d + 1))
        rc = lib().orc_patch_corrections(self.h, level, _dp(r), len(nodes), _lp(nodes), _dp(out))
        if rc == -4:
            raise np.linalg.LinAlgError("singular patch")
        return out.reshape(len(nodes), self.d + 1)

    def restrict(self, fine_level: int, rf: np.ndarray) -> np.ndarray:
        rf = np.ascontiguousarray(rf, dtype=np.float64)
        bc = np.zeros(self.ndofs(fine_level - 1))
        lib().orc_restrict(self.h, fine_level, _dp(rf), _dp(bc))
        return bc

    def prolong_add(self, fine_level: int, xc: np.ndarray, xf: np.ndarray) -> np.ndarray:
        xc = np.ascontiguousarray(xc, dtype=np.float64)
        xf = np.array(xf, dtype=np.float64, copy=True)
        lib().orc_prolong_add(self.h, fine_level, _dp(xc), _dp(xf))
        return xf

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        if lib().orc_coarse_solve(self.h, _dp(b), _dp(x)) != 0:
            raise np.linalg.LinAlgError("singular coarse operator")
        return x

    def vcycle(self, x: np.ndarray, b: np.ndarray, nu1=None, nu2=None, omega=None, mode=MODE_LU) -> np.ndarray:
        p = self.prob
        x = np.array(x, dtype=np.float64, copy=True)
        b = np.ascontiguousarray(b, dtype=np.float64)
        rc = lib().orc_vcycle(self.h, _dp(x), _dp(b), p.nu_pre if nu1 is None else nu1,
                              p.nu_post if nu2 is None else nu2, p.omega if omega is None else omega, mode)
        if rc != 0:
            raise np.linalg.LinAlgError(f"vcycle failed ({rc})")
        return x

    def solve(self, b: np.ndarray, x0=None, rtol=1e-8, max_iter=100, mode=MODE_INVERSE, nu1=None, nu2=None,
              omega=None):
        p = self.prob
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0)
        hist = np.zeros(max_iter + 1)
        rc = lib().orc_solve(self.h, _dp(x), _dp(b), rtol, max_iter, p.nu_pre if nu1 is None else nu1,
                             p.nu_post if nu2 is None else nu2, p.omega if omega is None else omega, mode,
                             ctypes.byref(it), ctypes.byref(rel), _dp(hist))
        return x, it.value, rel.value, hist[: it.value + 1], rc


def set_threads(n: int) -> None:
    lib().orc_set_threads(n)


def max_threads() -> int:
    return int(lib().orc_max_threads())
