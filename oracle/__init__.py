"""CPU oracle for the D2Q37 thermal lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the product path never does.  It shares
no code with the GPU library (``paper_1703_04594_amd``).

``lbm_ref.c`` is the plain serial FP64 implementation of the paper's step
(arXiv:1703.04594, section 3: eq. (1) BGK update, eq. (2) moments, eq. (4)
pull form; propagate -> bc -> collide order of the heterogeneous control flow,
section 5).  ``ref_torch`` re-states the same step with PyTorch CPU float64
operations so that autograd supplies the exact vector-Jacobian products the
GPU adjoint is compared with.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_ref.c")
LIB_SERIAL = os.path.join(HERE, "liblbm_ref.so")
LIB_OMP = os.path.join(HERE, "liblbm_ref_omp.so")

NPOP = 37
PERIODIC, WALL, OPEN = 1, 0, 2


def build(verbose: bool = False) -> None:
    """Compile the serial and the OpenMP build of the same source."""
    base = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
            "-fPIC", "-shared", "-D_GNU_SOURCE", SRC]
    cmds = [base + ["-o", LIB_SERIAL, "-lquadmath", "-lm"],
            base + ["-fopenmp", "-o", LIB_OMP, "-lquadmath", "-lm"]]
    for c in cmds:
        if verbose:
            print(" ".join(c))
        subprocess.run(c, check=True)


_libs: dict[bool, ctypes.CDLL] = {}


def load(openmp: bool = False) -> ctypes.CDLL:
    path = LIB_OMP if openmp else LIB_SERIAL
    if openmp in _libs:
        return _libs[openmp]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    d, i32, i64, vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.ref_velocity_table.argtypes = [P(i32), P(i32)]
    lib.ref_scale_c.restype = d
    lib.ref_weights.argtypes = [P(d)]
    lib.ref_quadrature_residuals.argtypes = [P(d)]
    lib.ref_feq.argtypes = [d, d, d, d, P(d)]
    lib.ref_create.restype = vp
    lib.ref_create.argtypes = [i32, i32, i32, i32, i32, d, d, d, d]
    lib.ref_destroy.argtypes = [vp]
    for name in ("ref_propagate", "ref_bc", "ref_collide"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = ctypes.c_int
    lib.ref_step.argtypes = [vp, i64]
    lib.ref_init.argtypes = [vp, P(d), P(d), P(d), P(d)]
    lib.ref_set_pops.argtypes = [vp, P(d)]
    lib.ref_get_pops.argtypes = [vp, P(d)]
    lib.ref_get_macros.argtypes = [vp, P(d), P(d), P(d), P(d)]
    lib.ref_conservation.argtypes = [vp, P(d)]
    lib.ref_threads.restype = ctypes.c_int
    _libs[openmp] = lib
    return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def velocity_table() -> tuple[np.ndarray, np.ndarray]:
    lib = load()
    ex = (ctypes.c_int32 * NPOP)()
    ey = (ctypes.c_int32 * NPOP)()
    lib.ref_velocity_table(ex, ey)
    return np.array(ex, dtype=np.int64), np.array(ey, dtype=np.int64)


def scale_c() -> float:
    return float(load().ref_scale_c())


def weights() -> np.ndarray:
    w = np.zeros(NPOP)
    load().ref_weights(_dp(w))
    return w


def quadrature_residuals() -> np.ndarray:
    r = np.zeros(9)
    load().ref_quadrature_residuals(_dp(r))
    return r


def feq(rho: float, ux: float, uy: float, T: float) -> np.ndarray:
    out = np.zeros(NPOP)
    load().ref_feq(rho, ux, uy, T, _dp(out))
    return out


class RefLattice:
    """ctypes handle on one oracle lattice (canonical [37][lx][ly] FP64)."""

    def __init__(self, lx: int, ly: int, tau: float, g_y: float = 0.0,
                 t_bottom: float = 1.0, t_top: float = 1.0,
                 xbc: int = PERIODIC, ybc: int | tuple[int, int] = WALL,
                 openmp: bool = False):
        self.lib = load(openmp)
        yb, yt = (ybc, ybc) if isinstance(ybc, int) else ybc
        h = self.lib.ref_create(lx, ly, xbc, yb, yt, tau, g_y, t_bottom, t_top)
        if not h:
            raise ValueError("ref_create rejected the parameters")
        self.h = ctypes.c_void_p(h)
        self.lx, self.ly = lx, ly

    def close(self):
        if self.h:
            self.lib.ref_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(np.broadcast_to(a, (self.lx, self.ly)), dtype=np.float64)
                for a in (rho, ux, uy, T)]
        self.lib.ref_init(self.h, *[_dp(a) for a in arrs])

    def set_pops(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (NPOP, self.lx, self.ly)
        self.lib.ref_set_pops(self.h, _dp(f))

    def get_pops(self) -> np.ndarray:
        f = np.empty((NPOP, self.lx, self.ly))
        self.lib.ref_get_pops(self.h, _dp(f))
        return f

    def propagate(self):
        assert self.lib.ref_propagate(self.h) == 0

    def bc(self):
        assert self.lib.ref_bc(self.h) == 0

    def collide(self):
        assert self.lib.ref_collide(self.h) == 0

    def step(self, n: int = 1):
        self.lib.ref_step(self.h, n)

    def macros(self):
        out = [np.empty((self.lx, self.ly)) for _ in range(4)]
        self.lib.ref_get_macros(self.h, *[_dp(a) for a in out])
        return tuple(out)

    def conservation(self) -> np.ndarray:
        out = np.zeros(4)
        self.lib.ref_conservation(self.h, _dp(out))
        return out


def threads(openmp: bool = False) -> int:
    return int(load(openmp).ref_threads())
