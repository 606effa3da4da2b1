"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Device memory and streams come from PyTorch: the workspace is a uint8 CUDA
tensor, every array argument is a contiguous CUDA tensor of the documented
dtype and shape, and all work is enqueued on the stream that was current when
the Lattice was created.  Every computation runs in the library's kernels;
if the library is missing this module raises instead of computing anything.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

NPOP = 37
FP64, FP32_SHIFTED, FP32_SHIFTED_F32SUMS = 0, 1, 2
Y_WALLS, Y_PERIODIC = 0, 1
X_WRAP, X_HALO = 0, 1
STEP_SPLIT, STEP_FUSED = 0, 1
LAYOUT_PLANES, LAYOUT_COLUMNS = 0, 1

# "fp32": FP32 deviations collided with FP64 moment sums; "fp32_f32sums":
# the same with the sums in FP32 too
_PREC = {"fp64": FP64, "fp32": FP32_SHIFTED, "fp32_shifted": FP32_SHIFTED, "fp32_f32sums": FP32_SHIFTED_F32SUMS}
_YBC = {"walls": Y_WALLS, "periodic": Y_PERIODIC}
_XMODE = {"wrap": X_WRAP, "halo": X_HALO}
_STEP = {"split": STEP_SPLIT, "fused": STEP_FUSED}
_LAYOUT = {"planes": LAYOUT_PLANES, "columns": LAYOUT_COLUMNS}


class LBMError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ybc", ctypes.c_int32), ("xmode", ctypes.c_int32), ("step_kind", ctypes.c_int32),
                ("adjoint", ctypes.c_int32), ("layout", ctypes.c_int32), ("tau", ctypes.c_double),
                ("g_y", ctypes.c_double), ("t_bottom", ctypes.c_double), ("t_top", ctypes.c_double)]


class RtProfileC(ctypes.Structure):
    _fields_ = [("t_mid", ctypes.c_double), ("t_amp", ctypes.c_double), ("p0", ctypes.c_double),
                ("width", ctypes.c_double), ("y_mid", ctypes.c_double)]


@dataclass
class RtProfile:
    """T0 = t_mid - t_amp tanh((y - y_mid - P) / width), rho0 = p0 / T0."""
    t_mid: float = 1.0
    t_amp: float = 1.0 / 3.0
    p0: float = 8.0 / 9.0
    width: float = 2.0
    y_mid: float | None = None   # default (ly - 1) / 2

    def c(self, ly: int) -> RtProfileC:
        ym = (ly - 1) / 2.0 if self.y_mid is None else self.y_mid
        return RtProfileC(self.t_mid, self.t_amp, self.p0, self.width, ym)


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LBMError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                       "(the library has no CPU fallback)")
    # torch first, so that liblbm binds to the HIP runtime torch already loaded
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, d, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    PP = ctypes.POINTER(Params)
    L.lbm_workspace_bytes.argtypes = [PP]
    L.lbm_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_state_bytes.argtypes = [PP]
    L.lbm_state_bytes.restype = ctypes.c_size_t
    L.lbm_create.argtypes = [PP, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_set_tau.argtypes = [vp, d]
    L.lbm_init.argtypes = [vp, vp, vp, vp, vp]
    L.lbm_init_rt.argtypes = [vp, vp, ctypes.POINTER(RtProfileC)]
    for n in ("lbm_propagate", "lbm_bc", "lbm_collide", "lbm_sync"):
        getattr(L, n).argtypes = [vp]
    L.lbm_step.argtypes = [vp, i64]
    L.lbm_get_macros.argtypes = [vp, vp, vp, vp, vp]
    for n in ("lbm_get_pops", "lbm_set_pops", "lbm_get_state", "lbm_set_state", "lbm_conservation",
              "lbm_adjoint_seed_temperature", "lbm_adjoint_get_lambda", "lbm_adjoint_set_lambda",
              "lbm_adjoint_take_dtau"):
        getattr(L, n).argtypes = [vp, vp]
    L.lbm_loss_temperature.argtypes = [vp, vp, vp]
    L.lbm_adjoint_step.argtypes = [vp, vp, vp]
    L.lbm_step_state.argtypes = [vp, vp, vp]
    L.lbm_adjoint_init_rt.argtypes = [vp, vp, ctypes.POINTER(RtProfileC), vp]
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_velocity_table.argtypes = [ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(ctypes.c_int8)]
    L.lbm_velocity_table.restype = None
    L.lbm_weights.argtypes = [ctypes.POINTER(ctypes.c_double)]
    L.lbm_weights.restype = None
    L.lbm_scale_c.restype = ctypes.c_double
    ci = ctypes.c_int
    L.lbm_host_lattice_bytes.argtypes = [PP]
    L.lbm_host_lattice_bytes.restype = ctypes.c_size_t
    L.lbm_host_pack.argtypes = [PP, vp, vp]
    L.lbm_host_unpack.argtypes = [PP, vp, vp]
    L.lbm_host_step.argtypes = [PP, vp, vp, i64, ci]
    L.lbm_hetero_workspace_bytes.argtypes = [PP, ci]
    L.lbm_hetero_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_hetero_create.argtypes = [PP, ci, ci, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbm_hetero_destroy.argtypes = [vp]
    L.lbm_hetero_destroy.restype = None
    L.lbm_hetero_set_pops.argtypes = [vp, vp]
    L.lbm_hetero_get_pops.argtypes = [vp, vp]
    L.lbm_hetero_step.argtypes = [vp, i64]
    L.lbm_hetero_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.lbm_hetero_last_error.argtypes = [vp]
    L.lbm_hetero_last_error.restype = ctypes.c_char_p
    for n in ("lbm_host_pack", "lbm_host_unpack", "lbm_host_step", "lbm_hetero_create", "lbm_hetero_set_pops",
              "lbm_hetero_get_pops", "lbm_hetero_step", "lbm_hetero_times"):
        getattr(L, n).restype = st
    L.lbm_conservation_noalloc.argtypes = [ci, ci, ci, vp, vp, vp]
    L.lbm_conservation_noalloc.restype = st
    L.lbm_study_bytes.argtypes = [ci, ci, ci, ci]
    L.lbm_study_bytes.restype = ctypes.c_size_t
    for n in ("lbm_study_pack", "lbm_study_unpack", "lbm_study_propagate"):
        getattr(L, n).argtypes = [ci, ci, ci, ci, vp, vp, vp]
        getattr(L, n).restype = st
    L.lbm_study_collide.argtypes = [ci, ci, ci, ci, d, d, vp, vp]
    L.lbm_study_collide.restype = st
    for n in ("lbm_create", "lbm_set_tau", "lbm_init", "lbm_init_rt", "lbm_propagate", "lbm_bc",
              "lbm_collide", "lbm_step", "lbm_get_macros", "lbm_get_pops", "lbm_set_pops",
              "lbm_get_state", "lbm_set_state", "lbm_step_state", "lbm_conservation", "lbm_loss_temperature",
              "lbm_adjoint_seed_temperature", "lbm_adjoint_step", "lbm_adjoint_take_dtau", "lbm_adjoint_init_rt",
              "lbm_adjoint_get_lambda", "lbm_adjoint_set_lambda", "lbm_sync"):
        getattr(L, n).restype = st
    _lib = L
    return L


def velocity_table():
    ex = (ctypes.c_int8 * NPOP)()
    ey = (ctypes.c_int8 * NPOP)()
    lib().lbm_velocity_table(ex, ey)
    return list(ex), list(ey)


def weights():
    w = (ctypes.c_double * NPOP)()
    lib().lbm_weights(w)
    return list(w)


def scale_c() -> float:
    return float(lib().lbm_scale_c())


_ADJ = {False: 0, None: 0, 0: 0, True: 1, 1: 1, "fp64": 1, 2: 2, "fp32": 2}


def make_params(lx, ly, tau, g_y=0.0, t_bottom=1.0, t_top=1.0, precision="fp64", ybc="walls",
                xmode="wrap", step="split", adjoint=False, layout="columns") -> Params:
    """adjoint: False (none), True / "fp64" (FP64 lambda) or "fp32" (FP32 lambda storage)."""
    return Params(lx, ly, _PREC[precision], _YBC[ybc], _XMODE[xmode], _STEP[step], _ADJ[adjoint],
                  _LAYOUT[layout], tau, g_y, t_bottom, t_top)


def workspace_bytes(p: Params) -> int:
    return int(lib().lbm_workspace_bytes(ctypes.byref(p)))


def _ptr(t: torch.Tensor, dtype, shape, device) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or t.device != device:
        raise ValueError(f"expected contiguous {dtype} {tuple(shape)} on {device}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")
    return t.data_ptr()


class Lattice:
    """One D2Q37 lattice on one GPU (a context of liblbm.so)."""

    def __init__(self, lx, ly, tau, g_y=0.0, t_bottom=1.0, t_top=1.0, precision="fp64",
                 ybc="walls", xmode="wrap", step="split", adjoint=False, layout="columns", device="cuda"):
        self.L = lib()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.p = make_params(lx, ly, tau, g_y, t_bottom, t_top, precision, ybc, xmode, step, adjoint, layout)
        self.lx, self.ly = lx, ly
        self.precision = precision
        self.store_dtype = torch.float64 if _PREC[precision] == FP64 else torch.float32
        nbytes = workspace_bytes(self.p)
        if nbytes == 0:
            raise LBMError("invalid lattice parameters")
        self.state_bytes = int(self.L.lbm_state_bytes(ctypes.byref(self.p)))
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            h = ctypes.c_void_p()
            st = self.L.lbm_create(ctypes.byref(self.p), ctypes.c_void_p(self._ws_ptr), nbytes,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise LBMError(f"lbm_create: {self.L.lbm_last_error(None).decode()} (status {st})")
        self.h = h

    # ------------------------------------------------------------------
    def _check(self, st: int, what: str):
        if st != 0:
            raise LBMError(f"{what}: {self.L.lbm_last_error(self.h).decode()} (status {st})")

    def _run(self, what: str, fn, *args):
        """fn(context, *args) with the lattice's device current (the C ABI's
        convention), then the status check."""
        if torch.cuda.current_device() == self.device.index:
            st = fn(self.h, *args)
        else:
            with torch.cuda.device(self.device):
                st = fn(self.h, *args)
        self._check(st, what)

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field(self, t):
        return ctypes.c_void_p(_ptr(t, torch.float64, (self.lx, self.ly), self.device))

    def _new_field(self):
        return torch.empty((self.lx, self.ly), dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------------
    def set_tau(self, tau: float):
        self._run("set_tau", self.L.lbm_set_tau, tau)

    def init(self, rho, ux, uy, T):
        self._run("init", self.L.lbm_init, self._field(rho), self._field(ux), self._field(uy), self._field(T))

    def init_rt(self, P, profile: RtProfile | None = None):
        prof = (profile or RtProfile()).c(self.ly)
        self._run("init_rt", self.L.lbm_init_rt, self._field(P), ctypes.byref(prof))

    def propagate(self):
        self._run("propagate", self.L.lbm_propagate)

    def bc(self):
        self._run("bc", self.L.lbm_bc)

    def collide(self):
        self._run("collide", self.L.lbm_collide)

    def step(self, n: int = 1):
        self._run("step", self.L.lbm_step, int(n))

    def macros(self):
        out = [self._new_field() for _ in range(4)]
        self._run("get_macros", self.L.lbm_get_macros, *[ctypes.c_void_p(t.data_ptr()) for t in out])
        return tuple(out)

    def get_pops(self) -> torch.Tensor:
        """Canonical (37, lx, ly) populations: float64 f for "fp64", float32
        deviations f - w for the FP32 forms (set_pops takes the same)."""
        out = torch.empty((NPOP, self.lx, self.ly), dtype=self.store_dtype, device=self.device)
        self._run("get_pops", self.L.lbm_get_pops, ctypes.c_void_p(out.data_ptr()))
        return out

    def set_pops(self, f: torch.Tensor):
        p = _ptr(f, self.store_dtype, (NPOP, self.lx, self.ly), self.device)
        self._run("set_pops", self.L.lbm_set_pops, ctypes.c_void_p(p))

    def new_state(self) -> torch.Tensor:
        return torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)

    def get_state(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.new_state() if out is None else out
        p = _ptr(out, torch.uint8, (self.state_bytes,), self.device)
        self._run("get_state", self.L.lbm_get_state, ctypes.c_void_p(p))
        return out

    def set_state(self, s: torch.Tensor):
        p = _ptr(s, torch.uint8, (self.state_bytes,), self.device)
        self._run("set_state", self.L.lbm_set_state, ctypes.c_void_p(p))

    def step_state(self, src: torch.Tensor, dst: torch.Tensor):
        """dst <- one step from the snapshot src (lbm_step_state); the
        lattice's own state is untouched."""
        ps = _ptr(src, torch.uint8, (self.state_bytes,), self.device)
        pd = _ptr(dst, torch.uint8, (self.state_bytes,), self.device)
        self._run("step_state", self.L.lbm_step_state, ctypes.c_void_p(ps), ctypes.c_void_p(pd))

    def conservation(self) -> torch.Tensor:
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        self._run("conservation", self.L.lbm_conservation, ctypes.c_void_p(out.data_ptr()))
        return out

    # -- adjoint ----------------------------------------------------------
    def loss_temperature(self, T_target) -> torch.Tensor:
        out = torch.empty((), dtype=torch.float64, device=self.device)
        self._run("loss_temperature", self.L.lbm_loss_temperature, self._field(T_target),
                  ctypes.c_void_p(out.data_ptr()))
        return out

    def seed_temperature(self, dT):
        self._run("seed_temperature", self.L.lbm_adjoint_seed_temperature, self._field(dT))

    def adjoint_step(self, state: torch.Tensor, dtau_acc: torch.Tensor | None):
        """One reverse step from the snapshot f_n.  Its d/dtau term is added
        to dtau_acc (a float64 scalar tensor), or, with None, kept in the
        context until take_dtau."""
        p = _ptr(state, torch.uint8, (self.state_bytes,), self.device)
        a = None if dtau_acc is None else _ptr(dtau_acc, torch.float64, (), self.device)
        self._run("adjoint_step", self.L.lbm_adjoint_step, ctypes.c_void_p(p), ctypes.c_void_p(a))

    def take_dtau(self, dtau_acc: torch.Tensor):
        """dtau_acc += the d/dtau terms kept by adjoint_step(..., None) calls."""
        a = _ptr(dtau_acc, torch.float64, (), self.device)
        self._run("take_dtau", self.L.lbm_adjoint_take_dtau, ctypes.c_void_p(a))

    def adjoint_init_rt(self, P, profile: RtProfile | None = None) -> torch.Tensor:
        prof = (profile or RtProfile()).c(self.ly)
        out = self._new_field()
        self._run("adjoint_init_rt", self.L.lbm_adjoint_init_rt, self._field(P), ctypes.byref(prof),
                  ctypes.c_void_p(out.data_ptr()))
        return out

    def get_lambda(self) -> torch.Tensor:
        out = torch.empty((NPOP, self.lx, self.ly), dtype=torch.float64, device=self.device)
        self._run("get_lambda", self.L.lbm_adjoint_get_lambda, ctypes.c_void_p(out.data_ptr()))
        return out

    def set_lambda(self, lam: torch.Tensor):
        p = _ptr(lam, torch.float64, (NPOP, self.lx, self.ly), self.device)
        self._run("set_lambda", self.L.lbm_adjoint_set_lambda, ctypes.c_void_p(p))

    def sync(self):
        self._run("sync", self.L.lbm_sync)


def conservation_noalloc(pops: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Lattice totals {sum rho, sum j_x, sum j_y, sum E} of a canonical
    population tensor (37, lx, ly): float64 populations, or float32
    deviations f - w (lbm_conservation_noalloc: the library allocates
    nothing; `out`, a float64 (4,) tensor on the same device, may be given
    so that this call allocates nothing either).  Runs on the tensor's device
    and current stream."""
    if pops.dtype == torch.float64:
        prec = FP64
    elif pops.dtype == torch.float32:
        prec = FP32_SHIFTED
    else:
        raise ValueError("pops must be float64 or float32 (deviation form)")
    if pops.dim() != 3 or pops.shape[0] != NPOP:
        raise ValueError(f"expected a ({NPOP}, lx, ly) tensor, got {tuple(pops.shape)}")
    _, lx, ly = pops.shape
    _ptr(pops, pops.dtype, (NPOP, lx, ly), pops.device)
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=pops.device)
    _ptr(out, torch.float64, (4,), pops.device)
    with torch.cuda.device(pops.device):
        st = lib().lbm_conservation_noalloc(prec, int(lx), int(ly), ctypes.c_void_p(pops.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), _stream(pops))
    if st != 0:
        raise LBMError(f"conservation_noalloc: {lib().lbm_last_error(None).decode()} (status {st})")
    return out


# ---------------------------------------------------------------------------
# Layout study (section 4, Table 2): stateless propagate / collide on FP64
# buffers in one of the paper's four layouts, periodic in x and y.
# ---------------------------------------------------------------------------
STUDY_LAYOUTS = {"aos": 0, "soa": 1, "csoa": 2, "caosoa": 3}


def _study_args(layout: str, vl: int, lx: int, ly: int):
    if layout not in STUDY_LAYOUTS:
        raise ValueError(f"unknown study layout {layout!r}")
    return STUDY_LAYOUTS[layout], int(vl), int(lx), int(ly)


def _study_check(st: int, what: str):
    if st != 0:
        raise LBMError(f"{what}: {lib().lbm_last_error(None).decode()} (status {st})")


def study_bytes(layout: str, vl: int, lx: int, ly: int) -> int:
    """Bytes of one population buffer; 0 for an invalid combination."""
    return int(lib().lbm_study_bytes(*_study_args(layout, vl, lx, ly)))


def _stream(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def study_pack(layout: str, vl: int, canon: torch.Tensor) -> torch.Tensor:
    """canonical FP64 (37, lx, ly) -> new flat FP64 buffer in the layout."""
    _, lx, ly = canon.shape
    a = _study_args(layout, vl, lx, ly)
    _ptr(canon, torch.float64, (NPOP, lx, ly), canon.device)
    buf = torch.empty(NPOP * lx * ly, dtype=torch.float64, device=canon.device)
    _study_check(lib().lbm_study_pack(*a, ctypes.c_void_p(canon.data_ptr()), ctypes.c_void_p(buf.data_ptr()),
                                      _stream(canon)), "study_pack")
    return buf


def study_unpack(layout: str, vl: int, lx: int, ly: int, buf: torch.Tensor) -> torch.Tensor:
    """flat FP64 buffer in the layout -> new canonical FP64 (37, lx, ly)."""
    a = _study_args(layout, vl, lx, ly)
    _ptr(buf, torch.float64, (NPOP * lx * ly,), buf.device)
    out = torch.empty((NPOP, lx, ly), dtype=torch.float64, device=buf.device)
    _study_check(lib().lbm_study_unpack(*a, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        _stream(buf)), "study_unpack")
    return out


def study_propagate(layout: str, vl: int, lx: int, ly: int, src: torch.Tensor, dst: torch.Tensor):
    a = _study_args(layout, vl, lx, ly)
    _ptr(src, torch.float64, (NPOP * lx * ly,), src.device)
    _ptr(dst, torch.float64, (NPOP * lx * ly,), src.device)
    _study_check(lib().lbm_study_propagate(*a, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                           _stream(src)), "study_propagate")


def study_collide(layout: str, vl: int, lx: int, ly: int, tau: float, g_y: float, buf: torch.Tensor):
    a = _study_args(layout, vl, lx, ly)
    _ptr(buf, torch.float64, (NPOP * lx * ly,), buf.device)
    _study_check(lib().lbm_study_collide(*a, float(tau), float(g_y), ctypes.c_void_p(buf.data_ptr()),
                                         _stream(buf)), "study_collide")


# ---------------------------------------------------------------------------
# Host cores, and host + GPU co-execution (sections 5 and 6).  FP64 only.
# ---------------------------------------------------------------------------
import numpy as _np  # noqa: E402


def _host_canon(a, lx, ly) -> _np.ndarray:
    a = _np.ascontiguousarray(a, dtype=_np.float64)
    if a.shape != (NPOP, lx, ly):
        raise ValueError(f"expected a ({NPOP}, {lx}, {ly}) array, got {a.shape}")
    return a


def _dp(a: _np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _aligned_zeros(n: int, align: int = 64) -> _np.ndarray:
    """n float64 zeros starting on an `align`-byte boundary (whole cache
    lines per block of 8 rows, so the host step can stream its stores)."""
    raw = _np.zeros(n + align // 8)
    off = (-raw.ctypes.data % align) // 8
    return raw[off:off + n]


class HostLattice:
    """A whole x-periodic lattice stepped on host cores (the host part's
    kernel), in host memory."""

    def __init__(self, lx, ly, tau, g_y=0.0, t_bottom=1.0, t_top=1.0, ybc="walls", threads=1):
        self.L = lib()
        self.p = make_params(lx, ly, tau, g_y, t_bottom, t_top, "fp64", ybc)
        n = int(self.L.lbm_host_lattice_bytes(ctypes.byref(self.p)))
        if n == 0:
            raise LBMError("invalid lattice parameters")
        self.lx, self.ly, self.threads = lx, ly, int(threads)
        self.buf = [_aligned_zeros(n // 8), _aligned_zeros(n // 8)]
        self.cur = 0

    def _check(self, st, what):
        if st != 0:
            raise LBMError(f"{what}: {self.L.lbm_last_error(None).decode()} (status {st})")

    def set_pops(self, canon):
        c = _host_canon(canon, self.lx, self.ly)
        self._check(self.L.lbm_host_pack(ctypes.byref(self.p), _dp(c), _dp(self.buf[self.cur])), "host_pack")

    def get_pops(self) -> _np.ndarray:
        out = _np.empty((NPOP, self.lx, self.ly))
        self._check(self.L.lbm_host_unpack(ctypes.byref(self.p), _dp(self.buf[self.cur]), _dp(out)), "host_unpack")
        return out

    def step(self, n: int = 1):
        a, b = self.buf[self.cur], self.buf[1 - self.cur]
        self._check(self.L.lbm_host_step(ctypes.byref(self.p), _dp(a), _dp(b), int(n), self.threads), "host_step")
        if n % 2:
            self.cur = 1 - self.cur


class Hetero:
    """A lattice split between host cores (m border columns on each side)
    and the GPU (the rest), halos swapped every step."""

    def __init__(self, lx, ly, tau, g_y=0.0, t_bottom=1.0, t_top=1.0, ybc="walls", m=0, host_threads=1,
                 device="cuda"):
        self.L = lib()
        self.p = make_params(lx, ly, tau, g_y, t_bottom, t_top, "fp64", ybc)
        self.lx, self.ly, self.m = lx, ly, int(m)
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        nbytes = int(self.L.lbm_hetero_workspace_bytes(ctypes.byref(self.p), self.m))
        if nbytes == 0:
            raise LBMError("invalid lattice parameters or split")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            ws = (self.workspace.data_ptr() + 255) // 256 * 256
            h = ctypes.c_void_p()
            st = self.L.lbm_hetero_create(ctypes.byref(self.p), self.m, int(host_threads), ctypes.c_void_p(ws),
                                          nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise LBMError(f"lbm_hetero_create: {self.L.lbm_hetero_last_error(None).decode()} (status {st})")
        self.h = h

    def _check(self, st, what):
        if st != 0:
            raise LBMError(f"{what}: {self.L.lbm_hetero_last_error(self.h).decode()} (status {st})")

    def _run(self, what: str, fn, *args):
        with torch.cuda.device(self.device):
            st = fn(self.h, *args)
        self._check(st, what)

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_hetero_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_pops(self, canon):
        c = _host_canon(canon, self.lx, self.ly)
        self._run("hetero_set_pops", self.L.lbm_hetero_set_pops, _dp(c))

    def get_pops(self) -> _np.ndarray:
        out = _np.empty((NPOP, self.lx, self.ly))
        self._run("hetero_get_pops", self.L.lbm_hetero_get_pops, _dp(out))
        return out

    def step(self, n: int = 1):
        self._run("hetero_step", self.L.lbm_hetero_step, int(n))

    def times(self) -> dict:
        """Per-step averages of the last step() call, seconds."""
        t = (ctypes.c_double * 4)()
        self._run("hetero_times", self.L.lbm_hetero_times, t)
        return {"wall": t[0], "host": t[1], "gpu": t[2], "swap": t[3]}
