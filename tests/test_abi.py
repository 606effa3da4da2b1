"""The C-ABI library loads, exports every symbol of include/lbm.h, agrees
with the oracle on the lattice constants, and validates arguments on the
host (CPU only: no call here reaches the device)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1703_04594_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = lbm.lib()
    names = declared_functions()
    assert len(names) == 48
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_constants_match_the_oracle_bitwise():
    ex, ey = lbm.velocity_table()
    oex, oey = oracle.velocity_table()
    assert ex == oex.tolist() and ey == oey.tolist()
    assert np.array_equal(np.array(lbm.weights()), oracle.weights())
    assert lbm.scale_c() == oracle.scale_c()


def test_host_side_validation():
    L = lbm.lib()
    good = lbm.make_params(64, 48, 0.7)
    n = lbm.workspace_bytes(good)
    assert n > 37 * 2 * 64 * 48 * 8
    for bad in (lbm.make_params(6, 48, 0.7), lbm.make_params(64, 6, 0.7), lbm.make_params(64, 48, 0.5),
                lbm.make_params(64, 48, float("nan")),
                lbm.make_params(1 << 16, (1 << 15) + 1, 0.7)):      # more than 2^31 sites
        assert lbm.workspace_bytes(bad) == 0
    assert lbm.workspace_bytes(lbm.make_params(1 << 16, 1 << 15, 0.7)) > 0      # exactly 2^31 sites
    p = lbm.make_params(64, 48, 0.7)
    p.precision = 7
    assert lbm.workspace_bytes(p) == 0
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(lbm.make_params(64, 48, 0.4)), ctypes.c_void_p(4096), 1 << 30,
                        None, ctypes.byref(h)) == 1
    assert b"invalid" in L.lbm_last_error(None)
    assert L.lbm_create(ctypes.byref(good), ctypes.c_void_p(4096), n - 1, None, ctypes.byref(h)) == 2
    assert L.lbm_create(ctypes.byref(good), ctypes.c_void_p(4096 + 8), n, None, ctypes.byref(h)) == 1
    assert not h.value
    assert L.lbm_step_state(None, None, None) == 1
    # every context call refuses a NULL context before touching the device
    for name, args in (("lbm_step", (1,)), ("lbm_propagate", ()), ("lbm_collide", ()), ("lbm_sync", ()),
                       ("lbm_adjoint_step", (None, None)), ("lbm_adjoint_take_dtau", (None,)),
                       ("lbm_conservation", (None,))):
        assert getattr(L, name)(None, *args) == 1, name
    # FP32 storage about halves the population buffers (on a lattice tall
    # enough for the ghost rows and padding not to dominate); the adjoint adds
    # FP64 lambda
    n64 = lbm.workspace_bytes(lbm.make_params(64, 1000, 0.7))
    n32 = lbm.workspace_bytes(lbm.make_params(64, 1000, 0.7, precision="fp32"))
    assert n32 < 0.6 * n64
    assert lbm.workspace_bytes(lbm.make_params(64, 48, 0.7, adjoint=True)) > n


def test_python_binding_refuses_missing_library(monkeypatch):
    monkeypatch.setattr(lbm, "_lib", None)
    monkeypatch.setattr(lbm, "LIB_PATH", "/nonexistent/liblbm.so")
    with pytest.raises(lbm.LBMError):
        lbm.lib()


def test_reference_copy_library_rejects_bad_arguments():
    """The benchmark's calibration copy (csrc/copy_probe.hip) loads, exports
    cp_copy, and refuses invalid arguments before any HIP call."""
    path = os.path.join(os.path.dirname(lbm.LIB_PATH), "libcopyprobe.so")
    lib = ctypes.CDLL(path)
    f = lib.cp_copy
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    f.restype = ctypes.c_int
    assert f(None, None, 16, 2048, None) == 1                  # null pointers
    assert f(0x1000, 0x100000, 24, 2048, None) == 1            # size not a multiple of 16
    assert f(0x1008, 0x100000, 32, 2048, None) == 1            # misaligned source
    assert f(0x1000, 0x1010, 64, 2048, None) == 1              # overlapping ranges
    assert f(0x1000, 0x100000, 64, 3000, None) == 1            # unsupported workgroup size
    # the fused step's access-pattern copy: sizes, and refusals before any launch
    nb = lib.cp_gather_bytes
    nb.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    nb.restype = ctypes.c_size_t
    assert nb(8, 64, 48) > 37 * 70 * 48 * 8 and nb(4, 64, 48) > 0
    assert nb(2, 64, 48) == 0 and nb(8, 6, 48) == 0 and nb(8, 1 << 16, (1 << 15) + 1) == 0
    g = lib.cp_gather_copy
    g.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    g.restype = ctypes.c_int
    n = nb(8, 64, 48)
    assert g(8, 64, 48, None, 0x100000, None) == 1                 # null source
    assert g(8, 64, 48, 0x1000, 0x1000, None) == 1                 # same buffer
    assert g(8, 64, 48, 0x1000, 0x1000 + n - 256, None) == 1       # overlapping buffers
    assert g(8, 64, 48, 0x1008, 0x1000 + 2 * n, None) == 1         # not 256-byte aligned
    assert g(3, 64, 48, 0x1000, 0x1000 + 2 * n, None) == 1         # element size


def test_layout_study_validates_arguments():
    """Sizes of the four layouts, and every invalid combination refused on
    the host before anything is launched (status 1 or 2, a message)."""
    L = lbm.lib()
    n = 37 * 64 * 96 * 8
    for layout, vl in (("aos", 1), ("soa", 1), ("csoa", 1), ("csoa", 8), ("caosoa", 32)):
        assert lbm.study_bytes(layout, vl, 64, 96) == n
    for layout, vl, lx, ly in (("aos", 2, 64, 96),      # AOS and SOA take vl = 1
                               ("soa", 4, 64, 96),
                               ("csoa", 3, 64, 96),     # not a power of two
                               ("csoa", 128, 64, 1024),  # wider than a wave
                               ("caosoa", 64, 64, 96),  # ly not a multiple of vl
                               ("csoa", 32, 64, 64),    # ly / vl < 3
                               ("csoa", 8, 6, 96),      # lx < 7
                               ("soa", 1, 1 << 14, 1 << 13)):   # more than 2^26 sites
        assert lbm.study_bytes(layout, vl, lx, ly) == 0, (layout, vl, lx, ly)
    assert L.lbm_study_bytes(4, 1, 64, 96) == 0
    fake = ctypes.c_void_p(4096)
    assert L.lbm_study_propagate(1, 1, 64, 96, None, fake, None) == 1
    assert b"NULL" in L.lbm_last_error(None)
    assert L.lbm_study_propagate(1, 1, 64, 96, fake, fake, None) == 1
    assert b"differ" in L.lbm_last_error(None)
    assert L.lbm_study_propagate(0, 2, 64, 96, fake, ctypes.c_void_p(8192), None) == 1
    assert L.lbm_study_collide(2, 8, 64, 96, 0.5, 0.0, fake, None) == 1
    assert L.lbm_study_collide(2, 8, 64, 96, float("nan"), 0.0, fake, None) == 1
    assert L.lbm_study_collide(2, 8, 64, 96, 0.7, float("inf"), fake, None) == 1
    assert L.lbm_study_pack(3, 8, 64, 96, None, fake, None) == 1
    assert L.lbm_study_unpack(7, 8, 64, 96, fake, fake, None) == 1
    # a thin lattice whose propagate would need more than one grid's workgroups
    assert L.lbm_study_propagate(1, 1, (1 << 26) // 7, 7, fake, ctypes.c_void_p(8192), None) == 2
    with pytest.raises(ValueError):
        lbm.study_bytes("aosoa", 1, 64, 96)


def test_conservation_noalloc_validates_on_the_host():
    """The no-allocation totals refuse a lattice beyond LBM_NOALLOC_MAX_SITES
    (status 2), unknown precisions, empty lattices and NULL pointers (status
    1), each with a message, before any HIP call."""
    L = lbm.lib()
    fake = ctypes.c_void_p(4096)
    assert L.lbm_conservation_noalloc(0, 1 << 16, (1 << 15) + 1, fake, fake, None) == 2
    assert b"exceeds" in L.lbm_last_error(None)
    assert L.lbm_conservation_noalloc(7, 8, 8, fake, fake, None) == 1
    assert b"precision" in L.lbm_last_error(None)
    assert L.lbm_conservation_noalloc(1, 0, 8, fake, fake, None) == 1
    assert L.lbm_conservation_noalloc(1, 8, 8, None, fake, None) == 1
    assert L.lbm_conservation_noalloc(1, 8, 8, fake, None, None) == 1
    assert b"NULL" in L.lbm_last_error(None)
