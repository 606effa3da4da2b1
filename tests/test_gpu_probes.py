"""The benchmark's access-pattern probes (csrc/copy_probe.hip) move exactly
the data they claim to: `cp_gather_copy` is a propagate evaluated per site
(bitwise the library's `lbm_propagate` on the same padded buffer), and
`cp_adjoint_pattern` stores lambda_l(x + e) + f_l(x - e) at every site.
Their times are the ceilings the bench quotes the fused and reverse steps
against, so they must perform the same loads and stores."""
import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1703_04594_amd import inputs, lbm
from paper_1703_04594_amd.lbm import Lattice

from _util import TB, TT, TAU, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def probe_lib():
    L = ctypes.CDLL(os.path.join(os.path.dirname(lbm.LIB_PATH), "libcopyprobe.so"))
    ci, vp = ctypes.c_int, ctypes.c_void_p
    L.cp_gather_bytes.argtypes = [ci, ci, ci]
    L.cp_gather_bytes.restype = ctypes.c_size_t
    L.cp_gather_copy.argtypes = [ci, ci, ci, vp, vp, vp]
    L.cp_gather_copy.restype = ci
    L.cp_adjoint_pattern.argtypes = [ci, ci, ci, vp, vp, vp, vp]
    L.cp_adjoint_pattern.restype = ci
    return L


def aligned_copy(t, n):
    """A 256-byte aligned device buffer (uint8 view) holding the first n bytes of t."""
    raw = torch.empty(n + 256, dtype=torch.uint8, device=DEV)
    off = (-raw.data_ptr()) % 256
    buf = raw[off:off + n]
    buf.copy_(t[:n])
    return raw, buf


@pytest.mark.parametrize("precision,lx,ly", [(p, lx, ly) for p in ("fp64", "fp32") for lx, ly in ((37, 45), (300, 1030))]
                         + [("fp64", 2048, 4096)])
def test_gather_copy_is_the_library_propagate(precision, lx, ly):
    """2048x4096 FP64 takes the probe's 512-thread, one-block-per-CU launch
    (the fused step's on the largest lattices)."""
    say(f"cp_gather_copy {precision} {lx}x{ly}")
    P = probe_lib()
    elem = 8 if precision == "fp64" else 4
    lat = Lattice(lx, ly, TAU, -1e-4, TB, TT, precision=precision, step="split", device=DEV)
    lat.init_rt(torch.tensor(inputs.rt_perturbation(lx, ly, 3), device=DEV))
    lat.step(3)
    n = P.cp_gather_bytes(elem, lx, ly)
    assert 0 < n <= lat.state_bytes
    src_raw, src = aligned_copy(lat.get_state(), n)
    dst_raw, dst = aligned_copy(torch.zeros(n, dtype=torch.uint8, device=DEV), n)
    assert P.cp_gather_copy(elem, lx, ly, src.data_ptr(), dst.data_ptr(), None) == 0
    torch.cuda.synchronize()
    lat.propagate()
    want = lat.get_pops()
    st = lat.new_state()
    st[:n].copy_(dst)
    lat.set_state(st)
    assert torch.equal(lat.get_pops(), want)


def test_adjoint_pattern_stores_the_sum_of_its_two_gathers():
    lx, ly = 40, 70
    say("cp_adjoint_pattern fp32")
    P = probe_lib()
    ex, ey = (np.asarray(v) for v in oracle.velocity_table())
    f = (0.01 * inputs.population_noise(lx, ly, 91)).astype(np.float32)
    lam = inputs.population_noise(lx, ly, 92).astype(np.float32)
    lat = Lattice(lx, ly, TAU, precision="fp32", ybc="periodic", device=DEV)
    n = P.cp_gather_bytes(4, lx, ly)
    assert 0 < n <= lat.state_bytes
    lat.set_pops(torch.tensor(f, device=DEV))
    f_raw, fb = aligned_copy(lat.get_state(), n)
    lat.set_pops(torch.tensor(lam, device=DEV))
    l_raw, lb = aligned_copy(lat.get_state(), n)
    m_raw, mb = aligned_copy(torch.zeros(n, dtype=torch.uint8, device=DEV), n)
    assert P.cp_adjoint_pattern(4, lx, ly, fb.data_ptr(), lb.data_ptr(), mb.data_ptr(), None) == 0
    torch.cuda.synchronize()
    st = lat.new_state()
    st[:n].copy_(mb)
    lat.set_state(st)
    mu = lat.get_pops().cpu().numpy()
    # rows whose y +- e_y stays inside the lattice (the probe reads ghost rows
    # beyond it, which it does not fill)
    x = np.arange(lx)[None, :, None]
    y = np.arange(3, ly - 3)[None, None, :]
    l = np.arange(37)[:, None, None]
    want = lam[l, (x + ex[:, None, None]) % lx, y + ey[:, None, None]] + \
        f[l, (x - ex[:, None, None]) % lx, y - ey[:, None, None]]
    assert np.array_equal(mu[:, :, 3:ly - 3], want.astype(np.float32))
