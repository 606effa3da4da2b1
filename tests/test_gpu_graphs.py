"""HIP graphs: the library's calls launch kernels only (no allocation, no
memset, no host synchronisation), so they can be captured on the context's
stream and replayed.  A replay repeats the captured launches with the
captured buffer pointers, so a capture of an even number of steps returns
the context to the buffers it started from, and every replay then advances
the state by that many steps.  Each test replays several times, with the
program's own eager work and synchronisations between replays, and checks
every replay bitwise against the same work done eagerly.  Everything runs
on one stream, so the order is the stream order."""
import pytest
import torch

from paper_1703_04594_amd import inputs, lbm
from paper_1703_04594_amd.lbm import Lattice

from _util import G, TAU, TB, TT, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("lx,ly", [(256, 128), (1024, 1024)])
@pytest.mark.parametrize("step", ["fused", "split"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_captured_steps_replay_like_eager_steps(precision, step, lx, ly):
    say(f"graph of lbm_step {precision} {step} {lx}x{ly}")
    n = 10
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        P = torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=DEV)
        lat = Lattice(lx, ly, TAU, G, TB, TT, precision=precision, step=step, device=DEV)
        ref = Lattice(lx, ly, TAU, G, TB, TT, precision=precision, step=step, device=DEV)
        lat.init_rt(P)
        ref.init_rt(P)
        lat.step(2)
        ref.step(2)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        lat.step(n)
    s.synchronize()
    for k in range(4):
        with torch.cuda.stream(s):
            g.replay()
            ref.step(n)
            a, b = lat.get_pops(), ref.get_pops()
        s.synchronize()
        assert torch.equal(a, b), k
        if k == 1:                       # eager steps on the captured lattice between replays
            with torch.cuda.stream(s):
                lat.step(4)
                ref.step(4)
            s.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_captured_noalloc_totals_replay_like_eager(precision):
    """lbm_conservation_noalloc inside a graph: its fixed scratch array is
    rewritten by every replay; each replay's totals equal lbm_conservation of
    the state copied into the captured input buffer."""
    lx, ly = 300, 211
    say(f"graph of conservation_noalloc {precision}")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        lat = Lattice(lx, ly, TAU, G, TB, TT, precision=precision, step="fused", device=DEV)
        lat.init_rt(torch.tensor(inputs.rt_perturbation(lx, ly, 2), device=DEV))
        lat.step(3)
        pops = lat.get_pops()
        out = torch.zeros(4, dtype=torch.float64, device=DEV)
        lbm.conservation_noalloc(pops, out)    # warm-up: the scratch address is looked up once
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        lbm.conservation_noalloc(pops, out)
    s.synchronize()
    for k in range(4):
        with torch.cuda.stream(s):
            lat.step(2)
            pops.copy_(lat.get_pops())
            want = lat.conservation()
            g.replay()
        s.synchronize()
        assert torch.equal(out, want), k
