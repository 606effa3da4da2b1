"""The co-execution performance model of section 6 (host logic, CPU only):
closed forms of the balance point and of T_exe, and the choice of m."""
import pytest

from paper_1703_04594_amd.hetero import Model


def test_balance_point_closed_form():
    m = Model(tau_d=1e-10, tau_h=3e-10, t_swap=0.0)
    # (lx - 2m) tau_d = 2m tau_h  =>  2m = lx tau_d / (tau_d + tau_h)
    assert m.m_balance(2048) == pytest.approx(2048 * 1e-10 / 4e-10 / 2)
    mb = Model(tau_d=2e-10, tau_h=2e-10, t_swap=0.0).m_balance(1000)
    assert mb == pytest.approx(250.0)
    # at the balance point both sides take the same time
    lx, ly = 1000, 64
    mod = Model(tau_d=2e-10, tau_h=2e-10, t_swap=0.0)
    assert (lx - 2 * 250) * ly * mod.tau_d == pytest.approx(2 * 250 * ly * mod.tau_h)
    assert mod.t_exe(lx, ly, 250) == pytest.approx(lx * ly * 2e-10 / 2)


def test_t_exe_terms():
    mod = Model(tau_d=1e-10, tau_h=1e-8, t_swap=5e-5)
    lx, ly = 2048, 4096
    assert mod.t_exe(lx, ly, 0) == pytest.approx(lx * ly * 1e-10)          # no split, no swap
    assert mod.t_exe(lx, ly, 4) == pytest.approx((lx - 8) * ly * 1e-10 + 5e-5)   # GPU-bound side
    assert mod.t_exe(lx, ly, 500) == pytest.approx(1000 * ly * 1e-8 + 5e-5)      # host-bound side
    assert mod.mlups(lx, ly, 0) == pytest.approx(lx * ly / mod.t_exe(lx, ly, 0) / 1e6)


def test_best_m():
    lx, ly = 2048, 4096
    # a host as fast as the GPU and a free swap: split in half
    assert Model(1e-10, 1e-10, 0.0).best_m(lx, ly) == 512
    # a slow host: the gain from its few columns is below the swap cost
    assert Model(1e-10, 1e-8, 1e-4).best_m(lx, ly) == 0
    # a slow host but a free swap: the balance point (lx tau_d / 2 (tau_d + tau_h) ~ 10)
    mod = Model(1e-10, 1e-8, 0.0)
    best = mod.best_m(lx, ly)
    assert best in (10, 11)
    assert mod.t_exe(lx, ly, best) < mod.t_exe(lx, ly, 0)
    # best_m is never beaten by any admissible m
    for mod in (Model(1e-10, 3e-9, 2e-5), Model(1e-10, 5e-10, 1e-4), Model(1e-10, 1e-10, 3e-4)):
        b = mod.best_m(lx, ly)
        others = [0] + list(range(2, (lx - 3) // 2 + 1))
        assert mod.t_exe(lx, ly, b) <= min(mod.t_exe(lx, ly, m) for m in others) * (1 + 1e-12)


def test_measured_host_times():
    """T_host(m) from host-only runs: exact at the measured widths, linear
    between them, the nearest width's per-site rate beyond them; best_m
    then searches every admissible m, and no admissible m beats it."""
    lx, ly = 2048, 4096
    ht = {2: 0.15e-3, 8: 0.32e-3, 32: 0.83e-3, 128: 3.38e-3}
    mod = Model(tau_d=1.04e-10, tau_h=3.0e-9, t_swap=0.13e-3, host_times=ht)
    for m, t in ht.items():
        assert mod.t_host(ly, m) == pytest.approx(t)
    assert mod.t_host(ly, 20) == pytest.approx(0.32e-3 + (0.83e-3 - 0.32e-3) * 12 / 24)
    assert mod.t_host(ly, 256) == pytest.approx(3.38e-3 * 2)
    assert mod.t_exe(lx, ly, 32) == pytest.approx(max((lx - 64) * ly * 1.04e-10, 0.83e-3) + 0.13e-3)
    b = mod.best_m(lx, ly)
    others = [0] + list(range(2, (lx - 3) // 2 + 1))
    assert mod.t_exe(lx, ly, b) <= min(mod.t_exe(lx, ly, m) for m in others)
    # with one tau_h and no host times the closed form is unchanged
    assert Model(1.04e-10, 3.0e-9, 0.13e-3).t_host(ly, 32) == pytest.approx(64 * ly * 3.0e-9)
