#!/usr/bin/env python3
"""Throughput of the D2Q37 thermal lattice Boltzmann step on one MI355X.

Workload (default): the 2048x4096 Rayleigh-Taylor lattice in FP64 -- walls at
T = 4/3 (bottom) and 2/3 (top), x periodic, gravity g_y = -1e-5, tau = 0.7,
two layers of density/temperature ratio 2:1 whose interface is displaced by
seeded uniform noise of amplitude 1e-3.  A step is one propagate + bc +
collide pass over the whole lattice; the metric is MLUPS (million lattice
site updates per second), inputs resident in HBM.

Printed: one JSON line with the FP64 MLUPS as `value`, the FP32-shifted
MLUPS and ratio, the adjoint/forward cost ratio, the roofline of the dominant
kernel (timed with HIP events on the library's stream) and the CPU oracle's
rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3


def kernel_source_sha256():
    """Hash of the GPU kernel sources (to tell whether stored counters still apply)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1703_04594_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hpp")) + glob.glob(os.path.join(csrc, "*.hip"))
                   + glob.glob(os.path.join(csrc, "*.inc")) + glob.glob(os.path.join(csrc, "*.h")))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(kernel_prefix):
    """Per-launch rocprofv3 counter figures of a kernel on the 2048x4096
    lattice -- HBM bytes (FETCH_SIZE/WRITE_SIZE, calibrated) and VALU FLOPs
    (SQ_INSTS_VALU_FLOPS_FP64/FP32) -- from the committed profile, or None
    if the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "d2q37_2048x4096_counters.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != kernel_source_sha256():
        return None
    for name, v in rec["kernels"].items():
        if name.startswith(kernel_prefix):
            return v
    return None


def measured_traffic(kernel_prefix):
    v = measured_counters(kernel_prefix)
    return None if v is None else v["traffic_bytes"]


def flop_fraction(kernel_prefix, seconds):
    """Achieved FP64 and FP32 FLOP rate of one launch over the vector peaks."""
    v = measured_counters(kernel_prefix)
    if v is None or "flops_fp64" not in v:
        return None
    return {"fp64": round(v["flops_fp64"] / seconds / 1e12 / FP64_PEAK_TFLOPS, 4),
            "fp32": round(v["flops_fp32"] / seconds / 1e12 / FP32_PEAK_TFLOPS, 4)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_launches(fn, stream, reps):
    """Average duration of fn() over reps launches, HIP events on `stream`."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps * 1e-3


def copy_reference(nbytes, stream, reps=20):
    """Plain device copy of nbytes (csrc/copy_probe.hip) with 1, 2 and 4 KB per
    workgroup, timed like the lattice kernels; returns GB/s moved (read +
    write) per workgroup size."""
    import ctypes

    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1703_04594_amd", "libcopyprobe.so"))
    lib.cp_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    lib.cp_copy.restype = ctypes.c_int
    a = torch.arange(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    out = {}
    for bb in (1024, 2048, 4096):
        def go():
            rc = lib.cp_copy(a.data_ptr(), b.data_ptr(), a.numel() * 8, bb, stream.cuda_stream)
            if rc:
                raise RuntimeError(f"cp_copy failed ({rc})")
        go()
        b.zero_()
        go()
        stream.synchronize()
        if not torch.equal(a, b):
            raise RuntimeError("reference copy produced wrong data")
        t = time_launches(go, stream, reps)
        out[f"{bb // 1024}KB_per_workgroup"] = round(2 * a.numel() * 8 / t / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def gather_copy_reference(lx, ly, stream, reps=20, runs=5):
    """The fused step's access pattern with no arithmetic (cp_gather_copy in
    csrc/copy_probe.hip: 37 gathered loads and 37 stores per site on the
    columns layout, the fused step's workgroups and block order), FP64 and
    FP32: median over `runs` runs of the mean time of `reps` launches, in
    seconds.  This is the ceiling that access pattern leaves the fused step."""
    import ctypes

    import numpy as np
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1703_04594_amd", "libcopyprobe.so"))
    lib.cp_gather_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.cp_gather_bytes.restype = ctypes.c_size_t
    lib.cp_gather_copy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]
    lib.cp_gather_copy.restype = ctypes.c_int
    out = {}
    for elem in (8, 4):
        n = lib.cp_gather_bytes(elem, lx, ly)
        if n == 0:
            raise RuntimeError("cp_gather_bytes refused the lattice")
        # 256-byte aligned views into two buffers
        a_raw = torch.ones(n + 256, dtype=torch.uint8, device="cuda:0")
        b_raw = torch.empty(n + 256, dtype=torch.uint8, device="cuda:0")
        a = (a_raw.data_ptr() + 255) // 256 * 256
        b = (b_raw.data_ptr() + 255) // 256 * 256

        def go():
            rc = lib.cp_gather_copy(elem, lx, ly, a, b, stream.cuda_stream)
            if rc:
                raise RuntimeError(f"cp_gather_copy failed ({rc})")
        go()
        stream.synchronize()
        t = float(np.median([time_launches(go, stream, reps) for _ in range(runs)]))
        out["fp64" if elem == 8 else "fp32"] = t
        del a_raw, b_raw
        torch.cuda.empty_cache()
    return out


def adjoint_pattern_reference(lx, ly, stream, reps=20, runs=5):
    """The reverse step's access pattern over FP32 states with no collide^T
    arithmetic (cp_adjoint_pattern in csrc/copy_probe.hip: 37 gathered state
    loads, 37 gathered lambda loads and 37 stores per site), for FP64 and FP32
    lambda: median over `runs` runs of the mean time of `reps` launches, s."""
    import ctypes

    import numpy as np
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1703_04594_amd", "libcopyprobe.so"))
    lib.cp_gather_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.cp_gather_bytes.restype = ctypes.c_size_t
    vp = ctypes.c_void_p
    lib.cp_adjoint_pattern.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]
    lib.cp_adjoint_pattern.restype = ctypes.c_int
    out = {}
    nf = lib.cp_gather_bytes(4, lx, ly)
    f_raw = torch.zeros(nf + 256, dtype=torch.uint8, device="cuda:0")
    f = (f_raw.data_ptr() + 255) // 256 * 256
    for lam_bytes in (8, 4):
        nl = lib.cp_gather_bytes(lam_bytes, lx, ly)
        l_raw = torch.zeros(nl + 256, dtype=torch.uint8, device="cuda:0")
        m_raw = torch.empty(nl + 256, dtype=torch.uint8, device="cuda:0")
        lp = (l_raw.data_ptr() + 255) // 256 * 256
        mp = (m_raw.data_ptr() + 255) // 256 * 256

        def go():
            rc = lib.cp_adjoint_pattern(lam_bytes, lx, ly, f, lp, mp, stream.cuda_stream)
            if rc:
                raise RuntimeError(f"cp_adjoint_pattern failed ({rc})")
        go()
        stream.synchronize()
        out["fp64" if lam_bytes == 8 else "fp32"] = float(np.median([time_launches(go, stream, reps)
                                                                      for _ in range(runs)]))
        del l_raw, m_raw
        torch.cuda.empty_cache()
    del f_raw
    torch.cuda.empty_cache()
    return out


def run(args):
    import numpy as np
    import torch

    from paper_1703_04594_amd import inputs
    from paper_1703_04594_amd.lbm import Lattice

    lx, ly = args.lx, args.ly
    tau, g, tb, tt = 0.7, -1e-5, 4 / 3, 2 / 3
    sites = lx * ly
    dev = "cuda:0"
    P = torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=dev)
    out = {}

    def make(precision, step, adjoint=False):
        lat = Lattice(lx, ly, tau, g, tb, tt, precision=precision, step=step, adjoint=adjoint, device=dev)
        lat.init_rt(P)
        return lat

    def mlups(lat, steps, warmup):
        """Wall-clock rate of `steps` steps (device synchronised on both
        sides), and the per-step time from HIP events recorded around the
        same call on the lattice's stream."""
        lat.step(warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(lat.stream)
        lat.step(steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["event_step_s"] = e0.elapsed_time(e1) * 1e-3 / steps
        return sites * steps / dt / 1e6, dt

    # ---- headline: FP64 step ------------------------------------------------
    log(f"bench: FP64 {lx}x{ly}, fused step, warmup {args.warmup}, steps {args.steps}")
    lat = make("fp64", "fused")
    fp64_mlups, dt = mlups(lat, args.steps, args.warmup)
    t_timed = out["event_step_s"]   # the headline kernel per launch, over the timed region
    out["fp64"] = dict(mlups=fp64_mlups, seconds=dt)
    s = lat.stream
    t_fused_runs = [time_launches(lambda: lat.step(1), s, 20) for _ in range(5)]
    t_fused = float(np.median(t_fused_runs))
    # five more timed runs of 100 steps each and their median (a protocol
    # robust to one slow run), beside the single timed run that gives `value`
    median5 = float(np.median([mlups(lat, 100, 0)[0] for _ in range(5)]))
    del lat
    torch.cuda.empty_cache()

    log("bench: FP64 fused step, planes layout")
    lat = Lattice(lx, ly, tau, g, tb, tt, precision="fp64", step="fused", layout="planes", device=dev)
    lat.init_rt(P)
    planes_mlups, _ = mlups(lat, max(50, args.steps // 5), 10)
    del lat
    torch.cuda.empty_cache()

    log("bench: FP64 split step and its kernels")
    lat = make("fp64", "split")
    split_mlups, _ = mlups(lat, max(20, args.steps // 10), 5)
    # propagate and collide: median of five runs of 20 back-to-back launches
    t_prop_runs = [time_launches(lat.propagate, s, 20) for _ in range(5)]
    t_coll_runs = [time_launches(lat.collide, s, 20) for _ in range(5)]
    t_prop, t_coll = float(np.median(t_prop_runs)), float(np.median(t_coll_runs))
    del lat
    torch.cuda.empty_cache()

    log("bench: reference copy of one lattice's populations")
    copy_ref = copy_reference(37 * 8 * sites, s)
    log("bench: the fused step's access pattern without arithmetic")
    t_pattern = gather_copy_reference(lx, ly, s)

    log("bench: FP32-shifted")
    lat = make("fp32", "fused")
    fp32_mlups, _ = mlups(lat, args.steps, args.warmup)
    t_fused32 = float(np.median([time_launches(lambda: lat.step(1), s, 20) for _ in range(5)]))
    del lat
    torch.cuda.empty_cache()

    log("bench: FP32-shifted with FP32 moment sums")
    lat = make("fp32_f32sums", "fused")
    fp32s_mlups, _ = mlups(lat, args.steps, args.warmup)
    t_fused32s = time_launches(lambda: lat.step(1), s, 20)
    del lat
    torch.cuda.empty_cache()

    t_adj = {}
    for lam in ("fp64", "fp32"):
        log(f"bench: adjoint step (FP32 state, {lam} lambda)")
        lat = make("fp32", "fused", adjoint=lam)
        lat.step(10)
        st = lat.get_state()
        lat.step(1)
        lat.seed_temperature(torch.ones((lx, ly), dtype=torch.float64, device=dev))
        # as the rollout runs it: d/dtau kept per block, one reduction per sweep
        t_adj[lam] = float(np.median([time_launches(lambda: lat.adjoint_step(st, None), s, 10) for _ in range(5)]))
        t_fwd32 = float(np.median([time_launches(lambda: lat.step(1), s, 10) for _ in range(5)]))
        del lat, st
        torch.cuda.empty_cache()

    log("bench: x-periodicity by 3-column halos against the wrapped index")
    xmode = {}
    for prec, step in (("fp64", "fused"), ("fp64", "split"), ("fp32", "fused")):
        row = {}
        for xm in ("wrap", "halo"):
            lat = Lattice(lx, ly, tau, g, tb, tt, precision=prec, step=step, xmode=xm, device=dev)
            lat.init_rt(P)
            lat.step(5)
            row[xm] = float(np.median([time_launches(lambda: lat.step(1), s, 20) for _ in range(5)]))
            del lat
            torch.cuda.empty_cache()
        xmode[f"{prec}_{step}"] = {"wrap_ms": round(row["wrap"] * 1e3, 4), "halo_ms": round(row["halo"] * 1e3, 4),
                                   "halo_over_wrap": round(row["halo"] / row["wrap"], 4)}

    log("bench: the reverse step's access pattern without arithmetic")
    t_adj_pattern = adjoint_pattern_reference(lx, ly, s)

    bytes_fp64 = 2 * 37 * 8 * sites   # one read + one write of every population
    bytes_fp32 = 2 * 37 * 4 * sites
    achieved = bytes_fp64 / t_timed / 1e9
    res = {
        "metric": "MLUPS D2Q37 step FP64 vs FP32 (+%HBM/%FLOP peak); adjoint/forward cost ratio",
        "value": round(fp64_mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"D2Q37 Rayleigh-Taylor {lx}x{ly} FP64, walls, tau=0.7, g=-1e-5",
                   "lx": lx, "ly": ly, "step": "fused gather+bc+collide", "layout": "columns"},
        "fp32_shifted_mlups": round(fp32_mlups, 1),
        "fp32_over_fp64": round(fp32_mlups / fp64_mlups, 3),
        "fp32_arithmetic": "FP32 storage of f - w and FP32 collide; the collide's 8 moment sums of 37 terms "
                           "(before and after relaxation) accumulate in FP64 (416 FP64 FLOP/site)",
        "fp32_f32sums_mlups": round(fp32s_mlups, 1),
        "fp32_f32sums_arithmetic": "FP32 storage and collide with every sum in FP32 (no FP64 in the step)",
        "fp64_mlups_median_of_5x100_steps": round(median5, 1),
        "fp64_split_mlups": round(split_mlups, 1),
        "fp64_fused_planes_layout_mlups": round(planes_mlups, 1),
        "adjoint_over_forward_fp32": round(t_adj["fp64"] / t_fwd32, 3),
        "adjoint_over_forward_fp32_lambda32": round(t_adj["fp32"] / t_fwd32, 3),
        "kernel_ms": {"fused_fp64": round(t_fused * 1e3, 4), "fused_fp32": round(t_fused32 * 1e3, 4),
                      "fused_fp32_f32sums": round(t_fused32s * 1e3, 4), "propagate_fp64": round(t_prop * 1e3, 4), "collide_fp64": round(t_coll * 1e3, 4),
                      "adjoint_step_fp32": round(t_adj["fp64"] * 1e3, 4),
                      "adjoint_step_fp32_lambda32": round(t_adj["fp32"] * 1e3, 4), "step_fp32": round(t_fwd32 * 1e3, 4)},
        "copy_reference_GBps": copy_ref,
        "propagate_fp64_over_copy": round(bytes_fp64 / t_prop / 1e9 / max(copy_ref.values()), 3),
        "access_pattern_copy_ms": {k: round(v * 1e3, 4) for k, v in t_pattern.items()},
        "fused_over_access_pattern_copy": {"fp64": round(t_pattern["fp64"] / t_fused, 3),
                                           "fp32": round(t_pattern["fp32"] / t_fused32, 3)},
        "x_halo_vs_wrap": xmode,
        "adjoint_access_pattern_copy_ms": {k: round(v * 1e3, 4) for k, v in t_adj_pattern.items()},
        "adjoint_over_access_pattern_copy": {"fp64_lambda": round(t_adj_pattern["fp64"] / t_adj["fp64"], 3),
                                             "fp32_lambda": round(t_adj_pattern["fp32"] / t_adj["fp32"], 3)},
        "adjoint_hbm_frac": {"fp64_lambda": round(740 * sites / t_adj["fp64"] / 1e9 / HBM_PEAK_GBS, 3),
                             "fp32_lambda": round(444 * sites / t_adj["fp32"] / 1e9 / HBM_PEAK_GBS, 3)},
        "kernel_times": "per-kernel figures: median of 5 runs of 10-20 back-to-back launches (HIP events); "
                        "reverse steps as the checkpointed rollout runs them (d/dtau kept per block, "
                        "reduced once per sweep)",
        "propagate_fp64_hbm_frac_runs": [round(bytes_fp64 / t / 1e9 / HBM_PEAK_GBS, 4) for t in t_prop_runs],
        "hbm_frac": {"fused_fp64": round(bytes_fp64 / t_fused / 1e9 / HBM_PEAK_GBS, 3),
                     "fused_fp32": round(bytes_fp32 / t_fused32 / 1e9 / HBM_PEAK_GBS, 3),
                     "propagate_fp64": round(bytes_fp64 / t_prop / 1e9 / HBM_PEAK_GBS, 3),
                     "collide_fp64": round(bytes_fp64 / t_coll / 1e9 / HBM_PEAK_GBS, 3)},
        "flop_frac": None if (lx, ly) != (2048, 4096) else {
            "fused_fp64": flop_fraction("lbm::k_step_fused<double, true, true, true, 512, true>", t_fused),
            "collide_fp64": flop_fraction("lbm::k_collide<double, true, true>", t_coll),
            "fused_fp32": flop_fraction("lbm::k_step_fused<float, true, true, true, 256, true>", t_fused32),
            "adjoint_fp64_lambda": flop_fraction("lbm::k_adj_collide<float, double, true, true, 256, true>", t_adj["fp64"]),
            "adjoint_fp32_lambda": flop_fraction("lbm::k_adj_collide<float, float, true, true, 64, true>", t_adj["fp32"])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("lbm::k_step_fused<double, true, true, true, 512, true>") if (lx, ly) == (2048, 4096) else None,
                     "kernel": "k_step_fused<double,wrap,walls>", "bytes_per_site": 592,
                     "algorithmic_bytes_per_launch": bytes_fp64},
    }
    return res


def fp32_accuracy(args, nsteps=5000, every=500):
    """Both FP32-shifted forms (FP64 moment sums, the default; FP32 sums) vs
    FP64 on the bench lattice, every `every` steps:

    * per-field relative errors against the GPU FP64 path (itself pinned to
      the oracle by the parity tests): rho and T relative to the field's
      spread, ||q32 - q64|| / ||q64 - mean(q64)||, and to its size,
      ||q32 - q64|| / ||q64||; u relative to max(||u64||, 1e-6 sqrt(S));
    * the FP64 lattice totals (lbm_conservation) of mass M and of
      E = sum |xi|^2 f, for every precision: the bulk step conserves both,
      so their change is what the walls let through; `wall_mass_flux` is
      the mean change of M per step over the interval, and `M_rel_vs_fp64`
      how far an FP32 form's total mass has moved from the FP64 run's."""
    import torch

    from paper_1703_04594_amd import inputs
    from paper_1703_04594_amd.lbm import Lattice

    lx, ly, dev = args.lx, args.ly, "cuda:0"
    P = torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=dev)
    lats = {}
    for prec in ("fp64", "fp32", "fp32_f32sums"):
        lats[prec] = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision=prec, step="fused", device=dev)
        lats[prec].init_rt(P)
    totals = {prec: lat.conservation().cpu().tolist() for prec, lat in lats.items()}
    rows = [{"step": 0, "totals": {prec: {"M": t[0], "E": t[3]} for prec, t in totals.items()}}]
    floor_u = 1e-6 * (lx * ly) ** 0.5
    for k in range(nsteps // every):
        for lat in lats.values():
            lat.step(every)
        a = lats["fp64"].macros()
        rho64, T64 = a[0], a[3]
        u64 = torch.stack([a[1], a[2]])
        row = {"step": (k + 1) * every, "u_norm": float(u64.norm())}   # a dip in |u| shows as a spike in "u"
        now = {prec: lat.conservation().cpu().tolist() for prec, lat in lats.items()}
        for prec in ("fp32", "fp32_f32sums"):
            b = lats[prec].macros()
            u32 = torch.stack([b[1], b[2]])
            r = {}
            for name, x64, x32 in (("rho", rho64, b[0]), ("T", T64, b[3])):
                d = float((x32 - x64).norm())
                r[name + "_vs_spread"] = d / float((x64 - x64.mean()).norm())
                r[name + "_vs_size"] = d / float(x64.norm())
            r["u"] = float((u32 - u64).norm()) / max(float(u64.norm()), floor_u)
            r["M_rel_vs_fp64"] = (now[prec][0] - now["fp64"][0]) / now["fp64"][0]
            r["E_rel_vs_fp64"] = (now[prec][3] - now["fp64"][3]) / now["fp64"][3]
            row[prec] = {k2: round(v, 12) for k2, v in r.items()}
        row["totals"] = {prec: {"M": t[0], "E": t[3], "wall_mass_flux": (t[0] - totals[prec][0]) / every}
                         for prec, t in now.items()}
        totals = now
        rows.append(row)
        log(f"bench: fp32 accuracy {row}")
    del lats
    torch.cuda.empty_cache()
    return rows


def adjoint_at_scale(lx=1024, ly=2048, nsteps=10000, budget=32 * 10 ** 9, lam="fp64"):
    """Gradient of 1/2 sum (T_N - T*)^2 w.r.t. the initial perturbation field
    P and tau on the 1024x2048 lattice, FP32 forward states, FP64 adjoint,
    binomial checkpointing; the job's peak device memory (workspace, stored
    states, temporaries) stays inside `budget` bytes (32 GB = 32e9 bytes,
    which is also inside 32 GiB)."""
    import torch

    from paper_1703_04594_amd import inputs
    from paper_1703_04594_amd.autograd import RolloutConfig, rt_temperature
    from paper_1703_04594_amd.lbm import Lattice

    dev = "cuda:0"
    P = torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=dev)
    P2 = torch.tensor(inputs.rt_perturbation(lx, ly, 2), device=dev)
    lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp32", step="fused", device=dev)
    lat.init_rt(P2)
    lat.step(nsteps)
    Tt = lat.macros()[3].clone()
    # plain forward wall time, and per-step kernel times
    lat.init_rt(P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del lat
    probe = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp32", step="fused", adjoint=lam, device=dev)
    probe.init_rt(P)
    ws_bytes = probe.workspace.numel()
    st = probe.get_state()
    probe.step(1)
    probe.seed_temperature(torch.ones((lx, ly), dtype=torch.float64, device=dev))
    t_adj = time_launches(lambda: probe.adjoint_step(st, None), probe.stream, 20)
    t_step = time_launches(lambda: probe.step(1), probe.stream, 20)
    state_bytes = probe.state_bytes
    del probe, st
    torch.cuda.empty_cache()
    # full gradient: forward with checkpoints + reverse sweep.  The stored
    # states get what the budget leaves after the workspace and the rollout's
    # field-sized temporaries (macros, loss terms, dL/dT, dL/dP: 12 fields
    # allowed), so the whole job's peak stays inside the budget.
    reserve = 12 * lx * ly * 8
    cfg = RolloutConfig(lx, ly, nsteps, precision="fp32", checkpoint="binomial",
                        memory_budget=budget - ws_bytes - reserve, lambda_precision=lam)
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    Pg = P.clone().requires_grad_(True)
    tg = torch.tensor(0.7, dtype=torch.float64, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = rt_temperature(Pg, tg, cfg)
    loss = 0.5 * ((T - Tt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    peak = torch.cuda.max_memory_allocated() - base_mem
    out = {"lattice": f"{lx}x{ly}", "steps": nsteps, "checkpoint": "binomial", "lambda": lam,
           "budget_bytes": budget, "state_bytes": state_bytes,
           "snapshot_slots": cfg.stats.get("slots"), "forward_steps_total": cfg.stats.get("forward_steps"),
           "adjoint_step_ms": round(t_adj * 1e3, 4), "forward_step_ms": round(t_step * 1e3, 4),
           "adjoint_over_forward_step": round(t_adj / t_step, 3),
           "forward_wall_s": round(t_fwd, 3), "gradient_wall_s": round(t_grad, 3),
           "gradient_over_forward_wall": round(t_grad / t_fwd, 3),
           "peak_memory_bytes": peak, "peak_within_budget": bool(peak <= budget),
           "workspace_bytes": ws_bytes, "loss": float(loss.detach()),
           "dL_dtau": float(tg.grad), "dL_dP_norm": float(Pg.grad.norm())}
    log(f"bench: adjoint at scale {out}")
    return out


def adjoint_c4(lx=512, ly=512, nsteps=2000, lam="fp64"):
    """The adjoint configuration's own lattice: 512x512, FP32 forward, FP64
    (or FP32) lambda, 2000 steps, sqrt(T) checkpointing, loss 1/2 sum (T_N -
    T*)^2 with T* the final temperature of the seed-2 run: per-step adjoint /
    forward time and the whole gradient's wall time over the forward's."""
    import numpy as np
    import torch

    from paper_1703_04594_amd import inputs
    from paper_1703_04594_amd.autograd import RolloutConfig, rt_temperature
    from paper_1703_04594_amd.lbm import Lattice

    dev = "cuda:0"
    P = torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=dev)
    lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp32", step="fused", device=dev)
    lat.init_rt(torch.tensor(inputs.rt_perturbation(lx, ly, 2), device=dev))
    lat.step(nsteps)
    Tt = lat.macros()[3].clone()
    lat.init_rt(P)
    lat.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del lat
    probe = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp32", step="fused", adjoint=lam, device=dev)
    probe.init_rt(P)
    st = probe.get_state()
    probe.step(1)
    probe.seed_temperature(torch.ones((lx, ly), dtype=torch.float64, device=dev))
    t_adj = float(np.median([time_launches(lambda: probe.adjoint_step(st, None), probe.stream, 50) for _ in range(5)]))
    t_step = float(np.median([time_launches(lambda: probe.step(1), probe.stream, 50) for _ in range(5)]))
    del probe, st
    cfg = RolloutConfig(lx, ly, nsteps, precision="fp32", checkpoint="sqrt", lambda_precision=lam)
    for rep in range(2):          # the first rollout pays one-time costs
        Pg = P.clone().requires_grad_(True)
        tg = torch.tensor(0.7, dtype=torch.float64, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = rt_temperature(Pg, tg, cfg)
        (0.5 * ((T - Tt) ** 2).sum()).backward()
        torch.cuda.synchronize()
        t_grad = time.perf_counter() - t0
    out = {"lattice": f"{lx}x{ly}", "steps": nsteps, "checkpoint": "sqrt", "lambda": lam,
           "adjoint_step_ms": round(t_adj * 1e3, 4), "forward_step_ms": round(t_step * 1e3, 4),
           "adjoint_over_forward_step": round(t_adj / t_step, 3), "forward_wall_s": round(t_fwd, 4),
           "gradient_wall_s": round(t_grad, 4), "gradient_over_forward_wall": round(t_grad / t_fwd, 3),
           "forward_steps_total": cfg.stats.get("forward_steps"), "snapshot_slots": cfg.stats.get("slots")}
    log(f"bench: adjoint 512x512 {out}")
    return out


def cpu_baseline(args, budget_s=15.0):
    """The oracle (OpenMP build of the plain C source) on the host cores, on a
    bounded number of steps of the same lattice."""
    import numpy as np

    import oracle
    from paper_1703_04594_amd import inputs

    lx, ly = args.lx, args.ly
    P = inputs.rt_perturbation(lx, ly, 1)
    y = np.arange(ly)[None, :]
    T0 = 1.0 - np.tanh((y - (ly - 1) / 2 - P) / 2.0) / 3.0
    L = oracle.RefLattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, openmp=True)
    L.init((8 / 9) / T0, 0.0, 0.0, T0)
    t0 = time.perf_counter()
    L.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, int(budget_s / max(t1, 1e-3)))
    log(f"bench: cpu oracle, {n} steps (1 step took {t1:.2f}s)")
    t0 = time.perf_counter()
    L.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(lx * ly * n / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.threads(True),
            "kind": "oracle", "sample": f"{n} FP64 steps of the {lx}x{ly} RT lattice after 1 untimed step"}


def cpu_oracle_serial(lx=256, ly=128, n=50):
    """The serial oracle (one core) on the small 256x128 RT lattice, 50 steps
    after one untimed step."""
    import numpy as np

    import oracle
    from paper_1703_04594_amd import inputs

    P = inputs.rt_perturbation(lx, ly, 1)
    y = np.arange(ly)[None, :]
    T0 = 1.0 - np.tanh((y - (ly - 1) / 2 - P) / 2.0) / 3.0
    L = oracle.RefLattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, openmp=False)
    L.init((8 / 9) / T0, 0.0, 0.0, T0)
    L.step(1)
    t0 = time.perf_counter()
    L.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(lx * ly * n / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "seconds": round(dt, 3), "sample": f"{n} FP64 steps of the {lx}x{ly} RT lattice, serial build"}


def layout_study(lx=2160, ly=8192, reps=20):
    """Per-kernel times of the FP64 step on the paper's 2160x8192 lattice
    (its Table 2 experiment): for each layout the library's step supports,
    planes (structure of arrays) and columns (the 37 segments of a column
    together), and for the paper's four layouts (AOS, SOA, CSOA and CAOSOA,
    cluster widths 8-64) with the study kernels.  HIP events over `reps`
    back-to-back launches per kernel."""
    import torch

    from paper_1703_04594_amd import inputs
    from paper_1703_04594_amd.lbm import Lattice

    dev = "cuda:0"
    P = torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=dev)
    sites = lx * ly
    nbytes = 2 * 37 * 8 * sites
    out = {"lattice": f"{lx}x{ly}", "precision": "fp64", "layouts": {}}
    for layout in ("planes", "columns"):
        row = {}
        lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp64", step="split", layout=layout, device=dev)
        lat.init_rt(P)
        s = lat.stream
        lat.step(2)
        t_prop = time_launches(lat.propagate, s, reps)
        t_bc = time_launches(lat.bc, s, reps)
        t_coll = time_launches(lat.collide, s, reps)
        t_split = time_launches(lambda: lat.step(1), s, reps)
        del lat
        torch.cuda.empty_cache()
        lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp64", step="fused", layout=layout, device=dev)
        lat.init_rt(P)
        lat.step(2)
        t_fused = time_launches(lambda: lat.step(1), lat.stream, reps)
        del lat
        torch.cuda.empty_cache()
        for name, t in (("propagate", t_prop), ("bc", t_bc), ("collide", t_coll), ("step_split", t_split),
                        ("step_fused", t_fused)):
            row[name + "_ms"] = round(t * 1e3, 4)
        row["propagate_GBps"] = round(nbytes / t_prop / 1e9, 1)
        row["collide_GBps"] = round(nbytes / t_coll / 1e9, 1)
        row["split_mlups"] = round(sites / t_split / 1e6, 1)
        row["fused_mlups"] = round(sites / t_fused / 1e6, 1)
        out["layouts"][layout] = row
        log(f"bench: layout {layout}: {row}")

    # The paper's four layouts (section 4), with the library's generic study
    # kernels (one element per thread in propagate, one site per thread in
    # collide; periodic in x and y), on an RT state of the same lattice.
    from paper_1703_04594_amd import lbm as L
    lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp64", step="fused", device=dev)
    lat.init_rt(P)
    lat.step(2)
    f = lat.get_pops()
    del lat
    torch.cuda.empty_cache()
    s = torch.cuda.current_stream()
    out["study_layouts"] = {}
    for layout, vl in [("aos", 1), ("soa", 1)] + [(k, v) for k in ("csoa", "caosoa") for v in (8, 16, 32, 64)]:
        buf = L.study_pack(layout, vl, f)
        dst = torch.empty_like(buf)
        prop = lambda: L.study_propagate(layout, vl, lx, ly, buf, dst)     # noqa: E731
        coll = lambda: L.study_collide(layout, vl, lx, ly, 0.7, -1e-5, buf)  # noqa: E731
        prop()
        coll()
        t_prop = time_launches(prop, s, reps)
        t_coll = time_launches(coll, s, reps)
        del buf, dst
        name = layout if layout in ("aos", "soa") else f"{layout}_vl{vl}"
        row = {"propagate_ms": round(t_prop * 1e3, 4), "collide_ms": round(t_coll * 1e3, 4),
               "propagate_GBps": round(nbytes / t_prop / 1e9, 1), "collide_GBps": round(nbytes / t_coll / 1e9, 1)}
        out["study_layouts"][name] = row
        log(f"bench: study layout {name}: {row}")
    return out


def hetero_study(lx=2048, ly=4096, steps=20):
    """Host + GPU co-execution (section 5) on an lx x ly RT lattice, FP64:
    the performance model's auto-tuned parameters (section 6) and predicted
    optimum, then the measured rate for a sweep of m (border columns per
    side on the host) beside the model's prediction."""
    import torch

    from paper_1703_04594_amd import inputs
    from paper_1703_04594_amd.hetero import Model, autotune
    from paper_1703_04594_amd.lbm import Hetero, HostLattice, Lattice

    threads = min(16, os.cpu_count() or 1)
    dev = "cuda:0"
    lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, step="fused", device=dev)
    lat.init_rt(torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=dev))
    f0 = lat.get_pops().cpu().numpy()
    del lat
    torch.cuda.empty_cache()

    def make(m):
        h = Hetero(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, m=m, host_threads=threads, device=dev)
        h.set_pops(f0)
        return h

    widths = [m for m in (2, 4, 8, 16, 32, 64, 128) if lx - 2 * m >= 3]

    def host_probe(m):
        """Host step seconds of the host part of an m-column split alone: its
        band of 2m columns plus 3 halo columns per side (lbm_host_step)."""
        hl = HostLattice(2 * m + 6, ly, 0.7, -1e-5, 4 / 3, 2 / 3, threads=threads)
        hl.set_pops(f0[:, :2 * m + 6])
        hl.step(3)
        t0 = time.perf_counter()
        hl.step(steps)
        return (time.perf_counter() - t0) / steps

    model = autotune(make, lx, ly, m_probe=32, steps=steps, host_probe=host_probe, host_widths=widths)
    single = Model(model.tau_d, model.tau_h, model.t_swap)    # the paper's form: one tau_h (m = 32)
    log(f"bench: hetero model tau_d={model.tau_d:.3e} tau_h={model.tau_h:.3e} t_swap={model.t_swap:.3e} "
        f"host_times={model.host_times}")
    sweep = []
    for m in [0] + widths:
        h = make(m)
        h.step(3)
        h.step(steps)
        t = h.times()
        h.close()
        meas = lx * ly / t["wall"] / 1e6
        p1, p2 = single.mlups(lx, ly, m), model.mlups(lx, ly, m)
        # the model's composition max(T_acc, T_host) + T_swap fed with this
        # run's own component times: checks the overlap assumption alone
        p3 = lx * ly / (max(t["gpu"], t["host"]) + t["swap"]) / 1e6
        row = {"m": m, "host_fraction": round(2 * m / lx, 4), "mlups": round(meas, 1),
               "model_mlups": round(p1, 1), "model_rel_err": round(p1 / meas - 1, 4),
               "model_host_times_mlups": round(p2, 1), "model_host_times_rel_err": round(p2 / meas - 1, 4),
               "composition_rel_err": round(p3 / meas - 1, 4),
               "host_ns_per_site": None if m == 0 else round(t["host"] / (2 * m * ly) * 1e9, 4),
               "host_alone_ms": None if m == 0 else round(model.host_times[m] * 1e3, 4),
               "ms": {k: round(v * 1e3, 4) for k, v in t.items()}}
        sweep.append(row)
        log(f"bench: hetero {row}")
    return {"lattice": f"{lx}x{ly}", "precision": "fp64", "host_threads": threads, "steps": steps,
            "tau_d_ns_per_site": round(model.tau_d * 1e9, 5), "tau_h_ns_per_site": round(model.tau_h * 1e9, 4),
            "tau_h_ns_per_site_by_m": {m: round(v / (2 * m * ly) * 1e9, 4) for m, v in model.host_times.items()},
            "t_swap_ms": round(model.t_swap * 1e3, 4), "m_balance": round(single.m_balance(lx), 2),
            "best_m": single.best_m(lx, ly), "best_m_host_times": model.best_m(lx, ly),
            "max_abs_rel_err": {"model": max(abs(r["model_rel_err"]) for r in sweep),
                                "model_host_times": max(abs(r["model_host_times_rel_err"]) for r in sweep),
                                "composition": max(abs(r["composition_rel_err"]) for r in sweep)},
            "sweep": sweep}


def profile_workload(args):
    """Short fixed sequence for rocprofv3 runs: a plain device copy of known
    size (calibrates the HBM byte counters), the reference copy of one
    lattice's populations, then FP64 and FP32 fused steps,
    FP64 and FP32 split steps, and adjoint steps over FP32 states with FP64
    and FP32 lambda, all on the bench lattice."""
    import torch

    from paper_1703_04594_amd import inputs
    from paper_1703_04594_amd.lbm import Lattice

    lx, ly, dev = args.lx, args.ly, "cuda:0"
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)                     # 1 GiB read + 1 GiB written per dispatch
    torch.cuda.synchronize()
    del a, b
    copy_reference(37 * 8 * lx * ly, torch.cuda.current_stream(), reps=5)
    P = torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=dev)
    for prec in ("fp64", "fp32"):
        lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision=prec, step="fused", device=dev)
        lat.init_rt(P)
        lat.step(args.steps)
        torch.cuda.synchronize()
        del lat
    for prec in ("fp64", "fp32"):
        lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision=prec, step="split", device=dev)
        lat.init_rt(P)
        lat.step(args.steps)
        torch.cuda.synchronize()
        del lat
    for lam in ("fp64", "fp32"):
        lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp32", step="fused", adjoint=lam, device=dev)
        lat.init_rt(P)
        st = lat.get_state()
        lat.step(1)
        lat.seed_temperature(torch.ones((lx, ly), dtype=torch.float64, device=dev))
        dacc = torch.zeros((), dtype=torch.float64, device=dev)
        for _ in range(args.steps):
            lat.adjoint_step(st, None)
        lat.take_dtau(dacc)
        torch.cuda.synchronize()
        del lat, st
    lat = Lattice(lx, ly, 0.7, -1e-5, 4 / 3, 2 / 3, precision="fp32_f32sums", step="fused", device=dev)
    lat.init_rt(P)
    lat.step(args.steps)
    torch.cuda.synchronize()
    del lat
    torch.cuda.empty_cache()
    s = torch.cuda.current_stream()
    gather_copy_reference(lx, ly, s, reps=args.steps, runs=1)
    adjoint_pattern_reference(lx, ly, s, reps=args.steps, runs=1)
    torch.cuda.synchronize()
    print(json.dumps({"profile_workload": "done", "steps": args.steps}), flush=True)


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {d}")
    return rows


def _short(name):
    """Kernel name without its return type and argument list."""
    name = name.replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    s = "".join(out).strip()
    return s[5:] if s.startswith("void ") else s


def summarize_counters(trace_dir, fetch_dir, write_dir, f64_dir, f32_dir, lx, ly):
    """Per-kernel averages from rocprofv3 runs of `bench.py --profile`
    (kernel-trace stats, FETCH_SIZE, WRITE_SIZE, and the FP64 / FP32 VALU
    instruction counters), written to profiles/d2q37_<lx>x<ly>_counters.json
    with the current kernel-source hash.  FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) are scaled by what they read for the workload's first kernel,
    a plain 1 GiB copy (2^30 bytes each way)."""
    from collections import defaultdict
    stats = {_short(r["Name"]): float(r["AverageNs"]) for r in _csv_rows(trace_dir, "kernel_stats.csv")}

    def per_kernel(d):
        acc = defaultdict(lambda: defaultdict(list))
        order = []
        for r in sorted(_csv_rows(d, "counter_collection.csv"), key=lambda r: int(r["Dispatch_Id"])):
            k = _short(r["Kernel_Name"])
            if k not in acc:
                order.append(k)
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return acc, order

    def avg(acc):
        return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}

    fetch_all, order = per_kernel(fetch_dir)
    write_all, _ = per_kernel(write_dir)
    # calibration: the three 1 GiB device-to-device copies that start the
    # workload (the runtime's copy kernel), first in dispatch order
    copy = "__amd_rocclr_copyBuffer"
    fscale = 2 ** 30 / (sum(fetch_all[copy]["FETCH_SIZE"][:3]) / 3 * 1024)
    wscale = 2 ** 30 / (sum(write_all[copy]["WRITE_SIZE"][:3]) / 3 * 1024)
    fetch, write = avg(fetch_all), avg(write_all)
    f64, f32 = avg(per_kernel(f64_dir)[0]), avg(per_kernel(f32_dir)[0])
    sites = lx * ly
    alg = {"k_step_fused<double": 592, "k_step_fused<float": 296, "k_propagate<double": 592,
           "k_propagate<float": 296, "k_collide<double": 592, "k_collide<float": 296, "k_gather_copy<double": 592,
           "k_gather_copy<float": 296, "k_adj_collide<float, double": 740, "k_adj_collide<float, float": 444,
           "k_adjoint_pattern<double": 740, "k_adjoint_pattern<float": 444}
    out = {"workload": f"{lx}x{ly} Rayleigh-Taylor, columns layout", "fetch_scale": round(fscale, 4),
           "write_scale": round(wscale, 4), "calibration": f"first three {copy} dispatches, 1 GiB each way",
           "flops_note": "flops_* = 64 x SQ_INSTS_VALU_FLOPS_FP64/FP32 (wave-instruction counts, FMA as 2), per launch",
           "source_sha256": kernel_source_sha256(), "kernels": {}}
    for k in order:
        rb = fetch[k]["FETCH_SIZE"] * 1024 * fscale
        wb = write.get(k, {}).get("WRITE_SIZE", 0.0) * 1024 * wscale
        row = {"read_bytes": int(rb), "write_bytes": int(wb), "traffic_bytes": int(rb + wb),
               "avg_ns": stats.get(k)}
        for key, b in alg.items():
            if key in k:
                row["algorithmic_bytes"] = b * sites
                row["traffic_over_algorithmic"] = round((rb + wb) / (b * sites), 4)
        if k in f64:
            row["flops_fp64"] = int(64 * f64[k].get("SQ_INSTS_VALU_FLOPS_FP64", 0))
            row["valu_f64_instr"] = {n: int(f64[k].get(f"SQ_INSTS_VALU_{n}_F64", 0)) for n in ("ADD", "MUL", "FMA", "TRANS")}
        if k in f32:
            row["flops_fp32"] = int(64 * f32[k].get("SQ_INSTS_VALU_FLOPS_FP32", 0))
            row["valu_f32_instr"] = {n: int(f32[k].get(f"SQ_INSTS_VALU_{n}_F32", 0)) for n in ("ADD", "MUL", "FMA", "TRANS")}
        out["kernels"][k] = row
    path = os.path.join(ROOT, "profiles", f"d2q37_{lx}x{ly}_counters.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({"summary": path, "kernels": len(order)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--lx", type=int, default=2048)
    ap.add_argument("--ly", type=int, default=4096)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-reports", action="store_true",
                    help="skip the FP32 accuracy and adjoint-at-scale measurements")
    ap.add_argument("--profile", action="store_true",
                    help="run the short fixed kernel sequence used under rocprofv3")
    ap.add_argument("--hetero", action="store_true",
                    help="host + GPU co-execution on 1024x2048, 2048x4096 and 2160x8192: model and m sweep "
                         "(one JSON line)")
    ap.add_argument("--hetero-size", default="1024x2048,2048x4096,2160x8192",
                    help="lattices for --hetero, as LXxLY[,LXxLY...]")
    ap.add_argument("--summarize-counters", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "F64", "F32"),
                    help="write profiles/d2q37_<lx>x<ly>_counters.json from rocprofv3 output directories of "
                         "`bench.py --profile` (kernel-trace stats, FETCH_SIZE, WRITE_SIZE, FP64 and FP32 VALU passes)")
    ap.add_argument("--fp32-accuracy", type=int, metavar="STEPS",
                    help="only the FP32-vs-FP64 accuracy table, over STEPS steps (every 500), one JSON line")
    ap.add_argument("--layout-study", action="store_true",
                    help="per-kernel FP64 times on the 2160x8192 lattice for each layout (one JSON line)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; multi-GPU X-slab sharding is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.lx, args.ly)
        return
    if args.profile:
        profile_workload(args)
        return
    if args.hetero:
        # by default three lattice sizes, as the paper's co-execution study uses
        sizes = [tuple(int(v) for v in s.split("x")) for s in args.hetero_size.split(",")]
        out = [hetero_study(lx, ly) for lx, ly in sizes]
        print(json.dumps({"hetero": out}), flush=True)
        return
    if args.fp32_accuracy:
        every = 500 if args.fp32_accuracy <= 10000 else 2500
        print(json.dumps({"fp32_accuracy": fp32_accuracy(args, nsteps=args.fp32_accuracy, every=every)}), flush=True)
        return
    if args.layout_study:
        print(json.dumps({"layout_study": layout_study()}), flush=True)
        return
    res = run(args)
    if not args.skip_reports:
        res["fp32_accuracy_5000_steps"] = fp32_accuracy(args)
        res["adjoint_1024x2048_10000_steps"] = adjoint_at_scale()
        res["adjoint_1024x2048_10000_steps_lambda32"] = adjoint_at_scale(lam="fp32")
        res["adjoint_512x512_2000_steps"] = adjoint_c4()
        res["adjoint_512x512_2000_steps_lambda32"] = adjoint_c4(lam="fp32")
    res["cpu_baseline"] = None if args.skip_cpu else cpu_baseline(args)
    res["cpu_oracle_serial_256x128"] = None if args.skip_cpu else cpu_oracle_serial()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
