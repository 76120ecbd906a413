#!/usr/bin/env python3
"""Benchmark of the EBIT hot path on one MI355X.

Workload (default): the 3D deformation test of paper sec. 3.2 on a 256^3
grid -- sphere R = 0.15 at (0.35, 0.35, 0.35), LeVeque's field times
cos(pi t / T), T = 3, CFL 0.5 on v_max (dt = h/2, 1536 steps per period).
One step = three advection sweeps (x, y, z) + Front2VOF, FP64.

Metric: interfacial cell-updates/s = sum over the timed steps of the number
of interfacial cells at the start of the step, divided by the wall time of
those steps (inputs resident in HBM).  The roofline object describes the
dominant kernel, timed with HIP events on the stream it runs on; the CPU
baseline is the plain C oracle timed on a bounded sample of the same
workload on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# algorithmic bytes per interfacial cell (FP64 / FP32 storage):
#   sweep: read s_x,s_y,s_z + flags + U_d, write s_x,s_y,s_z + flags
#   Front2VOF: read s_x,s_y,s_z + flags, write C
BYTES = {
    "fp64": {"sweep": 3 * 8 + 1 + 8 + 3 * 8 + 1, "f2v": 3 * 8 + 1 + 8},
    "fp32": {"sweep": 3 * 4 + 1 + 4 + 3 * 4 + 1, "f2v": 3 * 4 + 1 + 4},
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=16)
    p.add_argument("--n", type=int, default=256)
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2509_26361_amd import ebit as E
    from paper_2509_26361_amd import inputs as I

    n = a.n
    T_end = 3.0
    dt = 0.5 / n
    period = int(round(T_end / dt))
    K = a.steps if a.steps is not None else period - a.warmup
    W = a.warmup
    dev = torch.device("cuda:0")
    print(f"[bench] deformation n={n} precision={a.precision} warmup={W} steps={K}", file=sys.stderr, flush=True)

    sh = I.sphere_shape(n)
    U = I.deformation_velocity(n)
    tdev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    dtype = torch.float64 if a.precision == "fp64" else torch.float32
    Ud = [tdev(u).to(dtype) for u in U]
    e = E.Ebit(n, a.precision, dev)
    e.init(tdev(sh.phi_nodes), [tdev(f) for f in sh.phi_faces])
    C = torch.zeros((n, n, n), dtype=dtype, device=dev)
    e.front2vof(C)
    stream = torch.cuda.current_stream()

    step = 0
    for _ in range(W):
        g = I.deformation_time_factor(step * dt, T_end)
        e.step(Ud, g, dt)
        e.front2vof(C)
        step += 1
    st0 = e.stats(C)
    torch.cuda.synchronize()

    ev = []   # (kind, start, end)
    t0 = time.perf_counter()
    for _ in range(K):
        g = I.deformation_time_factor(step * dt, T_end)
        for d in range(3):
            s_ev = torch.cuda.Event(enable_timing=True)
            e_ev = torch.cuda.Event(enable_timing=True)
            s_ev.record(stream)
            e.sweep(d, Ud[d], g, dt)
            e_ev.record(stream)
            ev.append(("sweep", s_ev, e_ev))
        s_ev = torch.cuda.Event(enable_timing=True)
        e_ev = torch.cuda.Event(enable_timing=True)
        s_ev.record(stream)
        e.front2vof(C)
        e_ev.record(stream)
        ev.append(("f2v", s_ev, e_ev))
        step += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = e.stats(C)
    wall = t1 - t0

    # interfacial cells at the start of each timed step
    n_start = st0["n_interfacial"] + (st1["n_interfacial_sum"] - st0["n_interfacial_sum"]) - st1["n_interfacial"]
    value = n_start / wall
    kt = {"sweep": [], "f2v": []}
    for kind, s_ev, e_ev in ev:
        kt[kind].append(s_ev.elapsed_time(e_ev) * 1e-3)
    tot = {k: sum(v) for k, v in kt.items()}
    dom = max(tot, key=tot.get)
    avg_dur = tot[dom] / len(kt[dom])
    units_per_launch = n_start / K          # interfacial cells per launch (step-start count)
    bytes_per_launch = BYTES[a.precision][dom] * units_per_launch
    achieved = bytes_per_launch / avg_dur / 1e9

    out = {
        "metric": "interfacial cell-updates/s (advect+Front2VOF), 256^3; vol err vs FP64",
        "value": value,
        "unit": "interfacial cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"deformation_{n}: sphere R=0.15 at 0.35, LeVeque field x cos(pi t/3), "
                               f"CFL 0.5, steps {W}..{W + K} of {period}",
                   "n": n, "precision": a.precision, "sweeps_per_step": 3},
        "roofline": {
            "kernel": "k_sweep" if dom == "sweep" else "k_f2v",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_unit": BYTES[a.precision][dom],
            "units_per_launch": units_per_launch,
            "avg_launch_us": avg_dur * 1e6,
        },
        "time_split_ms": {k: v * 1e3 for k, v in tot.items()},
        "interfacial_cells": {"start": st0["n_interfacial"], "end": st1["n_interfacial"],
                              "mean": n_start / K},
        "volume": {"start": st0["volume"] + st0["volume_comp"], "end": st1["volume"] + st1["volume_comp"]},
        "counters": {k: st1[k] for k in ("n_fallback", "n_multi", "n_cfl", "n_merged")},
        "band_bricks_per_sweep": (st1["n_active_cells"] - st0["n_active_cells"]) / 64.0 / (3 * K),
    }

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline(n, budget_s):
    """The oracle as it stands, on the host cores, on the first steps of the
    same workload (bounded by `budget_s` seconds of work)."""
    from oracle import oracle as O
    from paper_2509_26361_amd import inputs as I
    sh = I.sphere_shape(n)
    U = I.deformation_velocity(n)
    dt = 0.5 / n
    st = O.init(sh)
    O.f2v(st)
    cells = 0
    steps = 0
    t0 = time.perf_counter()
    while True:
        cells += O.count_interfacial(st)
        g = I.deformation_time_factor(steps * dt, 3.0)
        st, _ = O.step(st, U, g, dt)
        O.f2v(st)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 50:
            break
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cells / el, "unit": "interfacial cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {steps} steps of deformation_{n} (3 sweeps + Front2VOF each), {el:.1f} s"}


if __name__ == "__main__":
    main()
