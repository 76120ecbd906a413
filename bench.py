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
# surrogate 20 -> 128 -> 128 -> 1: multiply-adds per row of the forward pass;
# the gradient adds dW2, dh1 (128 x 128 each) and dW1 (20 x 128)
MLP_FWD_FLOP = 2 * (20 * 128 + 128 * 128 + 128)
MLP_GRAD_FLOP = MLP_FWD_FLOP + 2 * (2 * 128 * 128 + 20 * 128 + 128)
# algorithmic bytes per interfacial cell (FP64 / FP32 storage):
#   sweep: read s_x,s_y,s_z + flags + U_d, write s_x,s_y,s_z + flags
#   Front2VOF: read s_x,s_y,s_z + flags, write C
#   Front2VOF with the next x sweep (one launch): both
BYTES = {
    "fp64": {"sweep": 3 * 8 + 1 + 8 + 3 * 8 + 1, "f2v": 3 * 8 + 1 + 8},
    "fp32": {"sweep": 3 * 4 + 1 + 4 + 3 * 4 + 1, "f2v": 3 * 4 + 1 + 4},
}
for _b in BYTES.values():
    _b["fused"] = _b["sweep"] + _b["f2v"]
# launch kinds timed by the library: kernel name (traffic key), description
KERNELS = {
    "sweep": ("k_sweep", "k_sweep (ebit_advect_sweep)"),
    "f2v": ("k_f2v", "k_f2v (ebit_front2vof)"),
    "fused": ("k_f2v_sweep_x", "k_f2v_sweep_x (ebit_advance: Front2VOF + next x sweep)"),
}


def launch_times(tm):
    """(timed launches, seconds) per launch kind from Ebit.timing()."""
    return {"sweep": (tm["sweeps"], tm["sweep_ms"] * 1e-3), "f2v": (tm["f2v"], tm["f2v_ms"] * 1e-3),
            "fused": (tm["fused"], tm["fused_ms"] * 1e-3)}


def roofline_of(kind, kt, units, precision, window):
    """Roofline entry of one launch kind: algorithmic bytes (per interfacial
    cell x cells per launch) over its mean launch duration from HIP events;
    `traffic` (HBM bytes per launch from counters) only when the counters
    were taken on this same window of this workload with these kernels."""
    cnt, secs = kt[kind]
    avg_dur = secs / max(1, cnt)
    achieved = BYTES[precision][kind] * units / avg_dur / 1e9 if cnt else None
    return {"kernel": KERNELS[kind][1], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if cnt else None,
            "traffic": stored_traffic(KERNELS[kind][0], window),
            "bytes_per_unit": BYTES[precision][kind], "units_per_launch": units,
            "avg_launch_us": avg_dur * 1e6 if cnt else None, "timed_launches": cnt,
            "window": window}


def roofline(kt, units, precision, window):
    """The dominant launch kind (largest timed total) and every kind."""
    tot = {k: v[1] for k, v in kt.items()}
    dom = max(tot, key=tot.get)
    kinds = {k: roofline_of(k, kt, units, precision, window) for k in kt if kt[k][0]}
    return roofline_of(dom, kt, units, precision, window), kinds


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=16)
    p.add_argument("--workload", default="deformation", choices=["deformation", "mixed", "tables"],
                   help="deformation: the 256^3 deformation test (the default line); mixed: 512^3, 4096 random "
                        "spheres in a random divergence-free field, 100 steps; tables: the paper's convergence "
                        "studies (translation and deformation, N = 32..256, CFL 0.125) with their errors")
    p.add_argument("--n", type=int, default=256)
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp32", action="store_true", help="skip the FP32 precision-form run")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-surrogate", action="store_true", help="skip training / running the learned Front2VOF")
    p.add_argument("--no-accuracy", action="store_true",
                   help="skip the untimed whole-period runs (errors of FP64, FP32 and FP32 + surrogate at T)")
    p.add_argument("--surr-rows", type=int, default=10_000_000, help="training rows (unambiguous cells)")
    p.add_argument("--surr-steps", type=int, default=20000, help="Adam steps")
    p.add_argument("--surr-batch", type=int, default=8192)
    p.add_argument("--timing-every", type=int, default=0,
                   help="in the bracketed pass, every k-th launch of each kind gets HIP events (the roofline's "
                        "durations); 0: every launch (deformation), or k so that at least 16 launches of each "
                        "kind are bracketed (mixed)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device copy of MIB MiB (float32 read + write), for scaling "
                        "memory-traffic counters, and exit")
    return p.parse_args()


def kernel_source_hash():
    """sha256 of the hot-path kernel sources: a stored traffic figure applies
    only to the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("ebit.hip", "ebit_device.h"):
        with open(os.path.join(ROOT, "paper_2509_26361_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def window_name(workload, precision, warmup, steps):
    """The step window a measurement covers, e.g. deformation_256_fp64_steps5-25."""
    return f"{workload}_{precision}_steps{warmup}-{warmup + steps}"


def stored_traffic(kernel, window):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this exact window (profiles/traffic_<window>.md: FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy), or None when there is none or the
    kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{window}.md")
    if not os.path.exists(path):
        return None
    sha = kernel_source_hash()
    for line in open(path):
        f = line.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == kernel and f[3] == "sha256":
            return float(f[2]) if f[4] == sha else None
    return None


def run_case(E, I, torch, n, precision, W, K, events, theta=None, every=8, keep=False):
    """W untimed steps, then K timed steps of the deformation workload
    (Front2VOF through the learned surrogate when `theta` is given)."""
    T_end = 3.0
    dt = 0.5 / n
    dev = torch.device("cuda:0")
    sh = I.sphere_shape(n)
    U = I.deformation_velocity(n)
    tdev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    Ud = [tdev(u).to(dtype) for u in U]
    e = E.Ebit(n, precision, dev)
    e.init(tdev(sh.phi_nodes), [tdev(f) for f in sh.phi_faces])
    del sh
    if theta is not None:
        e.set_surrogate(theta)
    C = torch.zeros((n, n, n), dtype=dtype, device=dev)
    e.front2vof(C)
    C0 = C.clone()
    gvals = [I.deformation_time_factor(k * dt, T_end) for k in range(W + K)]
    e.advance(Ud, gvals[:W], dt, C)
    st0 = e.stats(C)
    e.set_option(E.EBIT_OPT_TIMING, every if events else 0)
    e.timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.advance(Ud, gvals[W:], dt, C)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = e.timing()
    st1 = e.stats(C)
    n_start = st0["n_interfacial"] + (st1["n_interfacial_sum"] - st0["n_interfacial_sum"]) - st1["n_interfacial"]
    kt = launch_times(tm)
    out = {"wall": wall, "n_start": n_start, "st0": st0, "st1": st1, "kt": kt}
    if keep:
        out["ebit"], out["C"] = e, C
    return out


# algorithmic bytes per cell of the coupling kernels (full grid, FP64):
#   curvature: read C, write kappa and the status byte; CSF: read C, kappa,
#   status, write the three face forces; refinement band: read the flags,
#   write the mask (and a byte per 4^3 brick)
COUPLING_BYTES = {"curvature": 8 + 8 + 1, "csf": 8 + 8 + 1 + 3 * 8, "refine_band": 1 + 1 + 1.0 / 64}


def coupling_kernels(E, torch, e, C, reps=20):
    """Mean durations of the coupling entry points on the state at the end of
    the timed steps (HIP events on the stream they run on), and their rate
    on the algorithmic bytes of the whole grid."""
    n = C.shape[0]
    stream = torch.cuda.current_stream()
    kap = torch.empty_like(C)
    status = torch.empty(C.shape, dtype=torch.uint8, device=C.device)
    work = torch.empty(E.lib().ebit_curvature_work_bytes(n), dtype=torch.uint8, device=C.device)
    F = [torch.empty_like(C) for _ in range(3)]
    flags = e.state()[0]
    rb_out = (torch.empty_like(flags), torch.empty((n // 4,) * 3, dtype=torch.uint8, device=C.device),
              torch.empty(4, dtype=torch.int64, device=C.device),
              torch.empty(E.lib().ebit_refine_work_bytes(n), dtype=torch.uint8, device=C.device))
    calls = {
        "curvature": lambda: E.curvature(C, kap, status, work),
        "csf": lambda: E.csf(C, kap, status, 0.0728, F),
        "refine_band": lambda: E.refine_band(flags, out=rb_out),
    }
    out = {}
    for name, f in calls.items():
        for _ in range(3):
            f()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            f()
        b.record(stream)
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / reps
        gbs = COUPLING_BYTES[name] * n ** 3 / (us * 1e-6) / 1e9
        out[name] = {"us": us, "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
                     "bytes_per_cell": COUPLING_BYTES[name]}
    st = status.cpu()
    out["curvature"]["cells"] = {"interfacial": int((st > 0).sum()), "height_function": int(((st == 1) | (st == 2)).sum()),
                                 "neighbour_mean": int((st == 3).sum()), "none": int((st == 4).sum())}
    return out


def accuracy_run(E, I, torch, n, precision, theta=None):
    """A whole period of the deformation workload (sec. 3.2, CFL 0.5), not
    timed: E_mass over every step and E_shape at T from ebit_errors, and C at
    T (float64) for comparisons between forms."""
    T_end = 3.0
    dt = 0.5 / n
    steps = int(round(T_end / dt))
    dev = torch.device("cuda:0")
    sh = I.sphere_shape(n)
    tdev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    Ud = [tdev(u).to(dtype) for u in I.deformation_velocity(n)]
    e = E.Ebit(n, precision, dev)
    e.init(tdev(sh.phi_nodes), [tdev(f) for f in sh.phi_faces])
    del sh
    if theta is not None:
        e.set_surrogate(theta)
    C0 = torch.zeros((n, n, n), dtype=dtype, device=dev)
    e.front2vof(C0)
    C = torch.zeros_like(C0)
    for k in range(steps):
        e.advance(Ud, [I.deformation_time_factor(k * dt, T_end)], dt, C)
        r = e.errors(C, C0, reset=(k == 0))
    st = e.stats(C)
    return {"E_mass": r["e_mass"], "E_shape": r["e_shape"], "volume_T": r["volume"], "volume_0": r["volume_ref"],
            "volume_change_at_T": (r["volume"] - r["volume_ref"]) / r["volume_ref"], "steps": steps,
            "max_courant": st["max_courant"], "n_fallback": st["n_fallback"], "C": C.double()}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library and this benchmark run on one GPU; several GPUs are not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    if a.copy_calibration:
        nel = a.copy_calibration * (1 << 20) // 4
        x = torch.ones(nel, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nel * 4, "bytes_written": nel * 4,
                                               "kernel": "elementwise multiply by 1 (3 launches)"}}))
        return
    from paper_2509_26361_amd import ebit as E
    from paper_2509_26361_amd import inputs as I
    if a.workload == "mixed":
        return run_mixed(a, E, I, torch)
    if a.workload == "tables":
        return run_tables(a, E, I, torch)

    n = a.n
    dt = 0.5 / n
    period = int(round(3.0 / dt))
    K = a.steps if a.steps is not None else period - a.warmup
    W = a.warmup
    every = a.timing_every or 1
    window = window_name(f"deformation_{n}", a.precision, W, K)
    print(f"[bench] deformation n={n} precision={a.precision} warmup={W} steps={K}", file=sys.stderr, flush=True)
    # the timed steps, launched back to back (no events between launches)
    r = run_case(E, I, torch, n, a.precision, W, K, events=False)
    wall, n_start, st0, st1 = r["wall"], r["n_start"], r["st0"], r["st1"]
    value = n_start / wall
    units_per_launch = n_start / K          # interfacial cells per launch (step-start count)
    # the same window again from the same initial state, launches bracketed with HIP events
    # (every `every`-th of each kind; the brackets hold back the next dispatch, so this pass is
    # slower as a whole and serves only the per-launch durations)
    rb = run_case(E, I, torch, n, a.precision, W, K, events=True, every=every, keep=True)
    assert rb["n_start"] == n_start, "the bracketed pass took a different path"
    kt = rb["kt"]
    coupling = coupling_kernels(E, torch, rb.pop("ebit"), rb.pop("C"))
    dom, kinds = roofline(kt, units_per_launch, a.precision, window)
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
        "roofline": dom,
        "roofline_by_launch": kinds,
        "launch_us": {k: (kt[k][1] / kt[k][0] * 1e6 if kt[k][0] else None) for k in kt},
        "timing_pass": {"ms_per_step_with_events": rb["wall"] / K * 1e3, "every": every,
                        "note": "second pass over the same steps from the same state with launches bracketed "
                                "by HIP events; its per-launch durations make the roofline"},
        "interfacial_cells": {"start": st0["n_interfacial"], "end": st1["n_interfacial"],
                              "mean": n_start / K},
        "volume": {"start": st0["volume"] + st0["volume_comp"], "end": st1["volume"] + st1["volume_comp"]},
        "counters": {k: st1[k] for k in ("n_fallback", "n_multi", "n_cfl", "n_merged", "n_annihilated",
                                         "n_ambig_faces", "max_courant")},
        "band_bricks_per_sweep": (st1["n_active_cells"] - st0["n_active_cells"]) / 64.0 / (3 * K),
        "coupling_kernels": coupling,
    }
    print(f"[bench] {a.precision}: {out['ms_per_step']:.3f} ms/step, {value:.3e} cells/s", file=sys.stderr, flush=True)
    del r
    torch.cuda.empty_cache()

    if a.precision == "fp64" and not a.no_accuracy:
        # the whole period, not timed: the method's errors and the forms' errors against FP64
        acc = {}
        ref = accuracy_run(E, I, torch, n, "fp64")
        C64 = ref.pop("C")
        acc["fp64"] = ref
        print(f"[bench] fp64 period: E_mass {ref['E_mass']:.3e} E_shape {ref['E_shape']:.3e}", file=sys.stderr,
              flush=True)
        C32 = None
        if not a.no_fp32:
            q = run_case(E, I, torch, n, "fp32", W, K, events=False)
            qb = run_case(E, I, torch, n, "fp32", W, K, events=True, every=every)
            out["fp32_form"] = {"value": q["n_start"] / q["wall"], "ms_per_step": q["wall"] / K * 1e3,
                                "launch_us": {k: (qb["kt"][k][1] / qb["kt"][k][0] * 1e6 if qb["kt"][k][0] else None)
                                              for k in qb["kt"]}}
            f = accuracy_run(E, I, torch, n, "fp32")
            C32 = f.pop("C")
            f.update(form_vs_fp64(f, ref, C32, C64))
            acc["fp32"] = f
            print(f"[bench] fp32 form: {out['fp32_form']['ms_per_step']:.3f} ms/step; volume error at T "
                  f"{f['volume_rel_err_vs_fp64']:.2e}", file=sys.stderr, flush=True)
            del q, qb
            torch.cuda.empty_cache()
        if not a.no_surrogate:
            theta, info = train_surrogate(E, I, torch, a)
            q = run_case(E, I, torch, n, "fp32", W, K, events=False, theta=theta)
            qb = run_case(E, I, torch, n, "fp32", W, K, events=True, theta=theta, every=every)
            sf = {"value": q["n_start"] / q["wall"], "ms_per_step": q["wall"] / K * 1e3,
                  "launch_us": {k: (qb["kt"][k][1] / qb["kt"][k][0] * 1e6 if qb["kt"][k][0] else None)
                                for k in qb["kt"]}, "training": info,
                  # the last Front2VOF's cells: computed by the network, and geometric ambiguous ones
                  "cells_last_front2vof": {"surrogate": q["st1"]["n_surrogate"], "ambiguous": q["st1"]["n_ambiguous"]}}
            g = accuracy_run(E, I, torch, n, "fp32", theta=theta)
            Cs = g.pop("C")
            g.update(form_vs_fp64(g, ref, Cs, C64))
            acc["fp32_surrogate"] = g
            if C32 is not None:
                # the marker state does not depend on C: both FP32 runs hold the same state at T,
                # so C differs only by the surrogate's error on the unambiguous interfacial cells
                mixed = (C32 > 0) & (C32 < 1)
                dC = (Cs - C32).abs()
                sf["vs_geometric_fp32"] = {
                    "ms_per_step_ratio": sf["ms_per_step"] / out["fp32_form"]["ms_per_step"],
                    "mean_abs_C_diff_interfacial": float(dC[mixed].mean()) if bool(mixed.any()) else 0.0,
                    "max_abs_C_diff": float(dC.max()),
                    "volume_rel_diff_at_T": abs(g["volume_T"] - acc["fp32"]["volume_T"]) / acc["fp32"]["volume_T"]}
            out["fp32_surrogate_form"] = sf
            print(f"[bench] fp32 + surrogate: {sf['ms_per_step']:.3f} ms/step; volume error at T "
                  f"{g['volume_rel_err_vs_fp64']:.2e}, E_shape ratio {g['e_shape_ratio_vs_fp64']:.4f}",
                  file=sys.stderr, flush=True)
            del q, qb
            torch.cuda.empty_cache()
        out["accuracy_full_period"] = acc

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def form_vs_fp64(f, ref, C, C64):
    """A precision form's errors at T against the FP64 run (targets: volume
    within 1e-5 relative, E_shape at most twice the FP64 one)."""
    return {"volume_rel_err_vs_fp64": abs(f["volume_T"] - ref["volume_T"]) / ref["volume_T"],
            "e_shape_ratio_vs_fp64": f["E_shape"] / ref["E_shape"],
            "max_abs_C_diff_vs_fp64": float((C - C64).abs().max())}


def train_surrogate(E, I, torch, a):
    """Learned Front2VOF: training rows from the method's own FP64 runs of
    seeded ellipsoids at 128^3, training on the GPU (bf16 matrix cores).
    Returns the parameters and a report."""
    from paper_2509_26361_amd import surrogate as SG
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    calls = [0]

    def log(msg):
        calls[0] += 1
        if calls[0] % 50 == 1:
            print(f"[bench] surrogate rows: {msg}", file=sys.stderr, flush=True)
    X, c = SG.make_dataset(n=128, shapes=100000, snapshots=6, seed=0, device=dev, max_rows=a.surr_rows, log=log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    m = X.shape[0]
    nval = max(1, m // 20)
    g = torch.Generator(device="cpu").manual_seed(7)
    perm = torch.randperm(m, generator=g).to(dev)
    Xv, cv = X[perm[:nval]], c[perm[:nval]]
    Xt, ct = X[perm[nval:]], c[perm[nval:]]
    del X, c, perm
    theta = torch.from_numpy(I.mlp_init(0).astype(np.float32)).to(dev)
    mae0, _ = SG.evaluate(theta, Xv, cv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta = SG.train(Xt, ct, steps=a.surr_steps, batch=a.surr_batch, lr=2e-3, seed=0, theta=theta,
                     log=lambda msg: print(f"[bench] surrogate {msg}", file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    bias0 = float((E.mlp_forward(theta, Xv) - cv).mean().item())
    # output-bias calibration on training rows (not the hold-out)
    theta, shift = SG.calibrate_bias(theta, Xt[:1_000_000], ct[:1_000_000])
    mae, mx = SG.evaluate(theta, Xv, cv)
    bias = float((E.mlp_forward(theta, Xv) - cv).mean().item())
    # gradient kernel alone, timed with HIP events on its stream
    tr = E.MlpTrainer(theta.clone(), dev)
    xb, cb = Xt[:a.surr_batch].contiguous(), ct[:a.surr_batch].contiguous()
    stream = torch.cuda.current_stream()
    for _ in range(5):
        tr.gradient(xb, cb)
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record(stream)
    reps = 50
    for _ in range(reps):
        tr.gradient(xb, cb)
    e_ev.record(stream)
    torch.cuda.synchronize()
    grad_s = s_ev.elapsed_time(e_ev) * 1e-3 / reps
    fwd_rows = Xv
    s_ev.record(stream)
    for _ in range(reps):
        E.mlp_forward(theta, fwd_rows)
    e_ev.record(stream)
    torch.cuda.synchronize()
    fwd_s = s_ev.elapsed_time(e_ev) * 1e-3 / reps
    del Xt, ct, tr
    torch.cuda.empty_cache()
    info = {
        "rows": m, "holdout_rows": nval, "dataset_s": t_data, "train_s": t_train,
        "steps": a.surr_steps, "batch": a.surr_batch,
        "holdout_mae": mae, "holdout_max_err": mx, "holdout_bias": bias, "untrained_mae": mae0,
        "holdout_bias_before_calibration": bias0, "calibration_shift": shift,
        "train_us_per_step": t_train / a.surr_steps * 1e6,
        "gradient_us": grad_s * 1e6,
        "gradient_tflops": MLP_GRAD_FLOP * a.surr_batch / grad_s / 1e12,
        "forward_rows_per_s": nval / fwd_s,
        "forward_tflops": MLP_FWD_FLOP * nval / fwd_s / 1e12,
        "bf16_mfma_peak_tflops": 2500.0,
    }
    return theta, info


def mixed_case(E, I, torch, n, precision, W, K, phi, pf, U64, every, theta=None):
    """W untimed and K timed steps of the mixed workload (steady field, g = 1)."""
    dev = torch.device("cuda:0")
    dtype = torch.float64 if precision == "fp64" else torch.float32
    Ud = [u.to(dtype) for u in U64]
    dt = 0.5 / n
    e = E.Ebit(n, precision, dev)
    e.init(phi, pf)
    if theta is not None:
        e.set_surrogate(theta)
    C = torch.zeros((n, n, n), dtype=dtype, device=dev)
    e.front2vof(C)
    e.advance(Ud, [1.0] * W, dt, C)
    st0 = e.stats(C)
    e.set_option(E.EBIT_OPT_TIMING, every)
    e.timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.advance(Ud, [1.0] * K, dt, C)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = e.timing()
    st1 = e.stats(C)
    n_start = st0["n_interfacial"] + (st1["n_interfacial_sum"] - st0["n_interfacial_sum"]) - st1["n_interfacial"]
    res = {"wall": wall, "n_start": n_start, "st0": st0, "st1": st1, "C": C,
           "kt": launch_times(tm)}
    del e, Ud
    return res


def run_mixed(a, E, I, torch):
    """The large mixed run: 512^3, 4096 seeded non-overlapping spheres with
    radii U(3, 12) cells (surfaces at least 2 cells apart), a seeded
    divergence-free random Fourier field (8 modes per component, max |u| = 1),
    CFL 0.5, FP64; the FP32 form and the FP32 form with the surrogate are
    compared with it."""
    n, dev = 512, torch.device("cuda:0")
    K = a.steps if a.steps is not None else 100
    W = a.warmup
    log = lambda msg: print(f"[bench] mixed: {msg}", file=sys.stderr, flush=True)
    log("placing spheres")
    cs, rs = I.random_nonoverlapping_spheres(4096, 3.0, 12.0, n, gap_cells=2.0, seed=0)
    log(f"{len(rs)} spheres; sampling phi")
    sh = I.spheres_shape(n, cs, rs, with_s=False)
    phi = torch.from_numpy(sh.phi_nodes).to(dev)
    pf = [torch.from_numpy(f).to(dev) for f in sh.phi_faces]
    del sh
    U = I.fourier_velocity_device(n, seed=1, modes=8, device=dev)
    log("fp64 run")
    every = a.timing_every or 1
    window = window_name("mixed_512", "fp64", W, K)
    r = mixed_case(E, I, torch, n, "fp64", W, K, phi, pf, U, 0)
    log("fp64 run, launches bracketed by events")
    rb = mixed_case(E, I, torch, n, "fp64", W, K, phi, pf, U, every)
    assert rb["n_start"] == r["n_start"], "the bracketed pass took a different path"
    kt = rb["kt"]
    wall_events = rb["wall"]
    del rb
    torch.cuda.empty_cache()
    units = r["n_start"] / K
    V64 = r["st1"]["volume"] + r["st1"]["volume_comp"]
    out = {
        "metric": "interfacial cell-updates/s (advect+Front2VOF), 512^3 mixed run; vol err vs FP64",
        "value": r["n_start"] / r["wall"],
        "unit": "interfacial cell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": r["wall"] / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"mixed_512: {len(rs)} random spheres r U(3,12) cells, gap 2 cells, random "
                               f"divergence-free Fourier field (8 modes/component, max|u| = 1), CFL 0.5, "
                               f"steps {W}..{W + K}", "n": n, "precision": "fp64", "sweeps_per_step": 3},
        "roofline": roofline(kt, units, "fp64", window)[0],
        "roofline_by_launch": roofline(kt, units, "fp64", window)[1],
        "launch_us": {k: (kt[k][1] / kt[k][0] * 1e6 if kt[k][0] else None) for k in kt},
        "timing_pass": {"ms_per_step_with_events": wall_events / K * 1e3, "every": every},
        "interfacial_cells": {"start": r["st0"]["n_interfacial"], "end": r["st1"]["n_interfacial"], "mean": units},
        "volume": {"start": r["st0"]["volume"] + r["st0"]["volume_comp"], "end": V64},
        "counters": {k: r["st1"][k] for k in ("n_fallback", "n_multi", "n_cfl", "n_merged", "n_annihilated",
                                              "n_ambig_faces")},
    }
    C64 = r["C"]
    del r
    torch.cuda.empty_cache()
    forms = []
    if not a.no_fp32:
        forms.append(("fp32_form", None))
    if not a.no_surrogate:
        theta, info = train_surrogate(E, I, torch, a)
        forms.append(("fp32_surrogate_form", (theta, info)))
    for name, surr in forms:
        log(name)
        q = mixed_case(E, I, torch, n, "fp32", W, K, phi, pf, U, 0,
                       theta=surr[0] if surr else None)
        V = q["st1"]["volume"] + q["st1"]["volume_comp"]
        out[name] = {"value": q["n_start"] / q["wall"], "ms_per_step": q["wall"] / K * 1e3,
                     "launch_us": {k: (q["kt"][k][1] / q["kt"][k][0] * 1e6 if q["kt"][k][0] else None)
                                   for k in q["kt"]},
                     "volume_rel_err_vs_fp64": abs(V - V64) / V64,
                     "max_abs_C_diff_vs_fp64": float((q["C"].double() - C64).abs().max())}
        if surr:
            out[name]["ambiguous_cells_end"] = q["st1"]["n_ambiguous"]
            out[name]["surrogate_cells_end"] = q["st1"]["n_surrogate"]
            out[name]["training"] = surr[1]
        del q
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


# the paper's mesh-convergence studies (sec. 3.1.2 Table 2, sec. 3.2 Table 3)
PAPER_TABLES = {
    "translation": {"N": [32, 64, 128, 256], "E_mass": [5.03e-4, 6.13e-5, 1.35e-5, 2.81e-6],
                    "E_shape": [1.56e-3, 3.68e-4, 1.25e-4, 2.95e-5]},
    "deformation": {"N": [32, 64, 128, 256], "E_mass": [3.06e-1, 9.78e-2, 3.22e-3, 1.49e-3],
                    "E_shape": [5.66e-1, 2.23e-1, 3.82e-2, 1.58e-2]},
}


def table_case(E, I, torch, case, n, precision="fp64"):
    """One convergence run on the GPU: translation (sphere R = 0.15 at 0.25,
    u = (1,1,1) reversed at T/2, T = 1) or deformation (sphere at 0.35,
    LeVeque's field x cos(pi t/3), T = 3), CFL 0.125; E_mass from the volume
    after every step, E_shape at T (ebit_errors)."""
    dev = torch.device("cuda:0")
    dtype = torch.float64 if precision == "fp64" else torch.float32
    tdev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev).to(dtype)
    if case == "translation":
        sh, U, T = I.sphere_shape(n, centre=(0.25, 0.25, 0.25)), I.uniform_velocity(n), 1.0
    else:
        sh, U, T = I.sphere_shape(n), I.deformation_velocity(n), 3.0
    dt = 0.125 / n
    steps = int(round(T / dt))
    e = E.Ebit(n, precision, dev)
    e.init(tdev(sh.phi_nodes).double(), [tdev(f).double() for f in sh.phi_faces])
    Ud = [tdev(u) for u in U]
    C0 = torch.zeros((n, n, n), dtype=dtype, device=dev)
    e.front2vof(C0)
    C = torch.zeros_like(C0)
    t0 = time.perf_counter()
    for k in range(steps):
        if case == "translation":
            g = 1.0 if k < steps // 2 else -1.0
        else:
            g = I.deformation_time_factor(k * dt, T)
        e.advance(Ud, [g], dt, C)
        r = e.errors(C, C0, reset=(k == 0))
    wall = time.perf_counter() - t0
    st = e.stats(C)
    return {"N": n, "steps": steps, "E_mass": r["e_mass"], "E_shape": r["e_shape"],
            "volume_change_at_T": (r["volume"] - r["volume_ref"]) / r["volume_ref"],
            "max_courant": st["max_courant"], "n_merged": st["n_merged"], "n_multi": st["n_multi"],
            "n_fallback": st["n_fallback"], "wall_s": wall}


def run_tables(a, E, I, torch):
    """Both convergence studies at N = 32, 64, 128, 256 against the paper's
    printed errors (context: the same algorithm's readings, not a target)."""
    out = {"workload": "paper convergence studies, CFL 0.125, FP64", "precision": a.precision, "cases": {}}
    for case in ("translation", "deformation"):
        rows = []
        for n, pm, ps in zip(PAPER_TABLES[case]["N"], PAPER_TABLES[case]["E_mass"], PAPER_TABLES[case]["E_shape"]):
            r = table_case(E, I, torch, case, n, a.precision)
            r["paper_E_mass"], r["paper_E_shape"] = pm, ps
            r["ratio_E_mass"], r["ratio_E_shape"] = r["E_mass"] / pm, r["E_shape"] / ps
            print(f"[bench] {case} N={n}: E_mass {r['E_mass']:.3e} (paper {pm:.2e}), "
                  f"E_shape {r['E_shape']:.3e} (paper {ps:.2e}), {r['wall_s']:.1f} s", file=sys.stderr, flush=True)
            rows.append(r)
            torch.cuda.empty_cache()
        out["cases"][case] = rows
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
