"""Benchmark: cell-stage updates per second of the WENO-3 residual inside
SSP-RK3 steps on one MI355X, with the roofline of the dominant kernel (the
reconstruction, bound by FP32 vector arithmetic), the HBM fraction of the
whole stage, and the oracle timed on the host as a baseline.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c5|c4|c2q|c2t|c3|c1]
                [--precision fp32|fp64] [--no-cpu-baseline] [--no-check]

A step is one full SSP-RK3 step: the CFL time step, then three stages of
reconstruction, flux, residual gather and stage combination, all on the
device.  Steps are issued as calls of several steps each (one captured
graph per call), inside which each step's last flux launch also forms the
next step's CFL bound.  Inputs are synthetic (seeded meshes and
closed-form initial data) and resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# FP32 vector peak without packed FP32 instructions: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz x 2 (an FMA counts as two flops).  The published 157.3
# TFLOP/s needs two FP32 operations per lane per cycle (packed FP32), which
# this library does not emit.
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
PEAK_FP32_PUBLISHED = 157.3
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_recon_mixed16M_fp32.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1712_08317_amd", "csrc", "kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic bytes of the reconstruction kernel per cell (minimal table
# representation, one linear weight per Gauss point and candidate): stencil
# indices 4(S-1), Gauss-point offsets 4n, candidate operators 4M and linear
# weights 2nM values of p bytes, and the cell's own state V * 8 bytes.  The
# split sums the kernel also reads (3 per Gauss point) and the face states it
# writes for the flux kernel are implementation traffic and are not counted.
def recon_bytes(nf, p, nvar):
    S, M = (13, 12) if nf == 4 else (10, 9)
    return 4 * (S - 1) + p * (4 * nf + 4 * M + 2 * nf * M) + nvar * 8


# Whole cell-stage (both kernels): recon bytes plus the face table (3n
# values + 4 bytes of pairing) and the state traffic of the stage
# combination: W_in read, W_out written, W^n read in two of three stages.
def stage_bytes(nf, p, nvar):
    return recon_bytes(nf, p, nvar) - nvar * 8 + 4 + p * 3 * nf + (8 / 3) * nvar * 8


# Algorithmic flops of the WENO reconstruction per cell, counted on the
# formulas of Sec. 3.4 (an add, multiply or division is one flop, a fused
# multiply-add two, |.| none): differences to the stencil cells (S-1)V;
# candidate gradients Y_j dW (6) and beta_j = |g_j|^2 (3) per (j, v); per
# Gauss point and candidate the split gamma~+- = ((gamma + theta|gamma|)/2,
# gamma~+ - gamma) (4), their sums (2) and normalisation (2), plus the two
# reciprocals of sigma+- (the kernel takes the sums, which depend on the mesh
# only, from the precompute and does less); per (Gauss point, j, v) the
# candidate value
# d = ox gx + oy gy (3) and, for each sign, t = gamma~ beta (1), 1 + t + t^2
# (3), beta (.) + eps (2), its square (1), alpha = gamma~ / (.)^2 (1),
# sum alpha d (2), sum alpha (1); per (Gauss point, v) the two ratios (2),
# the sigma scalings (2), their difference (1) and the increment (1).
#
# Characteristic variables (Sec. 4, Euler): per face the Roe mean and the two
# eigenvector matrices (80, counting a square root or division as one), per
# face and field the projected differences (S-1) x 7, gradients, indicators
# and eps (10 per candidate); per Gauss point the projection back (4 x 8).
def recon_flops(nf, nvar, characteristic=False):
    S, M = (13, 12) if nf == 4 else (10, 9)
    G = 2 * nf
    per_sign = 1 + 3 + 2 + 1 + 1 + 2 + 1
    common = G * (8 * M + 2) + G * M * nvar * (3 + 2 * per_sign) + G * nvar * 6
    if characteristic and nvar == 4:
        return ((S - 1) * nvar + common + nf * (80 + nvar * ((S - 1) * 7 + 10 * M))
                + G * nvar * 8)
    return (S - 1) * nvar + 9 * M * nvar + common


def l1_errors(a, b):
    """Relative L1 differences of a state a against a reference b ([V, n]):
    per variable sum|a - b| / sum|b|, their maximum, and the whole state
    sum over variables and cells of |a - b| over that of |b|."""
    num = np.abs(a - b).sum(1)
    den = np.abs(b).sum(1)
    per = num / den
    return {"max_over_variables": float(per.max()), "per_variable": [float(x) for x in per],
            "state": float(num.sum() / den.sum())}


def committed_traffic():
    """HBM bytes per reconstruction pass (both cell-type launches) from the
    committed FETCH_SIZE / WRITE_SIZE profile, or None when the kernel source
    has changed since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    try:
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if fields.get("kernels.hip sha256") != sha:
            return None
        return float(fields["traffic bytes per pass"])
    except (KeyError, ValueError, OSError):
        return None


def make_workload(name):
    import workloads as wl
    if name == "c5":
        return wl.mesh_c5(), "c5", "mixed 3264x3264 squares on [0,2]^2, 64x64 checkerboard, 30% jitter, periodic; density wave x vortex"
    if name == "c2q":
        return wl.mesh_c2q(), "c2q", "400x400 quads on [0,2]^2, 20% jitter, periodic; density wave"
    if name == "c2t":
        return wl.mesh_c2t(), "c2t", "283x283x2 triangles on [0,2]^2, 20% jitter, periodic; density wave"
    if name == "c3":
        return wl.mesh_c3(), "c3", "1340x1340 squares on [0,1]^2 with a triangle band, 15% jitter, transmissive; rotated Sod"
    if name == "c1":
        return wl.mesh_c1(), "c1", "20x20x2 triangles on [0,2]^2, 10% jitter, periodic; scalar density wave"
    raise SystemExit(f"unknown config {name}")


def cpu_baseline(seconds_hint=20.0):
    """The oracle (FP64 NumPy, as it stands) on a bounded sample of the same
    workload kind: a 128x128-square mixed periodic mesh with the same block
    checkerboard, jitter and initial data, one residual per stage of
    SSP-RK3 steps until about ``seconds_hint`` seconds have passed."""
    import workloads as wl
    from oracle import weights as ow
    from oracle import scheme as osc
    import contextlib
    try:
        from threadpoolctl import threadpool_limits
        one_thread = threadpool_limits(1)     # NumPy's BLAS and OpenMP pools
    except ImportError:
        one_thread = contextlib.nullcontext()
    mesh = wl.mesh_c5(n=128, block=64, jitter=0.30, seed=6)
    T = ow.precompute(mesh)
    W = wl.initial_state("c5", mesh)
    ph = osc.Physics("euler")
    dt = osc.cfl_dt(T, W, ph, 0.5)
    with one_thread:
        c0 = os.times()
        t0 = time.perf_counter()
        steps = 0
        while True:
            W = osc.rk3_step(T, W, ph, dt)
            steps += 1
            el = time.perf_counter() - t0
            if el > seconds_hint or steps >= 50:
                break
        c1 = os.times()
    busy = (c1.user - c0.user + c1.system - c0.system) / el   # CPU seconds per second
    rate = mesh.n_cells * 3 * steps / el
    return {"value": rate, "unit": "cell-stage updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle rk3 on a {mesh.n_cells}-cell mixed mesh (128x128 squares, "
                      f"64x64 checkerboard, 30% jitter), {steps} steps, {el:.1f} s, one thread "
                      f"(thread pools limited to 1; {busy:.2f} CPU-s per s measured)"}


def copy_bandwidth():
    """Achievable HBM rate on this device: a 1 GiB device-to-device copy
    (bytes read plus bytes written over the time), median of five after a
    warm-up copy, timed with events on torch's stream (the copy runs there)."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ms = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / (sorted(ms)[2] * 1e-3) / 1e9


def host_cores():
    """CPUs this process may run on (its affinity mask), capped at the
    box's CPU share of one GPU (16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_worker(seconds_hint):
    """One oracle instance of the CPU baseline's sample, run in a child
    process (``--cpu-worker``): prints its step count and time as JSON."""
    r = cpu_baseline(seconds_hint)
    print(json.dumps({"rate": r["value"], "sample": r["sample"]}), flush=True)


def cpu_baseline_all_cores(seconds_hint=20.0):
    """The same oracle on every host core at once: one independent oracle
    instance of the sample per core, each in its own child process with
    one thread (the oracle has no parallel decomposition of one mesh; the
    host's aggregate throughput on the workload is the sum of the
    instances' rates over the same window)."""
    import subprocess
    n = host_cores()
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker",
                               str(seconds_hint)], stdout=subprocess.PIPE, env=env, text=True)
             for _ in range(n)]
    rates = []
    for pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"cpu baseline worker failed with status {pr.returncode}")
        rates.append(json.loads(out.strip().splitlines()[-1])["rate"])
    return {"value": float(sum(rates)), "unit": "cell-stage updates/s", "cores": n,
            "kind": "oracle",
            "sample": f"{n} concurrent single-thread processes, each the oracle rk3 on the "
                      f"24576-cell mixed mesh (128x128 squares, 64x64 checkerboard, 30% "
                      f"jitter) for about {seconds_hint:.0f} s; value = sum of their rates "
                      f"(per process {min(rates):.3g} to {max(rates):.3g})"}


def run_batch(args):
    """The 256-instance batch: every instance advanced by the same graph-
    captured launches, each with its own CFL time step.  Prints one JSON
    line (no per-kernel roofline: the launches run inside a graph)."""
    import torch
    import workloads as wl
    import paper_1712_08317_amd as uw

    t0 = time.perf_counter()
    meshes = [wl.mesh_c4(k) for k in range(256)]
    Ms = [uw.Mesh.from_workload(m, device=0) for m in meshes]
    for M in Ms:
        M.precompute()
    states = [wl.initial_state("c2q", m, q=2) for m in meshes]
    ncell = sum(m.n_cells for m in meshes)
    nq = sum(M.n_quads for M in Ms)
    del meshes
    log(f"256 instances, {ncell} cells, set up in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    prec = uw.UW_FP32 if args.precision == "fp32" else uw.UW_FP64
    ph = uw.make_physics(uw.UW_EULER, 1.0, 1.0, 1.4, prec)
    B = uw.Batch(Ms, ph)
    B.autotune(ph)
    W0 = B.to_internal(states)
    W = torch.from_numpy(W0).to(dev)
    t = torch.zeros(256, dtype=torch.float64, device=dev)
    # steps go in calls of `chunk` steps (one captured graph per call); the
    # first warm-up call captures it, the timed calls replay it
    chunk = max(c for c in (10, 5, 4, 2, 1) if args.steps % c == 0 and c <= max(args.warmup, 1))

    def warm(b, Wd, td):
        if args.warmup == 0:
            return
        b.rk3_step(Wd, td, cfl=0.5, n_steps=chunk)
        for _ in range(args.warmup - chunk):
            b.rk3_step(Wd, td, cfl=0.5, n_steps=1)
        torch.cuda.synchronize()

    def timed_steps(b, Wd, td):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps // chunk):
            b.rk3_step(Wd, td, cfl=0.5, n_steps=chunk)
        torch.cuda.synchronize()
        return time.perf_counter() - a

    warm(B, W, t)
    B.check()
    el = timed_steps(B, W, t)
    B.check()
    err = None
    fp64 = None
    if not args.no_check and prec == uw.UW_FP32:
        ph64 = uw.make_physics(uw.UW_EULER, 1.0, 1.0, 1.4, uw.UW_FP64)
        B64 = uw.Batch(Ms, ph64)
        B64.autotune(ph64)
        W64 = torch.from_numpy(W0).to(dev)
        t64 = torch.zeros(256, dtype=torch.float64, device=dev)
        warm(B64, W64, t64)
        el64 = timed_steps(B64, W64, t64)
        B64.check()
        fp64 = {"value": ncell * 3 * args.steps / el64, "ms_per_step": el64 / args.steps * 1e3}
        a = B.to_original(W.cpu().numpy())
        b = B64.to_original(W64.cpu().numpy())
        errs = [l1_errors(x, y) for x, y in zip(a, b)]
        err = max(errs, key=lambda e: e["max_over_variables"])
        log(f"fp32 vs fp64 relative L1, worst instance: {err}")
    p = 4 if prec == uw.UW_FP32 else 8
    sbytes = nq * stage_bytes(4, p, 4) + (ncell - nq) * stage_bytes(3, p, 4)
    stage_s = el / args.steps / 3
    out = {
        "metric": "cell-stage updates/s, FP32 vs FP64 at L1 err<=1e-5; % of HBM roofline",
        "value": ncell * 3 * args.steps / el, "unit": "cell-stage updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == uw.UW_FP32 else "f64", "data": "synthetic",
        "config": {"workload": "256 periodic density-wave instances, 2k-200k cells "
                               "log-uniform, quad or triangle, jitter 0-30%",
                   "cells": ncell, "quads": nq, "instances": 256, "state": "f64",
                   "rk3_steps": args.steps, "cfl": 0.5,
                   "graph": f"graph replays of {chunk}-step calls"},
        "roofline": None,
        "schedule": B.schedule(),
        "tile": B.tile_size(),
        "stage": {"algorithmic_bytes": sbytes, "ms": stage_s * 1e3,
                  "achieved_GBs": sbytes / stage_s / 1e9,
                  "hbm_frac": sbytes / stage_s / 1e9 / PEAK_HBM_GBS},
        "hbm_roofline_frac": sbytes / stage_s / 1e9 / PEAK_HBM_GBS,
        "fp64_value": None if fp64 is None else fp64["value"],
        "fp64_ms_per_step": None if fp64 is None else fp64["ms_per_step"],
        "host_cores": host_cores(),
        "fp32_vs_fp64_rel_l1": None if err is None else err["max_over_variables"],
        "fp32_vs_fp64_rel_l1_detail": err,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--variables", default="conserved", choices=["conserved", "characteristic"],
                    help="reconstruct the conserved or the characteristic variables (Euler)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 reference run")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library runs each "
              "mesh on a single device and has no multi-GPU decomposition.", file=sys.stderr)
        sys.exit(2)
    if args.config == "c4":
        run_batch(args)
        return

    import torch
    import workloads as wl
    import paper_1712_08317_amd as uw

    t0 = time.perf_counter()
    mesh, cname, desc = make_workload(args.config)
    log(f"mesh {cname}: {mesh.n_cells} cells ({time.perf_counter() - t0:.1f} s)")
    t1 = time.perf_counter()
    M = uw.Mesh.from_workload(mesh, device=0)
    log(f"upload/connectivity/stencils {time.perf_counter() - t1:.1f} s")
    t1 = time.perf_counter()
    char = args.variables == "characteristic"
    diag = M.precompute(uw.make_scheme(
        variables=uw.UW_CHARACTERISTIC if char else uw.UW_CONSERVED))
    log(f"FP64 precompute {time.perf_counter() - t1:.1f} s; max|gamma| raw "
        f"{diag['max_abs_gamma_raw']:.3g} opt {diag['max_abs_gamma_opt']:.3g}")
    eq = uw.UW_ADVECTION if cname == "c1" else uw.UW_EULER
    nvar = 1 if eq == uw.UW_ADVECTION else 4
    W0 = wl.initial_state(cname, mesh)
    W0i = M.to_internal(W0)
    del mesh
    dev = torch.device("cuda:0")
    prec = uw.UW_FP32 if args.precision == "fp32" else uw.UW_FP64
    phys = uw.make_physics(eq, 1.0, 1.0, 1.4, prec)
    W = torch.from_numpy(W0i).to(dev)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written")
        del a, b
    t1 = time.perf_counter()
    M.autotune(phys)
    tile = M.tile_size()
    sched = M.schedule()
    log(f"autotune {time.perf_counter() - t1:.1f} s; tile {tile}, schedule {sched}")
    # steps go in calls of `chunk` steps (one captured graph per call); the
    # first warm-up call captures it, the timed calls replay it
    chunk = max(c for c in (10, 5, 4, 2, 1) if args.steps % c == 0 and c <= max(args.warmup, 1))

    def warm(ph, Wd, td):
        if args.warmup == 0:
            return
        M.rk3_steps(ph, Wd, td, chunk, cfl=0.5)
        for _ in range(args.warmup - chunk):
            M.rk3_step(ph, Wd, td, cfl=0.5)
        torch.cuda.synchronize()

    def timed_steps(ph, Wd, td):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps // chunk):
            M.rk3_steps(ph, Wd, td, chunk, cfl=0.5)
        torch.cuda.synchronize()
        return time.perf_counter() - a

    warm(phys, W, t)
    M.check()
    el = timed_steps(phys, W, t)
    M.check()
    # the same number of steps again, launched one kernel at a time with HIP
    # events on the library's stream around each launch: per-kernel times
    M.profile(enable=1)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for k in range(args.steps // chunk):
        M.rk3_steps(phys, W, t, chunk, cfl=0.5)
    torch.cuda.synchronize()
    el_prof = time.perf_counter() - s0
    (rms, fms), (rn, fn) = M.profile(enable=0)
    M.check()
    log(f"timed {args.steps} steps in {el:.3f} s (graph replays of {chunk}-step calls); per-kernel pass "
        f"{el_prof:.3f} s: recon {rms / max(rn, 1):.3f} ms x {rn}, "
        f"flux {fms / max(fn, 1):.3f} ms x {fn}")

    N, Nq = M.n_cells, M.n_quads
    N_cells = N
    p = 4 if prec == uw.UW_FP32 else 8
    value = N * 3 * args.steps / el
    rbytes = Nq * recon_bytes(4, p, nvar) + (N - Nq) * recon_bytes(3, p, nvar)
    ravg = rms / max(rn, 1) / 1e3
    rflops = Nq * recon_flops(4, nvar, char) + (N - Nq) * recon_flops(3, nvar, char)
    achieved = rflops / ravg / 1e12
    hbm_achieved = rbytes / ravg / 1e9
    sbytes = Nq * stage_bytes(4, p, nvar) + (N - Nq) * stage_bytes(3, p, nvar)

    err = None
    fp64 = None
    if not args.no_check and prec == uw.UW_FP32:
        # the same steps in FP64 on the device: its throughput (timed like
        # the FP32 steps) and the FP32 result's error against it
        W64 = torch.from_numpy(W0i).to(dev)
        t64 = torch.zeros(1, dtype=torch.float64, device=dev)
        ph64 = uw.make_physics(eq, 1.0, 1.0, 1.4, uw.UW_FP64)
        M.autotune(ph64)          # FP64 stages use 256-cell tiles
        warm(ph64, W64, t64)
        el64 = timed_steps(ph64, W64, t64)
        for _ in range(args.steps // chunk):
            M.rk3_steps(ph64, W64, t64, chunk, cfl=0.5)
        torch.cuda.synchronize()
        M.check()
        fp64 = {"value": N_cells * 3 * args.steps / el64, "ms_per_step": el64 / args.steps * 1e3}
        a = W.cpu().numpy()
        b = W64.cpu().numpy()
        err = l1_errors(a, b)
        log(f"fp64: {fp64['value']:.3g} cell-stage/s; fp32 vs fp64 relative L1 after "
            f"{args.warmup + 2 * args.steps} steps: {err}")
        del W64

    base = None
    if not args.no_cpu_baseline:
        t1 = time.perf_counter()
        single = cpu_baseline()
        log(f"cpu baseline, one core: {single['value']:.3g} cell-stage/s "
            f"({time.perf_counter() - t1:.1f} s)")
        t1 = time.perf_counter()
        base = cpu_baseline_all_cores()
        base["one_core"] = {"value": single["value"], "cores": 1, "sample": single["sample"]}
        log(f"cpu baseline, {base['cores']} cores: {base['value']:.3g} cell-stage/s "
            f"({time.perf_counter() - t1:.1f} s)")

    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.0f} GB/s")
    traffic = committed_traffic()
    out = {
        "metric": "cell-stage updates/s, FP32 vs FP64 at L1 err<=1e-5; % of HBM roofline",
        "value": value,
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == uw.UW_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": N, "quads": Nq, "triangles": N - Nq,
                   "state": "f64", "rk3_steps": args.steps, "cfl": 0.5,
                   "variables": args.variables},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": (traffic if prec == uw.UW_FP32 and nvar == 4 and args.config == "c5"
                                 and not char else None),
                     "kernel": "k_recon (WENO reconstruction, both cell types; one pass = "
                               "one launch per cell type)",
                     "flops_per_launch": rflops, "avg_launch_ms": ravg * 1e3,
                     "peak_note": "FP32 vector without packed FP32; published 157.3",
                     "frac_of_published": achieved / PEAK_FP32_PUBLISHED,
                     "hbm": {"algorithmic_bytes": rbytes, "achieved_GBs": hbm_achieved,
                             "frac": hbm_achieved / PEAK_HBM_GBS}},
        "hbm_roofline_frac": sbytes / (el / args.steps / 3) / 1e9 / PEAK_HBM_GBS,
        "schedule": sched,
        "tile": tile,
        "stage": {"algorithmic_bytes": sbytes, "ms": el / args.steps / 3 * 1e3,
                  "achieved_GBs": sbytes / (el / args.steps / 3) / 1e9,
                  "hbm_frac": sbytes / (el / args.steps / 3) / 1e9 / PEAK_HBM_GBS,
                  "recon_ms": ravg * 1e3, "flux_ms": fms / max(fn, 1),
                  "timing": f"value: graph replays of {chunk}-step calls; per-kernel times: a "
                            "second pass of as many steps launched one kernel at a time with HIP "
                            "events",
                  "per_kernel_pass_ms_per_step": el_prof / args.steps * 1e3,
                  "copy_GBs": copy_gbs,
                  "frac_of_copy": sbytes / (el / args.steps / 3) / 1e9 / copy_gbs},
        "fp64_value": None if fp64 is None else fp64["value"],
        "fp64_ms_per_step": None if fp64 is None else fp64["ms_per_step"],
        "host_cores": host_cores(),
        "fp32_vs_fp64_rel_l1": None if err is None else err["max_over_variables"],
        "fp32_vs_fp64_rel_l1_detail": err,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
