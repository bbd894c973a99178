#!/usr/bin/env python3
"""Throughput of the Z-Model high-order step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one SSP-RK3 step: three evaluations of (surface derivatives ->
all-pairs Birkhoff-Rott sweep -> tie correction -> reduction -> RK3 stage),
each evaluation doing N^2 pair interactions.  The default workload is the
1024 x 1024 (1,048,576-point) sixteen-mode interface with FP32 pair
interactions and FP64 state, sums and RK3.  Inputs are seeded synthetic
rocket-rig interfaces resident in HBM before the timed region.

The last stdout line is one JSON object: the throughput, the pair kernel's
place on its VALU roofline (timed with HIP events inside the library, on the
stream it launches on) with the FP64 form of the same 1M-point sweep beside
it, the CPU oracle timed on a bounded sample of the same workload, and short
summaries of the other measurements (the five-step trajectory against the
FP64 path and the oracle, the 256 x 256 FP64 run, the 64 x 64 trajectory,
the 64-member ensemble, the served request stream).  Progress lines come
before it; --detail-out writes every measured figure to a JSON file.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import rocket_rig as rr  # noqa: E402

METRIC = "BR pair-interactions/s & % VALU peak (FP32 vs FP64); served p50/p99 step ms"
# Algorithmic work of one pair in the direct form (the roofline unit): r (3
# sub), |r|^2 + eps^2 (3 FMA), rsqrt (1), cube (2 mul), w gamma (3 mul),
# r x (w gamma) accumulated (6 FMA), an FMA counted as 2 flop.  The kernels'
# factored far form executes fewer operations per pair; the flop they do
# execute is read from the committed VALU counters (executed_flops_per_pair).
FLOPS_PER_PAIR = 27
PEAK_TFLOPS = {"fp64": 78.6, "fp32_pairs": 157.3}   # MI355X vector peaks
DEFAULT_WORKLOAD = "periodic1024_multimode16_fp32"


def log(msg: str):
    """Progress line on stdout (the JSON result is always the last line)."""
    print(f"[bench] {msg}", flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed RK3 steps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(rr.WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample (0 = skip)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="time the workload's RK3 steps only (no precision sweep, trajectory "
                         "checks, ensemble or model sections)")
    ap.add_argument("--no-sections", action="store_true",
                    help="skip the cutoff, low-order, medium-order and free-sheet sections")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the served stream (0 = skip serving)")
    ap.add_argument("--serve-max-seconds", type=float, default=420.0,
                    help="stop serving after this long even if requests remain")
    ap.add_argument("--detail-out", default=None, metavar="PATH",
                    help="also write every measured figure to this JSON file")
    ap.add_argument("--tune-report", action="store_true",
                    help="only autotune the pair kernel for a range of mesh sides and print "
                         "the choice table (default shape vs tuned)")
    ap.add_argument("--cutoff-only", action="store_true",
                    help="only measure the cutoff solver (paper workloads, accuracy curve)")
    ap.add_argument("--low-order-only", action="store_true",
                    help="only measure the low-order (FFT) model at 4096 x 4096")
    ap.add_argument("--medium-only", action="store_true",
                    help="only measure the medium-order model against the high-order one")
    ap.add_argument("--free-only", action="store_true",
                    help="only measure the non-periodic single-mode case (exact, cutoff, "
                         "far-field check)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only measure the 64-member ensemble")
    ap.add_argument("--serve-only", action="store_true",
                    help="only serve the request stream")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def sig(x, digits: int = 4):
    """Floats rounded to a few significant digits, recursively (for the
    one-line summary)."""
    if isinstance(x, float):
        if x == 0.0 or not math.isfinite(x):
            return x
        return float(f"{x:.{digits}g}")
    if isinstance(x, dict):
        return {k: sig(v, digits) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [sig(v, digits) for v in x]
    return x


def rel(a, b):
    """Normwise relative error max |a - b| / max |b|."""
    den = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


PAIR_KERNEL_SOURCES = ("zm_device.h", "zm_internal.h", "zm_kernels.hip")


def code_only(text: str) -> str:
    """C/C++ source with comments removed and whitespace runs collapsed, so
    that comment and layout edits leave it unchanged (string and character
    literals are kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def library_source_hash() -> str:
    """SHA-256 over the code (comments and whitespace runs removed) of the
    sources that define the single-instance pair kernels (name, then code,
    in this order)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2406_05490_amd", "csrc")
    for f in PAIR_KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()


def measured_counters(kernel: str, workload: str):
    """The committed counter record of this kernel and workload
    (profiles/<kernel>_<workload>.counters.json: HBM bytes per launch from
    FETCH_SIZE / WRITE_SIZE scaled by a plain copy's reading, and VALU
    instructions per 64 pairs by kind), or None when there is none or the
    pair-kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel") != kernel or rec.get("workload") != workload:
        return None
    if rec.get("source_sha256") != library_source_hash():
        return None
    return rec


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter record, or None."""
    rec = measured_counters(kernel, workload)
    if rec is None or "read_bytes_per_launch" not in rec:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def executed_flops_per_pair(kernel: str, workload: str):
    """Flop the kernel executes per pair by the committed VALU counters:
    (2 FMA + MUL + ADD + TRANS) wave instructions per 64 pairs (each wave
    instruction is 64 lane operations), or None."""
    rec = measured_counters(kernel, workload)
    if rec is None or "valu_per_64_pairs" not in rec:
        return None
    v = rec["valu_per_64_pairs"]
    return 2.0 * v["fma"] + v["mul"] + v["add"] + v["trans"]


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))


def to_dev(torch, a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to(dev)


def params_of(zm, wl, precision=None, flags=0):
    prec = precision if precision is not None else (
        zm.ZM_FP32_PAIRS if wl.precision == "fp32_pairs" else zm.ZM_FP64)
    return zm.Params(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt,
                     precision=prec, flags=flags)


class ClockSampler:
    """Mean GPU core clock (MHz) over a timed region: a background thread
    reads torch.cuda.clock_rate (amd-smi's current GFX clock) every `period`
    seconds and prints nothing; mean() is None when the query is not
    available.  The first query, which loads amd-smi, runs before the region."""

    def __init__(self, torch, period: float = 0.05):
        self.torch, self.period, self.samples, self.ok = torch, period, [], True
        self._stop = threading.Event()
        self._thread = None

    def _run(self):
        while not self._stop.is_set():
            try:
                v = self.torch.cuda.clock_rate(0)
            except Exception:
                self.ok = False
                return
            if v:
                self.samples.append(float(v))
            self._stop.wait(self.period)

    def __enter__(self):
        try:
            self.torch.cuda.clock_rate(0)
        except Exception:
            self.ok = False
            return self
        self._thread = threading.Thread(target=self._run, daemon=True)
        self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self._thread is not None:
            self._thread.join()
        return False

    def mean(self):
        return round(statistics.mean(self.samples)) if self.ok and self.samples else None


def trajectory_run(zm, torch, wl, steps: int, warmup: int):
    """The workload's RK3 steps from its initial state: warmup steps, then
    `steps` timed steps with per-kernel HIP events on the context stream."""
    dev = torch.device("cuda:0")
    p = params_of(zm, wl)
    z0, w0 = wl.state()
    zd, wd = to_dev(torch, z0, dev), to_dev(torch, w0, dev)
    ctx = zm.Context(p)
    ctx.init_state(zd, wd)
    info = ctx.launch_info()
    stream = ctx.stream
    ctx.step(warmup)
    torch.cuda.synchronize()
    ctx.profile_read()                      # discard warm-up timings
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with ClockSampler(torch) as clock:
        t0 = time.perf_counter()
        ev0.record(stream)
        ctx.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    stats = ctx.profile_read()
    ctx.profile_enable(False)
    del ctx
    elapsed = max(wall, gpu_s)
    launches, pair_ms = stats["pairs"]
    return {"info": info, "elapsed": elapsed, "steps": steps, "stats": stats,
            "pair_launches": launches, "avg_pair_s": pair_ms / 1e3 / max(launches, 1),
            "pairs_per_step": 3 * info.pairs_per_eval, "clock_mhz": clock.mean()}


def br_sweep(zm, torch, wl, reps: int = 2):
    """One BR evaluation of the workload's state with the synthetic
    vorticity in the FP64 and FP32 forms: pair-kernel time from HIP events,
    roofline fraction against each form's vector peak, speedup and the
    difference between the forms on every target."""
    z, _ = wl.state()
    w = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
    dev = torch.device("cuda:0")
    zd, wd = to_dev(torch, z, dev), to_dev(torch, w, dev)
    res, us = {}, {}
    for name, prec in (("fp64", zm.ZM_FP64), ("fp32_pairs", zm.ZM_FP32_PAIRS)):
        ctx = zm.Context(params_of(zm, wl, precision=prec))
        ud = torch.empty_like(zd)
        ctx.br_velocity(zd, wd, ud)          # warm-up
        torch.cuda.synchronize()
        ctx.profile_read()
        ctx.profile_enable(True)
        for _ in range(reps):
            ctx.br_velocity(zd, wd, ud)
        st = ctx.profile_read()
        torch.cuda.synchronize()
        n, ms = st["pairs"]
        pairs = ctx.launch_info().pairs_per_eval
        sec = ms / 1e3 / n
        tf = FLOPS_PER_PAIR * pairs / sec / 1e12
        res[name] = {"kernel": "k_pairs_f64f" if prec == zm.ZM_FP64 else "k_pairs_f32",
                     "pair_kernel_ms": sec * 1e3, "pairs_per_s": pairs / sec, "tflops": tf,
                     "peak_tflops": PEAK_TFLOPS[name], "frac": tf / PEAK_TFLOPS[name],
                     "eval_ms": sum(v[1] / max(v[0], 1) for v in st.values() if v[0])}
        us[name] = ud.cpu().numpy().reshape(3, -1)
        del ctx
    res["fp32_over_fp64_speedup"] = res["fp32_pairs"]["pairs_per_s"] / res["fp64"]["pairs_per_s"]
    res["fp32_vs_fp64_max_rel_err"] = rel(us["fp32_pairs"], us["fp64"])
    res["workload"] = f"{wl.name}: one BR evaluation, synthetic vorticity, {wl.n} points"
    return res, (z, w), us


def precision_trajectory(zm, torch, wl, oracle_targets: int = 256, threads: int = 0):
    """The workload's own RK3 trajectory (its step count from its initial
    state) in the FP32 pair form and in FP64: the two final states compared
    (motion z - z0 and w), then F at the FP32 final state in both forms
    against the oracle's F at seeded targets (the oracle also evaluates the
    BR velocity at their stencil neighbours).  With oracle_targets = 0 the
    oracle leg is skipped."""
    dev = torch.device("cuda:0")
    z0, w0 = wl.state()
    out, final, ctxs = {}, {}, {}
    for name, prec in (("fp32_pairs", zm.ZM_FP32_PAIRS), ("fp64", zm.ZM_FP64)):
        ctx = zm.Context(params_of(zm, wl, precision=prec))
        zd, wd = to_dev(torch, z0, dev), to_dev(torch, w0, dev)
        ctx.init_state(zd, wd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(wl.steps)
        torch.cuda.synchronize()
        out[f"{name}_ms_per_step"] = (time.perf_counter() - t0) / wl.steps * 1e3
        z1, w1 = torch.empty_like(zd), torch.empty_like(wd)
        ctx.get_state(z1, w1)
        torch.cuda.synchronize()
        final[name] = (z1.cpu().numpy().reshape(3, -1), w1.cpu().numpy().reshape(2, -1))
        ctxs[name] = ctx
    (z32, w32), (z64, w64) = final["fp32_pairs"], final["fp64"]
    out["steps"] = wl.steps
    out["pairs"] = 3.0 * wl.steps * wl.n * wl.n
    out["fp32_vs_fp64_state"] = {"z_motion": rel(z32 - z0, z64 - z0), "w": rel(w32, w64)}
    if oracle_targets > 0:
        import oracle
        zs, ws = to_dev(torch, z32, dev), to_dev(torch, w32, dev)
        g = {}
        for name, ctx in ctxs.items():
            zt, wt = torch.empty_like(zs), torch.empty_like(ws)
            ctx.rhs(zs, ws, zt, wt)
            torch.cuda.synchronize()
            g[name] = (zt.cpu().numpy().reshape(3, -1), wt.cpu().numpy().reshape(2, -1))
        tg = rr.sample_targets(wl.n, oracle_targets, seed=wl.seed + 11)
        P = oracle.Problem(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity,
                           dt=wl.dt)
        t0 = time.perf_counter()
        zr, wr = oracle.rhs_sampled(P, z32, w32, tg, threads=threads)
        dt = time.perf_counter() - t0
        out["F_vs_oracle"] = {"targets": int(tg.size), "oracle_seconds": dt}
        for name, (zt, wt) in g.items():
            out["F_vs_oracle"][name] = {"z_t": rel(zt[:, tg], zr), "w_t": rel(wt[:, tg], wr)}
    for ctx in ctxs.values():
        del ctx
    return out


def small_mesh_latency(zm, torch, steps: int = 50):
    """64 x 64 FP64 (launch-latency bound): ms per RK3 step with direct
    launches and with the captured graph; also returns the state after the
    workload's own trajectory (its step count from its initial state), which
    the oracle leg compares."""
    wl = rr.WORKLOADS["periodic64_single_fp64"]
    z, w = wl.state()
    dev = torch.device("cuda:0")
    out = {}
    p = zm.Params(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt)
    ctx = zm.Context(p)
    zd = torch.from_numpy(z.ravel()).to(dev); wd = torch.from_numpy(w.ravel()).to(dev)
    ctx.init_state(zd, wd)
    ctx.step(wl.steps)
    z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
    ctx.get_state(z1, w1)
    torch.cuda.synchronize()
    traj = (z1.cpu().numpy().reshape(3, -1), w1.cpu().numpy().reshape(2, -1))
    del ctx
    for name, flags in (("direct", 0), ("graph", zm.ZM_FLAG_GRAPH)):
        p = zm.Params(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt,
                      flags=flags)
        ctx = zm.Context(p)
        ctx.init_state(torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
        ctx.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(steps)
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
        del ctx
    out["pairs_per_s_graph"] = 3 * wl.n * wl.n / (out["graph_ms_per_step"] / 1e3)
    return out, traj


def cutoff_eval(zm, torch, p, z, w, reps: int = 3):
    """Timed cutoff BR evaluations: per-kernel ms, accepted / tested pairs."""
    dev = torch.device("cuda:0")
    ctx = zm.Context(p)
    zd = torch.from_numpy(np.ascontiguousarray(z).ravel()).to(dev)
    wd = torch.from_numpy(np.ascontiguousarray(w).ravel()).to(dev)
    ud = torch.empty_like(zd)
    ctx.br_velocity(zd, wd, ud)
    torch.cuda.synchronize()
    ctx.profile_read()
    ctx.profile_enable(True)
    ctx.cutoff_info()
    for _ in range(reps):
        ctx.br_velocity(zd, wd, ud)
    st = ctx.profile_read()
    info = ctx.cutoff_info()
    ms = {k: v[1] / max(v[0], 1) for k, v in st.items() if v[0]}
    eval_ms = sum(ms.values())
    acc = info.pairs_accepted / reps
    tested = info.pairs_tested / reps
    res = {"mesh": f"{p.n1}x{p.n2}", "cutoff": p.cutoff,
           "cells": [info.cells1, info.cells2], "block_cells": info.block_cells,
           "pairs_accepted_per_eval": acc, "pairs_tested_per_eval": tested,
           "accepted_fraction_of_all_pairs": acc / float(p.n) ** 2,
           "kernel_ms": ms, "eval_ms": eval_ms,
           "accepted_pairs_per_s": acc / (ms["pairs"] / 1e3),
           "pair_kernel_tflops_accepted": FLOPS_PER_PAIR * acc / (ms["pairs"] / 1e3) / 1e12}
    res["pair_kernel_frac_of_fp64_peak"] = res["pair_kernel_tflops_accepted"] / PEAK_TFLOPS["fp64"]
    return res, ud


def cutoff_section(zm, torch):
    """Cutoff BR solver: the paper's two cutoff workloads (per-GPU meshes,
    cutoff as the same fraction of the interface width: 0.2 of 6 and 0.5 of
    6 on a width-2 period cell), and the accuracy-vs-cutoff curve on the
    256 x 256 eight-mode interface against the exact all-pairs sweep."""
    out = {}
    n = 768
    z, _ = rr.multi_mode(n, n, 8, seed=1)
    w = rr.synthetic_vorticity(n, n, seed=1)
    rc = 0.2 * 2.0 / 6.0
    out["multimode768"], _ = cutoff_eval(zm, torch, zm.Params(n, n, eps=1.0 / n, cutoff=rc), z, w)
    n = 512
    z, _ = rr.single_mode(n, n, 0.05)
    w = rr.synthetic_vorticity(n, n, seed=2)
    rc = 0.5 * 2.0 / 6.0
    out["singlemode512"], _ = cutoff_eval(zm, torch, zm.Params(n, n, eps=1.0 / n, cutoff=rc), z, w)
    # accuracy against the exact sweep
    n = 256
    z, _ = rr.multi_mode(n, n, 8, seed=1)
    w = rr.synthetic_vorticity(n, n, seed=1)
    dev = torch.device("cuda:0")
    exact_ctx = zm.Context(zm.Params(n, n, eps=1.0 / n))
    ue = torch.empty(3 * n * n, dtype=torch.float64, device=dev)
    zd = torch.from_numpy(z.ravel()).to(dev); wd = torch.from_numpy(w.ravel()).to(dev)
    exact_ctx.br_velocity(zd, wd, ue)
    exact_ctx.profile_enable(True)
    exact_ctx.br_velocity(zd, wd, ue)
    est = exact_ctx.profile_read()
    exact_ms = sum(v[1] / max(v[0], 1) for v in est.values() if v[0])
    ue_h = ue.cpu().numpy()
    scale = float(np.max(np.abs(ue_h)))
    curve = []
    for rc in (0.05, 0.1, 0.2, 0.3, 0.45, 0.6, 0.9):
        r, uc = cutoff_eval(zm, torch, zm.Params(n, n, eps=1.0 / n, cutoff=rc), z, w, reps=2)
        err = float(np.max(np.abs(uc.cpu().numpy() - ue_h)) / scale)
        curve.append({"cutoff": rc, "max_rel_err_vs_exact": err, "eval_ms": r["eval_ms"],
                      "speedup_vs_exact": exact_ms / r["eval_ms"],
                      "accepted_fraction_of_all_pairs": r["accepted_fraction_of_all_pairs"]})
    out["accuracy_vs_cutoff_256"] = {"exact_eval_ms": exact_ms, "curve": curve}
    return out


def free_section(zm, torch):
    """Non-periodic single-mode interface (the paper's second test case:
    extrapolated ghosts, no images):
      exact256      RK3 steps at 256 x 256, FP64, exact BR: ms/step, pairs/s,
                    pair-kernel TFLOP/s;
      cutoff512     one cutoff BR evaluation at 512 x 512, rc = 1/6 (0.5 of a
                    6-wide domain scaled to the width-2 sheet);
      far_field128  the far-field check: 128 x 128 from a 0.05 single mode,
                    eps = 2h = 1/32 (with eps = h/2 the unfiltered sheet
                    reaches its singularity before t = 2 at this mesh),
                    A = 0.5, g = 1, dt = 5e-3, 400 steps (t = 2) with the exact
                    sum and with cutoffs 0.15 .. 1.2; peak-to-peak z3 of each
                    run and the deviation of every point from the exact
                    trajectory, in the edge band (|alpha_a| > 0.75) and inside."""
    dev = torch.device("cuda:0")
    out = {}
    n, steps = 256, 20
    z, _ = rr.single_mode(n, n, 0.05)
    w = rr.synthetic_vorticity(n, n, seed=3)
    p = zm.Params(n, n, eps=1.0 / n, dt=1e-3, boundary=zm.ZM_BOUNDARY_FREE)
    ctx = zm.Context(p)
    ctx.init_state(torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
    ctx.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile_enable(True)
    ctx.step(1)
    st = ctx.profile_read()
    ppe = ctx.launch_info().pairs_per_eval
    pair_ms = st["pairs"][1] / max(st["pairs"][0], 1)
    out["exact256"] = {"mesh": f"{n}x{n}", "steps": steps, "ms_per_step": wall / steps * 1e3,
                       "pairs_per_s": 3 * ppe * steps / wall, "pair_kernel_ms": pair_ms,
                       "pair_kernel_tflops": FLOPS_PER_PAIR * ppe / (pair_ms / 1e3) / 1e12}
    out["exact256"]["pair_kernel_frac_of_fp64_peak"] = (out["exact256"]["pair_kernel_tflops"] /
                                                         PEAK_TFLOPS["fp64"])
    del ctx
    n = 512
    z, _ = rr.single_mode(n, n, 0.05)
    w = rr.synthetic_vorticity(n, n, seed=2)
    out["cutoff512"], _ = cutoff_eval(zm, torch, zm.Params(n, n, eps=1.0 / n, cutoff=1.0 / 6.0,
                                                           boundary=zm.ZM_BOUNDARY_FREE), z, w)
    n, steps = 128, 400
    z, _ = rr.single_mode(n, n, 0.05)
    w = np.zeros((2, n * n))
    A1, A2 = rr.grid(n, n)
    edge = ((np.abs(A1) > 0.75) | (np.abs(A2) > 0.75)).ravel()
    runs = {}
    for rc in (0.0, 0.15, 0.3, 0.6, 1.2):
        p = zm.Params(n, n, eps=4.0 / n, dt=5e-3, cutoff=rc, boundary=zm.ZM_BOUNDARY_FREE)
        ctx = zm.Context(p)
        ctx.init_state(torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        zd = torch.empty(3 * p.n, dtype=torch.float64, device=dev)
        wd = torch.empty(2 * p.n, dtype=torch.float64, device=dev)
        ctx.get_state(zd, wd)
        runs[rc] = (zd.cpu().numpy().reshape(3, -1), ms)
        del ctx
    ze = runs[0.0][0]
    curve = []
    for rc, (zc, ms) in runs.items():
        d = np.linalg.norm(zc - ze, axis=0)
        curve.append({"cutoff": rc, "ms_per_step": ms,
                      "z3_peak_to_peak": float(zc[2].max() - zc[2].min()),
                      "dev_max": float(d.max()), "dev_mean_edge": float(d[edge].mean()),
                      "dev_mean_inner": float(d[~edge].mean()),
                      "finite": bool(np.all(np.isfinite(zc)))})
    out["far_field128"] = {"mesh": f"{n}x{n}", "eps": 4.0 / n, "steps": steps, "t_end": steps * 5e-3,
                           "runs": curve}
    return out


def medium_section(zm, torch, steps: int = 3):
    """Medium-order model (BR moves the sheet, FFT velocity in the vorticity
    law) against the high-order model on the same inputs: ms per RK3 step and
    per-kernel ms per evaluation, for the exact sum at 512 x 512 and for the
    cutoff sum (rc = 0.2 of a 6-wide domain scaled to width 2) at
    1024 x 1024; eight modes with the synthetic vorticity."""
    dev = torch.device("cuda:0")
    out = {}
    for name, n, rc in (("exact512", 512, 0.0), ("cutoff1024", 1024, 0.2 * 2.0 / 6.0)):
        z, _ = rr.multi_mode(n, n, 8, seed=1)
        w = rr.synthetic_vorticity(n, n, seed=1)
        row = {"mesh": f"{n}x{n}", "cutoff": rc}
        for label, model in (("high", zm.ZM_MODEL_HIGH), ("medium", zm.ZM_MODEL_MEDIUM)):
            p = zm.Params(n, n, eps=1.0 / n, dt=1e-3, cutoff=rc, model=model)
            ctx = zm.Context(p)
            ctx.init_state(torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
            ctx.step(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.step(steps)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            ctx.profile_enable(True)
            ctx.step(1)
            st = ctx.profile_read()
            row[label] = {"ms_per_step": ms,
                          "kernel_ms_per_eval": {k: v[1] / v[0] for k, v in st.items() if v[0]}}
            del ctx
        row["medium_over_high"] = row["medium"]["ms_per_step"] / row["high"]["ms_per_step"]
        out[name] = row
    return out


def low_order_section(zm, torch, n: int = 4096, steps: int = 5):
    """Low-order model (FFT velocity): RK3 steps on an n x n eight-mode
    interface (n = 4096 stands in for the paper's 4864 x 4864 per-GPU mesh,
    the largest power of two below it), per-kernel times, mesh points
    advanced per second, and the HBM rate of the FFT velocity against its
    algorithmic traffic: pack + row FFT (w in, complex out), transpose,
    FFT-symbol-inverse-FFT rows, transpose, inverse row FFT (complex in, S
    out), point kernel (S, z, w in; u, V out)."""
    z, _ = rr.multi_mode(n, n, 8, seed=1)
    w = rr.synthetic_vorticity(n, n, seed=1)
    dev = torch.device("cuda:0")
    p = zm.Params(n, n, eps=1.0 / n, dt=1e-3, model=zm.ZM_MODEL_LOW)
    ctx = zm.Context(p)
    ctx.init_state(torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
    ctx.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile_enable(True)
    ctx.step(1)
    st = ctx.profile_read()
    ms = {k: v[1] / v[0] for k, v in st.items() if v[0]}
    N = n * n
    # bytes of one FFT-velocity evaluation per point: pack + FFT rows (w 16
    # in, 16 out), two transposes and the symbol rows (16 in + 16 out each),
    # inverse FFT rows (16 in, S 8 out), point kernel (S 8, z 24 with its
    # stencil neighbours from cache, w 16 in; u 24, V 8 out)
    fft_bytes = N * (32 + 3 * 32 + 24 + 80)
    return {"mesh": f"{n}x{n}", "steps": steps, "ms_per_step": wall / steps * 1e3,
            "points_per_s": N * steps / wall, "kernel_ms_per_eval": ms,
            "fft_velocity_bytes_per_eval": fft_bytes,
            "fft_velocity_gb_per_s": fft_bytes / (ms["fft"] / 1e3) / 1e9,
            "fft_velocity_frac_of_hbm": fft_bytes / (ms["fft"] / 1e3) / 8e12}


def pair_kernel_ms(zm, torch, n: int, prec: int, reps: int = 3) -> float:
    """Average pair-kernel time (HIP events) of one BR evaluation on an n x n
    seeded interface with the shape a new context gets."""
    z, w = rr.random_state(n, n, seed=5, height=0.05)
    dev = torch.device("cuda:0")
    ctx = zm.Context(zm.Params(n, n, eps=1.0 / n, precision=prec))
    zd = torch.from_numpy(z.ravel()).to(dev); wd = torch.from_numpy(w.ravel()).to(dev)
    ud = torch.empty_like(zd)
    ctx.br_velocity(zd, wd, ud)
    torch.cuda.synchronize()
    ctx.profile_read()
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.br_velocity(zd, wd, ud)
    n_, ms = ctx.profile_read()["pairs"]
    return ms / n_


def tune_report(zm, torch, sides=(32, 48, 64, 96, 128, 192, 256, 512, 1024),
                precisions=("fp64", "fp32_pairs")):
    """Autotune the pair kernel per (side, precision); report the default and
    tuned shapes with their measured pair-kernel times.  The process-wide
    tuning entries are removed again afterwards."""
    rows = []
    for prec, name in ((zm.ZM_FP64, "fp64"), (zm.ZM_FP32_PAIRS, "fp32_pairs")):
        if name not in precisions:
            continue
        for n in sides:
            zm.tuning_set(n, n, prec)
            d = zm.tuning_get(n, n, prec)
            ms_d = pair_kernel_ms(zm, torch, n, prec)
            R, S, _ = zm.autotune(zm.Params(n, n, eps=1.0 / n, precision=prec))
            ms_t = pair_kernel_ms(zm, torch, n, prec)
            zm.tuning_set(n, n, prec)
            rows.append({"side": n, "precision": name,
                         "default": {"R": d[0], "splits": d[1], "pair_ms": ms_d},
                         "tuned": {"R": R, "splits": S, "pair_ms": ms_t},
                         "tuned_pairs_per_s": float(n) ** 4 / (ms_t / 1e3),
                         "tuned_tflops": FLOPS_PER_PAIR * float(n) ** 4 / (ms_t / 1e3) / 1e12})
    return rows


def ensemble64(zm, torch, steps: int = 20):
    """The 64-member uneven ensemble (sides 32..256, FP32 form) advanced by
    one batch with graph-captured RK3 steps.  The same batch is timed with
    the untuned default shapes, then the batch tuner picks the pair-kernel
    shape of every side by timing the batched sweep itself (entries kept for
    the timed run).  One member of each side is rerun alone and compared bit
    for bit with the tuned batch (the solo context takes the same shape)."""
    ms = rr.ensemble(64, seed=3)
    ps = [zm.Params(m.n, m.n, eps=m.eps, atwood=m.atwood, gravity=1.0, dt=1e-3,
                    precision=zm.ZM_FP32_PAIRS) for m in ms]
    dev = torch.device("cuda:0")
    sides = sorted({m.n for m in ms})
    prec = zm.ZM_FP32_PAIRS

    def timed_batch():
        b = zm.Batch(ps, flags=zm.ZM_FLAG_GRAPH)
        for i, m in enumerate(ms):
            z, w = m.state()
            b.init_state(i, to_dev(torch, z, dev), to_dev(torch, w, dev))
        b.step(1)                                   # capture + warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        return b, time.perf_counter() - t0

    for n in sides:
        zm.tuning_set(n, n, prec)                  # defaults
    defaults = {n: zm.tuning_get(n, n, prec) for n in sides}
    b, dt_default = timed_batch()
    info = b.info()
    b.destroy()
    shapes, sweep_ms = zm.batch_autotune(ps)
    tuned = {m.n: shapes[i] for i, m in enumerate(ms)}
    b, dt = timed_batch()
    info_t = b.info()
    # one member of each side rerun alone for the same 1 + steps steps: its
    # state must be bitwise equal to the batch's
    firsts = {}
    for i, m in enumerate(ms):
        firsts.setdefault(m.n, i)
    equal = 0
    for i in sorted(firsts.values()):
        m = ms[i]
        zb = torch.empty(3 * m.n * m.n, dtype=torch.float64, device=dev)
        wb = torch.empty(2 * m.n * m.n, dtype=torch.float64, device=dev)
        b.get_state(i, zb, wb)
        z, w = m.state()
        ctx = zm.Context(ps[i])
        ctx.init_state(to_dev(torch, z, dev), to_dev(torch, w, dev))
        ctx.step(1 + steps)
        zs, ws = torch.empty_like(zb), torch.empty_like(wb)
        ctx.get_state(zs, ws)
        torch.cuda.synchronize()
        equal += int(torch.equal(zs, zb) and torch.equal(ws, wb))
        del ctx
    b.destroy()
    for n in sides:
        zm.tuning_set(n, n, prec)                  # leave the table as found
    pps = info_t.pairs_per_step
    tf = FLOPS_PER_PAIR * pps * steps / dt / 1e12
    return {"members": 64, "sides": sides, "steps": steps,
            "solo_vs_batch": {"members_checked": len(firsts), "bitwise_equal": equal},
            "shapes": [{"side": n, "default": list(defaults[n]), "tuned": list(tuned[n])}
                       for n in sides],
            "tuned_batch_pair_sweep_ms": sweep_ms,
            "pairs_per_step": pps, "work_items": info_t.work_items[1],
            "work_items_default": info.work_items[1],
            "persistent_groups": info_t.persistent_groups, "seconds": dt,
            "pairs_per_s": pps * steps / dt, "tflops": tf, "frac_of_fp32_peak": tf / 157.3,
            "default_shapes_pairs_per_s": pps * steps / dt_default,
            "tuned_over_default": dt_default / dt}


def serving(zm, torch, count: int = 200, budget: int = 1 << 30, step_scale: int = 10,
            solo_checks: int = 8, max_seconds: float = 420.0):
    """Poisson request stream (sides log-uniform 64..512, A ~ U[0.1, 0.9],
    100..1000 RK3 steps, FP32 form) served by one pool with a 1 GiB budget
    until every request has arrived and finished (or max_seconds pass).
    Capacity is measured first on a saturated pool; the arrival rate is then
    0.8 x capacity.

    Time compression: every request's step count is divided by step_scale
    (10..100 steps) and the rate multiplied by it.  The mean number of live
    requests (rate x residence time) and hence the per-step latency
    distribution of the steady state are unchanged, while the whole stream
    is served in step_scale times less wall time.  The first solo_checks
    requests to finish are rerun alone afterwards and compared bit for bit
    with their pooled result."""
    dev = torch.device("cuda:0")

    def params(m):
        return zm.Params(m.n, m.n, eps=m.eps, atwood=m.atwood, gravity=1.0, dt=1e-3,
                         precision=zm.ZM_FP32_PAIRS)

    smin, smax = 100 // step_scale, 1000 // step_scale
    probe = rr.request_stream(count, rate=1.0, seed=4, steps_min=smin, steps_max=smax)
    mean_pairs = float(np.mean([3.0 * m.n ** 4 * m.steps for m in probe]))
    # capacity: a saturated pool (requests waiting), pairs/s over 40 iterations
    pool = zm.Pool(budget)
    keep = []
    for m in probe[:40]:
        z, w = m.state()
        zt, wt = to_dev(torch, z, dev), to_dev(torch, w, dev)
        keep.append((zt, wt))
        pool.submit(params(m), zt, wt, m.steps)
    pool.iterate()
    s0 = pool.stats().pairs_done
    t0 = time.perf_counter()
    for _ in range(40):
        pool.iterate()
    dt = time.perf_counter() - t0
    cap_pairs = (pool.stats().pairs_done - s0) / dt
    pool.destroy()
    del keep
    rate = 0.8 * cap_pairs / mean_pairs
    stream = rr.request_stream(count, rate=rate, seed=4, steps_min=smin, steps_max=smax)
    log(f"serving {count} requests at {rate:.2f}/s (0.8 x capacity), steps / {step_scale}")
    pool = zm.Pool(budget)
    lat, queue_delay, admitted_at, finished = [], [], {}, 0
    ids = {}
    checked = []   # (stream index, final z, final w) of the first finished requests
    nxt = 0
    start = time.perf_counter()
    last_log = start
    p0 = pool.stats().pairs_done
    timed_out = False
    while True:
        now = time.perf_counter() - start
        if now >= max_seconds:
            timed_out = True
            break
        while nxt < len(stream) and stream[nxt].arrival <= now:
            m = stream[nxt]
            z, w = m.state()
            rid = pool.submit(params(m), to_dev(torch, z, dev), to_dev(torch, w, dev), m.steps)
            ids[rid] = nxt
            nxt += 1
        recs = pool.iterate()
        t_now = time.perf_counter() - start
        for rid, done, state, ms in recs:
            lat.append(ms)
            if rid not in admitted_at:
                admitted_at[rid] = t_now
                queue_delay.append(t_now - stream[ids[rid]].arrival)
            if state == zm.ZM_REQ_FINISHED:
                finished += 1
                if len(checked) < solo_checks:
                    m = stream[ids[rid]]
                    zf = torch.empty(3 * m.n * m.n, dtype=torch.float64, device=dev)
                    wf = torch.empty(2 * m.n * m.n, dtype=torch.float64, device=dev)
                    pool.fetch(rid, zf, wf)
                    checked.append((ids[rid], zf, wf))
                pool.release(rid)
        if time.perf_counter() - last_log > 20.0:
            last_log = time.perf_counter()
            log(f"serving: {t_now:.0f} s, arrived {nxt}, finished {finished}")
        if not recs:
            if nxt >= len(stream):
                break
            time.sleep(min(0.01, max(0.0, stream[nxt].arrival - t_now)))
    wall = time.perf_counter() - start
    st = pool.stats()
    # solo vs mix: each checked request rerun alone in its own context from
    # the same state must end bitwise equal to its run inside the pool
    equal = 0
    for k, zf, wf in checked:
        m = stream[k]
        z, w = m.state()
        ctx = zm.Context(params(m))
        ctx.init_state(to_dev(torch, z, dev), to_dev(torch, w, dev))
        ctx.step(m.steps)
        zs, ws = torch.empty_like(zf), torch.empty_like(wf)
        ctx.get_state(zs, ws)
        torch.cuda.synchronize()
        equal += int(torch.equal(zs, zf) and torch.equal(ws, wf))
        del ctx
    out = {
        "requests_total": count, "steps_per_request": [smin, smax],
        "time_compression": step_scale, "arrived": nxt, "admitted": len(admitted_at),
        "finished": finished, "stopped_at_time_limit": timed_out,
        "makespan_s": wall, "budget_bytes": budget,
        "capacity_requests_per_s": cap_pairs / mean_pairs, "rate_requests_per_s": rate,
        "step_samples": len(lat), "iterations": st.iterations,
        "p50_step_ms": float(np.percentile(lat, 50)) if lat else None,
        "p99_step_ms": float(np.percentile(lat, 99)) if lat else None,
        "mean_step_ms": float(np.mean(lat)) if lat else None,
        "queue_delay_p50_s": float(np.percentile(queue_delay, 50)) if queue_delay else None,
        "queue_delay_p99_s": float(np.percentile(queue_delay, 99)) if queue_delay else None,
        "pairs_per_s": (st.pairs_done - p0) / wall,
        "saturated_pairs_per_s": cap_pairs,
        "live_at_end": st.live, "queued_at_end": st.queued,
        "solo_vs_mix": {"requests_checked": len(checked), "bitwise_equal": equal,
                        "sides": [stream[k].n for k, _, _ in checked]},
    }
    pool.destroy()
    return out


def oracle_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()


def cpu_baseline(zm, torch, wl, target_seconds: float, sweep=None):
    """The CPU oracle on a bounded sample of the same workload.

    If one full oracle RK3 step (3 N^2 pairs) fits in about 3x target_seconds
    of host time, time exactly that from the workload's initial state and
    compare the GPU's step from the same state with it, element by element.
    Otherwise time the BR velocity of seeded targets (against all sources)
    sized to target_seconds, on the workload's state with the synthetic
    vorticity, and compare the GPU's velocity at those targets: in both pair
    forms when the precision sweep's velocities are given (sweep =
    ((z, w), {form: u})), else in the workload's own form.
    """
    import oracle
    threads = oracle_threads()
    P = oracle.Problem(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt)
    z0, w0 = wl.state()
    w_syn = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
    probe = rr.sample_targets(wl.n, 256, seed=99)
    t0 = time.perf_counter()
    oracle.br_velocity(P, z0, w_syn, targets=probe, threads=threads)
    rate = probe.size * wl.n / (time.perf_counter() - t0)        # pairs/s
    full_step = 3.0 * wl.n * wl.n / rate
    dev = torch.device("cuda:0")

    if full_step <= 3.0 * target_seconds:
        t0 = time.perf_counter()
        zr, wr = oracle.rk3(P, z0, w0, 1, threads=threads)
        dt = time.perf_counter() - t0
        ctx = zm.Context(params_of(zm, wl))
        zd, wd = to_dev(torch, z0, dev), to_dev(torch, w0, dev)
        ctx.init_state(zd, wd)
        ctx.step(1)
        z1, w1 = torch.empty_like(zd), torch.empty_like(wd)
        ctx.get_state(z1, w1)
        torch.cuda.synchronize()
        zg = z1.cpu().numpy().reshape(3, -1); wg = w1.cpu().numpy().reshape(2, -1)
        return {
            "value": 3.0 * wl.n * wl.n / dt, "unit": "pair-interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one full RK3 step of the workload from its initial state "
                      f"({3.0 * wl.n * wl.n:.3e} pairs, {dt:.1f} s)",
            "seconds": dt,
            "gpu_vs_oracle_max_rel_err": {"z": rel(zg, zr), "w": rel(wg, wr) if np.any(wr) else 0.0,
                                          "z_motion": rel(zg - z0, zr - z0)},
        }

    count = int(min(wl.n, max(64, target_seconds * rate / wl.n)))
    tg = rr.sample_targets(wl.n, count, seed=wl.seed)
    if sweep is not None:
        us = sweep[1]
    else:
        ctx = zm.Context(params_of(zm, wl))
        zd, wd = to_dev(torch, z0, dev), to_dev(torch, w_syn, dev)
        ud = torch.empty_like(zd)
        ctx.br_velocity(zd, wd, ud)
        torch.cuda.synchronize()
        us = {wl.precision: ud.cpu().numpy().reshape(3, -1)}
        del ctx
    t0 = time.perf_counter()
    ref = oracle.br_velocity(P, z0, w_syn, targets=tg, threads=threads)
    dt = time.perf_counter() - t0
    return {
        "value": tg.size * wl.n / dt, "unit": "pair-interactions/s", "cores": threads,
        "kind": "oracle",
        "sample": f"BR at {tg.size} seeded targets x {wl.n} sources ({tg.size * wl.n:.2e} pairs)",
        "seconds": dt,
        "gpu_vs_oracle_max_rel_err": {form: rel(u[:, tg], ref) for form, u in us.items()},
    }


def small_mesh_oracle(threads: int, traj64):
    """The oracle's own runs on the 64 x 64 workload (a few seconds of host
    time): one full BR evaluation with all threads and with one, and the
    workload's trajectory (its step count from its initial state), timed
    and compared with the GPU's."""
    import oracle
    out = {"threads": threads}
    wl = rr.WORKLOADS["periodic64_single_fp64"]
    z, _ = wl.state()
    w = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
    P = oracle.Problem(wl.n1, wl.n2, eps=wl.eps)
    for name, nt in (("full_br", threads), ("full_br_1thread", 1)):
        t0 = time.perf_counter()
        oracle.br_velocity(P, z, w, threads=nt)
        dt = time.perf_counter() - t0
        out[name] = {"pairs": wl.n * wl.n, "seconds": dt, "pairs_per_s": wl.n * wl.n / dt,
                     "threads": nt}
    z0, w0 = wl.state()
    P = oracle.Problem(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt)
    t0 = time.perf_counter()
    zr, wr = oracle.rk3(P, z0, w0, wl.steps, threads=threads)
    dt = time.perf_counter() - t0
    zg, wg = traj64
    out["trajectory"] = {
        "steps": wl.steps, "pairs": 3.0 * wl.steps * wl.n * wl.n, "seconds": dt,
        "pairs_per_s": 3.0 * wl.steps * wl.n * wl.n / dt, "threads": threads,
        "gpu_vs_oracle_max_rel_err": {"z": rel(zg, zr), "w": rel(wg, wr),
                                      "z_motion": rel(zg - z0, zr - z0)}}
    return out


def fp64_256(zm, torch, steps: int = 50, warmup: int = 2):
    """The 256 x 256 eight-mode FP64 workload: its RK3 steps timed, the
    FP64 pair kernel on its roofline."""
    wl = rr.WORKLOADS["periodic256_multimode8_fp64"]
    r = trajectory_run(zm, torch, wl, steps, warmup)
    ach = FLOPS_PER_PAIR * r["info"].pairs_per_eval / r["avg_pair_s"] / 1e12
    return {"workload": wl.name, "steps": steps, "ms_per_step": r["elapsed"] / steps * 1e3,
            "pairs_per_s": r["pairs_per_step"] * steps / r["elapsed"],
            "pair_kernel_ms": r["avg_pair_s"] * 1e3, "pair_kernel_tflops": ach,
            "frac_of_fp64_peak": ach / PEAK_TFLOPS["fp64"],
            "pair_share_of_step": r["avg_pair_s"] * 3 * steps / r["elapsed"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch
    import paper_2406_05490_amd as zm

    only = {"cutoff": args.cutoff_only, "low_order_4096": args.low_order_only,
            "medium_order": args.medium_only, "free_single_mode": args.free_only,
            "tune_report": args.tune_report, "ensemble64": args.ensemble_only}
    runners = {"cutoff": cutoff_section, "low_order_4096": low_order_section,
               "medium_order": medium_section, "free_single_mode": free_section,
               "tune_report": tune_report, "ensemble64": ensemble64}
    for key, on in only.items():
        if on:
            print(json.dumps({key: runners[key](zm, torch)}), flush=True)
            return
    if args.serve_only:
        print(json.dumps({"serving": serving(zm, torch, count=args.serve_requests,
                                             max_seconds=args.serve_max_seconds)}), flush=True)
        return

    wl = rr.WORKLOADS[args.workload]
    steps = wl.steps if args.steps is None else args.steps
    torch.cuda.set_device(torch.device("cuda:0"))
    threads = oracle_threads()
    detail = {}

    log(f"{wl.name}: {args.warmup} warm-up + {steps} timed RK3 steps")
    r = trajectory_run(zm, torch, wl, steps, args.warmup)
    info = r["info"]
    prec32 = wl.precision == "fp32_pairs"
    kernel = "k_pairs_f32" if prec32 else "k_pairs_f64f"
    peak = PEAK_TFLOPS[wl.precision]
    value = r["pairs_per_step"] * steps / r["elapsed"]
    achieved = FLOPS_PER_PAIR * info.pairs_per_eval / r["avg_pair_s"] / 1e12
    roof = {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(kernel, wl.name),
            "flops_per_pair": FLOPS_PER_PAIR, "avg_launch_ms": r["avg_pair_s"] * 1e3,
            "launches": r["pair_launches"], "clock_mhz": r["clock_mhz"]}
    xf = executed_flops_per_pair(kernel, wl.name)
    if xf is not None:
        roof["executed_flops_per_pair"] = xf
        roof["frac_executed"] = xf / FLOPS_PER_PAIR * achieved / peak
    detail["kernel_ms"] = {k: {"launches": n, "total_ms": ms} for k, (n, ms) in r["stats"].items()}
    detail["pair_kernel_share"] = r["avg_pair_s"] * r["pair_launches"] / r["elapsed"]

    sweep = None
    extras = {}
    if not args.no_sweep and wl.n1 * wl.n2 >= 1 << 20:
        log("one BR evaluation in each pair form")
        sw, zw, us = br_sweep(zm, torch, wl)
        detail["br_sweep"] = sw
        sweep = (zw, us)
        f64 = sw["fp64"]
        roof["fp64_form"] = {"kernel": f64["kernel"], "avg_launch_ms": f64["pair_kernel_ms"],
                             "achieved": f64["tflops"], "peak": PEAK_TFLOPS["fp64"],
                             "frac": f64["frac"]}
        roof["fp32_over_fp64_speedup"] = sw["fp32_over_fp64_speedup"]
        roof["fp32_vs_fp64_max_rel_err"] = sw["fp32_vs_fp64_max_rel_err"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["elapsed"] / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": wl.name, "mesh": f"{wl.n1}x{wl.n2}",
            "modes": wl.modes, "eps_over_h": wl.eps_over_h, "atwood": wl.atwood, "dt": wl.dt,
            "precision": wl.precision,
            "pair_shape": f"R{info.targets_per_lane} S{info.source_splits} WG{info.workgroups}",
        },
        "roofline": roof,
    }

    if args.cpu_seconds > 0:
        log("CPU oracle sample")
        cb = cpu_baseline(zm, torch, wl, args.cpu_seconds, sweep=sweep)
        cb["gpu_speedup"] = value / cb["value"]
        out["cpu_baseline"] = cb

    if not args.no_sweep:
        if wl.n1 * wl.n2 >= 1 << 20:
            log(f"{wl.steps}-step trajectory in both forms, F against the oracle")
            pt = precision_trajectory(zm, torch, wl, threads=threads,
                                      oracle_targets=256 if args.cpu_seconds > 0 else 0)
            detail["precision_trajectory"] = pt
            extras["traj5"] = {"fp32_vs_fp64_state": pt["fp32_vs_fp64_state"]}
            if "F_vs_oracle" in pt:
                f = pt["F_vs_oracle"]
                extras["traj5"]["F_vs_oracle"] = {
                    "targets": f["targets"],
                    "fp32": max(f["fp32_pairs"].values()), "fp64": max(f["fp64"].values())}
        log("256 x 256 FP64 workload")
        detail["fp64_256"] = fp64_256(zm, torch)
        extras["fp64_256"] = {k: detail["fp64_256"][k] for k in
                              ("pairs_per_s", "pair_kernel_ms", "frac_of_fp64_peak")}
        log("64 x 64 workload")
        lat, traj64 = small_mesh_latency(zm, torch)
        detail["periodic64_latency"] = lat
        if args.cpu_seconds > 0:
            so = small_mesh_oracle(threads, traj64)
            detail["periodic64_oracle"] = so
            extras["c64"] = {"graph_ms_per_step": lat["graph_ms_per_step"],
                             "traj_vs_oracle": max(so["trajectory"]["gpu_vs_oracle_max_rel_err"]
                                                   [k] for k in ("z", "w"))}
        log("64-member ensemble")
        en = ensemble64(zm, torch)
        detail["ensemble64"] = en
        extras["ensemble64"] = {"tera_pairs_per_s": en["pairs_per_s"] / 1e12,
                                "frac_of_fp32_peak": en["frac_of_fp32_peak"],
                                "default_shapes_tera_pairs_per_s":
                                    en["default_shapes_pairs_per_s"] / 1e12,
                                "solo_bitwise": f"{en['solo_vs_batch']['bitwise_equal']}/"
                                                f"{en['solo_vs_batch']['members_checked']}"}
        if not args.no_sections:
            for key, fn in (("cutoff", cutoff_section), ("low_order_4096", low_order_section),
                            ("free_single_mode", free_section), ("medium_order", medium_section)):
                log(f"section {key}")
                detail[key] = fn(zm, torch)
            cut = detail["cutoff"]
            extras["cutoff"] = {
                side: {"giga_acc_per_s": c["accepted_pairs_per_s"] / 1e9,
                       "tested_per_acc": c["pairs_tested_per_eval"] / c["pairs_accepted_per_eval"],
                       "pair_ms": c["kernel_ms"]["pairs"]}
                for side, c in (("768", cut["multimode768"]), ("512", cut["singlemode512"]))}
    if args.serve_requests > 0:
        sv = serving(zm, torch, count=args.serve_requests, max_seconds=args.serve_max_seconds)
        detail["serving"] = sv
        extras["serving"] = {k: sv[k] for k in ("p50_step_ms", "p99_step_ms", "queue_delay_p99_s",
                                                "arrived", "finished", "time_compression")}
        extras["serving"]["tera_pairs_per_s"] = sv["pairs_per_s"] / 1e12
        extras["serving"]["solo_bitwise"] = (f"{sv['solo_vs_mix']['bitwise_equal']}/"
                                             f"{sv['solo_vs_mix']['requests_checked']}")
    if args.detail_out:
        full = dict(out, **detail)
        os.makedirs(os.path.dirname(os.path.abspath(args.detail_out)), exist_ok=True)
        with open(args.detail_out, "w") as fh:
            json.dump(full, fh, indent=1)
    out.update(sig(extras, 3))
    print(json.dumps(sig(out), separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
