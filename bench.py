#!/usr/bin/env python3
"""Throughput of the Z-Model high-order step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one SSP-RK3 step: three evaluations of (surface derivatives ->
all-pairs Birkhoff-Rott sweep -> tie correction -> reduction -> RK3 stage),
each evaluation doing N^2 pair interactions.  Inputs are seeded synthetic
rocket-rig interfaces resident in HBM before the timed region.  Prints one
JSON line with the throughput, the pair kernel's place on its VALU roofline
(timed with HIP events inside the library, on the stream it launches on) and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import rocket_rig as rr  # noqa: E402

METRIC = "BR pair-interactions/s & % VALU peak (FP32 vs FP64); served p50/p99 step ms"
FLOPS_PER_PAIR = 27          # 3 sub, 3 fma, 1 rsqrt, 2 mul, 3 mul, 6 fma (fma = 2)
PEAK_TFLOPS = {"fp64": 78.6, "fp32_pairs": 157.3}   # MI355X vector peaks
DEFAULT_WORKLOAD = "periodic256_multimode8_fp64"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed RK3 steps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(rr.WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample (0 = skip)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the 1M-point BR sweep (FP64 and FP32 forms)")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the real-time serving window (0 = skip)")
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
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


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


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary of this kernel
    and workload (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's reading),
    or None when there is none or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel") != kernel or rec.get("workload") != workload:
        return None
    if rec.get("source_sha256") != library_source_hash():
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))


def br_sweep_1m(zm, torch, reps: int = 2):
    """One BR evaluation on the 1024 x 1024 precision workload (synthetic
    vorticity) in the FP64 and FP32 forms: pair-kernel time from HIP events,
    roofline fraction against each form's vector peak, speedup and error."""
    wl = rr.WORKLOADS["periodic1024_multimode16_fp32"]
    z, _ = wl.state()
    w = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
    dev = torch.device("cuda:0")
    zd = torch.from_numpy(z.ravel()).to(dev)
    wd = torch.from_numpy(w.ravel()).to(dev)
    res, us = {}, {}
    for name, prec in (("fp64", zm.ZM_FP64), ("fp32_pairs", zm.ZM_FP32_PAIRS)):
        p = zm.Params(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity,
                      dt=wl.dt, precision=prec)
        ctx = zm.Context(p)
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
        res[name] = {"pair_kernel_ms": sec * 1e3, "pairs_per_s": pairs / sec, "tflops": tf,
                     "peak_tflops": PEAK_TFLOPS[name], "frac": tf / PEAK_TFLOPS[name]}
        us[name] = ud.cpu().numpy()
        del ctx
    err = float(np.max(np.abs(us["fp32_pairs"] - us["fp64"])) / np.max(np.abs(us["fp64"])))
    res["fp32_over_fp64_speedup"] = res["fp32_pairs"]["pairs_per_s"] / res["fp64"]["pairs_per_s"]
    res["fp32_vs_fp64_max_rel_err"] = err
    res["workload"] = f"{wl.name}: one BR evaluation, synthetic vorticity, {wl.n} points"
    return res, us


def ensemble64(zm, torch, steps: int = 20):
    """The 64-member uneven ensemble (sides 32..256, FP32 form) advanced by
    one batch with graph-captured RK3 steps: aggregate pair-interactions/s,
    one member of each side checked bit for bit against a solo run, and the
    autotuner's choice per side (default and tuned shape, pair-kernel ms;
    measured after the timed run, entries removed afterwards)."""
    ms = rr.ensemble(64, seed=3)
    ps = [zm.Params(m.n, m.n, eps=m.eps, atwood=m.atwood, gravity=1.0, dt=1e-3,
                    precision=zm.ZM_FP32_PAIRS) for m in ms]
    b = zm.Batch(ps, flags=zm.ZM_FLAG_GRAPH)
    dev = torch.device("cuda:0")
    for i, m in enumerate(ms):
        z, w = m.state()
        b.init_state(i, torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
    b.step(1)                                   # capture + warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = b.info()
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
        ctx.init_state(torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
        ctx.step(1 + steps)
        zs = torch.empty_like(zb); ws = torch.empty_like(wb)
        ctx.get_state(zs, ws)
        torch.cuda.synchronize()
        equal += int(torch.equal(zs, zb) and torch.equal(ws, wb))
        del ctx
    b.destroy()
    sides = sorted({m.n for m in ms})
    tuned = tune_report(zm, torch, sides=tuple(sides), precisions=("fp32_pairs",))
    return {"members": 64, "sides": sides, "steps": steps,
            "solo_vs_batch": {"members_checked": len(firsts), "bitwise_equal": equal},
            "autotune_fp32": [{"side": r["side"], "default": [r["default"]["R"], r["default"]["splits"]],
                               "tuned": [r["tuned"]["R"], r["tuned"]["splits"]],
                               "default_ms": r["default"]["pair_ms"], "tuned_ms": r["tuned"]["pair_ms"]}
                              for r in tuned],
            "pairs_per_step": info.pairs_per_step, "work_items": info.work_items[1],
            "persistent_groups": info.persistent_groups, "seconds": dt,
            "pairs_per_s": info.pairs_per_step * steps / dt,
            "tflops": FLOPS_PER_PAIR * info.pairs_per_step * steps / dt / 1e12,
            "frac_of_fp32_peak": FLOPS_PER_PAIR * info.pairs_per_step * steps / dt / 1e12 / 157.3}


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
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return rows


def serving(zm, torch, window_s: float = 30.0, budget: int = 1 << 30, count: int = 200,
            step_scale: int = 10, solo_checks: int = 8):
    """Poisson request stream (sides log-uniform 64..512, A ~ U[0.1, 0.9],
    100..1000 RK3 steps, FP32 form) served by one pool with a 1 GiB budget.
    Capacity is measured first on a saturated pool; the arrival rate is then
    0.8 x capacity and the stream is replayed in real time for window_s.

    Time compression: every request's step count is divided by step_scale
    (10..100 steps) and the rate multiplied by it.  The mean number of live
    requests (rate x residence time) and hence the per-step latency
    distribution of the steady state are unchanged, while a bounded window
    sees step_scale times more arrivals and completions.  The first
    solo_checks requests to finish are rerun alone afterwards and compared
    bit for bit with their pooled result."""
    import numpy as np
    dev = torch.device("cuda:0")

    def params(m):
        return zm.Params(m.n, m.n, eps=m.eps, atwood=m.atwood, gravity=1.0, dt=1e-3,
                         precision=zm.ZM_FP32_PAIRS)

    probe = rr.request_stream(count, rate=1.0, seed=4, steps_min=100 // step_scale,
                              steps_max=1000 // step_scale)
    mean_pairs = float(np.mean([3.0 * m.n ** 4 * m.steps for m in probe]))
    # capacity: a saturated pool (requests waiting), pairs/s over 40 iterations
    pool = zm.Pool(budget)
    keep = []
    for m in probe[:40]:
        z, w = m.state()
        zt = torch.from_numpy(z.ravel()).to(dev); wt = torch.from_numpy(w.ravel()).to(dev)
        keep.append((zt, wt))
        pool.submit(params(m), zt, wt, m.steps)
    pool.iterate()
    s0 = pool.stats().pairs_done
    t0 = time.perf_counter()
    for _ in range(40):
        pool.iterate()
    dt = time.perf_counter() - t0
    cap_pairs = (pool.stats().pairs_done - s0) / dt
    pool.destroy(); del keep
    rate = 0.8 * cap_pairs / mean_pairs
    stream = rr.request_stream(count, rate=rate, seed=4, steps_min=100 // step_scale,
                               steps_max=1000 // step_scale)
    pool = zm.Pool(budget)
    lat, queue_delay, admitted_at = [], [], {}
    ids = {}
    checked = []   # (stream index, final z, final w) of the first finished requests
    nxt = 0
    start = time.perf_counter()
    p0 = pool.stats().pairs_done
    while True:
        now = time.perf_counter() - start
        if now >= window_s:
            break
        while nxt < len(stream) and stream[nxt].arrival <= now:
            m = stream[nxt]
            z, w = m.state()
            rid = pool.submit(params(m), torch.from_numpy(z.ravel()).to(dev),
                              torch.from_numpy(w.ravel()).to(dev), m.steps)
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
                if len(checked) < solo_checks:
                    m = stream[ids[rid]]
                    zf = torch.empty(3 * m.n * m.n, dtype=torch.float64, device=dev)
                    wf = torch.empty(2 * m.n * m.n, dtype=torch.float64, device=dev)
                    pool.fetch(rid, zf, wf)
                    checked.append((ids[rid], zf, wf))
                pool.release(rid)
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
        ctx.init_state(torch.from_numpy(z.ravel()).to(dev), torch.from_numpy(w.ravel()).to(dev))
        ctx.step(m.steps)
        zs = torch.empty_like(zf); ws = torch.empty_like(wf)
        ctx.get_state(zs, ws)
        torch.cuda.synchronize()
        equal += int(torch.equal(zs, zf) and torch.equal(ws, wf))
        del ctx
    out = {
        "requests_total": count, "steps_per_request": [100 // step_scale, 1000 // step_scale],
        "time_compression": step_scale, "arrived": nxt, "admitted": len(admitted_at),
        "finished_in_window": sum(1 for r in ids if pool.query(r)[0] == zm.ZM_REQ_UNKNOWN),
        "window_s": wall, "budget_bytes": budget,
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


def cpu_baseline(wl, ctx_factory, z0, w0, target_seconds: float):
    """The CPU oracle on a bounded sample of the same workload.

    If one full oracle RK3 step (3 N^2 pairs) fits in about 3x target_seconds
    of host time, time exactly that from the workload's initial state and
    compare the GPU's step from the same state with it, element by element.
    Otherwise time the BR velocity of seeded targets (against all sources)
    sized to target_seconds and compare those targets.
    """
    import oracle
    import torch
    threads = oracle_threads()
    P = oracle.Problem(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt)
    w_probe = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
    probe = rr.sample_targets(wl.n, 256, seed=99)
    t0 = time.perf_counter()
    oracle.br_velocity(P, z0, w_probe, targets=probe, threads=threads)
    rate = probe.size * wl.n / (time.perf_counter() - t0)        # pairs/s
    full_step = 3.0 * wl.n * wl.n / rate

    def rel(a, b):
        return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

    if full_step <= 3.0 * target_seconds:
        t0 = time.perf_counter()
        zr, wr = oracle.rk3(P, z0, w0, 1, threads=threads)
        dt = time.perf_counter() - t0
        ctx = ctx_factory()
        dev = ctx.workspace.device
        zd = torch.from_numpy(z0.ravel()).to(dev); wd = torch.from_numpy(w0.ravel()).to(dev)
        ctx.init_state(zd, wd)
        ctx.step(1)
        z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
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
    ctx = ctx_factory()
    dev = ctx.workspace.device
    zd = torch.from_numpy(z0.ravel()).to(dev); wd = torch.from_numpy(w_probe.ravel()).to(dev)
    ud = torch.empty_like(zd)
    ctx.br_velocity(zd, wd, ud)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = oracle.br_velocity(P, z0, w_probe, targets=tg, threads=threads)
    dt = time.perf_counter() - t0
    return {
        "value": tg.size * wl.n / dt, "unit": "pair-interactions/s", "cores": threads,
        "kind": "oracle",
        "sample": f"BR velocity of {tg.size} seeded targets x {wl.n} sources "
                  f"({tg.size * wl.n:.3e} pairs, {dt:.1f} s), synthetic vorticity",
        "seconds": dt,
        "gpu_vs_oracle_max_rel_err": {"u": rel(ud.cpu().numpy().reshape(3, -1)[:, tg], ref)},
    }


def cpu_oracle_detail(threads: int, sweep_u=None, traj64=None):
    """The oracle's own rates on the other workloads (a few seconds of host
    time in all): one full BR evaluation of the 64 x 64 workload, 1024 seeded
    targets of the 1024 x 1024 workload, and the 64 x 64 evaluation on one
    thread.  With the 1M-point sweep's GPU velocities (FP64 and FP32 forms,
    same state and vorticity) their error on those 1024 targets as well.
    With the GPU's 64 x 64 trajectory, the oracle's own trajectory of the
    workload (its step count from its initial state), timed and compared."""
    import oracle
    out = {"threads": threads}
    for name, key, targets, nthreads in (
            ("periodic64_full_br", "periodic64_single_fp64", None, threads),
            ("periodic1024_sampled_br", "periodic1024_multimode16_fp32", 1024, threads),
            ("periodic64_full_br_1thread", "periodic64_single_fp64", None, 1)):
        wl = rr.WORKLOADS[key]
        z, _ = wl.state()
        w = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
        P = oracle.Problem(wl.n1, wl.n2, eps=wl.eps)
        tg = rr.sample_targets(wl.n, targets, seed=7) if targets else None
        t0 = time.perf_counter()
        ref = oracle.br_velocity(P, z, w, targets=tg, threads=nthreads)
        dt = time.perf_counter() - t0
        pairs = (tg.size if targets else wl.n) * wl.n
        out[name] = {"pairs": pairs, "seconds": dt, "pairs_per_s": pairs / dt, "threads": nthreads}
        if targets and sweep_u is not None:
            scale = float(np.max(np.abs(ref)))
            for form, u in sweep_u.items():
                ug = u.reshape(3, -1)[:, tg]
                out[name][f"{form}_vs_oracle_max_rel_err"] = float(np.max(np.abs(ug - ref)) / scale)
    if traj64 is not None:
        wl = rr.WORKLOADS["periodic64_single_fp64"]
        z0, w0 = wl.state()
        P = oracle.Problem(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt)
        t0 = time.perf_counter()
        zr, wr = oracle.rk3(P, z0, w0, wl.steps, threads=threads)
        dt = time.perf_counter() - t0
        zg, wg = traj64
        out["periodic64_trajectory"] = {
            "steps": wl.steps, "pairs": 3.0 * wl.steps * wl.n * wl.n, "seconds": dt,
            "pairs_per_s": 3.0 * wl.steps * wl.n * wl.n / dt, "threads": threads,
            "gpu_vs_oracle_max_rel_err": {
                "z": float(np.max(np.abs(zg - zr)) / np.max(np.abs(zr))),
                "w": float(np.max(np.abs(wg - wr)) / np.max(np.abs(wr))),
                "z_motion": float(np.max(np.abs((zg - z0) - (zr - z0))) / np.max(np.abs(zr - z0)))}}
    return out


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

    if args.cutoff_only:
        print(json.dumps({"cutoff": cutoff_section(zm, torch)}), flush=True)
        return
    if args.low_order_only:
        print(json.dumps({"low_order_4096": low_order_section(zm, torch)}), flush=True)
        return
    if args.medium_only:
        print(json.dumps({"medium_order": medium_section(zm, torch)}), flush=True)
        return
    if args.free_only:
        print(json.dumps({"free_single_mode": free_section(zm, torch)}), flush=True)
        return
    if args.tune_report:
        print(json.dumps({"tune_report": tune_report(zm, torch)}), flush=True)
        return

    sweep_u = traj64 = None
    wl = rr.WORKLOADS[args.workload]
    prec = zm.ZM_FP32_PAIRS if wl.precision == "fp32_pairs" else zm.ZM_FP64
    steps = wl.steps if args.steps is None else args.steps
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = zm.Params(wl.n1, wl.n2, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt,
                  precision=prec)
    z0, w0 = wl.state()
    zd = torch.from_numpy(z0.ravel()).to(dev)
    wd = torch.from_numpy(w0.ravel()).to(dev)
    ctx = zm.Context(p)
    ctx.init_state(zd, wd)
    info = ctx.launch_info()
    stream = ctx.stream

    ctx.step(args.warmup)
    torch.cuda.synchronize()
    ctx.profile_read()                      # discard warm-up timings
    ctx.profile_enable(True)

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    ctx.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    stats = ctx.profile_read()
    ctx.profile_enable(False)

    pairs_per_step = 3 * info.pairs_per_eval
    elapsed = max(wall, gpu_s)
    value = pairs_per_step * steps / elapsed
    launches, pair_ms = stats["pairs"]
    avg_pair_s = pair_ms / 1e3 / max(launches, 1)
    achieved = FLOPS_PER_PAIR * info.pairs_per_eval / avg_pair_s / 1e12
    peak = PEAK_TFLOPS[wl.precision]
    kernel = "k_pairs_f64f" if prec == zm.ZM_FP64 else "k_pairs_f32"

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == zm.ZM_FP64 else "f32",
        "data": "synthetic",
        "config": {
            "workload": wl.name, "mesh": f"{wl.n1}x{wl.n2}", "points": wl.n,
            "eps_over_h": wl.eps_over_h, "atwood": wl.atwood, "dt": wl.dt,
            "precision": wl.precision, "image_layers": 0,
            "pairs_per_step": pairs_per_step, "pair_kernel_workgroups": info.workgroups,
            "source_splits": info.source_splits, "targets_per_lane": info.targets_per_lane,
        },
        "roofline": {
            "kernel": kernel, "bound": "alu", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(kernel, wl.name), "traffic_unit": "bytes/launch",
            "flops_per_pair": FLOPS_PER_PAIR, "pairs_per_launch": info.pairs_per_eval,
            "avg_launch_ms": avg_pair_s * 1e3, "launches": launches,
        },
        "kernel_ms": {k: {"launches": n, "total_ms": ms} for k, (n, ms) in stats.items()},
        "pair_kernel_share": pair_ms / 1e3 / elapsed,
    }

    if not args.no_sweep:
        out["br_sweep_1m"], sweep_u = br_sweep_1m(zm, torch)
        out["ensemble64_fp32_graph"] = ensemble64(zm, torch)
        out["periodic64_latency"], traj64 = small_mesh_latency(zm, torch)
        out["cutoff"] = cutoff_section(zm, torch)
        out["low_order_4096"] = low_order_section(zm, torch)
        out["free_single_mode"] = free_section(zm, torch)
        out["medium_order"] = medium_section(zm, torch)
    if args.serve_seconds > 0:
        out["serving"] = serving(zm, torch, window_s=args.serve_seconds)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(wl, lambda: zm.Context(p), z0, w0, args.cpu_seconds)
        out["cpu_baseline"]["gpu_speedup"] = value / out["cpu_baseline"]["value"]
        out["cpu_oracle_detail"] = cpu_oracle_detail(out["cpu_baseline"]["cores"], sweep_u, traj64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
