#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X: multistep EPI steps of the DFR
shallow-water model, each one KIOPS phi-combination driven by complex-step
J*v products, plus the J*v kernel alone.

Default workload (the headline): an ensemble of 64 independent members (ne in
{8, 12, 16, 24, 32, 40}, p in {4, 5, 6}), EPI4, dt = 900 s, Krylov dimension
<= 32, in the mixed batched form (complex-FP32 products, FP32 Krylov basis,
FP64 inner products, Hessenberg, exponential and update) at KIOPS tol 1e-6,
on the balanced zonal flow with seeded perturbations (synthetic; see
paper_2101_05617_amd/inputs.py).  One "step" is one EPI step of every member;
the value is member EPI steps per second.  Alongside: the other ensemble
forms (plain FP64, sequential, device-driven rounds) with their errors after
one simulated day, and the single-grid workloads (--workload NAME for one).

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(ROOT, "profiles")   # committed rocprofv3 summaries
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6    # MI355X, FP64 vector (and FP64 matrix) peak
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X, FP32 vector peak
METRIC = "complex-step Jv/s + EPI steps/s, FP64 plain vs FP32-Jv batched at stated error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def jv_bytes_per_node(form):
    # algorithmic bytes of one complex-step J*v per node: read q, read v, write J*v
    # (the FP32-basis form's stand-alone product reads and writes FP64 like
    # the FP32 form; inside KIOPS its basis reads and writes are 12 B)
    return {"fp64": 72, "fp32_jv": 12 + 24 + 24, "fp32_jv_basis32": 12 + 24 + 24}[form]


def arnoldi_jv_bytes_per_node(p, iop=2, prec="fp64"):
    # the J*v kernel as launched inside KIOPS additionally reads the p scaled
    # b-columns of the augmented operator (FP64) and the previous basis
    # vector for the fused inner products: 72 + 24 p + 24 in FP64 (iop = 2);
    # with FP32 products on an FP64 basis the state is read as an FP32 copy
    # (60 + 24 p + 24); with an FP32 basis the basis vectors read and written
    # and the b-columns are FP32 too (36 + 12 p + 12)
    if prec == "fp64":
        return 72 + 24 * p + (24 if iop >= 2 else 0)
    if prec == "fp32_jv":
        return 60 + 24 * p + (24 if iop >= 2 else 0)
    return 36 + 12 * p + (12 if iop >= 2 else 0)


EPI_M = {2: 1, 3: 2, 4: 3, 5: 4, 6: 4}   # phi-columns b_1..b_M of an EPI step


def time_jv(g, q, vs, outs, eps, prec, reps):
    """Mean duration (ms) of back-to-back J*v launches, HIP events on the
    library's (torch's current) stream; v and out rotate through buffers."""
    import torch
    from paper_2101_05617_amd import dfrsw
    for k in range(3):
        dfrsw.dfr_jvp_complex_step(g, q, vs[k % len(vs)], eps, prec, outs[k % len(outs)])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(reps):
        dfrsw.dfr_jvp_complex_step(g, q, vs[k % len(vs)], eps, prec, outs[k % len(outs)])
    e1.record()
    torch.cuda.synchronize()
    dfrsw.dfr_sync(g)
    return e0.elapsed_time(e1) / reps


CAL_BYTES = 256 * 1024 * 1024


def calibration_copy():
    """A plain device-to-device copy of exactly 256 MiB: the calibration point
    of the FETCH_SIZE / WRITE_SIZE counters in profiled runs."""
    import torch
    a = torch.ones(CAL_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


MEASURED_COPY_BYTES = 2 * 1024 ** 3


def measured_copy_gbs(reps=5):
    """Bandwidth the library's streaming copy (dfr_stream_copy: 16 bytes per
    lane) reaches over 2 GiB (read + write bytes over its duration, best of
    `reps`, HIP events on torch's current stream, where it is launched): the
    practical ceiling of a streaming kernel on this GPU, reported beside the
    published peak."""
    import torch
    from paper_2101_05617_amd import dfrsw
    a = torch.ones(MEASURED_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream().cuda_stream
    dfrsw.dfr_stream_copy(a, b, s)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dfrsw.dfr_stream_copy(a, b, s)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.synchronize()
    return 2 * MEASURED_COPY_BYTES / (best * 1e-3) / 1e9


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "dfrsw_internal.h"):
        with open(os.path.join(ROOT, "paper_2101_05617_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def summarize_profile(args):
    """Text summary of rocprofv3 output: per-kernel durations (--kernel-trace
    --stats) and, from FETCH_SIZE / WRITE_SIZE passes, the HBM bytes per launch
    of the kernel named by --kernel, scaled by what the same counter reads for
    the 256 MiB calibration copy."""
    import csv
    lines = []
    rows = list(csv.DictReader(open(os.path.join(args.summarize_profile, "run_kernel_stats.csv"))))
    lines.append(f"{'kernel':90s} {'calls':>6s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}")
    for r in rows[:12]:
        lines.append(f"{r['Name'][:90]:90s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:9.3f} {float(r['Percentage']):6.2f}")
    sel = [r for r in rows if re.search(args.kernel, r["Name"])]
    if sel:
        calls = sum(int(r["Calls"]) for r in sel)
        total_ns = sum(float(r["TotalDurationNs"]) for r in sel)
        for r in sel:
            lines.append(f"selected kernel: {r['Name'][:120]}")
        lines.append(f"selected_avg_us (all launches, tuning included): {total_ns / calls / 1e3:.3f} "
                     f"over {calls} launches")
        tr = [r for r in csv.DictReader(open(os.path.join(args.summarize_profile, "run_kernel_trace.csv")))
              if re.search(args.kernel, r["Kernel_Name"])]
        tr.sort(key=lambda r: int(r["Start_Timestamp"]))
        last = tr[-args.last:] if args.last else tr
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in last]
        lines.append(f"timed_region_avg_us: {sum(d) / len(d):.3f} over the last {len(d)} launches")
    traffic = {}
    for counter, d in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        if not d:
            continue
        cc = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
        cal = max(float(r["Counter_Value"]) for r in cc
                  if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"])
        vals = [float(r["Counter_Value"]) for r in cc
                if r["Counter_Name"] == counter and re.search(args.kernel, r["Kernel_Name"])]
        if not vals:
            lines.append(f"{counter}: no dispatch of a kernel matching {args.kernel!r}")
            continue
        factor = (CAL_BYTES / 1024.0) / cal
        per = sum(vals) / len(vals) * factor * 1024.0
        traffic[counter] = per
        lines.append(f"{counter}: the calibration copy counts {cal:.1f} KiB for {CAL_BYTES // 1024} KiB "
                     f"(factor {factor:.3f}); kernel mean {sum(vals) / len(vals):.1f} KiB over {len(vals)} "
                     f"dispatches -> {per / 1e6:.3f} MB per launch")
    if len(traffic) == 2:
        lines.append(f"traffic_bytes_per_launch: {traffic['FETCH_SIZE'] + traffic['WRITE_SIZE']:.0f} "
                     f"fetch {traffic['FETCH_SIZE']:.0f} write {traffic['WRITE_SIZE']:.0f} "
                     f"kernel_source: {kernel_source_digest()}")
    # further counter passes: the mean of every counter over the selected
    # kernel's last N dispatches
    util = {}
    for d in args.counters or []:
        cc = [r for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv")))
              if re.search(args.kernel, r["Kernel_Name"])]
        by = {}
        for r in cc:
            by.setdefault(r["Counter_Name"], []).append((int(r.get("Dispatch_Id") or 0), float(r["Counter_Value"])))
        for name, v in sorted(by.items()):
            v.sort()
            v = [x for _, x in (v[-args.last:] if args.last else v)]
            util[name] = sum(v) / len(v)
            lines.append(f"counter {name}: mean {util[name]:.6g} over {len(v)} dispatches")
    if "SQ_WAVES" in util and util["SQ_WAVES"] > 0:
        # instruction mix per wave and the share of wave cycles spent waiting
        waves = util["SQ_WAVES"]
        per = {k[len("SQ_INSTS_"):]: util[k] / waves for k in sorted(util) if k.startswith("SQ_INSTS_")
               and not k.startswith("SQ_INSTS_VALU_FLOPS")}
        lines.append("per_wave: " + " ".join(f"{k}={v:.1f}" for k, v in per.items()))
        if util.get("SQ_WAVE_CYCLES"):
            for k in ("SQ_WAIT_INST_ANY", "SQ_WAIT_ANY"):
                if k in util:
                    lines.append(f"{k} / SQ_WAVE_CYCLES: {util[k] / util['SQ_WAVE_CYCLES']:.3f}")
    if util:
        lines.append("utilisation: " + " ".join(f"{k}={v:.6g}" for k, v in sorted(util.items())) +
                     f" kernel_source: {kernel_source_digest()}")
    print("\n".join(lines))
    return 0


def profiled_utilisation(name):
    """Counter means (VALUBusy, LdsUtil, ...) recorded in profiles/<name> for
    the current kernel source, or None."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("utilisation:"):
            parts = line.split()
            if parts[-1] != kernel_source_digest():
                return None
            return {k: float(v) for k, v in (p.split("=") for p in parts[1:-2])}
    return None


def utilisation_summary(name, avg_us):
    """The recorded counter means of profiles/<name> as percentages against the
    chip (VALU busy, LDS busy, occupancy, matrix-core busy, active lanes per
    VALU instruction) and the FP64 / FP32 vector flops per launch as TFLOP/s
    over `avg_us` (default: the profile's own timed average) against the
    vector peaks; None without a record for the current kernel source."""
    u = profiled_utilisation(name)
    if not u:
        return None
    if not avg_us:   # the profile's own timed average
        for line in open(os.path.join(PROFILES, name)):
            if line.startswith("timed_region_avg_us:"):
                avg_us = float(line.split()[1])
    out = {k2: u.get(k1) for k1, k2 in (("VALUBusy", "valu_busy_pct"), ("LdsUtil", "lds_util_pct"),
                                         ("OccupancyPercent", "occupancy_pct"), ("MfmaUtil", "mfma_util_pct"),
                                         ("VALUUtilization", "valu_active_lanes_pct"))}
    if u.get("SQ_WAVES"):
        for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"):
            if k in u:
                out[k[len("SQ_INSTS_"):].lower() + "_insts_per_wave"] = u[k] / u["SQ_WAVES"]
        if u.get("SQ_WAVE_CYCLES") and "SQ_WAIT_ANY" in u:
            out["wait_fraction_of_wave_cycles"] = u["SQ_WAIT_ANY"] / u["SQ_WAVE_CYCLES"]
    for key, peak, tag in (("SQ_INSTS_VALU_FLOPS_FP64", FP64_VECTOR_PEAK_TFLOPS, "fp64"),
                           ("SQ_INSTS_VALU_FLOPS_FP32", FP32_VECTOR_PEAK_TFLOPS, "fp32")):
        if key in u and avg_us:
            # the counter adds an instruction's flops once per wave: x 64 lanes
            # (issued lane slots; inactive lanes included)
            tf = u[key] * 64 / (avg_us * 1e-6) / 1e12
            out[f"valu_{tag}_tflops"] = tf
            out[f"valu_{tag}_frac_of_peak"] = tf / peak
    return out


def profiled_traffic(name):
    """HBM bytes per launch recorded in profiles/<name> for the current kernel
    source, or None (no record, or the kernels changed since)."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            parts = line.split()
            if parts[-1] == kernel_source_digest():
                return float(parts[1])
    return None


def mixed_study(steps):
    """c2_ne60_p6_jet: the same EPI6 integration with the plain FP64 product and
    with the complex-FP32 product; steps/s of each (start-up included) and the
    relative L2 difference in h after `steps` steps."""
    import numpy as np
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    w = inputs.WORKLOADS["c2_ne60_p6_jet"]
    opts = dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max)
    # the stated-error comparison: KIOPS tolerance one decade above the
    # relative noise of a complex-FP32 product (about 1e-7)
    tol_matched = 1e-6
    opts_matched = dfrsw.kiops_opts(tol=tol_matched, m_max=w.m_max)
    res, finals = {}, {}
    for name, prec, eps, opts in (("fp64", "fp64", 1e-150, opts), ("fp32_jv", "fp32_jv", w.eps, opts),
                                  ("fp32_jv_tol1e-6", "fp32_jv", w.eps, opts_matched),
                                  ("fp32_jv_basis32_tol1e-6", "fp32_jv_basis32", w.eps, opts_matched),
                                  ("fp64_tol1e-6", "fp64", 1e-150, opts_matched)):
        g = dfrsw.Grid(w.ne, w.p, *w.constants())
        dfrsw.dfr_autotune(g, prec)
        P, B1, B2 = g.node_frames()
        Q, _ = inputs.initial_state(w, P, B1, B2)
        st = dfrsw.epi_create(g, w.order, w.dt_nd, torch.from_numpy(Q).cuda(),
                              startup_substeps=w.startup_substeps, eps=eps, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nmv = 0
        t_startup = None
        for k in range(steps):
            nmv += dfrsw.epi_step(g, st, opts)["n_matvec"]
            if k + 1 == w.order - 2:
                torch.cuda.synchronize()
                t_startup = time.perf_counter()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        finals[name] = dfrsw.epi_get_state(st).cpu().numpy()
        n_after = steps - (w.order - 2)
        res[name] = {"steps_per_s": steps / (t1 - t0), "wall_s": t1 - t0, "jv_per_step": nmv / steps,
                     "epi6_steps_per_s_after_startup": n_after / (t1 - t_startup) if t_startup else None,
                     "tile": dfrsw.dfr_get_tile(g), "tile_krylov": dfrsw.dfr_get_krylov_tile(g)}
        log(f"c2 {name}: {steps} steps in {t1 - t0:.2f}s, {nmv / steps:.0f} J*v/step")
        del st, g
        torch.cuda.synchronize()
    N = w.n_nodes

    def errs(name):
        a, b = finals[name], finals["fp64"]
        err_h = float(np.linalg.norm(a[:N] - b[:N]) / np.linalg.norm(b[:N]))
        err_all = max(float(np.linalg.norm(a[f * N:(f + 1) * N] - b[f * N:(f + 1) * N]) /
                            np.linalg.norm(b[f * N:(f + 1) * N])) for f in range(3))
        return err_h, err_all
    err_h, err_all = errs("fp32_jv")
    em_h, em_all = errs("fp32_jv_tol1e-6")
    eb_h, eb_all = errs("fp32_jv_basis32_tol1e-6")
    e64_h, e64_all = errs("fp64_tol1e-6")
    base = res["fp64"]["steps_per_s"]
    return {"workload": f"{w.name}: ne={w.ne}, p={w.p} ({N} nodes), EPI6, dt={w.dt_s:g}s, {steps} steps "
                        f"({steps * w.dt_s / 86400:g} days), tol {w.tol:g}, m<={w.m_max}",
            "fp64": res["fp64"], "fp32_jv": res["fp32_jv"],
            "speedup_mixed_over_fp64": res["fp32_jv"]["steps_per_s"] / base,
            "rel_l2_error_h_mixed_vs_fp64": err_h, "rel_l2_error_max_field": err_all,
            "at_stated_error": {
                "note": f"KIOPS tol {tol_matched:g} (one decade above the complex-FP32 product's relative "
                        f"noise); error and speed-up against plain FP64 at tol {w.tol:g}",
                "fp32_jv": res["fp32_jv_tol1e-6"], "fp64": res["fp64_tol1e-6"],
                "fp32_jv_basis32": res["fp32_jv_basis32_tol1e-6"],
                "speedup_mixed_over_fp64": res["fp32_jv_tol1e-6"]["steps_per_s"] / base,
                "speedup_mixed_basis32_over_fp64": res["fp32_jv_basis32_tol1e-6"]["steps_per_s"] / base,
                "rel_l2_error_h_mixed_basis32": eb_h, "rel_l2_error_max_field_mixed_basis32": eb_all,
                "speedup_fp64_over_fp64": res["fp64_tol1e-6"]["steps_per_s"] / base,
                "rel_l2_error_h_mixed": em_h, "rel_l2_error_max_field_mixed": em_all,
                "rel_l2_error_h_fp64": e64_h, "rel_l2_error_max_field_fp64": e64_all}}


# the ensemble forms compared in the headline: (name, precision, form, KIOPS
# tolerance).  The first is the headline's mixed batched form at the stated
# error (FP32 products, FP32 Krylov basis; inner products, norms, Hessenberg,
# exponential and EPI update FP64; tolerance one decade above the relative
# noise of a complex-FP32 product); the last is plain FP64, one member after
# another, the reference of every error.
# (name, precision, form, KIOPS tol, who drives the batched form's rounds)
ENSEMBLE_FORMS = [
    ("fp32_jv_basis32_batched_tol1e-6", "fp32_jv_basis32", "batched", 1e-6, "host"),
    ("fp32_jv_basis32_batched_device_rounds_tol1e-6", "fp32_jv_basis32", "batched", 1e-6, "device"),
    ("fp32_jv_batched_tol1e-6", "fp32_jv", "batched", 1e-6, "host"),
    ("fp64_batched_tol1e-6", "fp64", "batched", 1e-6, "host"),
    ("fp64_sequential_tol1e-6", "fp64", "sequential", 1e-6, "host"),
    ("fp32_jv_batched", "fp32_jv", "batched", 1e-10, "host"),
    ("fp64_batched", "fp64", "batched", 1e-10, "host"),
    ("fp64_batched_device_rounds", "fp64", "batched", 1e-10, "device"),
    ("fp64_sequential", "fp64", "sequential", 1e-10, "host"),
]


def ensemble_headline(args, forms=None):
    """The ensemble workload (64 members, ne in {8..40}, p in {4,5,6}, EPI4,
    dt 900 s, m <= 32) in every form of ENSEMBLE_FORMS: W untimed steps (the
    EPI2 start-up steps first), K timed steps of all members, then untimed
    steps to the end of the simulated day (96 steps), whose states give the
    error in h of each form against plain FP64 sequential at tol 1e-10.  In
    the headline form's timed steps HIP events bracket the launches of its
    Krylov-form product (the roofline); after the day, up to 20 more steps
    bracket every batched launch (the per-kind breakdown)."""
    import numpy as np
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    from paper_2101_05617_amd.ensemble import Ensemble
    members = inputs.ensemble_members(args.ensemble_members)
    w0 = members[0]
    W, K = args.warmup, args.steps
    day = int(round(86400.0 / w0.dt_s))
    total_nodes = sum(w.n_nodes for w in members)
    forms = forms or ENSEMBLE_FORMS
    res, finals = {}, {}
    for name, prec, form, tol, rounds in forms:
        opts = dfrsw.kiops_opts(tol=tol, m_max=w0.m_max)
        ens = Ensemble(members, prec=prec, form=form, rounds=rounds)
        for _ in range(W):
            ens.step(opts)
        headline = name == forms[0][0]
        if headline and form == "batched":
            dfrsw.dfr_ensemble_timing_kinds(ens.eg, ["jv_arnoldi"])
            dfrsw.dfr_ensemble_timing_enable(ens.eg, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        agg = {"n_matvec": 0, "n_substeps": 0, "n_rejected": 0, "n_expm": 0}
        for _ in range(K):
            for st in ens.step(opts):
                for k in agg:
                    agg[k] += st[k]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r = {"member_steps_per_s": len(members) * K / wall, "wall_s": wall, "ms_per_step": 1e3 * wall / K,
             "jv_per_member_step": agg["n_matvec"] / (len(members) * K),
             "expm_per_member_step": agg["n_expm"] / (len(members) * K),
             "substeps_per_member_step": agg["n_substeps"] / (len(members) * K),
             "rejections_per_member_step": agg["n_rejected"] / (len(members) * K), "kiops_tol": tol,
             "rounds": rounds if form == "batched" else None}
        if form == "batched" and rounds == "device":
            r["rounds_with_work_and_launched"] = dfrsw.dfr_ensemble_round_counts(ens.eg)
        done = W + K
        if headline and form == "batched":
            r["roofline_kernel"] = dfrsw.dfr_ensemble_timing_read(ens.eg, "jv_arnoldi")
            dfrsw.dfr_ensemble_timing_enable(ens.eg, False)
        if not args.headline_only:
            for _ in range(max(0, day - done)):
                ens.step(opts)
            done = max(done, day)
            finals[name] = [ens.state(k) for k in range(len(members))]
        r["steps_at_error_check"] = done
        if headline and form == "batched":
            # after the states of the error check: steps with every batched
            # launch bracketed (the time of each kind)
            n2 = min(K, 20) if not args.headline_only else 0
            if n2:
                dfrsw.dfr_ensemble_timing_kinds(ens.eg, None)
                dfrsw.dfr_ensemble_timing_enable(ens.eg, True)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(n2):
                    ens.step(opts)
                torch.cuda.synchronize()
                wall2 = time.perf_counter() - t1
                r["kernels"] = {k: dfrsw.dfr_ensemble_timing_read(ens.eg, k) for k in dfrsw.KERNEL_KINDS}
                r["kernels_steps"], r["kernels_wall_s"] = n2, wall2
                r["member_steps_per_s_every_launch_evented"] = len(members) * n2 / wall2
                dfrsw.dfr_ensemble_timing_enable(ens.eg, False)
        res[name] = r
        log(f"ensemble {name}: {len(members)} members x {K} timed steps in {wall:.3f}s "
            f"({r['member_steps_per_s']:.0f} member steps/s, {r['jv_per_member_step']:.1f} J*v per member step)")
        ens.close()
        del ens
        torch.cuda.synchronize()

    def err(name):
        num = den = worst = 0.0
        for w, a, b in zip(members, finals[name], finals["fp64_sequential"]):
            N = w.n_nodes
            e2, r2 = float(np.sum((a[:N] - b[:N]) ** 2)), float(np.sum(b[:N] ** 2))
            num += e2
            den += r2
            worst = max(worst, (e2 / r2) ** 0.5)
        return {"all_members": (num / den) ** 0.5, "worst_member": worst}
    if "fp64_sequential" in finals:
        for name in finals:
            res[name]["rel_l2_error_h_vs_fp64_sequential"] = err(name)
    out = {"members": len(members), "nodes_all_members": total_nodes, "forms": res,
           "simulated_days_at_error_check": (res[forms[0][0]]["steps_at_error_check"]) * w0.dt_s / 86400.0,
           "day_steps": day}
    if "fp64_sequential" in res:
        base = res["fp64_sequential"]["member_steps_per_s"]
        out["speedup_over_fp64_sequential"] = {n: v["member_steps_per_s"] / base for n, v in res.items()}
    if "fp64_sequential_tol1e-6" in res:
        base6 = res["fp64_sequential_tol1e-6"]["member_steps_per_s"]
        out["speedup_over_fp64_sequential_tol1e-6"] = {n: v["member_steps_per_s"] / base6 for n, v in res.items()}
    if "fp64_batched_tol1e-6" in res:
        b6 = res["fp64_batched_tol1e-6"]["member_steps_per_s"]
        out["precision_share"] = {
            "note": "at tol 1e-6: each batched form over FP64 batched (what the precision adds to batching)",
            **{n: v["member_steps_per_s"] / b6 for n, v in res.items() if "batched_tol1e-6" in n}}
    return out


def c4_study(steps, reps):
    """c4_ne120_p6_mountain (4,233,600 nodes, orography): the J*v kernel in
    FP64 and complex FP32 (three rotating buffers, beyond the last-level
    cache), and EPI6 with each product form: the start-up steps untimed, then
    `steps` timed steps; relative L2 difference in h between the two forms."""
    import numpy as np
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    w = inputs.WORKLOADS["c4_ne120_p6_mountain"]
    N = w.n_nodes
    opts = dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max)
    out = {"workload": f"{w.name}: ne={w.ne}, p={w.p} ({N} nodes), Gaussian mountain, EPI6, dt={w.dt_s:g}s, "
                       f"tol {w.tol:g}, m<={w.m_max}; {w.order - 2} start-up steps untimed, {steps} timed"}
    # the stated-error comparison: KIOPS tolerance one decade above the
    # relative noise of a complex-FP32 product (about 1e-7)
    tol_matched = 1e-6
    opts_matched = dfrsw.kiops_opts(tol=tol_matched, m_max=w.m_max)
    finals = {}
    for name, prec, eps, opts, with_jv in (("fp64", "fp64", 1e-150, opts, True),
                                           ("fp32_jv", "fp32_jv", 1e-20, opts, True),
                                           ("fp32_jv_basis32", "fp32_jv_basis32", 1e-20, opts, True),
                                           ("fp32_jv_basis32_tol1e-6", "fp32_jv_basis32", 1e-20, opts_matched, False),
                                           ("fp64_tol1e-6", "fp64", 1e-150, opts_matched, False)):
        g0 = dfrsw.Grid(w.ne, w.p, *w.constants())
        P, B1, B2 = g0.node_frames()
        g0.close()
        Q, hB = inputs.initial_state(w, P, B1, B2)
        g = dfrsw.Grid(w.ne, w.p, *w.constants(), hB=hB)
        tile = dfrsw.dfr_autotune(g, prec)
        q = torch.from_numpy(Q).cuda()
        if with_jv:
            vs = [torch.randn(3 * N, dtype=torch.float64, device="cuda") * 1e-3 for _ in range(3)]
            outs = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(3)]
            t_jv = time_jv(g, q, vs, outs, eps, prec, reps)
            bpn = jv_bytes_per_node(prec)
            del vs, outs
        st = dfrsw.epi_create(g, w.order, w.dt_nd, q, startup_substeps=w.startup_substeps, eps=eps, prec=prec)
        for _ in range(w.order - 2):
            dfrsw.epi_step(g, st, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nmv = 0
        for _ in range(steps):
            nmv += dfrsw.epi_step(g, st, opts)["n_matvec"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        finals[name] = dfrsw.epi_get_state(st).cpu().numpy()
        r = {"tile": tile, "epi6_steps_per_s": steps / dt, "jv_per_step": nmv / steps,
             "sim_days_per_wall_hour": (steps * w.dt_s / 86400.0) / (dt / 3600.0)}
        if with_jv:
            r.update({"jv_us": t_jv * 1e3, "jv_per_s": 1e3 / t_jv, "jv_GBs": bpn * N / (t_jv * 1e-3) / 1e9,
                      "jv_frac_hbm": bpn * N / (t_jv * 1e-3) / 1e9 / HBM_PEAK_GBS})
        out[name] = r
        log(f"c4 {name}: {steps} EPI6 steps in {dt:.2f}s" + (f", J*v {t_jv * 1e3:.1f} us" if with_jv else ""))
        del st, g, q
        torch.cuda.synchronize()
    b = finals["fp64"]

    def err_h(name):
        a = finals[name]
        return float(np.linalg.norm(a[:N] - b[:N]) / np.linalg.norm(b[:N]))
    out["rel_l2_error_h_fp32_vs_fp64"] = err_h("fp32_jv")
    out["rel_l2_error_h_fp32_basis32_vs_fp64"] = err_h("fp32_jv_basis32")
    base = out["fp64"]["epi6_steps_per_s"]
    out["at_stated_error"] = {
        "note": f"KIOPS tol {tol_matched:g} (one decade above the complex-FP32 product's relative noise); "
                f"error and speed-up against plain FP64 at tol {w.tol:g} after the same steps",
        "fp32_jv_basis32": out.pop("fp32_jv_basis32_tol1e-6"), "fp64": out.pop("fp64_tol1e-6"),
        "rel_l2_error_h_fp32_basis32": err_h("fp32_jv_basis32_tol1e-6"),
        "rel_l2_error_h_fp64": err_h("fp64_tol1e-6")}
    a = out["at_stated_error"]
    a["speedup_fp32_basis32_over_fp64"] = a["fp32_jv_basis32"]["epi6_steps_per_s"] / base
    a["speedup_fp64_over_fp64"] = a["fp64"]["epi6_steps_per_s"] / base
    return out


def ausm_study(steps, reps):
    """The AUSM interface flux (App. D): the FP64 J*v kernel at ne = 60, p = 6
    (eight rotating buffers, beyond the last-level cache) and EPI5 at
    ne = 30, p = 5 (start-up untimed, then `steps` timed steps)."""
    import numpy as np
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    out = {}
    w2 = inputs.WORKLOADS["c2_ne60_p6_jet"]
    g2 = dfrsw.Grid(w2.ne, w2.p, *w2.constants())
    dfrsw.dfr_set_riemann(g2, "ausm")
    tile = dfrsw.dfr_autotune(g2, "fp64")
    P, B1, B2 = g2.node_frames()
    Q2, _ = inputs.initial_state(w2, P, B1, B2)
    q2 = torch.from_numpy(Q2).cuda()
    N2 = w2.n_nodes
    vs = [torch.randn(3 * N2, dtype=torch.float64, device="cuda") * 1e-3 for _ in range(8)]
    outs = [torch.empty(3 * N2, dtype=torch.float64, device="cuda") for _ in range(8)]
    t = time_jv(g2, q2, vs, outs, 1e-150, "fp64", reps)
    out["jv_ne60_p6_fp64"] = {"tile": tile, "us": t * 1e3, "jv_per_s": 1e3 / t,
                              "GBs": 72 * N2 / (t * 1e-3) / 1e9, "frac_hbm": 72 * N2 / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log(f"AUSM ne=60 p=6 J*v fp64 {t * 1e3:.1f} us")
    del vs, outs, q2, g2
    torch.cuda.synchronize()

    w = inputs.WORKLOADS["c1_ne30_p5"]
    opts = dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max)
    finals = {}
    for flux in ("rusanov", "ausm"):
        g = dfrsw.Grid(w.ne, w.p, *w.constants())
        dfrsw.dfr_set_riemann(g, flux)
        dfrsw.dfr_autotune(g, "fp64")
        P, B1, B2 = g.node_frames()
        Q, _ = inputs.initial_state(w, P, B1, B2)
        st = dfrsw.epi_create(g, w.order, w.dt_nd, torch.from_numpy(Q).cuda(), startup_substeps=w.startup_substeps)
        for _ in range(w.order - 2):
            dfrsw.epi_step(g, st, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nmv = 0
        for _ in range(steps):
            nmv += dfrsw.epi_step(g, st, opts)["n_matvec"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        finals[flux] = dfrsw.epi_get_state(st).cpu().numpy()
        if flux == "ausm":
            out["epi5_c1_ne30_p5"] = {"steps_per_s": steps / dt, "jv_per_step": nmv / steps,
                                      "sim_days_per_wall_hour": (steps * w.dt_s / 86400.0) / (dt / 3600.0)}
        log(f"c1 EPI5 {flux}: {steps} steps in {dt:.3f}s, {nmv / steps:.0f} J*v/step")
        del st, g
        torch.cuda.synchronize()
    N = w.n_nodes
    a, b = finals["ausm"], finals["rusanov"]
    out["epi5_c1_ne30_p5"]["rel_l2_diff_h_vs_rusanov"] = float(np.linalg.norm(a[:N] - b[:N]) / np.linalg.norm(b[:N]))
    return out


def diagnostics_study(reps):
    """dfr_diagnostics at ne = 60, p = 6: the state check, the per-node
    vorticity / density kernel and the final sums, per call (library kernel
    timing), and the algorithmic bytes of the first two (read q twice, write
    zeta: 56 B per node)."""
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    w = inputs.WORKLOADS["c2_ne60_p6_jet"]
    g = dfrsw.Grid(w.ne, w.p, *w.constants())
    P, B1, B2 = g.node_frames()
    Q, _ = inputs.initial_state(w, P, B1, B2)
    q = torch.from_numpy(Q).cuda()
    for _ in range(3):
        dfrsw.dfr_diagnostics(g, q)
    dfrsw.dfr_timing_enable(g, True)
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, it = dfrsw.dfr_diagnostics(g, q)
    wall = (time.perf_counter() - t0) / reps
    k_ms = sum(dfrsw.dfr_timing_read(g, k)[0] for k in ("other", "finalize")) / reps
    dfrsw.dfr_timing_enable(g, False)
    N = w.n_nodes
    log(f"diagnostics ne=60 p=6: {k_ms * 1e3:.1f} us kernels, {wall * 1e6:.0f} us per call")
    out = {"nodes": N, "kernel_us_per_call": k_ms * 1e3, "wall_us_per_call": wall * 1e6,
           "bytes_per_node": 56, "GBs": 56 * N / (k_ms * 1e-3) / 1e9,
           "frac_hbm": 56 * N / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "mass_energy_enstrophy": list(it)}
    del q, g
    return out


def large_dt_study(steps):
    """The large-time-step regime: the mountain flow on ne = 20, p = 5 (86,400
    nodes) with dt = 4 h, EPI3..EPI6 (start-up untimed, then `steps` timed
    steps each), and EPI6 with dt = 1 h over the same simulated time for
    comparison; KIOPS statistics per step."""
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    w0 = inputs.WORKLOADS["f2_ne20_p5_mountain_dt4h"]
    out = {"workload": f"{w0.name}: ne={w0.ne}, p={w0.p} ({w0.n_nodes} nodes), Gaussian mountain, "
                       f"tol {w0.tol:g}, m<={w0.m_max}"}
    g0 = dfrsw.Grid(w0.ne, w0.p, *w0.constants())
    P, B1, B2 = g0.node_frames()
    g0.close()
    Q, hB = inputs.initial_state(w0, P, B1, B2)
    g = dfrsw.Grid(w0.ne, w0.p, *w0.constants(), hB=hB)
    dfrsw.dfr_autotune(g, "fp64")
    opts = dfrsw.kiops_opts(tol=w0.tol, m_max=w0.m_max)
    for order, dt_s, nsteps in [(3, 14400.0, steps), (4, 14400.0, steps), (5, 14400.0, steps), (6, 14400.0, steps),
                                (6, 3600.0, 4 * steps)]:
        dt = dt_s * inputs.EARTH_OMEGA
        st = dfrsw.epi_create(g, order, dt, torch.from_numpy(Q).cuda(), startup_substeps=4)
        for _ in range(order - 2):
            dfrsw.epi_step(g, st, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        agg = {"n_matvec": 0, "n_substeps": 0, "n_rejected": 0}
        mmax = 0
        for _ in range(nsteps):
            s = dfrsw.epi_step(g, st, opts)
            for k in agg:
                agg[k] += s[k]
            mmax = max(mmax, s["m_last"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        key = f"epi{order}_dt{int(dt_s / 3600)}h"
        out[key] = {"steps_per_s": nsteps / el, "sim_days_per_wall_hour": (nsteps * dt_s / 86400.0) / (el / 3600.0),
                    "jv_per_step": agg["n_matvec"] / nsteps, "substeps_per_step": agg["n_substeps"] / nsteps,
                    "rejections_per_step": agg["n_rejected"] / nsteps, "max_krylov_m": mmax}
        log(f"large dt {key}: {nsteps} steps in {el:.3f}s, {agg['n_matvec'] / nsteps:.0f} J*v/step")
        del st
    del g
    torch.cuda.synchronize()
    return out


def ode_suite_study():
    """The stiff test problems of Sec. 5.1 on the GPU path: EPI4 and EPI6 over
    each problem's interval at one of Fig. 2's step sizes, KIOPS tol 1e-14;
    the error is the 2-norm against the exact solution (semilinear) or
    against EPI6 with a quarter of the step (the other two)."""
    import numpy as np
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    cases = [("adr", 40, 0.1, 2.2e-4), ("burgers", 1024, 1.0, 1.8e-3), ("semilinear", 400, 1.0, 5.0e-2)]
    out = {}
    opts = dfrsw.kiops_opts(tol=1e-14, m_max=64)
    for name, n, T, h in cases:
        D = dfrsw.OdeProblem(name, n)
        u0 = inputs.ode_initial_state(name, n)
        x = np.arange(1, n + 1) / (n + 1)

        def run(order, hh):
            nst = int(round(T / hh))
            st = dfrsw.epi_create(D, order, T / nst, torch.from_numpy(u0).cuda(), startup_substeps=4)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nmv = 0
            for _ in range(nst):
                nmv += dfrsw.epi_step(D, st, opts)["n_matvec"]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            q = dfrsw.epi_get_state(st).cpu().numpy()
            st.close()
            return q, el, nst, nmv

        if name == "semilinear":
            ref = np.concatenate([x * (1 - x) * np.exp(1.0), [1.0]])
        else:
            ref = run(6, h / 4)[0]
        res = {"n_unknowns": int(u0.size), "t_final": T, "dt": h}
        for order in (4, 6):
            q, el, nst, nmv = run(order, h)
            res[f"epi{order}"] = {"wall_s": el, "steps": nst, "steps_per_s": nst / el, "jv_per_step": nmv / nst,
                                  "error_2norm": float(np.linalg.norm(q[: n if name == 'semilinear' else None] -
                                                                      ref[: n if name == 'semilinear' else None]))}
            log(f"ODE {name} EPI{order}: {nst} steps in {el:.3f}s, {nmv / nst:.0f} J*v/step")
        out[name] = res
        D.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_leg(workload_name):
    """Time the oracle on this host: one steady-state EPI step after the
    start-up steps (untimed, one EPI2 sub-step each)."""
    import numpy as np

    import oracle
    from oracle import epi as oepi
    from paper_2101_05617_amd import inputs
    w = inputs.WORKLOADS[workload_name]
    G = oracle.OracleGrid(w.ne, w.ns, *w.constants())
    P, B1, B2 = G.node_frames()
    Q, _ = inputs.initial_state(w, P, B1, B2)
    E = oepi.EPI(G.rhs, lambda a, b: G.jvp(a, b, w.eps), w.order, w.dt_nd, Q, startup_substeps=1,
                 kiops_opts=dict(tol=w.tol, m_max=w.m_max))
    for _ in range(E.P):
        E.step()
    t0 = time.perf_counter()
    E.step()
    dt = time.perf_counter() - t0
    st = E.stats[-1]
    V = np.random.default_rng(0).standard_normal(3 * G.N)
    t1 = time.perf_counter()
    for _ in range(10):
        G.jvp(Q, V, w.eps)
    tj = (time.perf_counter() - t1) / 10
    out = {"step_s": dt, "jv_s": tj, "n_matvec": st.n_matvec}
    del G, E
    # the product alone on the two largest grids (one call after one untimed)
    for key, name in (("jv_s_c2", "c2_ne60_p6_jet"), ("jv_s_c4", "c4_ne120_p6_mountain")):
        wk = inputs.WORKLOADS[name]
        G0 = oracle.OracleGrid(wk.ne, wk.ns, *wk.constants())
        P, B1, B2 = G0.node_frames()
        del G0
        Qk, hB = inputs.initial_state(wk, P, B1, B2)
        Gk = oracle.OracleGrid(wk.ne, wk.ns, *wk.constants(), hB=hB)
        Vk = np.random.default_rng(1).standard_normal(3 * Gk.N) * 1e-3
        Gk.jvp(Qk, Vk, 1e-150)
        t1 = time.perf_counter()
        Gk.jvp(Qk, Vk, 1e-150)
        out[key] = time.perf_counter() - t1
        del Gk, Qk, Vk, P, B1, B2
    return out


def cpu_baseline_ensemble(_name=None):
    """Time the oracle on the six smallest members of the ensemble: each
    member's EPI2 start-up steps untimed, then four EPI4 steps timed (KIOPS
    tol 1e-10, the plain method's)."""
    import oracle
    from oracle import epi as oepi
    from paper_2101_05617_amd import inputs
    members = inputs.ensemble_members(64)
    pick = sorted(range(len(members)), key=lambda k: (members[k].n_nodes, k))[:6]
    wall = 0.0
    steps = nmv = 0
    for k in pick:
        w = members[k]
        G = oracle.OracleGrid(w.ne, w.ns, *w.constants())
        P, B1, B2 = G.node_frames()
        Q, _ = inputs.initial_state(w, P, B1, B2)
        E = oepi.EPI(G.rhs, lambda a, b, G=G: G.jvp(a, b), w.order, w.dt_nd, Q,
                     startup_substeps=w.startup_substeps, kiops_opts=dict(tol=w.tol, m_max=w.m_max))
        for _ in range(E.P):
            E.step()
        n0 = len(E.stats)
        t0 = time.perf_counter()
        for _ in range(4):
            E.step()
        wall += time.perf_counter() - t0
        steps += 4
        nmv += sum(x.n_matvec for x in E.stats[n0:])
        del G, E
    return {"member_steps": steps, "wall_s": wall, "n_matvec": nmv,
            "members": [f"member {k}: ne={members[k].ne}, p={members[k].p}" for k in pick]}


def jv_only(w, args):
    """Time the plain J*v kernel alone on workload w (buffers rotated past the
    last-level cache); prints one JSON line."""
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    g = dfrsw.Grid(w.ne, w.p, *w.constants())
    tile = dfrsw.dfr_autotune(g, args.prec)
    P, B1, B2 = g.node_frames()
    Q, _ = inputs.initial_state(w, P, B1, B2)
    q = torch.from_numpy(Q).cuda()
    N = w.n_nodes
    nbuf = max(2, min(8, int(4e8 // (48 * N))))
    vs = [torch.randn(3 * N, dtype=torch.float64, device="cuda") * 1e-3 for _ in range(nbuf)]
    outs = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
    eps = 1e-20 if args.prec == "fp32_jv" else 1e-150
    t = time_jv(g, q, vs, outs, eps, args.prec, args.jv_reps)
    calibration_copy()
    bpn = jv_bytes_per_node(args.prec)
    print(json.dumps({"workload": w.name, "prec": args.prec, "nodes": N, "tile": tile, "us": t * 1e3,
                      "GBs": bpn * N / (t * 1e-3) / 1e9, "frac_hbm": bpn * N / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}),
          flush=True)
    return 0


def run_cpu_legs(workload):
    """The oracle leg of `workload` in a child process, with one thread and
    with all of this host's share; {threads: result}."""
    legs = {}
    n_all = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    for nt in sorted({1, n_all}):
        env = dict(os.environ, OMP_NUM_THREADS=str(nt), OPENBLAS_NUM_THREADS=str(nt), MKL_NUM_THREADS=str(nt))
        log(f"cpu baseline: oracle ({workload}), {nt} thread(s)")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                            "--workload", workload], capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            log("cpu baseline failed: " + r.stderr[-2000:])
            break
        legs[nt] = json.loads(r.stdout.strip().splitlines()[-1])
    return legs, n_all


def cpu_baseline_entry(args, ens):
    """The cpu_baseline object: the oracle on the headline's workload (for the
    ensemble, its six smallest members) and, beside it, the single-grid leg
    (one EPI5 step at ne = 30, p = 5 and the product alone at the three
    largest grids)."""
    from paper_2101_05617_amd import inputs
    out = None
    if ens:
        legs, n_all = run_cpu_legs("c3_ensemble")
        if 1 in legs:
            cb = legs[1]
            out = {"value": cb["member_steps"] / cb["wall_s"], "unit": "member EPI steps/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"the six smallest ensemble members ({'; '.join(cb['members'])}): each one's two "
                             f"EPI2 start-up steps untimed, then four EPI4 steps timed ({cb['n_matvec']} J*v in "
                             f"all), KIOPS tol 1e-10, FP64",
                   "cpu": cpu_model()}
            if n_all in legs and n_all != 1:
                cm = legs[n_all]
                out["all_threads"] = {"value": cm["member_steps"] / cm["wall_s"], "cores": n_all}
    w = inputs.WORKLOADS["c1_ne30_p5" if ens else args.workload]
    legs, n_all = run_cpu_legs(w.name)
    if 1 in legs:
        cb = legs[1]
        sg = {"value": 1.0 / cb["step_s"], "unit": "EPI steps/s", "cores": 1, "kind": "oracle",
              "sample": f"one EPI{w.order} step of {w.name} after {w.order - 2} untimed EPI2 start-up steps "
                        f"({cb['n_matvec']} J*v); J*v alone {cb['jv_s'] * 1e3:.1f} ms",
              "jv_per_s": 1.0 / cb["jv_s"], "jv_per_s_c2_ne60_p6": 1.0 / cb["jv_s_c2"],
              "jv_per_s_c4_ne120_p6": 1.0 / cb["jv_s_c4"], "cpu": cpu_model()}
        if n_all in legs and n_all != 1:
            cm = legs[n_all]
            sg["all_threads"] = {"value": 1.0 / cm["step_s"], "cores": n_all, "jv_per_s": 1.0 / cm["jv_s"],
                                 "jv_per_s_c2_ne60_p6": 1.0 / cm["jv_s_c2"],
                                 "jv_per_s_c4_ne120_p6": 1.0 / cm["jv_s_c4"]}
        if out is None:
            out = sg
        else:
            out["single_grid"] = sg
    return out


def ensemble_headline_line(args):
    """The JSON line of the ensemble headline: member EPI steps/s of the mixed
    batched form at the stated error, with the roofline of its batched
    Krylov-form product timed live in its timed region."""
    from paper_2101_05617_amd import inputs
    forms = ENSEMBLE_FORMS[:1] if args.headline_only else ENSEMBLE_FORMS
    e = ensemble_headline(args, forms)
    name, prec = forms[0][0], forms[0][1]
    h = e["forms"][name]
    members = inputs.ensemble_members(args.ensemble_members)
    w0 = members[0]
    M = EPI_M[w0.order]
    ms, n_launch, nodes = h["roofline_kernel"]
    bpn = arnoldi_jv_bytes_per_node(M, 2, prec)
    achieved = bpn * nodes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    prof = "dfr_kernel_batch_krylov_c3_ensemble.txt"
    out = {
        "metric": METRIC,
        "value": h["member_steps_per_s"],
        "unit": "member EPI steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 complex-step products, f64 Krylov/expm/update",
        "data": "synthetic",
        "config": {"workload": f"c3_ensemble: {e['members']} independent members ({e['nodes_all_members']} nodes "
                               f"in all), ne in {{8,12,16,24,32,40}}, p in {{4,5,6}}, EPI4, dt={w0.dt_s:g}s, "
                               f"m<={w0.m_max}; mixed batched form: complex-FP32 J*v and FP32 Krylov basis, FP64 "
                               f"inner products, Hessenberg, exponential and update, KIOPS tol {forms[0][3]:g}; "
                               f"one step = one EPI step of every member",
                   "members": e["members"], "nodes": e["nodes_all_members"], "order": w0.order,
                   "dt_s": w0.dt_s, "kiops_tol": forms[0][3], "form": name},
        "sim_days_per_wall_hour": (h["member_steps_per_s"] / e["members"]) * w0.dt_s / 86400.0 * 3600.0,
        "jv_in_step_per_s": h["member_steps_per_s"] * h["jv_per_member_step"],
        "kiops_per_member_step": {k: h[k] for k in ("jv_per_member_step", "substeps_per_member_step",
                                                     "rejections_per_member_step", "expm_per_member_step")},
        "roofline": {
            "kernel": "dfr_kernel_batch: batched complex-FP32 J*v with the fused Arnoldi epilogue, FP32 basis "
                      "and b-columns (every member's tiles in one launch per p group)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(prof),
            "bytes_per_node": bpn, "avg_launch_us": ms / max(n_launch, 1) * 1e3, "launches": n_launch,
            "nodes_per_launch": nodes / max(n_launch, 1),
            "algorithmic_bytes_per_launch": bpn * nodes / max(n_launch, 1),
            "utilisation": utilisation_summary(prof, ms / max(n_launch, 1) * 1e3),
        },
        "ensemble_c3": e,
    }
    if "kernels" in h:
        n2 = h["kernels_steps"]
        out["every_launch_evented"] = {
            "steps": n2, "member_steps_per_s": h["member_steps_per_s_every_launch_evented"],
            "kernel_ms_per_step": {k: v[0] / n2 for k, v in h["kernels"].items()},
            "kernel_launches_per_step": {k: v[1] / n2 for k, v in h["kernels"].items()},
            "gpu_busy_fraction": sum(v[0] for v in h["kernels"].values()) / (h["kernels_wall_s"] * 1e3)}
    if not args.headline_only:
        f = e["forms"]
        out["at_stated_error"] = {
            "target": ">= 2x plain FP64 EPI steps/s at <= 1e-6 relative L2 error in h after one simulated day",
            "rel_l2_error_h_vs_fp64_sequential_tol1e-10": f[name]["rel_l2_error_h_vs_fp64_sequential"],
            "speedup_over_fp64_sequential_tol1e-10": e["speedup_over_fp64_sequential"][name],
            "speedup_over_fp64_sequential_tol1e-6": e["speedup_over_fp64_sequential_tol1e-6"][name],
            "speedup_fp64_batched_tol1e-6_over_fp64_sequential_tol1e-6":
                e["speedup_over_fp64_sequential_tol1e-6"]["fp64_batched_tol1e-6"],
            "error_reference": "plain FP64 member by member at KIOPS tol 1e-10 on the GPU, itself checked against "
                               "the FP64 oracle (tests: batched and sequential members bit for bit, the smallest "
                               "members over the whole day against the oracle)",
        }
    return out


def single_grid_run(w, steps, warmup, jv_reps):
    """EPI steps of one grid in plain FP64 (warmup untimed, then `steps`
    timed), the same number of steps again with every kernel timed by HIP
    events on the library's stream, and the plain J*v kernel alone; the
    result carries the roofline of the Krylov-form product."""
    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    args = argparse.Namespace(steps=steps, warmup=warmup, jv_reps=jv_reps)
    g = dfrsw.Grid(w.ne, w.p, *w.constants())
    tile = dfrsw.dfr_autotune(g, "fp64")
    tile_kr = dfrsw.dfr_get_krylov_tile(g)
    log(f"autotuned tiles: plain {tile}, Krylov form {tile_kr}")
    P, B1, B2 = g.node_frames()
    Q, hB = inputs.initial_state(w, P, B1, B2)
    q0 = torch.from_numpy(Q).cuda()
    st = dfrsw.epi_create(g, w.order, w.dt_nd, q0, startup_substeps=w.startup_substeps, eps=w.eps, prec="fp64")
    opts = dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max)
    P_hist = 0 if w.order == 2 else w.order - 2

    for k in range(args.warmup):
        s = dfrsw.epi_step(g, st, opts)
        log(f"warmup step {k + 1}/{args.warmup}: {s}")
    timed_includes_startup = args.warmup < P_hist

    # ---- timed region: K whole EPI steps (no instrumentation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stats.append(dfrsw.epi_step(g, st, opts))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.3f}s")

    # ---- the same number of further steps with every kernel bracketed by HIP
    # events on the library's stream: per-kernel durations (the events add
    # some idle time of their own, so this pass is not the headline figure)
    dfrsw.dfr_timing_enable(g, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        dfrsw.epi_step(g, st, opts)
    torch.cuda.synchronize()
    wall_instr = time.perf_counter() - t1
    kern = {k: dfrsw.dfr_timing_read(g, k) for k in dfrsw.KERNEL_KINDS}
    dfrsw.dfr_timing_enable(g, False)
    log(f"instrumented pass {wall_instr:.3f}s; kernels {kern}")
    ms_per_step = 1e3 * wall / args.steps
    steps_per_s = args.steps / wall
    n_jv = sum(s["n_matvec"] for s in stats)
    kernel_ms_total = sum(v[0] for v in kern.values())

    N = w.n_nodes
    M = {2: 1, 3: 2, 4: 3, 5: 4, 6: 4}[w.order]   # phi-columns b_1..b_M of the EPI combination
    ms_jva, n_jva = kern["jv_arnoldi"]
    avg_jva_ms = ms_jva / max(n_jva, 1)
    bytes_jva = arnoldi_jv_bytes_per_node(M) * N
    achieved = bytes_jva / (avg_jva_ms * 1e-3) / 1e9 if n_jva else 0.0

    # ---- the J*v kernel alone (plain FP64), rotating buffers
    vs = [torch.randn(3 * N, dtype=torch.float64, device="cuda") * 1e-3 for _ in range(4)]
    outs = [torch.empty(3 * N, dtype=torch.float64, device="cuda") for _ in range(4)]
    q = dfrsw.epi_get_state(st)
    jv_ms = time_jv(g, q, vs, outs, w.eps, "fp64", args.jv_reps)
    jv32_ms = time_jv(g, q, vs, outs, 1e-20, "fp32_jv", args.jv_reps)
    log(f"plain J*v: fp64 {jv_ms * 1e3:.1f} us, fp32 {jv32_ms * 1e3:.1f} us")

    sim_days_per_hour = (args.steps * w.dt_s / 86400.0) / (wall / 3600.0)

    out = {
        "steps_per_s": steps_per_s,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "config": {"workload": f"{w.name}: rotated cubed sphere ne={w.ne}, p={w.p} ({N} nodes, {3 * N} unknowns), "
                               f"EPI{w.order}, dt={w.dt_s:g}s, KIOPS tol={w.tol:g}, m<={w.m_max}, plain FP64",
                   "ne": w.ne, "p": w.p, "nodes": N, "order": w.order, "dt_s": w.dt_s,
                   "timed_steps_include_startup": timed_includes_startup},
        "tile": tile,
        "tile_krylov": tile_kr,
        "jv_per_s": 1e3 / jv_ms,
        "jv_per_s_fp32": 1e3 / jv32_ms,
        "jv_in_step_per_s": n_jv / wall,
        "sim_days_per_wall_hour": sim_days_per_hour,
        "kiops_per_step": {"n_matvec": n_jv / args.steps,
                           "n_substeps": sum(s["n_substeps"] for s in stats) / args.steps,
                           "n_rejected": sum(s["n_rejected"] for s in stats) / args.steps,
                           "n_expm": sum(s["n_expm"] for s in stats) / args.steps},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kern.items()},
        "kernel_launches_per_step": {k: v[1] / args.steps for k, v in kern.items()},
        "gpu_busy_fraction_instrumented": kernel_ms_total / (1e3 * wall_instr),
        "ms_per_step_instrumented": 1e3 * wall_instr / args.steps,
        "roofline": {
            "kernel": "dfr_kernel complex-step J*v with fused Arnoldi epilogue (inside KIOPS)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(f"dfr_kernel_krylov_{w.name}.txt"),
            "bytes_per_node": arnoldi_jv_bytes_per_node(M), "avg_launch_us": avg_jva_ms * 1e3,
            "launches": n_jva,
            "utilisation": utilisation_summary(f"dfr_kernel_krylov_{w.name}.txt", avg_jva_ms * 1e3),
        },
        "roofline_plain_jv": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "fp64": {"bytes_per_node": 72, "avg_launch_us": jv_ms * 1e3,
                     "achieved": 72 * N / (jv_ms * 1e-3) / 1e9,
                     "frac": 72 * N / (jv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "fp32_jv": {"bytes_per_node": 60, "avg_launch_us": jv32_ms * 1e3,
                        "achieved": 60 * N / (jv32_ms * 1e-3) / 1e9,
                        "frac": 60 * N / (jv32_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        },
    }
    del st, vs, outs, q, q0
    torch.cuda.synchronize()
    calibration_copy()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 94 for the ensemble, one simulated day with the start-up; 8 otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 2 for the ensemble, its EPI2 start-up; 4 otherwise)")
    ap.add_argument("--workload", default="c3_ensemble",
                    help="c3_ensemble (the headline) or a single-grid workload of inputs.WORKLOADS")
    ap.add_argument("--jv-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="skip the ne=30, p=5 EPI5 run (with the ensemble headline)")
    ap.add_argument("--no-c2", action="store_true", help="skip the ne=60, p=6 J*v roofline figures")
    ap.add_argument("--no-mixed", action="store_true", help="skip the ne=60, p=6 mixed-precision EPI6 day")
    ap.add_argument("--mixed-steps", type=int, default=72)
    ap.add_argument("--no-c4", action="store_true", help="skip the ne=120, p=6 mountain figures")
    ap.add_argument("--c4-steps", type=int, default=2)
    ap.add_argument("--no-ausm", action="store_true", help="skip the AUSM-flux figures")
    ap.add_argument("--no-diagnostics", action="store_true", help="skip the conservation-diagnostics figures")
    ap.add_argument("--no-large-dt", action="store_true", help="skip the dt = 4 h figures")
    ap.add_argument("--no-ode", action="store_true", help="skip the Sec. 5.1 test problems")
    ap.add_argument("--ensemble-members", type=int, default=64)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline run (for the ensemble: its headline form, no error check; for profiling)")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--jv-only", action="store_true",
                    help="only time the plain complex-step J*v kernel of --workload (for profiling)")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32_jv"], help="precision of --jv-only")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="print a summary of rocprofv3 output in DIR (kernel trace) and exit")
    ap.add_argument("--fetch", metavar="DIR", help="with --summarize-profile: a FETCH_SIZE pass")
    ap.add_argument("--write", metavar="DIR", help="with --summarize-profile: a WRITE_SIZE pass")
    ap.add_argument("--counters", metavar="DIR", action="append",
                    help="with --summarize-profile: a further counter pass (repeatable)")
    ap.add_argument("--kernel", default="true, true>",
                    help="with --summarize-profile: regular expression matched against kernel names")
    ap.add_argument("--last", type=int, default=0,
                    help="with --summarize-profile: average over the last N launches (the timed region)")
    args = ap.parse_args()

    if args.summarize_profile:
        return summarize_profile(args)
    ens = args.workload == "c3_ensemble"
    if args.steps is None:
        args.steps = 94 if ens else 8
    if args.warmup is None:
        args.warmup = 2 if ens else 4
    if args.headline_only:
        args.no_c1 = args.no_c2 = args.no_mixed = args.no_c4 = args.no_ausm = args.no_diagnostics = \
            args.no_large_dt = args.no_ode = args.no_cpu_baseline = True

    if args.cpu_baseline_only:
        leg = cpu_baseline_ensemble if ens else cpu_baseline_leg
        print(json.dumps(leg(args.workload)), flush=True)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the hot path on a single MI355X "
              "(the multi-GPU design is described, not built); use --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_2101_05617_amd import dfrsw, inputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    if not ens and args.workload not in inputs.WORKLOADS:
        print(f"unknown workload {args.workload}", file=sys.stderr)
        return 2
    if args.jv_only:
        return jv_only(inputs.WORKLOADS[args.workload], args)

    if ens:
        out = ensemble_headline_line(args)
        calibration_copy()   # the 256 MiB reference of the traffic counters in profiled runs
        copy_gbs = measured_copy_gbs()
        log(f"a plain 2 GiB device copy: {copy_gbs:.0f} GB/s")
        out["roofline"]["measured_copy"] = {"GBs": copy_gbs, "frac_of_peak": copy_gbs / HBM_PEAK_GBS,
                                            "achieved_frac_of_copy": out["roofline"]["achieved"] / copy_gbs}
        if not args.no_c1:
            w1 = inputs.WORKLOADS["c1_ne30_p5"]
            out["epi5_c1_ne30_p5"] = single_grid_run(w1, 8, 4, args.jv_reps)
    else:
        w = inputs.WORKLOADS[args.workload]
        log(f"workload {w.name}: ne={w.ne} p={w.p} N={w.n_nodes} EPI{w.order} dt={w.dt_s}s tol={w.tol} m<={w.m_max}")
        r = single_grid_run(w, args.steps, args.warmup, args.jv_reps)
        out = {"metric": METRIC, "value": r.pop("steps_per_s"), "unit": "EPI steps/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": r.pop("ms_per_step"),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic", **r}

    # ---- the ne = 60, p = 6 J*v (the roofline target size), buffers rotated
    if not args.no_c2:
        w2 = inputs.WORKLOADS["c2_ne60_p6_jet"]
        g2 = dfrsw.Grid(w2.ne, w2.p, *w2.constants())
        tile2 = dfrsw.dfr_autotune(g2, "fp64")
        P2, B12, B22 = g2.node_frames()
        Q2, _ = inputs.initial_state(w2, P2, B12, B22)
        q2 = torch.from_numpy(Q2).cuda()
        N2 = w2.n_nodes
        nbuf = 8   # 8 x (v, out) x 25 MB = 406 MB > 256 MB last-level cache
        v2 = [torch.randn(3 * N2, dtype=torch.float64, device="cuda") * 1e-3 for _ in range(nbuf)]
        o2 = [torch.empty(3 * N2, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
        t64 = time_jv(g2, q2, v2, o2, 1e-150, "fp64", args.jv_reps)
        tile2_32 = dfrsw.dfr_autotune(g2, "fp32_jv")
        t32 = time_jv(g2, q2, v2, o2, 1e-20, "fp32_jv", args.jv_reps)
        log(f"ne=60 p=6 J*v: fp64 {t64 * 1e3:.1f} us, fp32 {t32 * 1e3:.1f} us")
        copy_gbs = measured_copy_gbs()
        out["jv_ne60_p6"] = {
            "nodes": N2, "tile_fp64": tile2, "tile_fp32": tile2_32,
            "measured_copy_GBs": copy_gbs,
            "fp64_frac_of_copy": 72 * N2 / (t64 * 1e-3) / 1e9 / copy_gbs,
            "fp64": {"us": t64 * 1e3, "jv_per_s": 1e3 / t64, "GBs": 72 * N2 / (t64 * 1e-3) / 1e9,
                     "frac_hbm": 72 * N2 / (t64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": profiled_traffic("dfr_kernel_jv_fp64_c2_ne60_p6_jet.txt"),
                     "utilisation": utilisation_summary("dfr_kernel_jv_fp64_c2_ne60_p6_jet.txt", t64 * 1e3)},
            "fp32_jv": {"us": t32 * 1e3, "jv_per_s": 1e3 / t32, "GBs": 60 * N2 / (t32 * 1e-3) / 1e9,
                        "frac_hbm": 60 * N2 / (t32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": profiled_traffic("dfr_kernel_jv_fp32_c2_ne60_p6_jet.txt"),
                        "utilisation": utilisation_summary("dfr_kernel_jv_fp32_c2_ne60_p6_jet.txt", None),
                        "note": "timed per call including the FP32 copy of q (to_f32_kernel)"},
        }
        del v2, o2, q2, g2

    # ---- mixed precision on the jet workload: complex-FP32 J*v inside the
    # FP64 Krylov / EPI6 machinery against the plain FP64 path, one simulated day
    if not args.no_mixed:
        out["mixed_c2"] = mixed_study(args.mixed_steps)

    # ---- the largest grid (ne = 120, p = 6, orography)
    if not args.no_c4:
        out["c4_ne120_p6"] = c4_study(args.c4_steps, 50)

    # ---- the AUSM interface flux (App. D) on the same path
    if not args.no_ausm:
        out["ausm"] = ausm_study(8, 50)

    # ---- conservation diagnostics (Sec. 5.4)
    if not args.no_diagnostics:
        out["diagnostics_c2"] = diagnostics_study(20)

    # ---- the large-time-step regime (dt = 4 h)
    if not args.no_large_dt:
        out["large_dt"] = large_dt_study(4)

    # ---- the stiff test problems of Sec. 5.1 on the same KIOPS / EPI path
    if not args.no_ode:
        out["ode_suite"] = ode_suite_study()

    # ---- the oracle on this host's cores (bounded samples): one thread, then
    # every thread of this host's share (its element loop runs under OpenMP)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_entry(args, ens)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
