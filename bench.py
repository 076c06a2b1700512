#!/usr/bin/env python3
"""Throughput of the gas-phase NNP MD step on one MI355X.

Workload: one 2,500-atom cluster (H:C:N:O = 50:30:10:10, 0.1 atoms/A^3,
seeded RSA in a ball of radius 18.14 A, Maxwell-Boltzmann velocities at
300 K, Xavier-normal weights), NVE velocity Verlet at dt = 0.5 fs, pair-list
rebuild every 20 steps with a 1 A skin (earlier when an atom moved more than
half the skin).  One step = one full energy + force evaluation (pair list when
due, descriptors, network, adjoint, FP64 force gather, FP64 integration and
energy sums), so evals/s = MD steps/s and ns/day = steps/s * 0.5 fs * 86400 / 1e6.

Variants (all through the C ABI, multi-step blocks replayed from HIP graphs):
  fp32  / plain   one kernel per stage, FP32 network on the vector ALUs
  fp32  / fused   one kernel per evaluation, FP32 network on the vector ALUs
  bf16  / fused   one kernel per evaluation, BF16 MFMA network
  bf16x3/ fused   one kernel per evaluation, split-BF16 MFMA network
  fp8   / fused   one kernel per evaluation, FP8 (E4M3) MFMA network
The headline value is the fastest variant whose max force error against the
FP64 oracle is <= 1e-2 eV/A on the initial configuration and on 10 snapshots
of a trajectory (the rerun check).

Per variant the timed region is K graph-replayed steps after W warm-up steps,
repeated REPEATS times from the same initial state; value is the median and
the spread (max - min) / median is reported.  The graphs of every block
length the timed steps use are captured and instantiated before the timed
region (nnp_capture), so it replays cached graphs only.  The same K steps
are then replayed from the same state without a graph, with HIP events on
the context stream around every kernel launch, which gives the average
duration of the evaluation kernel for the roofline report.

Other modes (not part of the default run): --precision (errors per network
dtype on a second 2,500-atom cluster and on 23,000 atoms, and NVE drift),
--profile-only (one variant's steps, for rocprofv3), --pmc-summary (turns
two rocprofv3 counter databases into the traffic summary kept in profiles/),
--counter-summary (per-kernel counters of one variant: MFMA utilisation and
rate, vector-ALU and LDS activity, HBM rate, as a markdown section).

Prints ONE JSON line on stdout.
"""

import argparse
import hashlib
import json
import os
import re
import sqlite3
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DT_FS = 0.5
F_TOL = 1e-2
REPEATS = 5
N_SNAPSHOTS = 10
VARIANTS = (("fp32", "plain"), ("fp32", "fused"), ("bf16", "fused"), ("bf16x3", "fused"), ("fp8", "fused"))
KERNEL_MODE = {"fp32": 0, "bf16": 1, "bf16x3": 2, "fp8": 3}  # template MODE of the evaluation kernels

# Algorithmic FLOPs (see the design notes): per radial pair (r < 5.2 A) and
# per angular triple (both neighbours within 3.5 A), forward descriptor plus
# adjoint, and per atom for the network forward + input gradient.
FLOP_RADIAL_PAIR = 96 + 150
FLOP_ANGULAR_TRIPLE = 170 + 360
FLOP_MLP_ATOM = 2 * 2 * (384 * 160 + 160 * 128 + 128 * 96 + 96)

MI355X_FP32_VECTOR_TFLOPS = 157.3
MI355X_BF16_MFMA_TFLOPS = 2500.0
MI355X_FP8_MFMA_TFLOPS = 5000.0
MI355X_HBM_GBS = 8000.0

TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_eval_pooled_bf16x3_cluster2500_traffic.md")
KERNEL_SOURCES = ("nnp_kernels.hip", "nnp_network.hip", "nnp_device.h", "nnp_internal.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 over the sources the evaluation kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2412_18271_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def neighbour_counts(pos):
    from scipy.spatial import cKDTree
    t = cKDTree(pos)
    rad = 2 * len(t.query_pairs(5.2))
    nA = np.array([len(x) - 1 for x in t.query_ball_point(pos, 3.5)])
    tri = int((nA * (nA - 1) // 2).sum())
    return rad, tri


def drift(U, K, n_atoms):
    H = U + K
    t = np.arange(H.shape[0]) * DT_FS * 1e-3  # ps
    slope = np.polyfit(t, H, 1)[0] if H.shape[0] > 2 else 0.0
    return float(np.max(np.abs(H - H[0]))), float(slope * 1e3 / n_atoms)


def snapshots(P, s, n, block):
    """Positions every `block` steps of an FP32 trajectory (rerun inputs)."""
    ctx = P.Context.from_system(s, dtype="fp32", path="fused")
    try:
        ctx.set_state(s.pos, s.vel)
        out = []
        for _ in range(n):
            ctx.step(DT_FS, block, graph=True)
            out.append(ctx.get_state()["pos"])
        return out
    finally:
        ctx.close()


def event_timed(ctx, s, warmup, steps):
    """The timed segment again, without a graph: per-kernel averages from HIP
    events, and the radial-pair / triple counts along it (mean of chunk ends)."""
    ctx.set_state(s.pos, s.vel)
    ctx.step(DT_FS, warmup, graph=True)
    c0 = neighbour_counts(ctx.get_state()["pos"])
    ev = ga = tot = 0.0
    rad = tri = 0.0
    left = steps
    while left > 0:
        n = min(100, left)
        a, b, c = ctx.time_steps(DT_FS, n)
        c1 = neighbour_counts(ctx.get_state()["pos"])
        ev += a * n
        ga += b * n
        tot += c * n
        rad += 0.5 * (c0[0] + c1[0]) * n
        tri += 0.5 * (c0[1] + c1[1]) * n
        c0 = c1
        left -= n
    return {"eval_ms": ev / steps, "gather_ms": ga / steps, "step_ms_eager": tot / steps,
            "radial_pairs": rad / steps, "angular_triples": tri / steps}


def timed_steps(ctx, s, steps, warmup, repeats=REPEATS):
    """Seconds of `steps` graph-replayed MD steps after `warmup` untimed
    ones, `repeats` times from the same initial state.  The graphs of the
    timed block lengths are captured before the clock starts."""
    out = []
    for _ in range(repeats):
        ctx.set_state(s.pos, s.vel)
        ctx.step(DT_FS, warmup, graph=True)
        ctx.capture(DT_FS, steps)
        ctx.stats()  # synchronises
        t0 = time.perf_counter()
        ctx.step(DT_FS, steps, graph=True)
        st = ctx.stats()
        out.append(time.perf_counter() - t0)
    return out, st


def rate_summary(seconds, steps, units=1):
    """Median rate over the repeats and its spread."""
    rates = [units * steps / x for x in seconds]
    med = float(np.median(rates))
    return {"rate": med, "ms_per_step": 1e3 * float(np.median(seconds)) / steps,
            "repeats": rates, "spread": (max(rates) - min(rates)) / med}


def run_variant(P, s, dtype, path, steps, warmup, refs, tune=True):
    """One network dtype / path: the autotuner picks the kernel configuration
    (path within the fused / split family, atoms per workgroup, network
    tile) on the initial positions, then the force errors on the reference
    configurations, the timed MD steps and the event-timed kernels."""
    ctx = P.Context.from_system(s, dtype=dtype, path=path)
    try:
        tuned = None
        if tune:
            ctx.set_state(s.pos, s.vel)
            tuned = ctx.autotune(None)
            log("   autotune:", tuned)
        errs = []
        for pos, F_ref in refs:
            _, F = ctx.compute(pos)
            errs.append(float(np.abs(F - F_ref).max()))
        secs, st = timed_steps(ctx, s, steps, warmup)
        rs = rate_summary(secs, steps)
        U, K = ctx.energy_log(min(steps + 1, 4096))
        dH, slope = drift(U[:, 0], K[:, 0], s.n_atoms)
        final_finite = bool(np.isfinite(ctx.get_state()["pos"]).all())
        kt = event_timed(ctx, s, warmup, steps)
        return {
            "dtype": dtype, "path": ctx.path, "requested_path": path, "steps_per_s": rs["rate"],
            "ms_per_step": rs["ms_per_step"], "repeats_steps_per_s": rs["repeats"], "spread": rs["spread"],
            "autotune": tuned, "max_force_err": errs[0],
            "max_force_err_snapshots": max(errs[1:]) if len(errs) > 1 else None,
            "drift_max_abs_eV": dH, "drift_slope_meV_per_atom_ps": slope,
            "rebuilds": st["rebuilds"], "forced_rebuilds": st["forced_rebuilds"],
            "kernel_ms_eval": kt["eval_ms"], "kernel_ms_gather_vv": kt["gather_ms"],
            "step_ms_eager": kt["step_ms_eager"], "radial_pairs_mean": kt["radial_pairs"],
            "angular_triples_mean": kt["angular_triples"], "final_finite": final_finite,
        }
    finally:
        ctx.close()


def langevin_leg(P, s, dtype, path, steps, warmup):
    """The paper's timed integrator: Langevin dynamics (BAOAB) at 300 K with a
    friction of 0.1 ps^-1, same graph-replayed blocks as the NVE run."""
    ctx = P.Context.from_system(s, dtype=dtype, path=path)
    try:
        ctx.set_thermostat(300.0, 0.1, 0)
        secs, _ = timed_steps(ctx, s, steps, warmup)
        rs = rate_summary(secs, steps)
        _, K = ctx.energy_log(min(steps, 4096))
        return {"dtype": dtype, "path": path, "temperature_K": 300.0, "friction_per_ps": 0.1,
                "steps_per_s": rs["rate"], "ms_per_step": rs["ms_per_step"], "spread": rs["spread"],
                "ns_per_day": rs["rate"] * DT_FS * 86400 / 1e6,
                "kinetic_temperature_K": float(2.0 * K[:, 0].mean() / (3 * s.n_atoms * 8.617333262e-5))}
    finally:
        ctx.close()


def periodic_leg(P, dtype, path, steps, warmup):
    """A periodic 2,500-atom box (L = 29.24 A, same density): NVE MD steps/s
    with nearest-image pair lists, and the force error against the oracle's
    explicit-image periodic forces at the initial configuration."""
    import oracle
    import synth
    s = synth.make_config("box2500")
    _, _, F_ref = oracle.periodic_energy_forces(s.pos, s.species, s.weights, s.box)
    ctx = P.Context.from_system(s, dtype=dtype, path=path)
    try:
        _, F = ctx.compute(s.pos)
        secs, st = timed_steps(ctx, s, steps, warmup)
        rs = rate_summary(secs, steps)
        return {"workload": "box2500: 2,500 atoms, periodic cube L = %.2f A" % s.box[0], "dtype": dtype,
                "path": path, "steps_per_s": rs["rate"], "ms_per_step": rs["ms_per_step"], "spread": rs["spread"],
                "max_force_err": float(np.abs(F - F_ref).max()), "rebuilds": st["rebuilds"]}
    finally:
        ctx.close()


def large_leg(P, steps, warmup):
    """The 23,000-atom cluster (cell lists), split-BF16 network, kernel
    configuration from the autotuner: MD steps/s, the evaluation kernels'
    event-timed duration and their VALU / MFMA rates against the peaks."""
    import synth
    s = synth.make_config("cluster23k")
    ctx = P.Context.from_system(s, dtype="bf16x3", path="fused")
    try:
        ctx.set_state(s.pos, s.vel)
        tuned = ctx.autotune(None)
        log("   autotune:", tuned)
        secs, st = timed_steps(ctx, s, steps, warmup, repeats=3)
        rs = rate_summary(secs, steps)
        kt = event_timed(ctx, s, warmup, steps)
    finally:
        ctx.close()
    t = kt["eval_ms"] * 1e-3
    valu = kt["radial_pairs"] * FLOP_RADIAL_PAIR + kt["angular_triples"] * FLOP_ANGULAR_TRIPLE
    mlp = s.n_atoms * FLOP_MLP_ATOM
    sol = valu / (MI355X_FP32_VECTOR_TFLOPS * 1e12) + mlp / (MI355X_BF16_MFMA_TFLOPS * 1e12)
    var = "bf16x3:%s" % tuned["path"]
    traffic = load_traffic(var, traffic_summary_path(var, "cluster23k"), tile_of_choice(tuned))
    return {"workload": "cluster23k: 23,000-atom gas-phase cluster, NVE dt 0.5 fs, rebuild 20 / skin 1 A",
            "dtype": "bf16x3", "autotune": tuned, "steps_per_s": rs["rate"], "ms_per_step": rs["ms_per_step"],
            "spread": rs["spread"], "ns_per_day": rs["rate"] * DT_FS * 86400 / 1e6,
            "kernel_ms_eval": kt["eval_ms"], "kernel_ms_gather_vv": kt["gather_ms"],
            "valu_tflops": valu / t / 1e12, "mlp_tflops": mlp / t / 1e12, "combined_frac": sol / t,
            "traffic": traffic, "hbm_gbs_from_traffic": None if traffic is None else traffic / t / 1e9,
            "rebuilds": st["rebuilds"]}


def batch_leg(P, steps, warmup):
    """256 molecules of 10-300 atoms: molecule-steps/s of one batched context
    (one evaluation launch per step for all molecules, graph-replayed) against
    a loop of one context per molecule (graph-replayed, and eager)."""
    import synth
    s = synth.make_config("batch256")
    M = s.n_molecules
    out = {"n_molecules": M, "n_atoms": int(s.n_atoms), "steps": steps, "dtype": "bf16x3"}
    ctx = P.Context.from_system(s, dtype="bf16x3", path="fused")
    try:
        ctx.set_state(s.pos, s.vel)
        out["autotune"] = ctx.autotune(None)
        log("   autotune:", out["autotune"])
        secs, _ = timed_steps(ctx, s, steps, warmup)
        rs = rate_summary(secs, steps, M)
        out["batched_molecule_steps_per_s"] = rs["rate"]
        out["batched_spread"] = rs["spread"]
        try:
            ctx.get_state()  # synchronising: raises on the sticky device flags
            out["within_capacity"] = True
        except P.NNPError as e:
            out["within_capacity"] = False
            out["capacity_error"] = str(e)
    finally:
        ctx.close()
    ctxs = []
    try:
        for m in range(M):
            sl = s.molecule(m)
            c = P.Context(s.species[sl], s.masses[sl], s.weights, None, dtype="bf16x3", path="fused")
            c.set_state(s.pos[sl], s.vel[sl])
            ctxs.append(c)
        for graph, key in ((True, "per_molecule_graph_molecule_steps_per_s"),
                           (False, "per_molecule_eager_molecule_steps_per_s")):
            for c in ctxs:
                c.step(DT_FS, warmup, graph=graph)
                if graph:
                    c.capture(DT_FS, steps)
            for c in ctxs:
                c.stats()
            t0 = time.perf_counter()
            for c in ctxs:
                c.step(DT_FS, steps, graph=graph)
            for c in ctxs:
                c.stats()
            out[key] = M * steps / (time.perf_counter() - t0)
    finally:
        for c in ctxs:
            c.close()
    out["speedup_vs_per_molecule_graph"] = (out["batched_molecule_steps_per_s"]
                                            / out["per_molecule_graph_molecule_steps_per_s"])
    return out


def copy_calibration(mib):
    """One elementwise kernel of known traffic (reads and writes `mib` MiB),
    to scale the FETCH_SIZE / WRITE_SIZE counters of a profile."""
    import torch
    n = (int(mib) << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    log("copy calibration: 3 x torch.neg over %d MiB (read %d MiB, write %d MiB)" % (mib, mib, mib))


# Evaluation kernels per path (one launch each per evaluation; the split path's
# traffic is the sum of its three kernels' per-dispatch means).
EVAL_KERNELS = {"fused": [r"k_eval_(fused|pooled)<\d+, %d,"], "split": [r"k_desc_pooled<", r"k_mlp_wide<",
                                                                       r"k_adj_pooled<"]}


def tile_of_kernels(names):
    """Tile configuration named by the evaluation kernels seen: "10" (fused:
    atoms per workgroup), "5x32" (split: descriptor / adjoint tile x network
    tile), or None."""
    fused = {int(m.group(1)) for n in names for m in [re.search(r"k_eval_(?:fused|pooled)<(\d+),", n)] if m}
    desc = {int(m.group(1)) for n in names for m in [re.search(r"k_desc_pooled<(\d+)>", n)] if m}
    wide = {int(m.group(1)) for n in names for m in [re.search(r"k_mlp_wide<(\d+),", n)] if m}
    if len(fused) == 1 and not desc:
        return "%d" % fused.pop()
    if len(desc) == 1 and len(wide) == 1 and not fused:
        return "%dx%d" % (desc.pop(), 16 * wide.pop())
    return None


def tile_of_choice(choice):
    """The same string for an autotuner choice ({path, atoms_per_tile,
    network_tile})."""
    if not choice:
        return None
    if choice["path"] == "split":
        return "%dx%d" % (choice["atoms_per_tile"], choice["network_tile"])
    return "%d" % choice["atoms_per_tile"]


def pmc_summary(fetch_db, write_db, variant, mib, command, workload="cluster2500"):
    """Markdown summary of a FETCH_SIZE run and a WRITE_SIZE run: per-dispatch
    KiB of the evaluation kernel(s), scaled by the calibration kernel's
    reading."""
    dtype, path = variant.split(":")[:2]
    pats = [p % KERNEL_MODE[dtype] if "%d" in p else p for p in EVAL_KERNELS[path]]

    def per_kernel(db, counter):
        c = sqlite3.connect(db)
        rows = c.execute("select kernel_name, value from counters_collection where counter_name = ?",
                         (counter,)).fetchall()
        return rows

    known_kib = mib * 1024.0
    res = {}
    for db, counter in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        rows = per_kernel(db, counter)
        cal = [v for k, v in rows if "neg" in k and v > 0.25 * known_kib]
        ker = [(k, v) for k, v in rows if any(re.search(p, k) for p in pats)]
        names = sorted({k for k, _ in ker})
        per = [[v for k, v in ker if re.search(p, k)] for p in pats]
        res[counter] = {"cal_kib": float(np.median(cal)) if cal else None,
                        "kernel_kib": float(sum(np.mean(x) for x in per)) if all(per) else None,
                        "dispatches": min(len(x) for x in per), "names": names}
    fr = res["FETCH_SIZE"]
    wr = res["WRITE_SIZE"]
    f_factor = known_kib / fr["cal_kib"]
    w_factor = known_kib / wr["cal_kib"]
    fetch_b = fr["kernel_kib"] * f_factor * 1024
    write_b = wr["kernel_kib"] * w_factor * 1024
    lines = [
        "# Evaluation kernel HBM traffic, %s, %s network, %s path" % (workload, dtype, path),
        "",
        "Commands (run from the repository root, TMPDIR=/tmp):",
        "",
        "```",
        command.replace("COUNTER", "FETCH_SIZE"),
        command.replace("COUNTER", "WRITE_SIZE"),
        "python3 bench.py --pmc-summary <fetch run db> <write run db> --variant %s --workload %s "
        "--copy-calibration-mib %d" % (variant, workload, mib),
        "```",
        "",
        "Calibration kernel: torch.neg over %d MiB of float32 (reads %d MiB, writes %d MiB)." % (mib, mib, mib),
        "",
        "| counter | calibration reading (KiB) | known (KiB) | scale | evaluation kernel per dispatch (KiB) | dispatches | scaled bytes per launch |",
        "|---|---|---|---|---|---|---|",
        "| FETCH_SIZE | %.1f | %.0f | %.4f | %.1f | %d | %.0f |" % (fr["cal_kib"], known_kib, f_factor,
                                                                  fr["kernel_kib"], fr["dispatches"], fetch_b),
        "| WRITE_SIZE | %.1f | %.0f | %.4f | %.1f | %d | %.0f |" % (wr["cal_kib"], known_kib, w_factor,
                                                                  wr["kernel_kib"], wr["dispatches"], write_b),
        "",
        "Kernels seen: %s" % ", ".join(fr["names"]),
        "",
        "- variant: %s" % variant,
        "- tile: %s" % tile_of_kernels(fr["names"]),
        "- hbm_bytes_per_launch: %d" % int(round(fetch_b + write_b)),
        "- fetch_bytes_per_launch: %d" % int(round(fetch_b)),
        "- write_bytes_per_launch: %d" % int(round(write_b)),
        "- kernel_source_sha256: %s" % kernel_source_hash(),
    ]
    print("\n".join(lines))


def counter_summary(variant, stats_csv, dbs, mib, profile_args):
    """Markdown section for one variant: per kernel, its mean duration (from a
    kernel-trace statistics file of the same variant) and the mean value per
    dispatch of every counter in the rocprofv3 counter databases, with the
    MFMA rate against the dtype's dense peak and, where FETCH_SIZE and
    WRITE_SIZE were taken next to the calibration kernel, the HBM rate
    against 8 TB/s."""
    import csv
    dtype, path = variant.split(":")[:2]
    dur = {}
    with open(stats_csv) as fh:
        for row in csv.DictReader(fh):
            dur[row["Name"]] = (float(row["AverageNs"]), int(row["Calls"]))
    vals, names, passes = {}, {}, []
    known_kib = mib * 1024.0
    scale = {}
    for db in dbs:
        c = sqlite3.connect(db)
        rows = c.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
        c.close()
        passes.append(sorted({r[1] for r in rows}))
        for k, n, v in rows:
            if "neg" in k and n in ("FETCH_SIZE", "WRITE_SIZE") and v > 0.25 * known_kib:
                scale.setdefault(n, []).append(v)
            if not re.search(r"nnp::k_", k):
                continue
            vals.setdefault(k, {}).setdefault(n, []).append(float(v))
            names[n] = True
    factor = {n: known_kib / float(np.median(v)) for n, v in scale.items()}
    counters = list(names)
    mfma_peak = MI355X_FP8_MFMA_TFLOPS if dtype == "fp8" else MI355X_BF16_MFMA_TFLOPS
    head = ["kernel", "mean us (trace)", "dispatches"] + counters
    derived = []
    if "MfmaFlopsBF16" in names:
        head += ["MFMA TFLOP/s", "of %g" % mfma_peak]
        derived.append("mfma")
    if "FETCH_SIZE" in factor and "WRITE_SIZE" in factor:
        head += ["HBM bytes (scaled)", "GB/s", "of 8000"]
        derived.append("hbm")
    out = ["## %s network, %s path" % (dtype, path), "",
           "Counter passes (one rocprofv3 run each, `--profile-only %s %s`):" % (variant, profile_args), ""]
    out += ["- `%s`" % " ".join(p) for p in passes]
    if factor:
        out += ["", "HBM counters scaled by the calibration kernel (torch.neg over %d MiB): %s." % (
            mib, ", ".join("%s x %.3f" % kv for kv in sorted(factor.items())))]
    out += ["", "| " + " | ".join(head) + " |", "|" + "---|" * len(head)]
    order = sorted(vals, key=lambda k: -dur.get(k, (0.0, 0))[0])
    for k in order:
        us = dur.get(k, (float("nan"), 0))[0] / 1e3
        row = [k.replace("nnp::", "").replace("(nnp::Sys)", "").split("(")[0], "%.2f" % us,
               str(len(next(iter(vals[k].values()))))]
        mean = {n: float(np.mean(v)) for n, v in vals[k].items()}
        row += ["%.4g" % mean[n] if n in mean else "" for n in counters]
        if "mfma" in derived:
            f = mean.get("MfmaFlopsBF16", 0.0)
            t = f / (us * 1e-6) / 1e12 if us == us and us > 0 else float("nan")
            row += ["%.1f" % t, "%.2f %%" % (100 * t / mfma_peak)]
        if "hbm" in derived:
            if "FETCH_SIZE" in mean and "WRITE_SIZE" in mean:
                b = (mean["FETCH_SIZE"] * factor["FETCH_SIZE"] + mean["WRITE_SIZE"] * factor["WRITE_SIZE"]) * 1024
                g = b / (us * 1e-6) / 1e9 if us == us and us > 0 else float("nan")
                row += ["%.0f" % b, "%.0f" % g, "%.2f %%" % (100 * g / MI355X_HBM_GBS)]
            else:
                row += ["", "", ""]
        out.append("| " + " | ".join(row) + " |")
    out.append("")
    print("\n".join(out))


def traffic_summary_path(variant, workload):
    """Committed HBM-traffic summary of a dtype:path on a workload."""
    dtype, path = variant.split(":")[:2]
    kern = "k_split" if path == "split" else "k_eval_pooled"
    return os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.md" % (kern, dtype, workload))


def load_traffic(variant, summary=None, tile=None):
    """HBM bytes per launch from the committed counter summary, or None when
    it covers another variant or tile configuration (tile given), or the
    kernel sources changed since."""
    try:
        txt = open(summary or TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^- (\w+): (\S+)$", txt, re.M))
    if kv.get("variant") != variant or kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if tile is not None and kv.get("tile") != tile:
        return None
    return int(kv["hbm_bytes_per_launch"])


def cpu_baseline(s, seconds):
    import oracle
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.energy_forces(s.pos, s.species, s.weights)
        n += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    cores = oracle.threads()
    # one core, a few evaluations
    oracle.set_threads(1)
    n1 = 0
    t1 = time.perf_counter()
    while n1 < 2 or time.perf_counter() - t1 < min(5.0, seconds / 3):
        oracle.energy_forces(s.pos, s.species, s.weights)
        n1 += 1
    one = n1 / (time.perf_counter() - t1)
    oracle.set_threads(cores)
    return {"value": n / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "%d FP64 energy+force evaluations of the 2,500-atom cluster at its initial "
                      "positions (no integration), %.1f s on %d threads; one thread: %.2f evals/s"
                      % (n, dt, cores, one),
            "single_core_value": one}


def nve_energies(P, ctx, s, n, chunk=500):
    """H = U + K at every step of an n-step NVE run from the initial state
    (the device keeps the last 4096 steps; read after every chunk).  The
    device flags are checked after every chunk: the run stops at the first
    chunk in which an atom's environment exceeded the library's capacity
    (or a result was not finite), and only the steps before that chunk are
    returned, with the error."""
    ctx.set_state(s.pos, s.vel)
    H = []
    done = 0
    while done < n:
        c = min(chunk, n - done)
        ctx.step(DT_FS, c, graph=True)
        try:
            U, K = ctx.energy_log(c + 1 if done == 0 else c)  # raises on the sticky device flags
        except P.NNPError as e:
            return (np.concatenate(H) if H else np.zeros(0)), done, str(e)
        H.append(U[:, 0] + K[:, 0])
        done += c
    return np.concatenate(H), done, None


def precision_study(P, steps_drift):
    """Force / energy errors per network dtype against the oracle, and NVE
    drift over `steps_drift` steps, on a second 2,500-atom cluster and on
    23,000 atoms (sampled atoms there)."""
    import oracle
    import synth
    out = {}
    for name in ("cluster2500b", "cluster23k"):
        s = synth.make_config(name)
        res = {"n_atoms": int(s.n_atoms)}
        if s.n_atoms <= 5000:
            Eo, Eio, Fo = oracle.energy_forces(s.pos, s.species, s.weights)
            sel = np.arange(s.n_atoms)
        else:
            Eo, Eio, _ = oracle.energy_forces(s.pos, s.species, s.weights, forces=False)
            rng = np.random.Generator(np.random.PCG64(5))
            sel = np.sort(rng.choice(s.n_atoms, size=64, replace=False))
            Fo = np.zeros((s.n_atoms, 3))
            for a in sel:
                env = oracle.local_environment(s.pos, int(a), 10.4)
                loc = int(np.nonzero(env == a)[0][0])
                Fo[a] = oracle.forces_on(s.pos[env], s.species[env], s.weights, [loc])[0]
        S = float(np.abs(Eio).sum())
        for dtype in ("fp32", "bf16x3", "bf16", "fp8"):
            ctx = P.Context.from_system(s, dtype=dtype, path="fused")
            try:
                E, F = ctx.compute(s.pos)
                r = {"rel_energy_err": float(abs(E[0] - Eo) / S),
                     "max_force_err": float(np.abs(F[sel] - Fo[sel]).max()),
                     "rms_force_err": float(np.sqrt(np.mean((F[sel] - Fo[sel]) ** 2))),
                     "force_atoms_checked": int(len(sel))}
                H, n, err = nve_energies(P, ctx, s, steps_drift)
                r["stats"] = ctx.stats()
                r["drift_steps"] = n  # steps with every environment within capacity
                if err is not None:
                    r["drift_stopped"] = err
                if n >= 2:
                    t = np.arange(H.shape[0]) * DT_FS * 1e-3
                    r["drift_max_abs_eV"] = float(np.max(np.abs(H - H[0])))
                    r["drift_slope_meV_per_atom_ps"] = float(np.polyfit(t, H, 1)[0] * 1e3 / s.n_atoms)
            except Exception as e:  # report the failure for this dtype
                r = {"error": str(e)}
            finally:
                ctx.close()
            log(name, dtype, json.dumps(r))
            res[dtype] = r
        out[name] = res
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--variants", default=",".join("%s:%s" % v for v in VARIANTS))
    ap.add_argument("--profile-only", default=None,
                    help="dtype:path[:atoms_per_tile[:network_tile]]; run only that variant's timed steps "
                         "(for rocprofv3)")
    ap.add_argument("--workload", default="cluster2500", help="with --profile-only: the synthetic system")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="with --profile-only: also run an elementwise kernel over this many MiB")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"), default=None)
    ap.add_argument("--variant", default="bf16x3:fused", help="with --pmc-summary")
    ap.add_argument("--pmc-command", default="timeout -s KILL 60 rocprofv3 --pmc COUNTER -d <dir> -o run -- "
                    "python3 bench.py --profile-only bf16x3:fused --steps 20 --warmup 5 "
                    "--copy-calibration-mib 256")
    ap.add_argument("--counter-summary", nargs="+", metavar="DB", default=None,
                    help="rocprofv3 counter databases of one variant (--variant) -> markdown section")
    ap.add_argument("--trace-stats", default=None, help="with --counter-summary: kernel_stats.csv of the variant")
    ap.add_argument("--profile-args", default="--steps 200 --warmup 20",
                    help="with --counter-summary: the --profile-only arguments the runs used")
    ap.add_argument("--precision", action="store_true",
                    help="run the precision / drift study instead of the benchmark")
    ap.add_argument("--drift-steps", type=int, default=10000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.variant,
                    args.copy_calibration_mib or 256, args.pmc_command, args.workload)
        return

    if args.counter_summary:
        counter_summary(args.variant, args.trace_stats, args.counter_summary, args.copy_calibration_mib or 256,
                        args.profile_args)
        return

    import synth
    import paper_2412_18271_amd as P

    if args.precision:
        print(json.dumps({"precision_study": precision_study(P, args.drift_steps)}), flush=True)
        return

    s = synth.make_config("cluster2500")
    if args.profile_only:
        parts = args.profile_only.split(":")
        dtype, path = parts[0], parts[1]
        T = int(parts[2]) if len(parts) > 2 else 0
        nt = int(parts[3]) if len(parts) > 3 else 0
        s = synth.make_config(args.workload)
        ctx = P.Context.from_system(s, dtype=dtype, path=path, atoms_per_tile=T, network_tile=nt)
        ctx.set_state(s.pos, s.vel)
        ctx.step(DT_FS, args.warmup, graph=True)
        ctx.step(DT_FS, args.steps, graph=True)
        log("profiled", dtype, path, ctx.stats())
        ctx.close()
        if args.copy_calibration_mib:
            copy_calibration(args.copy_calibration_mib)
        return

    import oracle
    log("oracle forces at the initial configuration and at %d trajectory snapshots" % N_SNAPSHOTS)
    snaps = snapshots(P, s, N_SNAPSHOTS, 100)
    refs = [(p, oracle.energy_forces(p, s.species, s.weights)[2]) for p in [s.pos] + snaps]
    variants = [tuple(v.split(":")) for v in args.variants.split(",") if v]
    res = []
    for dtype, path in variants:
        log("variant", dtype, path)
        r = run_variant(P, s, dtype, path, args.steps, args.warmup, refs)
        log("  ", json.dumps(r))
        res.append(r)
    ok = [r for r in res if r["max_force_err"] <= F_TOL
          and (r["max_force_err_snapshots"] is None or r["max_force_err_snapshots"] <= F_TOL)]
    best = max(ok, key=lambda r: r["steps_per_s"])
    plain = next((r for r in res if r["dtype"] == "fp32" and r["path"] == "plain"), None)

    rad, tri = best["radial_pairs_mean"], best["angular_triples_mean"]
    valu_flop = rad * FLOP_RADIAL_PAIR + tri * FLOP_ANGULAR_TRIPLE
    mlp_flop = s.n_atoms * FLOP_MLP_ATOM
    t_eval = best["kernel_ms_eval"] * 1e-3
    valu_tflops = valu_flop / t_eval / 1e12
    mfma_peak = MI355X_FP8_MFMA_TFLOPS if best["dtype"] == "fp8" else MI355X_BF16_MFMA_TFLOPS
    mlp_peak = MI355X_FP32_VECTOR_TFLOPS if best["dtype"] == "fp32" else mfma_peak
    traffic = load_traffic("%s:%s" % (best["dtype"], best["path"]), tile=tile_of_choice(best.get("autotune")))
    sol_s = valu_flop / (MI355X_FP32_VECTOR_TFLOPS * 1e12) + mlp_flop / (mlp_peak * 1e12)
    roofline = {
        "bound": "alu", "achieved": valu_tflops, "peak": MI355X_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s", "frac": valu_tflops / MI355X_FP32_VECTOR_TFLOPS, "traffic": traffic,
        "kernel": "evaluation kernel (%s path, %s network): pair list, descriptors, network, adjoint" % (
            best["path"], best["dtype"]),
        "kernel_ms": best["kernel_ms_eval"],
        "flop_per_launch_valu": valu_flop, "flop_per_launch_mlp": mlp_flop,
        "radial_pairs_per_launch": rad, "angular_triples_per_launch": tri,
        "mlp_tflops": mlp_flop / t_eval / 1e12, "mlp_peak_tflops": mlp_peak,
        "mlp_frac": mlp_flop / t_eval / 1e12 / mlp_peak,
        # time at peak of both halves (descriptor VALU work at the FP32 vector
        # peak + network work at its dtype's peak) over the kernel's time
        "combined_frac": sol_s / t_eval, "speed_of_light_us": sol_s * 1e6,
        "hbm_gbs_from_traffic": None if traffic is None else traffic / t_eval / 1e9,
    }
    out = {
        "metric": "NNP energy+force evals/s & ns/day (2.5k atoms), BF16-MFMA vs FP32 plain",
        "value": best["steps_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
        "repeats": REPEATS, "repeats_value": best["repeats_steps_per_s"], "spread": best["spread"],
        "scaling": "weak", "vs_baseline": None, "dtype": best["dtype"], "data": "synthetic",
        "ns_per_day": best["steps_per_s"] * DT_FS * 86400 / 1e6,
        "config": {"workload": "cluster2500: 2,500-atom gas-phase cluster, NVE dt 0.5 fs, "
                               "rebuild 20 / skin 1 A", "n_atoms": s.n_atoms, "path": best["path"],
                   "mlp": best["dtype"]},
        "fp32_plain": None if plain is None else {
            "evals_per_s": plain["steps_per_s"], "ns_per_day": plain["steps_per_s"] * DT_FS * 86400 / 1e6,
            "max_force_err": plain["max_force_err"]},
        "speedup_vs_fp32_plain": None if plain is None else best["steps_per_s"] / plain["steps_per_s"],
        "variants": res,
        "roofline": roofline,
    }
    log("langevin")
    out["langevin"] = langevin_leg(P, s, best["dtype"], best["path"], args.steps, args.warmup)
    log("  ", json.dumps(out["langevin"]))
    log("periodic")
    out["periodic_box2500"] = periodic_leg(P, best["dtype"], best["path"], args.steps, args.warmup)
    log("  ", json.dumps(out["periodic_box2500"]))
    if not args.no_large:
        log("cluster23k")
        out["cluster23k"] = large_leg(P, 200, 20)
        log("  ", json.dumps(out["cluster23k"]))
    if not args.no_batch:
        log("batch256")
        out["batch256"] = batch_leg(P, 100, 20)
        log("  ", json.dumps(out["batch256"]))
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
