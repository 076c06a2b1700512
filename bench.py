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
The headline value is the fastest variant whose max force error against the
FP64 oracle is <= 1e-2 eV/A.

Prints ONE JSON line on stdout.
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

DT_FS = 0.5
F_TOL = 1e-2
VARIANTS = (("fp32", "plain"), ("fp32", "fused"), ("bf16", "fused"), ("bf16x3", "fused"))

# Algorithmic FLOPs (see the design notes): per radial pair (r < 5.2 A) and
# per angular triple (both neighbours within 3.5 A), forward descriptor plus
# adjoint, and per atom for the network forward + input gradient.
FLOP_RADIAL_PAIR = 96 + 150
FLOP_ANGULAR_TRIPLE = 170 + 360
FLOP_MLP_ATOM = 2 * 2 * (384 * 160 + 160 * 128 + 128 * 96 + 96)

MI355X_FP32_VECTOR_TFLOPS = 157.3
MI355X_BF16_MFMA_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def run_variant(P, s, dtype, path, steps, warmup, F_ref):
    ctx = P.Context.from_system(s, dtype=dtype, path=path)
    try:
        E, F = ctx.compute(s.pos)
        ferr = float(np.abs(F - F_ref).max()) if F_ref is not None else None
        ctx.set_state(s.pos, s.vel)
        ctx.step(DT_FS, warmup, graph=True)
        ctx.stats()  # synchronises
        t0 = time.perf_counter()
        ctx.step(DT_FS, steps, graph=True)
        st = ctx.stats()
        t1 = time.perf_counter()
        U, K = ctx.energy_log(min(steps + 1, 4096))
        dH, slope = drift(U[:, 0], K[:, 0], s.n_atoms)
        state = ctx.get_state()
        ms_eval, ms_gather = ctx.time_kernels(50)
        return {
            "dtype": dtype, "path": path, "steps_per_s": steps / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / steps, "max_force_err": ferr,
            "drift_max_abs_eV": dH, "drift_slope_meV_per_atom_ps": slope,
            "rebuilds": st["rebuilds"], "forced_rebuilds": st["forced_rebuilds"],
            "kernel_ms_eval": ms_eval, "kernel_ms_gather_vv": ms_gather,
            "final_finite": bool(np.isfinite(state["pos"]).all()),
        }
    finally:
        ctx.close()


def copy_calibration(mib):
    """One device-to-device copy of a known size (the HIP runtime's blit
    kernel), to scale the FETCH_SIZE / WRITE_SIZE counters of a profile."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    n = int(mib) << 20
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(n)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(n)) == 0
    assert hip.hipMemset(a, 1, ctypes.c_size_t(n)) == 0
    for _ in range(3):
        assert hip.hipMemcpy(b, a, ctypes.c_size_t(n), 3) == 0  # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    log("copy calibration: 3 x %d MiB device-to-device" % mib)


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
    return {"value": n / dt, "unit": "evals/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": "%d FP64 energy+force evaluations of the 2,500-atom cluster at its initial "
                      "positions (no integration), %.1f s" % (n, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default=",".join("%s:%s" % v for v in VARIANTS))
    ap.add_argument("--profile-only", default=None,
                    help="dtype:path; run only that variant's timed steps (for rocprofv3)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="with --profile-only: also run a device-to-device copy of this size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import synth
    import paper_2412_18271_amd as P

    s = synth.make_config("cluster2500")
    if args.profile_only:
        dtype, path = args.profile_only.split(":")
        ctx = P.Context.from_system(s, dtype=dtype, path=path)
        ctx.set_state(s.pos, s.vel)
        ctx.step(DT_FS, args.warmup, graph=True)
        ctx.step(DT_FS, args.steps, graph=True)
        log("profiled", dtype, path, ctx.stats())
        ctx.close()
        if args.copy_calibration_mib:
            copy_calibration(args.copy_calibration_mib)
        return

    import oracle
    log("oracle forces at the initial configuration")
    _, _, F_ref = oracle.energy_forces(s.pos, s.species, s.weights)
    variants = [tuple(v.split(":")) for v in args.variants.split(",") if v]
    res = []
    for dtype, path in variants:
        log("variant", dtype, path)
        r = run_variant(P, s, dtype, path, args.steps, args.warmup, F_ref)
        log("  ", json.dumps(r))
        res.append(r)
    ok = [r for r in res if r["max_force_err"] is not None and r["max_force_err"] <= F_TOL]
    best = max(ok, key=lambda r: r["steps_per_s"])
    plain = next((r for r in res if r["dtype"] == "fp32" and r["path"] == "plain"), None)

    rad, tri = neighbour_counts(s.pos)
    valu_flop = rad * FLOP_RADIAL_PAIR + tri * FLOP_ANGULAR_TRIPLE
    mlp_flop = s.n_atoms * FLOP_MLP_ATOM
    t_eval = best["kernel_ms_eval"] * 1e-3
    valu_tflops = valu_flop / t_eval / 1e12
    roofline = {
        "kernel": "k_eval_fused (%s network): descriptors + network + adjoint" % best["dtype"],
        "bound": "alu", "achieved": valu_tflops, "peak": MI355X_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s", "frac": valu_tflops / MI355X_FP32_VECTOR_TFLOPS, "traffic": None,
        "flop_per_launch_valu": valu_flop, "flop_per_launch_mlp": mlp_flop,
        "mlp_tflops": mlp_flop / t_eval / 1e12,
        "mlp_frac_of_bf16_mfma_peak": mlp_flop / t_eval / 1e12 / MI355X_BF16_MFMA_TFLOPS,
        "kernel_ms": best["kernel_ms_eval"],
        "radial_pairs": rad, "angular_triples": tri,
    }
    out = {
        "metric": "NNP energy+force evals/s & ns/day (2.5k atoms), BF16-MFMA vs FP32 plain",
        "value": best["steps_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
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
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
