"""Benchmark: Metropolis spin updates/s of the batched FP32 multipath engine on one MI355X.

Default workload (one step): L = 16 classical Heisenberg lattices at T = 1.2, 1.443 and 1.7,
4096 independent paths per temperature, each from a random start through 2000 thermalisation
and 8000 measured checkerboard sweeps (FP32 spins and fields, FP64 accumulators), then the
FP64 cross-path statistics -- 5.03e11 spin updates per step, in one persistent hipGraph launch.

Also reported on the same GPU: the plain per-instance FP64 engine on the same workload, the
4-standard-error agreement of the FP32 results with the FP64 CPU oracle (sampled paths,
stored by tests/golden/make_oracle_golden.py), the VALU and device-memory rooflines of the
batch kernels (the one they come closer to as "roofline"; the VALU ceiling is the update's
instruction mix measured in the same process), and the oracle itself timed on the host cores.
The default run adds one timed pass each of the largest configuration (the uneven batch of 96
instances, "largest_config") and of the two device-memory configurations (L = 32 and L = 64,
"device_memory_configs"), with their rooflines and oracle agreement.

--workload selects another batched FP32 workload of paper_1305_6758_amd/workloads.py (same
JSON line; the plain FP64 comparison runs only where its resident spins fit). For the
Binder-cumulant workload the line also carries the cumulants, their ratio and the crossing.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--skip-plain] [--skip-cpu]
                      [--skip-largest]
"""
import argparse
import json
import re
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Metropolis spin updates/sec (batched FP32 vs plain FP64) at 4σ oracle agreement"
WORKLOAD = "L16-T3-p4096-fp32"

# VALU roofline of the batch kernel. Peak: the published MI355X FP32 vector rate, 157.3
# TFLOP/s = 256 CUs x 2.4 GHz x 128 lanes x 2 FLOP per FMA, i.e. 7.86e13 lane-operations/s.
# Each instruction class costs PEAK / rate lane-slots, with the sustained rates measured on
# gfx950 by `python -m paper_1305_6758_amd.opbench` (profiles/valu_op_rates_gfx950.md).
VALU_PEAK = 256 * 2.4e9 * 128
OP_RATES = {  # lane-operations per second, whole GPU
    "v_add_f32": 6.2467e13, "v_sub_f32": 6.2675e13, "v_mul_f32": 6.2759e13, "v_fma_f32": 3.6725e13,
    "v_cndmask_b32": 3.6135e13, "v_cmp_lt_f32": 3.2484e13, "v_alignbit_b32": 3.4979e13, "v_xor_b32": 5.4277e13,
    "v_bitop3_b32": 5.6564e13, "v_mad_u64_u32": 2.9577e13, "v_exp_f32": 1.8809e13, "v_sin_f32": 1.8770e13,
    "v_cos_f32": 1.8820e13, "v_sqrt_f32": 1.8793e13,
}
# Instructions one FP32 Metropolis update needs (per lane): Philox4x32-10 with the wave-uniform
# half of its first two rounds on the scalar unit (18 64-bit products, 15 three-way and 4
# two-way xors); three exact uniforms (alignbit + subtract each) and z = 2u - 1 (fma);
# proposal (fma, sqrt, sin, cos, 2 mul); local field (15 add); dE and test (3 sub, mul,
# 2 fma, mul, exp2, compare); new-spin select (3 cndmask); fused measurement (3 add for M,
# 3 fma for S.h on the odd half, 1.5 on average). Site addresses are immediate offsets.
UPDATE_OPS_F32 = {
    "v_mad_u64_u32": 18, "v_bitop3_b32": 15, "v_xor_b32": 4, "v_alignbit_b32": 3, "v_sub_f32": 6,
    "v_fma_f32": 5.5, "v_mul_f32": 4, "v_sqrt_f32": 1, "v_sin_f32": 1, "v_cos_f32": 1, "v_exp_f32": 1,
    "v_add_f32": 18, "v_cmp_lt_f32": 1, "v_cndmask_b32": 3,
}
# Summed class by class these cost 153.9 lane-slots; the classes partly overlap in the
# hardware, so the ceiling is measured instead: the same 81.5 instructions per update (163 per
# two updates, checked in the compiled loop) on independent chains with no memory traffic run
# at 5.874e11 updates/s on one MI355X (`opbench` "update_mix"), i.e. 133.9 lane-slots of the
# peak per update.
SUMMED_SLOTS_PER_UPDATE_F32 = sum(n * VALU_PEAK / OP_RATES[op] for op, n in UPDATE_OPS_F32.items())
# The mix's rate, hence the lane-slots per update, follows each box's sustained clock: it is
# measured in the benchmarking process itself (measure_update_mix) right after the timed steps.
# 2-D Ising update (per site): a quarter of one Philox4x32-10 call (one call serves four
# sites); the field (3 adds), a = s h (multiply), the threshold index (2) and the
# always-accept flag (2), the threshold select (4 cndmask) and compare, the flipped spin
# (cndmask), the accept and magnetisation counts (2 adds), s h on the odd half (1/2 multiply
# and add).
UPDATE_OPS_ISING = {
    "v_mad_u64_u32": 4.5, "v_bitop3_b32": 3.75, "v_xor_b32": 1.0, "v_add_u32": 9.5, "v_mul_lo_u32": 1.5,
    "v_cndmask_b32": 5.0, "v_cmp_lt_f32": 1.0,
}
OP_RATES.update({"v_add_u32": 5.2908e13, "v_mul_lo_u32": 3.4925e13})
# (summed class by class: like the FP32 update's summed cost, an upper estimate of the cost, so
# the Ising VALU fraction is an upper estimate too)
SLOTS_PER_UPDATE_ISING = sum(n * VALU_PEAK / OP_RATES[op] for op, n in UPDATE_OPS_ISING.items())
# resident FP64 spins the plain engine may hold (its comparison is skipped above this)
PLAIN_FP64_MAX_BYTES = 64 << 30


def counters_file(workload, kernel="k_batch_f32"):
    """The committed counter summary of a workload's dominant kernel (family k_batch_f32,
    k_resident_f32 or k_window_f32)."""
    short = workload[:-5] if workload.endswith("-fp32") else workload
    return os.path.join(ROOT, "profiles", f"{kernel}_{short}_counters.md")


def measured_traffic(workload, kernel="k_batch_f32", plan=None):
    """HBM bytes per launch from the committed counter summary of the workload's dominant
    kernel, or None when there is none, the kernels have changed since those counters were
    taken, or the counters were taken with another plan (the tuners may pick other variants on
    another box)."""
    import hashlib
    try:
        text = open(counters_file(workload, kernel)).read()
    except OSError:
        return None
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1305_6758_amd", "csrc", "kernels.hip"), "rb").read()).hexdigest()[:16]
    fields = dict(l.split(": ", 1) for l in text.splitlines()
                  if l.startswith(("kernels_sha256:", "traffic_bytes_per_launch:", "plan:")))
    if fields.get("kernels_sha256") != sha:
        return None
    if plan is not None and fields.get("plan") not in (None, plan):
        return None
    return float(fields["traffic_bytes_per_launch"])


# Algorithmic device-memory bytes per update by placement (the variant name's marker): 36 for
# the device-memory variants (read own 12 B, write 12 B, read the other colour 12 B per
# half-sweep), 18 for the colour split (colour 1 in device memory: read once per colour-0
# update, read and written per colour-1 update), 24 for the x/y split (as the colour split,
# plus colour 0's z: read and written per colour-0 update, read once per colour-1 update);
# LDS-resident lattices (and windows, whose traffic depends on the pass length) move none here.
BYTES_PER_UPDATE = {"-hbm-": 36.0, "-split-": 18.0, "-splitxy-": 24.0, "-ring-": None, "-hring-": None,
                    "-ring2-": None}
BYTES_PER_UPDATE_BY_KIND = {"device-memory": 36, "split": 18, "splitxy": 24, "ring": "24 + 24/L",
                            "half ring": "24 + 12/L", "two-sweep ring": "12 + 36/L + 24/64"}


def ring_bytes_per_update(L, half=False):
    """The plane ring reads each half-plane once per sweep plus four half-planes twice
    (12 (2L + 4) / (2L) B per update) and writes every site once (12 B); the half ring reads
    only colour 0's two planes twice (colour 1 once, from device memory through the L2)."""
    return 12.0 * (2 * L + (2 if half else 4)) / (2 * L) + 12.0


def ring2_bytes_per_update(L, renorm_every=64):
    """The two-sweep ring, per pass of two sweeps (2 L^3 updates): reads 2L + 8 half-planes
    (each once, plus the wrap-around reloads) and writes 2L + 4, 12 L^2 / 2 B each, i.e.
    12 (1 + 3/L) B per update; plus the in-place renormalisation (every site read and written
    once every renorm_every sweeps)."""
    return 12.0 * (1.0 + 3.0 / L) + 24.0 / renorm_every


def device_memory_bytes(instances, plan):
    """(algorithmic device-memory bytes of one step, updates on device-memory variants, updates
    on split variants) for the instances and the plan string of their run (a single variant
    name, or a batch plan whose part after ';' names each instance's variant)."""
    variants = plan.split(";", 1)[1].split() if ";" in plan else [plan] * len(instances)
    if len(variants) != len(instances):
        raise ValueError(f"plan names {len(variants)} variants for {len(instances)} instances")
    upd_of = dict.fromkeys(BYTES_PER_UPDATE, 0)
    total = 0.0
    for (L, T, p, nt, nm), v in zip(instances, variants):
        for k in BYTES_PER_UPDATE:
            if k in v:
                upd = p * L ** 3 * (nt + nm)
                upd_of[k] += upd
                total += upd * (ring_bytes_per_update(L, k == "-hring-") if k in ("-ring-", "-hring-")
                                else ring2_bytes_per_update(L) if k == "-ring2-" else BYTES_PER_UPDATE[k])
    return (total, upd_of["-hbm-"] + upd_of["-ring-"] + upd_of["-hring-"] + upd_of["-ring2-"],
            upd_of["-split-"] + upd_of["-splitxy-"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure_update_mix(target_ms=1500.0):
    """The FP32 update's instruction mix alone (opbench's update_mix: the 81.5 algorithmic VALU
    instructions of one update on independent register chains, no memory traffic) on this GPU,
    in this process, run for about target_ms at full occupancy: its updates/s is the VALU
    ceiling the sweep kernels are measured against. Also returns the mean shader clock of that
    run (MHz, s_memtime cycles over wall-clock ticks)."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_1305_6758_amd", "libmmc_opbench.so"))
    fn = lib.mmc_opbench_update_mix
    fn.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    rate, ms, mhz = C.c_double(), C.c_double(), C.c_double()
    iters = 4096
    for _ in range(6):
        rc = fn(iters, C.byref(rate), C.byref(ms), C.byref(mhz))
        if rc != 0:
            raise RuntimeError(f"mmc_opbench_update_mix failed ({rc})")
        if ms.value >= 0.8 * target_ms:
            break
        iters = int(iters * min(64.0, max(2.0, target_ms / max(ms.value, 1e-3))))
    log(f"update mix: {rate.value:.4e} updates/s over {ms.value:.0f} ms at {mhz.value:.0f} MHz")
    return {"updates_per_s": rate.value, "ms": ms.value, "clock_mhz": mhz.value,
            "lane_slots_per_update": VALU_PEAK / rate.value}


def valu_roofline(updates, kernel_ms, mix, kernel):
    """VALU roofline of a sweep kernel: the update mix's cost per update (lane-slots of the
    published peak, from its rate measured on this GPU) times the updates, over the kernel time."""
    slots = mix["lane_slots_per_update"]
    achieved = slots * updates / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12, "unit": "T VALU lane-op/s",
            "frac": achieved / VALU_PEAK, "traffic": None, "kernel": kernel, "kernel_ms": kernel_ms,
            "lane_slots_per_update": slots, "ceiling_updates_per_s": mix["updates_per_s"],
            "ceiling_clock_mhz": mix["clock_mhz"],
            "ceiling_source": "measured in this run: the update's instruction mix alone (opbench update_mix)"}


def four_sigma_vs_oracle(results, golden):
    """Per instance and observable x = e, |m|, m^2, m^4: |<x>_gpu - <x>_oracle| against
    4 sqrt(SE_gpu^2 + SE_oracle^2). SE_oracle is the oracle sample's standard deviation over
    sqrt(K) when it holds K >= 16 paths; with fewer its own spread is too noisy an estimate
    (a t-law with K - 1 degrees of freedom) and the GPU's per-path spread of the same instance
    stands in for it (both sides sample the same law when the engine is right). With fewer
    than 16 oracle paths and at least 16 instances the z-scores must also have a mean square
    below 2 over all instances and observables (a systematic shift well inside each 4-sigma
    bound still fails that). With fewer instances that check is left out: the four observables
    of an instance are strongly correlated, so their mean square behaves like a chi-square with
    one or two degrees of freedom and exceeds 2 by chance in about one case in seven."""
    import numpy as np
    out = []
    ok = True
    zs = []
    small = golden.get("paths_per_instance", 16) < 16
    pooled = small and len(golden["instances"]) >= 16
    for inst, res in zip(golden["instances"], results):
        row = {"L": inst["L"], "T": inst["T"], "oracle_paths": len(inst["e_mean"])}
        for key in ("e_mean", "absm_mean", "m2_mean", "m4_mean"):
            a = np.asarray(res[key])
            b = np.asarray(inst[key])
            d = abs(a.mean() - b.mean())
            sa = a.std(ddof=1) / math.sqrt(a.size)
            sb = (a.std(ddof=1) if small else b.std(ddof=1)) / math.sqrt(b.size)
            bound = 4 * math.hypot(sa, sb)
            row[key] = {"gpu": float(a.mean()), "oracle": float(b.mean()), "diff": float(d), "bound_4sigma": float(bound)}
            ok = bool(ok and d <= bound)
            zs.append((a.mean() - b.mean()) / math.hypot(sa, sb))
        out.append(row)
    if pooled:
        zs = np.asarray(zs)
        ok = bool(ok and np.mean(zs * zs) < 2.0)
        out.append({"pooled_z": {"n": int(zs.size), "max_abs": float(np.max(np.abs(zs))),
                                 "mean_square": float(np.mean(zs * zs))}})
    return ok, out


def run_batched(instances, steps, warmup, init="sphere", batch_launch="auto"):
    import torch
    from paper_1305_6758_amd import mmc
    inits = {"sphere": mmc.MMC_INIT_SPHERE, "angles": mmc.MMC_INIT_ANGLES, "ordered": mmc.MMC_INIT_ORDERED,
             "mixed": mmc.MMC_INIT_MIXED}
    launch = {"auto": mmc.MMC_BATCH_AUTO, "fused": mmc.MMC_BATCH_FUSED, "per-variant": mmc.MMC_BATCH_PER_VARIANT}
    ctx = mmc.mmc_batch_create([(L, T, 1.0, p, nt, nm) for (L, T, p, nt, nm) in instances], 1234,
                               mmc.config(precision=mmc.MMC_FP32, init=inits[init], batch_launch=launch[batch_launch]))
    ws = mmc.Workspace(ctx)
    plan = mmc.mmc_plan(ctx)
    log("plan:", plan)
    kernel_ms = []
    results = None
    for it in range(warmup + steps):
        if it == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        mmc.mmc_batch_run(ctx)
        kms = mmc.mmc_last_timing_ms(ctx)
        stats = [mmc.mmc_batch_stats(ctx, i) for i in range(len(instances))]
        if it >= warmup:
            kernel_ms.append(kms)
        log(f"batched step {it} ({'warmup' if it < warmup else 'timed'}): kernel {kms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    results = [mmc.mmc_batch_results(ctx, i, inst[2]) for i, inst in enumerate(instances)]
    ws.stream.synchronize()
    mmc.mmc_destroy(ctx)
    return wall, kernel_ms, results, stats, plan


def run_single(instance, steps, warmup, placement, variant=None):
    """A one-instance workload on the tuned (or pinned) single-instance FP32 engine (spins
    resident in device memory between launches): every step reruns all sweeps from the random
    start."""
    import torch
    from paper_1305_6758_amd import mmc
    L, T, p, nt, nm = instance
    ctx = mmc.mmc_create_ex(L, T, 1.0, p, nt, nm, 1234, mmc.config(precision=mmc.MMC_FP32, placement=placement))
    kernel_ms = []
    try:
        if variant:
            mmc.mmc_set_variant(ctx, variant)
        mmc.mmc_tune(ctx)
        plan = mmc.mmc_plan(ctx)
        log("plan:", plan)
        for it in range(warmup + steps):
            if it == warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            if it:
                mmc.mmc_reset(ctx)
            mmc.mmc_run(ctx)
            stats = [mmc.mmc_stats(ctx)]
            kms = mmc.mmc_last_timing_ms(ctx)
            if it >= warmup:
                kernel_ms.append(kms)
            log(f"single step {it} ({'warmup' if it < warmup else 'timed'}): kernel {kms:.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        results = [mmc.mmc_results(ctx, p)]
    finally:
        mmc.mmc_destroy(ctx)
    return wall, kernel_ms, results, stats, plan


def run_plain_fp64(instances, init="sphere"):
    """One pass of the same workload on the plain per-instance FP64 engine."""
    import torch
    from paper_1305_6758_amd import mmc
    init_id = {"sphere": mmc.MMC_INIT_SPHERE, "angles": mmc.MMC_INIT_ANGLES, "ordered": mmc.MMC_INIT_ORDERED,
               "mixed": mmc.MMC_INIT_MIXED}[init]
    total_ms = 0.0
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (L, T, p, nt, nm) in enumerate(instances):
        ctx = mmc.mmc_create_ex(L, T, 1.0, p, nt, nm, 1234,
                                mmc.config(precision=mmc.MMC_FP64, placement=mmc.MMC_PLACE_PLAIN, instance_id=i,
                                           init=init_id))
        try:
            mmc.mmc_run(ctx)
            total_ms += mmc.mmc_last_timing_ms(ctx)
            results.append(mmc.mmc_results(ctx, p))
        finally:
            mmc.mmc_destroy(ctx)
        log(f"plain fp64 instance {i}: {total_ms:.0f} ms so far")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, total_ms, results


def cpu_baseline(instances, init="sphere", proposal="sphere", trace=False, ising=False, idx=None):
    """The FP64 CPU oracle as it stands, on the host cores, on a bounded sample of the
    workload: paths of one instance (idx; by default the second, or the only one), as many per thread as keep
    the sample near 1.5e8 updates per thread (about 15 s); where one path's full sweep count
    exceeds that, the sample paths run fewer sweeps (same thermalised/measured proportion) --
    the oracle's cost per update does not depend on the sweep count."""
    from oracle import oracle as O
    threads = O.max_threads()
    if idx is None:
        idx = 1 if len(instances) > 1 else 0
    L, T, p, nt, nm = instances[idx]
    N = L * L if ising else L ** 3
    budget = 1.5e8  # updates per thread
    sweeps = min(nt + nm, max(1, int(budget / N)))
    nm_s = round(sweeps * nm / (nt + nm)) if nt + nm else 0
    nt_s = sweeps - nm_s
    per_path = N * sweeps
    per_thread = max(1, min(3, int(budget / per_path)))
    n = min(p, per_thread * threads)
    log(f"cpu baseline: {n} paths of L={L}, {nt_s}+{nm_s} sweeps on {threads} threads")
    t0 = time.perf_counter()
    if ising:
        O.ising_run_paths(L, T, n_therm=nt_s, n_meas=nm_s, seed=1234, path_begin=0, path_end=n, instance=idx,
                          init=init, trace_sweeps=sweeps if trace else 0, n_threads=threads)
    else:
        O.run_paths(L, T, n_therm=nt_s, n_meas=nm_s, seed=1234, path_begin=0, path_end=n, instance=idx,
                    n_threads=threads, init=init, proposal=proposal, trace_sweeps=sweeps if trace else 0)
    dt = time.perf_counter() - t0
    upd = n * per_path
    full = "all " if sweeps == nt + nm else f"the first {sweeps} of the "
    # the same oracle on one core: the first path, sweeps bounded to about 2e7 updates
    s1 = min(sweeps, max(1, int(2e7 / N)))
    m1 = round(s1 * nm / (nt + nm)) if nt + nm else 0
    t1 = time.perf_counter()
    if ising:
        O.ising_run_paths(L, T, n_therm=s1 - m1, n_meas=m1, seed=1234, path_begin=0, path_end=1, instance=idx,
                          init=init, n_threads=1)
    else:
        O.run_paths(L, T, n_therm=s1 - m1, n_meas=m1, seed=1234, path_begin=0, path_end=1, instance=idx,
                    n_threads=1, init=init, proposal=proposal)
    d1 = time.perf_counter() - t1
    return {"value": upd / dt, "unit": "spin updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} paths of the L={L}, T={T:g} instance (instance {idx}), {full}"
                      f"{nt}+{nm} sweeps ({nt_s}+{nm_s}): {upd:.3e} updates in {dt:.1f} s",
            "single_core": {"value": N * s1 / d1, "unit": "spin updates/s",
                            "sample": f"path 0 of the same instance, {s1 - m1}+{m1} sweeps on one thread"},
            "cpu_model": cpu_model()}


def fp32_vs_fp64(instances, r32, r64):
    """Per instance and observable: the FP32 and FP64 population means over all paths (same
    seeds, trajectories apart after the first flipped decision), their difference, the 4-sigma
    bound of the two standard errors, and the difference relative to the FP64 mean."""
    import numpy as np
    rows = []
    for (L, T, *_), a, b in zip(instances, r32, r64):
        row = {"L": L, "T": T}
        for key in ("e_mean", "absm_mean", "m2_mean", "m4_mean"):
            x, y = np.asarray(a[key], dtype=np.float64), np.asarray(b[key], dtype=np.float64)
            mx, my = float(x.mean()), float(y.mean())
            bound = 4.0 * float(np.hypot(x.std(ddof=1) / np.sqrt(x.size), y.std(ddof=1) / np.sqrt(y.size)))
            row[key] = {"fp32": mx, "fp64": my, "diff": mx - my, "bound_4sigma": bound,
                        "rel_diff": (mx - my) / abs(my) if my else None, "within": abs(mx - my) <= bound}
        rows.append(row)
    return rows


def tune_only(name):
    """Creates the workload's contexts as its run would and tunes them, without running."""
    from paper_1305_6758_amd import mmc
    from paper_1305_6758_amd.workloads import EXPERIMENTS, WORKLOADS, experiment_instances
    cfg = mmc.config(precision=mmc.MMC_FP32)
    if name in WORKLOADS:
        instances = WORKLOADS[name]["instances"]
        if len(instances) == 1:
            L, T, p, nt, nm = instances[0]
            ctx = mmc.mmc_create_ex(L, T, 1.0, p, nt, nm, 1234, cfg)
            try:
                mmc.mmc_tune(ctx)
                log("tuned:", mmc.mmc_plan(ctx))
            finally:
                mmc.mmc_destroy(ctx)
        else:
            ctx = mmc.mmc_batch_create([(L, T, 1.0, p, nt, nm) for (L, T, p, nt, nm) in instances], 1234, cfg)
            log("tuned:", mmc.mmc_plan(ctx)[:200])
            mmc.mmc_destroy(ctx)
        return
    spec = EXPERIMENTS[name]
    if spec.get("fp64") or spec.get("model", 0) == 1 or spec["kind"].startswith("ising"):
        return  # the plain FP64 engine and the Ising kernels have no variants to choose between
    for (L, T, p, nt, nm) in experiment_instances(spec):
        ctx = mmc.mmc_create_ex(L, T, 1.0, p, nt, nm, 1234, cfg)
        try:
            mmc.mmc_tune(ctx)
        finally:
            mmc.mmc_destroy(ctx)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def binder_summary(instances, results):
    """Cumulants of the four (L, T) instances, their ratio and the crossing (Sec. 4)."""
    from paper_1305_6758_amd import mmc
    cum = [mmc.mmc_binder_cumulant(r) for r in results]
    T1, T2 = instances[0][1], instances[2][1]
    cross = mmc.mmc_cumulant_crossing(T1, T2, [c[0] for c in cum], [c[1] for c in cum])
    return {"cumulants": [{"L": L, "T": T, "U": c[0], "se": c[1]} for (L, T, *_), c in zip(instances, cum)],
            "ratio": [{"T": T1, "R": cross["r_t1"], "se": cross["se_r_t1"]},
                      {"T": T2, "R": cross["r_t2"], "se": cross["se_r_t2"]}],
            "tc": cross["tc"], "se_tc": cross["se_tc"]}


def run_experiment(name, spec, steps, mix):
    """An experiment of Secs. 3-4 or of the 2-D Ising appendix through
    paper_1305_6758_amd.experiments; returns the JSON line."""
    from paper_1305_6758_amd import experiments as X
    from paper_1305_6758_amd.workloads import experiment_instances, site_count
    instances = experiment_instances(spec)
    upd = sum(p * site_count(spec, L) * (nt + nm) for (L, T, p, nt, nm) in instances)
    ising = spec.get("model", 0) == 1 or spec["kind"].startswith("ising")
    walls, kms, out = [], [], None
    for it in range(steps):
        t0 = time.perf_counter()
        if spec["kind"] == "thermalisation":
            out = X.thermalisation(L=spec["L"], T=spec["T"], n_paths=spec["n_paths"], sweeps=spec["sweeps"],
                                   init=spec["init"], fp64=spec["fp64"], model=spec.get("model", 0))
            kms.append(out["kernel_ms"])
        elif spec["kind"] == "ising_m":
            out = X.ising_magnetisation(Ls=spec["Ls"], Ts=spec["Ts"], n_paths=spec["n_paths"], sweeps=spec["sweeps"])
            kms.append(out["kernel_ms"])
        elif spec["kind"] == "ising_binder":
            out = X.ising_binder(Ls=spec["Ls"], Ts=spec["Ts"], n_paths=spec["n_paths"], sweeps=spec["sweeps"])
            kms.append(out["kernel_ms"])
        else:
            out = X.distribution_table(L=spec["L"], Ts=spec["Ts"], n_paths=spec["n_paths"], sweeps=spec["sweeps"],
                                       proposal=spec["proposal"], init=spec["init"], fp64=spec["fp64"])
            kms.append(sum(r["kernel_ms"] for r in out["rows"]))
        walls.append(time.perf_counter() - t0)
        log(f"{name} step {it}: kernels {kms[-1]:.1f} ms, wall {walls[-1]:.2f} s")
    wall, kms_avg = sum(walls) / steps, sum(kms) / steps
    plan = out["plan"] if "plan" in out else out["rows"][0]["plan"]
    kernel = "k_ising" if ising else ("k_plain_half" if plan.startswith("plain") else "k_resident<float>")
    line = {
        "metric": METRIC, "value": upd / wall, "unit": "spin updates/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8" if ising else ("f64" if spec["fp64"] else "f32"), "data": "synthetic",
        "config": {"workload": name, **{k: v for k, v in spec.items() if k != "fp64"}, "updates_per_step": upd,
                   "seed": 1234, "plan": plan},
        "kernel_updates_per_s": upd / (kms_avg * 1e-3),
        "experiment": {k: v for k, v in out.items() if k not in ("plan",)},
    }
    if not spec["fp64"] and not ising:
        line["roofline"] = valu_roofline(upd, kms_avg, mix, kernel)
    elif ising:
        slots = SLOTS_PER_UPDATE_ISING
        achieved = slots * upd / (kms_avg * 1e-3)
        line["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                            "unit": "T VALU lane-op/s", "frac": achieved / VALU_PEAK, "traffic": None,
                            "kernel": kernel, "kernel_ms": kms_avg, "lane_slots_per_update": slots,
                            "ceiling_updates_per_s": VALU_PEAK / slots,
                            "ceiling_source": "summed instruction-class model (an upper estimate of the cost)"}
    else:
        # plain FP64 engine: 72 B of algorithmic device-memory traffic per update
        achieved = 72.0 * upd / (kms_avg * 1e-3)
        line["roofline"] = {"bound": "hbm", "achieved": achieved / 1e9, "peak": 8000.0, "unit": "GB/s",
                            "frac": achieved / 8e12, "traffic": None, "kernel": kernel, "kernel_ms": kms_avg,
                            "bytes_per_update": 72}
    return line, instances


# The largest configuration: the uneven batch of 96 (L, T) instances, measured once per bench
# run beside the stepped default workload.
LARGEST = "uneven-batch-96-fp32"
# the two device-memory configurations: L = 32, 1024 paths, 5000 + 5000 sweeps; L = 64, 256
# paths, 10000 + 10000 sweeps (one timed pass each in the default run)
DEVICE_MEMORY_CONFIGS = ("L32-T1.443-p1024", "L64-T1.443-p256-fp32")


def parity_summary(rows):
    """Compact form of four_sigma_vs_oracle's rows: the largest |diff| / bound over every
    (instance, observable) and where it is."""
    worst = (0.0, None)
    n = 0
    for r in rows:
        for key in ("e_mean", "absm_mean", "m2_mean", "m4_mean"):
            if key in r:
                n += 1
                q = r[key]["diff"] / r[key]["bound_4sigma"] if r[key]["bound_4sigma"] > 0 else float("inf")
                if q > worst[0]:
                    worst = (q, {"L": r["L"], "T": r["T"], "observable": key, **r[key]})
    return {"comparisons": n, "max_diff_over_bound": worst[0], "worst": worst[1]}


def measure_workload(name, steps, warmup, mix, a, plain_paths=None, compact=False, cpu=True):
    """One batched (or single-instance) FP32 workload of workloads.WORKLOADS: `steps` timed
    passes after `warmup` untimed ones, parity with the stored oracle sample, the VALU and
    device-memory rooflines, the plain FP64 engine on the same seeds (all paths, or the first
    plain_paths of each instance), and the oracle on the host cores. Returns the JSON record."""
    import numpy as np
    from paper_1305_6758_amd.workloads import WORKLOADS, updates
    from paper_1305_6758_amd import mmc as _m
    instances = WORKLOADS[name]["instances"]
    upd_step = updates(instances)
    single = len(instances) == 1
    if single:
        place = {"auto": _m.MMC_PLACE_AUTO, "lds": _m.MMC_PLACE_LDS, "hbm": _m.MMC_PLACE_HBM,
                 "window": _m.MMC_PLACE_WINDOW}[a.placement]
        wall, kernel_ms, results, stats, plan = run_single(instances[0], steps, warmup, place, a.variant)
    else:
        wall, kernel_ms, results, stats, plan = run_batched(instances, steps, warmup,
                                                            init=WORKLOADS[name].get("init", "sphere"),
                                                            batch_launch=a.batch_launch)
    value = upd_step * steps / wall
    kms = sum(kernel_ms) / len(kernel_ms)
    hbm_bytes, hbm_upd, split_upd = device_memory_bytes(instances, plan)
    # the batch runs one persistent kernel per variant in use: name them by their variants
    launched = re.findall(r"\[(\S+) block=\d+ workgroups=", plan)
    fused = any(x.startswith("fused:") for x in launched)
    kernel_name = (("k_batch_fused<float> " if fused else "k_batch<float> ") + " + ".join(launched)) if not single else (
        "k_window<float>" if "win-" in plan else "k_resident<float>")
    kernel_family = kernel_name.split()[0].replace("<float>", "_f32")
    traffic = measured_traffic(name, kernel_family, plan)
    if mix is None:
        mix = measure_update_mix()

    golden_path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    parity = None
    if os.path.exists(golden_path):
        with open(golden_path) as f:
            ok, rows = four_sigma_vs_oracle(results, json.load(f))
        parity = {"agree_4sigma": ok, **({"summary": parity_summary(rows)} if compact else {"per_instance": rows})}

    Ls = sorted({x[0] for x in instances})
    config = {"workload": name, "L": Ls[0] if len(Ls) == 1 else Ls,
              "T": sorted({x[1] for x in instances}) if len(instances) <= 16 else [min(x[1] for x in instances),
                                                                               max(x[1] for x in instances)],
              "instances": len(instances),
              "paths": sum(x[2] for x in instances), "n_therm": sorted({x[3] for x in instances}),
              "n_meas": sorted({x[4] for x in instances}), "updates_per_step": upd_step, "seed": 1234,
              "plan": plan, "engine": "single-instance, tuned" if single else f"batch ({a.batch_launch} launch)",
              "init": WORKLOADS[name].get("init", "sphere")}
    roof = valu_roofline(upd_step, kms, mix, kernel_name)
    roof["traffic"] = traffic
    out = {
        "metric": METRIC, "value": value, "unit": "spin updates/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic", "config": config, "roofline": roof, "parity": parity,
    }
    if hbm_bytes > 0:
        # the bound reported is the one the kernels come closer to; the other rides along
        gbs = hbm_bytes / (kms * 1e-3) / 1e9
        hbm = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
               "traffic": traffic, "kernel": kernel_name, "kernel_ms": kms,
               "bytes_per_update": BYTES_PER_UPDATE_BY_KIND, "hbm_updates_per_step": hbm_upd,
               "split_updates_per_step": split_upd}
        if hbm["frac"] > out["roofline"]["frac"]:
            out["roofline_valu"] = out["roofline"]
            out["roofline"] = hbm
        else:
            out["roofline_hbm"] = hbm
    if len(instances) <= 16:
        out["stats"] = [{k: s[k] for k in ("mean_e", "se_e", "mean_absm", "se_absm", "chi", "cv_heat", "binder",
                                           "r_e", "p_norm_e", "accept_rate")} for s in stats]
    if name.startswith("binder-"):
        out["experiment"] = binder_summary(instances, results)
    plain_inst = [(L, T, min(p, plain_paths) if plain_paths else p, nt, nm) for (L, T, p, nt, nm) in instances]
    fits = sum(p * 3 * 8 * L ** 3 for (L, T, p, nt, nm) in plain_inst) <= PLAIN_FP64_MAX_BYTES
    if not a.skip_plain and fits:
        pwall, pms, presults = run_plain_fp64(plain_inst, init=WORKLOADS[name].get("init", "sphere"))
        pupd = updates(plain_inst)
        out["fp64_plain"] = {"value": pupd / pwall, "unit": "spin updates/s", "kernel_ms": pms,
                             "speedup_of_batched_fp32": value / (pupd / pwall)}
        if plain_paths:
            out["fp64_plain"]["sample"] = f"the first {plain_paths} paths of every instance, all sweeps ({pupd:.3e} updates)"
        if os.path.exists(golden_path):
            with open(golden_path) as f:
                ok, rows = four_sigma_vs_oracle(presults, json.load(f))
            out["fp64_plain"]["agree_4sigma"] = ok
        cmp = fp32_vs_fp64(plain_inst, [{k: np.asarray(r[k])[:q[2]] for k in r} for r, q in zip(results, plain_inst)],
                           presults)
        if len(instances) <= 16:
            out["fp32_vs_fp64"] = cmp
        else:
            within = [row[k]["within"] for row in cmp for k in ("e_mean", "absm_mean", "m2_mean", "m4_mean")]
            out["fp32_vs_fp64"] = {"comparisons": len(within), "within_4sigma": int(sum(within)),
                                   "max_abs_rel_diff": max(abs(row[k]["rel_diff"] or 0.0) for row in cmp
                                                           for k in ("e_mean", "absm_mean"))}
    if cpu and not a.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(instances, init=WORKLOADS[name].get("init", "sphere"),
                                           idx=None if len(instances) <= 16 else
                                           max(range(len(instances)), key=lambda i: instances[i][0]))
    return out, mix


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 3; 1 off the default workload)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (default 1; 0 off the default workload)")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--placement", default="auto", choices=["auto", "lds", "hbm", "window"],
                    help="one-instance workloads: spin placement of the single-instance engine")
    ap.add_argument("--variant", default=None,
                    help="one-instance workloads: pin the kernel variant by name instead of tuning")
    ap.add_argument("--tune-only", action="store_true",
                    help="run the tuners of the workload's contexts (their choices go to the MMC_TUNE_CACHE "
                         "file when set) and exit, so that a later (profiled) run launches only its steps")
    ap.add_argument("--batch-launch", default="auto", choices=["auto", "fused", "per-variant"],
                    help="batch workloads: one fused persistent kernel, or one kernel per variant (auto: the library's rule)")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-largest", action="store_true",
                    help="default workload only: leave out the one-pass records of the uneven batch and "
                         "of the two device-memory configurations")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the engine runs its paths on a single MI355X; several GPUs "
              "would each take a contiguous range of path indices, which is not built here.",
              file=sys.stderr)
        sys.exit(2)

    from paper_1305_6758_amd.workloads import EXPERIMENTS, WORKLOADS
    if a.workload not in WORKLOADS and a.workload not in EXPERIMENTS:
        print(f"unknown workload {a.workload}; one of {sorted(WORKLOADS) + sorted(EXPERIMENTS)}", file=sys.stderr)
        sys.exit(2)
    if a.tune_only:
        tune_only(a.workload)
        return
    if a.workload in EXPERIMENTS:
        spec = EXPERIMENTS[a.workload]
        ising = spec.get("model", 0) == 1 or spec["kind"].startswith("ising")
        mix = None if (spec["fp64"] or ising) else measure_update_mix()
        line, instances = run_experiment(a.workload, spec, a.steps or 1, mix)
        if not a.skip_cpu:
            line["cpu_baseline"] = cpu_baseline(instances, init=spec["init"], proposal=spec.get("proposal", "sphere"),
                                                trace=spec["kind"] == "thermalisation", ising=ising)
        print(json.dumps(line), flush=True)
        return
    default = a.workload == WORKLOAD
    steps = a.steps if a.steps is not None else (3 if default else 1)
    warmup = a.warmup if a.warmup is not None else (1 if default else 0)
    if steps < 1 or warmup < 0:
        print("need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    if a.variant and len(WORKLOADS[a.workload]["instances"]) != 1:
        print("--variant applies to one-instance workloads only", file=sys.stderr)
        sys.exit(2)
    out, mix = measure_workload(a.workload, steps, warmup, None, a)
    if default and not a.skip_largest:
        # the largest configuration, one timed pass (a step of it lasts about a minute or more)
        log(f"largest configuration: {LARGEST}, one pass")
        sub, _ = measure_workload(LARGEST, 1, 0, mix, a, plain_paths=64, compact=True)
        for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            sub.pop(k, None)
        out["largest_config"] = sub
    if default and not a.skip_largest:
        # the device-memory configurations, one timed pass each (the plain FP64 engine on a
        # sample of their paths; no CPU leg)
        out["device_memory_configs"] = {}
        for w in DEVICE_MEMORY_CONFIGS:
            log(f"device-memory configuration: {w}, one pass")
            sub, _ = measure_workload(w, 1, 0, mix, a, plain_paths=64, compact=True, cpu=False)
            for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
                sub.pop(k, None)
            out["device_memory_configs"][w] = sub
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
