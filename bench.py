"""Benchmark: Metropolis spin updates/s of the batched FP32 multipath engine on one MI355X.

Workload (one step): L = 16 classical Heisenberg lattices at T = 1.2, 1.443 and 1.7, 4096
independent paths per temperature, each from a random start through 2000 thermalisation and
8000 measured checkerboard sweeps (FP32 spins and fields, FP64 accumulators), then the FP64
cross-path statistics -- 5.03e11 spin updates per step, in one persistent hipGraph launch.

Also reported on the same GPU: the plain per-instance FP64 engine on the same workload, the
4-standard-error agreement of the FP32 results with the FP64 CPU oracle (sampled paths,
stored by tests/golden/make_oracle_golden.py), the VALU roofline of the batch kernel, and
the oracle itself timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-plain] [--skip-cpu]
"""
import argparse
import json
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
SLOTS_PER_UPDATE_F32 = sum(n * VALU_PEAK / OP_RATES[op] for op, n in UPDATE_OPS_F32.items())
COUNTERS = os.path.join(ROOT, "profiles", "k_batch_f32_L16-T3-p4096_counters.md")


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, or None when the kernels have
    changed since those counters were taken."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1305_6758_amd", "csrc", "kernels.hip"), "rb").read()).hexdigest()[:16]
    fields = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("kernels_sha256:", "traffic_bytes_per_launch:")))
    if fields.get("kernels_sha256") != sha:
        return None
    return float(fields["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def four_sigma_vs_oracle(results, golden):
    """Per instance: |<x>_gpu - <x>_oracle| against 4 sqrt(SE_gpu^2 + SE_oracle^2) for x = e, |m|."""
    import numpy as np
    out = []
    ok = True
    for inst, res in zip(golden["instances"], results):
        row = {"T": inst["T"], "oracle_paths": len(inst["e_mean"])}
        for key in ("e_mean", "absm_mean"):
            a = np.asarray(res[key])
            b = np.asarray(inst[key])
            d = abs(a.mean() - b.mean())
            bound = 4 * math.hypot(a.std(ddof=1) / math.sqrt(a.size), b.std(ddof=1) / math.sqrt(b.size))
            row[key] = {"gpu": float(a.mean()), "oracle": float(b.mean()), "diff": float(d), "bound_4sigma": float(bound)}
            ok = bool(ok and d <= bound)
        out.append(row)
    return ok, out


def run_batched(instances, steps, warmup):
    import torch
    from paper_1305_6758_amd import mmc
    ctx = mmc.mmc_batch_create([(L, T, 1.0, p, nt, nm) for (L, T, p, nt, nm) in instances], 1234,
                               mmc.config(precision=mmc.MMC_FP32))
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


def run_plain_fp64(instances):
    """One pass of the same workload on the plain per-instance FP64 engine."""
    import torch
    from paper_1305_6758_amd import mmc
    total_ms = 0.0
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (L, T, p, nt, nm) in enumerate(instances):
        ctx = mmc.mmc_create_ex(L, T, 1.0, p, nt, nm, 1234,
                                mmc.config(precision=mmc.MMC_FP64, placement=mmc.MMC_PLACE_PLAIN, instance_id=i))
        try:
            mmc.mmc_run(ctx)
            total_ms += mmc.mmc_last_timing_ms(ctx)
            results.append(mmc.mmc_results(ctx, p))
        finally:
            mmc.mmc_destroy(ctx)
        log(f"plain fp64 instance {i}: {total_ms:.0f} ms so far")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, total_ms, results


def cpu_baseline(instances):
    """The FP64 CPU oracle as it stands, on the host cores: three paths per thread of the
    T = 1.443 instance, all of their sweeps (about 10-30 s of CPU work)."""
    from oracle import oracle as O
    threads = O.max_threads()
    L, T, p, nt, nm = instances[1]
    n = 3 * threads
    t0 = time.perf_counter()
    O.run_paths(L, T, n_therm=nt, n_meas=nm, seed=1234, path_begin=0, path_end=n, instance=1, n_threads=threads)
    dt = time.perf_counter() - t0
    upd = n * L ** 3 * (nt + nm)
    return {"value": upd / dt, "unit": "spin updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} paths (3 per thread) of the L=16, T=1.443 instance, all "
                      f"{nt}+{nm} sweeps: {upd:.3e} updates in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs paths on a single MI355X; "
              "multi-GPU runs are not part of it (paths would shard by index, see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    from paper_1305_6758_amd.workloads import WORKLOADS, updates
    instances = WORKLOADS[WORKLOAD]["instances"]
    upd_step = updates(instances)

    wall, kernel_ms, results, stats, plan = run_batched(instances, a.steps, a.warmup)
    value = upd_step * a.steps / wall
    kms = sum(kernel_ms) / len(kernel_ms)
    achieved = SLOTS_PER_UPDATE_F32 * upd_step / (kms * 1e-3)

    golden_path = os.path.join(ROOT, "tests", "golden", f"oracle_{WORKLOAD}.json")
    parity = None
    if os.path.exists(golden_path):
        with open(golden_path) as f:
            ok, rows = four_sigma_vs_oracle(results, json.load(f))
        parity = {"agree_4sigma": ok, "per_temperature": rows}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "L": 16, "T": [1.2, 1.443, 1.7], "paths_per_T": 4096,
                   "n_therm": 2000, "n_meas": 8000, "updates_per_step": upd_step, "seed": 1234, "plan": plan},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "T VALU lane-op/s", "frac": achieved / VALU_PEAK, "traffic": measured_traffic(),
                     "kernel": "k_batch<float>", "kernel_ms": kms,
                     "lane_slots_per_update": SLOTS_PER_UPDATE_F32,
                     "ceiling_updates_per_s": VALU_PEAK / SLOTS_PER_UPDATE_F32},
        "parity": parity,
        "stats": [{k: s[k] for k in ("mean_e", "se_e", "mean_absm", "se_absm", "chi", "cv_heat", "binder",
                                     "r_e", "p_norm_e", "accept_rate")} for s in stats],
    }
    if not a.skip_plain:
        pwall, pms, presults = run_plain_fp64(instances)
        out["fp64_plain"] = {"value": upd_step / pwall, "unit": "spin updates/s", "kernel_ms": pms,
                             "speedup_of_batched_fp32": value / (upd_step / pwall)}
        if os.path.exists(golden_path):
            with open(golden_path) as f:
                ok, rows = four_sigma_vs_oracle(presults, json.load(f))
            out["fp64_plain"]["agree_4sigma"] = ok
    if not a.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(instances)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
