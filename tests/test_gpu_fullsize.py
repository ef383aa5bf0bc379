"""Full-size parity of the GPU engine with the FP64 oracle, in the launch configurations the
benchmark uses. The oracle's results for the first K paths of every instance are stored in
tests/golden/oracle_<workload>.json (written by tests/golden/make_oracle_golden.py, which
calls only the oracle).

  - FP64 engine: the sampled paths match the oracle to 1e-12 (same counter streams, same
    arithmetic order) over the full sweep counts;
  - FP32 engine: the cross-path means agree with the oracle's within 4 standard errors, and
    with the FP64 engine's over all paths (stating the FP32 - FP64 difference).
"""
import json
import math
import os

import numpy as np
import pytest

from helpers import assert_results_close, mean_se

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)


def golden(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"oracle sample {path} not written")
    with open(path) as f:
        return json.load(f)


def as_results(inst):
    out = {k: np.asarray(inst[k], dtype=np.float64) for k in
           ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e")}
    out["final_m"] = np.asarray(inst["final_m"], dtype=np.float64)
    out["n_accept"] = np.asarray(inst["n_accept"], dtype=np.uint64)
    return out


def run_batch(instances, fp64, n_paths_override=None):
    from paper_1305_6758_amd import mmc
    rows = [(L, T, 1.0, n_paths_override or p, nt, nm) for (L, T, p, nt, nm) in instances]
    ctx = mmc.mmc_batch_create(rows, 1234, mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32))
    try:
        mmc.mmc_batch_run(ctx)
        say("plan", mmc.mmc_plan(ctx), f"{mmc.mmc_last_timing_ms(ctx):.0f} ms")
        return [mmc.mmc_batch_results(ctx, i, r[3]) for i, r in enumerate(rows)]
    finally:
        mmc.mmc_destroy(ctx)


def run_single(L, T, n, nt, nm, fp64, instance_id=0):
    from paper_1305_6758_amd import mmc
    ctx = mmc.mmc_create_ex(L, T, 1.0, n, nt, nm, 1234,
                            mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32, instance_id=instance_id))
    try:
        mmc.mmc_run(ctx)
        say("plan", mmc.mmc_plan(ctx), f"{mmc.mmc_last_timing_ms(ctx):.0f} ms")
        return mmc.mmc_results(ctx, n)
    finally:
        mmc.mmc_destroy(ctx)


def four_sigma_ok(a, b, key):
    ma, sa = mean_se(a[key])
    mb, sb = mean_se(b[key])
    d, bound = abs(ma - mb), 4.0 * math.hypot(sa, sb)
    return d <= bound, d, bound


@pytest.mark.timeout(600)
def test_bench_workload_L16_three_temperatures():
    """L = 16, T in {1.2, 1.443, 1.7}, 4096 paths each, 2000 + 8000 sweeps: the batched FP32
    launch of the benchmark vs the oracle (4 sigma, 32 oracle paths per T) and vs the FP64
    engine over all paths; FP64 engine on the sampled paths vs the oracle to 1e-12."""
    g = golden("L16-T3-p4096-fp32")
    insts = [(i["L"], i["T"], i["n_paths"], i["n_therm"], i["n_meas"]) for i in g["instances"]]
    say("case L16 fp32 batch")
    r32 = run_batch(insts, fp64=False)
    say("case L16 fp64 batch, all paths")
    r64 = run_batch(insts, fp64=True)
    for i, inst in enumerate(g["instances"]):
        ora = as_results(inst)
        K = len(inst["e_mean"])
        assert_results_close({k: v[:K] for k, v in r64[i].items()}, ora, TOL64)
        for key in ("e_mean", "absm_mean"):
            ok, d, b = four_sigma_ok(r32[i], ora, key)
            assert ok, f"T={inst['T']} {key}: |FP32 - oracle| = {d:.3e} > {b:.3e}"
            ok, d, b = four_sigma_ok(r32[i], r64[i], key)
            say(f"T={inst['T']} {key}: FP32 - FP64 (all 4096 paths) = {d:.2e} (4 sigma {b:.2e})")
            assert ok


@pytest.mark.timeout(900)
def test_L32_fp32_and_fp64():
    """L = 32, T = 1.443, 1024 paths, 5000 + 5000 sweeps, device-memory spins: FP32 and FP64
    runs side by side; FP64 sampled paths match the oracle to 1e-12; FP32 within 4 sigma of
    the oracle and of the FP64 run."""
    g = golden("L32-T1.443-p1024")
    inst = g["instances"][0]
    L, T, n, nt, nm = inst["L"], inst["T"], inst["n_paths"], inst["n_therm"], inst["n_meas"]
    say("case L32 fp32")
    r32 = run_single(L, T, n, nt, nm, fp64=False)
    say("case L32 fp64")
    r64 = run_single(L, T, n, nt, nm, fp64=True)
    ora = as_results(inst)
    K = len(inst["e_mean"])
    assert_results_close({k: v[:K] for k, v in r64.items()}, ora, TOL64)
    for key in ("e_mean", "absm_mean"):
        ok, d, b = four_sigma_ok(r32, ora, key)
        assert ok, f"{key}: |FP32 - oracle| = {d:.3e} > {b:.3e}"
        ok, d, b = four_sigma_ok(r32, r64, key)
        say(f"L32 {key}: FP32 - FP64 (1024 paths) = {d:.2e} (4 sigma {b:.2e})")
        assert ok


@pytest.mark.timeout(900)
def test_uneven_batch():
    """The uneven batch (96 instances, L = 8 ... 48, T = 1 ... 2, 64-2048 paths, 2000 + 2000
    sweeps) in one persistent launch: FP64 batch on the sampled paths matches the oracle to
    1e-12; the FP32 batch agrees with the oracle per instance and observable within 4 sigma,
    SE_oracle taken from the GPU's per-path spread of the instance over sqrt(K) while the
    oracle sample has fewer than 16 paths, and the z-scores' mean square stays below 2."""
    g = golden("uneven-batch-96-fp32")
    insts = [(i["L"], i["T"], i["n_paths"], i["n_therm"], i["n_meas"]) for i in g["instances"]]
    K = g["paths_per_instance"]
    say("case uneven fp64 sample")
    r64 = run_batch(insts, fp64=True, n_paths_override=K)
    for i, inst in enumerate(g["instances"]):
        assert_results_close(r64[i], as_results(inst), TOL64)
    say("case uneven fp32 full")
    r32 = run_batch(insts, fp64=False)
    z = []
    for i, inst in enumerate(g["instances"]):
        ora = as_results(inst)
        for key in ("e_mean", "absm_mean", "m2_mean", "m4_mean"):
            m32, s32 = mean_se(r32[i][key])
            sd = float(np.std(r32[i][key] if K < 16 else ora[key], ddof=1))
            mo = float(np.mean(ora[key]))
            z.append((m32 - mo) / math.hypot(s32, sd / math.sqrt(K)))
            assert abs(z[-1]) <= 4.0, f"instance {i} (L={inst['L']}, T={inst['T']:.4g}) {key}: z = {z[-1]:.2f}"
    z = np.array(z)
    say(f"uneven batch: max |z| = {np.max(np.abs(z)):.2f}, mean z^2 = {np.mean(z * z):.2f} over {z.size}")
    assert np.mean(z * z) < 2.0


@pytest.mark.timeout(900)
def test_L64():
    """L = 64, T = 1.443, 256 paths, 10^4 + 10^4 sweeps, FP32 device-memory spins: within 4
    sigma of the oracle's sampled paths; normality statistics of the per-path means reported."""
    g = golden("L64-T1.443-p256-fp32")
    inst = g["instances"][0]
    L, T, n, nt, nm = inst["L"], inst["T"], inst["n_paths"], inst["n_therm"], inst["n_meas"]
    say("case L64 fp32")
    r32 = run_single(L, T, n, nt, nm, fp64=False)
    from paper_1305_6758_amd import mmc
    st = mmc.mmc_stats_from_results(r32, L, T)
    say(f"L64: <e> {st['mean_e']:.6f} +- {st['se_e']:.1e}, <|m|> {st['mean_absm']:.5f} +- {st['se_absm']:.1e}, "
        f"r_e {st['r_e']:.4f}, p_norm_e {st['p_norm_e']:.3g}")
    ora = as_results(inst)
    for key in ("e_mean", "absm_mean"):
        ok, d, b = four_sigma_ok(r32, ora, key)
        assert ok, f"{key}: |FP32 - oracle| = {d:.3e} > {b:.3e}"


@pytest.mark.timeout(600)
def test_ising_binder_full_size_sampled_paths_bit_exact():
    """The 2-D Ising cumulant workload at its full size (L = 60 and 50, 5 * 10^4 single-output
    paths, 3 * 10^4 sweeps, the contexts the experiment driver creates): integer spins and
    decisions, so sampled paths from both ends of the path range equal the oracle's exactly
    (accept counts, final m and e, moments)."""
    from oracle import oracle as O
    from paper_1305_6758_amd import mmc
    from paper_1305_6758_amd.experiments import SEED
    n, sweeps = 5 * 10 ** 4, 3 * 10 ** 4
    for (L, T, inst) in [(60, 2.264, 0), (50, 2.268, 3)]:
        say(f"case ising full size L={L} T={T} instance {inst}")
        ctx = mmc.mmc_create_ex(L, T, 1.0, n, sweeps - 1, 1, SEED,
                                mmc.config(model=mmc.MMC_MODEL_ISING2D, instance_id=inst))
        try:
            mmc.mmc_run(ctx)
            say("plan", mmc.mmc_plan(ctx), f"{mmc.mmc_last_timing_ms(ctx):.0f} ms")
            eng = mmc.mmc_results(ctx, n)
        finally:
            mmc.mmc_destroy(ctx)
        for (a, b) in [(0, 3), (n - 2, n)]:
            ora = O.ising_run_paths(L, T, n_therm=sweeps - 1, n_meas=1, seed=SEED, path_begin=a, path_end=b,
                                    instance=inst)
            assert np.array_equal(eng["n_accept"][a:b], ora["n_accept"]), (L, a)
            for k in ("e_mean", "absm_mean", "m2_mean", "m4_mean", "final_e"):
                assert np.max(np.abs(eng[k][a:b] - ora[k])) <= 1e-15, (L, a, k)
            assert np.max(np.abs(eng["final_m"][a:b] - ora["final_m"])) <= 1e-15, (L, a)
