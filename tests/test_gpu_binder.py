"""Parity of the Binder-cumulant experiment (Sec. 4, eq. (kum)) with the FP64 oracle.

Workload binder-L30-L20-p1e6-fp32: L = 30 and 20 at T = 1.44 and 1.45, single-output paths
(random start, 199 + 1 sweeps), instance ids 0..3 in (T, L) order. The oracle's results for the
first 256 paths of every instance are stored in tests/golden/oracle_binder-L30-L20-p1e6-fp32.json
(written by tests/golden/make_oracle_golden.py, which calls only the oracle).

  - FP64 batch: every sampled path matches the oracle to 1e-12;
  - FP32 batch at 10^5 paths per instance: <M^2>, <M^4>, <e> and the cumulant U agree with the
    oracle's sampled paths within 4 standard errors; the library's crossing equals the
    oracle's formula applied to the same cumulants.
"""
import json
import math
import os

import numpy as np
import pytest

from helpers import assert_results_close, mean_se
from oracle import stats as S

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_binder-L30-L20-p1e6-fp32.json")
# the equilibrated form: 10^4 paths per (L, T), 4000 + 4000 sweeps, time-averaged moments
GOLDEN_EQ = os.path.join(os.path.dirname(__file__), "golden", "oracle_binder-L30-L20-p1e4-s8000-fp32.json")


def say(*a):
    print(*a, flush=True)


def golden(path=GOLDEN):
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


@pytest.mark.timeout(300)
def test_binder_fp64_sampled_paths_match_oracle():
    from paper_1305_6758_amd import mmc
    g = golden()
    K = g["paths_per_instance"]
    rows = [(i["L"], i["T"], 1.0, K, i["n_therm"], i["n_meas"]) for i in g["instances"]]
    say("case binder fp64 batch", K, "paths per instance")
    ctx = mmc.mmc_batch_create(rows, g["seed"], mmc.config(precision=mmc.MMC_FP64))
    try:
        mmc.mmc_batch_run(ctx)
        say("plan", mmc.mmc_plan(ctx))
        for i, inst in enumerate(g["instances"]):
            assert_results_close(mmc.mmc_batch_results(ctx, i, K), as_results(inst), 1e-12)
    finally:
        mmc.mmc_destroy(ctx)


@pytest.mark.timeout(300)
def test_binder_fp32_cumulants_and_crossing():
    from paper_1305_6758_amd.experiments import binder_crossing
    g = golden()
    Ts = sorted({i["T"] for i in g["instances"]})
    Ls = [g["instances"][0]["L"], g["instances"][1]["L"]]
    say("case binder fp32, 1e5 paths per instance")
    out = binder_crossing(Ls=Ls, Ts=Ts, n_paths=10 ** 5, sweeps=200, seed=g["seed"], keep_results=True)
    say("plan", out["plan"], f"{out['kernel_ms']:.0f} ms, {out['updates_per_s']:.3e} updates/s")
    for inst, res, cum in zip(g["instances"], out["results"], out["cumulants"]):
        assert (cum["L"], cum["T"]) == (inst["L"], inst["T"])
        ora = as_results(inst)
        for key in ("m2_mean", "m4_mean", "e_mean"):
            ma, sa = mean_se(res[key])
            mb, sb = mean_se(ora[key])
            bound = 4.0 * math.hypot(sa, sb)
            assert abs(ma - mb) <= bound, f"L={inst['L']} T={inst['T']} {key}: {ma} vs {mb} (4 sigma {bound})"
        Uo, seo = S.binder_cumulant(ora["m2_mean"], ora["m4_mean"])
        Ur, ser = S.binder_cumulant(res["m2_mean"], res["m4_mean"])
        assert abs(cum["U"] - Ur) < 1e-12 and abs(cum["se"] - ser) < 1e-12
        say(f"L={inst['L']} T={inst['T']}: U = {cum['U']:.5f} +- {cum['se']:.5f} (oracle, "
            f"{len(inst['e_mean'])} paths: {Uo:.5f} +- {seo:.5f})")
        assert abs(cum["U"] - Uo) <= 4.0 * math.hypot(cum["se"], seo)
    u = [c["U"] for c in out["cumulants"]]
    se = [c["se"] for c in out["cumulants"]]
    Tc, sTc, R1, s1, R2, s2 = S.cumulant_crossing(Ts[0], Ts[1], u, se)
    assert abs(out["tc"] - Tc) < 1e-12 and abs(out["se_tc"] - sTc) < 1e-12
    assert abs(out["ratio"][0]["R"] - R1) < 1e-14 and abs(out["ratio"][1]["R"] - R2) < 1e-14
    say(f"U30/U20: {R1:.4f} +- {s1:.4f} (T={Ts[0]}), {R2:.4f} +- {s2:.4f} (T={Ts[1]}); crossing {Tc:.4f} +- {sTc:.4f}")


def _batch(rows, seed, fp64):
    from paper_1305_6758_amd import mmc
    ctx = mmc.mmc_batch_create(rows, seed, mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32))
    try:
        mmc.mmc_batch_run(ctx)
        say("plan", mmc.mmc_plan(ctx), f"{mmc.mmc_last_timing_ms(ctx):.0f} ms")
        return [mmc.mmc_batch_results(ctx, i, r[3]) for i, r in enumerate(rows)]
    finally:
        mmc.mmc_destroy(ctx)


@pytest.mark.timeout(300)
def test_equilibrated_binder_fp64_sampled_paths_match_oracle():
    """Workload binder-L30-L20-p1e4-s8000-fp32 (the equilibrated crossing: L = 30 and 20 at
    T = 1.44 and 1.45, 4000 + 4000 sweeps): the FP64 batch's first 8 paths of every instance
    match the oracle's to 1e-12 over all 8000 sweeps."""
    g = golden(GOLDEN_EQ)
    K = 8
    rows = [(i["L"], i["T"], 1.0, K, i["n_therm"], i["n_meas"]) for i in g["instances"]]
    say("case equilibrated binder fp64 batch,", K, "paths per instance")
    res = _batch(rows, g["seed"], fp64=True)
    for i, inst in enumerate(g["instances"]):
        ora = {k: v[:K] for k, v in as_results(inst).items()}
        assert_results_close(res[i], ora, 1e-12)


@pytest.mark.timeout(600)
def test_equilibrated_binder_fp32_cumulants_and_crossing():
    """The same workload at full size in FP32 (10^4 paths per instance, the benchmark's batch):
    <e>, <M^2>, <M^4> and the cumulant U of every instance agree with the oracle's 64 sampled
    paths within 4 standard errors; the crossing of U_30/U_20 from the engine's cumulants lies
    within the paper's T_c = 1.442(20) (Sec. 4), widened by 4 of its own standard errors."""
    g = golden(GOLDEN_EQ)
    rows = [(i["L"], i["T"], 1.0, i["n_paths"], i["n_therm"], i["n_meas"]) for i in g["instances"]]
    say("case equilibrated binder fp32 batch, full size")
    res = _batch(rows, g["seed"], fp64=False)
    u, se = [], []
    for inst, r in zip(g["instances"], res):
        ora = as_results(inst)
        for key in ("e_mean", "m2_mean", "m4_mean"):
            ma, sa = mean_se(r[key])
            mb, sb = mean_se(ora[key])
            bound = 4.0 * math.hypot(sa, sb)
            assert abs(ma - mb) <= bound, f"L={inst['L']} T={inst['T']} {key}: {ma} vs {mb} (4 sigma {bound})"
        Ur, ser = S.binder_cumulant(r["m2_mean"], r["m4_mean"])
        Uo, seo = S.binder_cumulant(ora["m2_mean"], ora["m4_mean"])
        say(f"L={inst['L']} T={inst['T']}: U = {Ur:.5f} +- {ser:.5f} (oracle, {len(inst['e_mean'])} paths: "
            f"{Uo:.5f} +- {seo:.5f})")
        assert abs(Ur - Uo) <= 4.0 * math.hypot(ser, seo)
        u.append(Ur)
        se.append(ser)
    Ts = [g["instances"][0]["T"], g["instances"][2]["T"]]
    Tc, sTc, R1, s1, R2, s2 = S.cumulant_crossing(Ts[0], Ts[1], u, se)
    say(f"U30/U20: {R1:.4f} +- {s1:.4f} (T={Ts[0]}), {R2:.4f} +- {s2:.4f} (T={Ts[1]}); crossing {Tc:.4f} +- {sTc:.4f}")
    assert abs(Tc - 1.442) <= 0.020 + 4.0 * sTc
