"""Host-side checks of the engine library that need no GPU: the C ABI loads and exports every
function the header declares, arguments are validated before any device work, and the host
FP64 statistics agree with the oracle's statistics and with scipy."""
import math
import os
import re
import subprocess
import sys

import numpy as np
import pytest
import scipy.stats as ss

from oracle import oracle as O
from oracle import stats as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "mmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mmc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_1305_6758_amd import mmc
    lib = mmc.lib()
    declared = header_functions()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(mmc.EXPORTED) == declared


def test_arguments_validated_without_gpu():
    from paper_1305_6758_amd import mmc
    bad = [(7, 1.0, 1.0, 4, 1, 1, 1), (0, 1.0, 1.0, 4, 1, 1, 1), (8, 0.0, 1.0, 4, 1, 1, 1),
           (8, -1.0, 1.0, 4, 1, 1, 1), (8, float("nan"), 1.0, 4, 1, 1, 1), (8, 1.0, float("inf"), 4, 1, 1, 1),
           (8, 1.0, 1.0, 0, 1, 1, 1), (8, 1.0, 1.0, 4, -1, 1, 1), (8, 1.0, 1.0, 4, 1, -2, 1)]
    for args in bad:
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_create(*args)
        assert e.value.code == mmc.MMC_EINVAL
        assert mmc.mmc_last_error()
    with pytest.raises(mmc.MMCError) as e:
        mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, mmc.config(precision=mmc.MMC_FP32, placement=mmc.MMC_PLACE_PLAIN))
    assert e.value.code == mmc.MMC_EUNSUPPORTED
    with pytest.raises(mmc.MMCError):
        mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, mmc.config(precision=7))
    with pytest.raises(mmc.MMCError):
        mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, mmc.config(instance_id=1 << 24))
    # a valid context is created without touching a device; its first run reports the missing GPU
    ctx = mmc.mmc_create(8, 1.5, 1.0, 4, 2, 2, 1)
    try:
        assert mmc.mmc_workspace_bytes(ctx) > 4 * 3 * 512 * 4
        assert mmc.mmc_sweeps_done(ctx) == 0
        lib = mmc.lib()
        assert lib.mmc_set_variant(ctx, None) == mmc.MMC_EINVAL
        assert lib.mmc_set_variant(None, b"f32-lds-L8-g64-b256") == mmc.MMC_EINVAL
    finally:
        mmc.mmc_destroy(ctx)
    mmc.mmc_destroy(None)


def test_measurement_library_exports_what_bench_calls():
    """libmmc_opbench.so (the instruction-rate and streaming probes) exports the calls bench.py
    and opbench.py make: the update-mix ceiling with its clock, and the streaming kernels."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_1305_6758_amd", "libmmc_opbench.so"))
    for name in ("mmc_opbench_update_mix", "mmc_opbench_stream", "mmc_opbench_copy", "mmc_opbench_run",
                 "mmc_opbench_count", "mmc_opbench_name"):
        assert hasattr(lib, name), name


def test_load_rejects_missing_or_foreign_files(tmp_path):
    from paper_1305_6758_amd import mmc
    with pytest.raises(mmc.MMCError):
        mmc.mmc_load(str(tmp_path / "nope.bin"))
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a checkpoint at all")
    with pytest.raises(mmc.MMCError):
        mmc.mmc_load(str(junk))


@pytest.mark.parametrize("done", [-1, -(1 << 30), 7, 1 << 30])
def test_load_rejects_sweep_count_out_of_range(tmp_path, done):
    """A checkpoint whose sweep count lies outside 0 .. n_therm + n_meas (here 2 + 4) is
    refused before any device work: the count indexes the trace and divides the measured sums.
    The header is written field by field in the order mmc_save writes it."""
    import ctypes as C
    import struct
    from paper_1305_6758_amd import mmc
    L, n_paths, n_therm, n_meas = 8, 2, 2, 4
    cfg = mmc.config(trace_sweeps=3)
    head = (b"MMCCKPT3" + struct.pack("<iddiiiQ", L, 1.5, 1.0, n_paths, n_therm, n_meas, 1234)
            + bytes(C.string_at(C.addressof(cfg), C.sizeof(cfg))) + struct.pack("<i", done)
            + b"f32-lds-L8-g64-b256".ljust(64, b"\0"))
    body = bytes(n_paths * 3 * L ** 3 * 4 + n_paths * 128 + n_paths * 3 * 4 * 8)
    f = tmp_path / "ckpt.bin"
    f.write_bytes(head + struct.pack("<Q", len(body)) + body)
    with pytest.raises(mmc.MMCError) as e:
        mmc.mmc_load(str(f))
    assert e.value.code == mmc.MMC_EIO
    assert "sweep count" in mmc.mmc_last_error()


def test_host_statistics_match_oracle_statistics():
    """mmc_stats_from_results (C++ host code: AS241 quantiles, Filliben Q-Q fit, K^2) against
    the oracle's statistics (numpy, scipy ndtri) on real oracle output."""
    from paper_1305_6758_amd import mmc
    L, T = 4, 1.3
    r = O.run_paths(L, T, n_therm=50, n_meas=100, path_end=200)
    ref = S.path_statistics(r, L, T)
    got = mmc.mmc_stats_from_results(r, L, T)
    for k in ("mean_e", "se_e", "mean_absm", "se_absm", "e2", "m2", "m4", "chi", "cv_heat", "binder",
              "r_e", "r_absm", "cv_absm", "p_norm_e", "p_norm_absm"):
        assert abs(got[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k
    assert got["n"] == 200


def test_host_normality_and_qq_against_scipy():
    from paper_1305_6758_amd import mmc
    rng = np.random.default_rng(11)
    for n, x in [(25, rng.standard_normal(25)), (400, rng.exponential(size=400)), (4096, rng.standard_normal(4096))]:
        res = {k: np.zeros(n) for k in ("e2_mean", "m2_mean", "m4_mean", "final_e")}
        res["e_mean"] = x
        res["absm_mean"] = np.abs(x) + 1.0
        res["final_m"] = np.zeros((n, 3))
        res["n_accept"] = np.zeros(n, dtype=np.uint64)
        got = mmc.mmc_stats_from_results(res, 4, 1.0)
        assert abs(got["r_e"] - ss.probplot(x)[1][2] ** 2) < 1e-12
        assert abs(got["p_norm_e"] - ss.normaltest(x).pvalue) < 1e-9
        assert abs(got["mean_e"] - x.mean()) < 1e-14 * n
        assert abs(got["se_e"] - x.std(ddof=1) / math.sqrt(n)) < 1e-13


def test_workload_recipes():
    from paper_1305_6758_amd.workloads import WORKLOADS, uneven_batch, updates
    b = uneven_batch()
    assert len(b) == 96
    assert [x[0] for x in b[::16]] == [8, 12, 16, 24, 32, 48]
    assert abs(b[0][1] - 1.0) < 1e-15 and abs(b[15][1] - 2.0) < 1e-15
    assert all(64 <= x[2] <= 2048 for x in b) and all(x[3:] == (2000, 2000) for x in b)
    assert updates(WORKLOADS["L16-T3-p4096-fp32"]["instances"]) == 3 * 4096 * 4096 * 10000


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_device_memory_bytes_by_placement():
    """bench.py prices each instance by its variant's placement: 36 B per update in device
    memory, 18 B for the colour split, 24 B for the x/y split, 24 + 24/L B for the plane ring,
    none in LDS or a multi-sweep window."""
    sys.path.insert(0, ROOT)
    import bench
    insts = [(48, 1.0, 10, 1, 1), (32, 1.2, 4, 2, 2), (24, 1.4, 3, 1, 0), (16, 1.6, 5, 3, 3), (32, 1.8, 2, 1, 1)]
    plan = ("batch launches=4 [...]; L48:f32-hbm-L48-g512 L32:f32-splitxy-L32-g1024 L24:f32-split-L24-g1024 "
            "L16:f32-lds-L16-g512 L32:f32-hbm-any-g512")
    total, hbm_upd, split_upd = bench.device_memory_bytes(insts, plan)
    u = [p * L ** 3 * (nt + nm) for (L, T, p, nt, nm) in insts]
    assert hbm_upd == u[0] + u[4] and split_upd == u[1] + u[2]
    assert total == 36 * (u[0] + u[4]) + 24 * u[1] + 18 * u[2]
    assert bench.device_memory_bytes([(32, 1.4, 8, 5, 5)], "f32-win-L32-d2-b1024") == (0, 0, 0)
    assert bench.device_memory_bytes([(32, 1.4, 8, 5, 5)], "f32-split-L30-g1024-b1024")[0] == 18 * 8 * 32 ** 3 * 10
    # the plane ring: 12 (2L + 4)/(2L) B read + 12 B written per update, 24.5 B at L = 48
    assert bench.device_memory_bytes([(48, 1.4, 2, 3, 3)], "f32-ring-L48-b1024") == (24.5 * 2 * 48 ** 3 * 6,
                                                                                   2 * 48 ** 3 * 6, 0)
    # the half ring: colour 1 read once from device memory, 24 + 12/L B per update
    assert bench.device_memory_bytes([(64, 1.4, 2, 3, 3)], "f32-hring-L64-b1024")[0] == (24 + 12 / 64) * 2 * 64 ** 3 * 6
    with pytest.raises(ValueError):
        bench.device_memory_bytes(insts, "batch launches=1 [x]; L48:f32-hbm-L48-g512")


def test_host_binder_crossing_and_r_match_oracle_statistics():
    """mmc_binder_cumulant, mmc_cumulant_crossing and mmc_distribution_coefficient (C++ host
    code) against the oracle's statistics on oracle snapshot output (n_meas = 1)."""
    from paper_1305_6758_amd import mmc
    us, ses = [], []
    for (L, T) in [(4, 1.3), (2, 1.3), (4, 1.6), (2, 1.6)]:
        r = O.run_paths(L, T, n_therm=40, n_meas=1, path_end=300, seed=5)
        U, se = mmc.mmc_binder_cumulant(r)
        Ur, ser = S.binder_cumulant(r["m2_mean"], r["m4_mean"])
        assert abs(U - Ur) < 1e-13 and abs(se - ser) < 1e-13 * max(1.0, ser)
        us.append(U)
        ses.append(se)
        for a in range(3):
            x = r["final_m"][:, a]
            assert abs(mmc.mmc_distribution_coefficient(x) - S.distribution_coefficient(x)) < 1e-12
    got = mmc.mmc_cumulant_crossing(1.3, 1.6, us, ses)
    ref = S.cumulant_crossing(1.3, 1.6, us, ses)
    for k, v in zip(("tc", "se_tc", "r_t1", "se_r_t1", "r_t2", "se_r_t2"), ref):
        assert abs(got[k] - v) <= 1e-12 * max(1.0, abs(v)), k
    with pytest.raises(mmc.MMCError):
        mmc.mmc_cumulant_crossing(1.0, 1.0, us, ses)
    with pytest.raises(mmc.MMCError):
        mmc.mmc_distribution_coefficient([1.0, 2.0])


def test_host_trace_stats_match_oracle_and_config_checks():
    """mmc_trace_stats (C++ host) against the oracle's per-sweep statistics of an oracle trace
    with the mixed start, for all paths and for each half; configuration checks of the mixed
    start and the both-angles proposal (no GPU needed)."""
    from paper_1305_6758_amd import mmc
    r = O.run_paths(4, 1.0, n_therm=30, n_meas=0, path_end=21, init="mixed", trace_sweeps=30)
    for b, st in ((0, 1), (0, 2), (1, 2)):
        got = mmc.mmc_trace_stats(r["trace"], b, st)
        ref = S.trace_statistics(r["trace"], b, st)
        assert np.max(np.abs(got - ref)) < 1e-13
    with pytest.raises(mmc.MMCError):
        mmc.mmc_trace_stats(r["trace"][:1])
    ctx = mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, mmc.config(init=mmc.MMC_INIT_MIXED))
    mmc.mmc_destroy(ctx)
    ctx = mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, mmc.config(precision=mmc.MMC_FP64, placement=mmc.MMC_PLACE_PLAIN,
                                                               proposal=mmc.MMC_PROPOSAL_ANGLES))
    mmc.mmc_destroy(ctx)
    for cfg in (mmc.config(proposal=mmc.MMC_PROPOSAL_ANGLES),
                mmc.config(precision=mmc.MMC_FP64, placement=mmc.MMC_PLACE_HBM, proposal=mmc.MMC_PROPOSAL_ANGLES)):
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, cfg)
        assert e.value.code == mmc.MMC_EUNSUPPORTED
    for cfg in (mmc.config(init=4), mmc.config(proposal=2)):
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, cfg)
        assert e.value.code == mmc.MMC_EINVAL
