"""The split placements: colour 0 of each path in LDS and colour 1 swept in place in device
memory (variants *-split-*), or only colour 0's x and y components in LDS (*-splitxy-*).
FP64 reproduces the oracle like every other FP64 kernel; FP32 gives
spins and accept counts bit-identical to the device-memory kernels (a site's update does not
depend on where its spins live), including renormalisation and runs split at any sweep; the
batch forms run beside LDS and device-memory kernels in one batch."""
import numpy as np
import pytest

from helpers import assert_results_close, engine_run, max_abs_diff, oracle_run

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("L,variant", [(2, "f64-split-any-g512-b512"), (6, "f64-split-any-g512-b512"),
                                       (10, "f64-split-any-g512-b512"), (20, "f64-split-any-g512-b512"),
                                       (4, "f64-splitxy-any-g512-b512"), (10, "f64-splitxy-any-g512-b512"),
                                       (24, "f64-splitxy-any-g512-b512")])
def test_fp64_split_matches_oracle(L, variant):
    """Generic FP64 split variants against the oracle: results, per-sweep trace and final spins
    within 1e-12 (L = 20: colour 0 takes 96 KB of LDS; L = 24: colour 0's x and y take 110 KB;
    the whole lattice would fit in neither)."""
    n, nt, nm, T = 3, 3, 4, 1.3
    say(f"case fp64 split L={L} {variant}")
    ora = oracle_run(L, T, n, nt, nm, trace=nt + nm, want_spins=True)
    eng, tr, sp, plan, _ = engine_run(L, T, n, nt, nm, trace=nt + nm, spins_of=range(n), variant=variant)
    assert plan == variant
    assert_results_close(eng, ora, TOL64)
    assert max_abs_diff(tr, ora["trace"]) <= TOL64
    for p in range(n):
        assert max_abs_diff(sp[p], ora["spins"][p]) <= TOL64, p


@pytest.mark.parametrize("L,variant", [(24, "f32-split-L24-g1024-b1024"), (30, "f32-split-L30-g1024-b1024"),
                                       (14, "f32-split-any-g512-b512"), (32, "f32-splitxy-L32-g1024-b1024"),
                                       (14, "f32-splitxy-any-g512-b512")])
def test_fp32_split_bitwise_equals_device_memory_kernel(L, variant):
    """FP32 split variants against the generic device-memory kernel: identical final spins and
    accept counts, with renormalisation every 4 sweeps; energies equal to FP32 rounding."""
    n, nt, nm, T = 3, 5, 4, 1.35
    say(f"case fp32 split L={L} {variant}")
    ref, _, sp_ref, _, _ = engine_run(L, T, n, nt, nm, fp64=False, renorm_every=4, spins_of=range(n),
                                      variant="f32-hbm-any-g512-b512")
    got, _, sp, plan, _ = engine_run(L, T, n, nt, nm, fp64=False, renorm_every=4, spins_of=range(n),
                                     variant=variant)
    assert plan == variant
    assert np.array_equal(got["n_accept"], ref["n_accept"])
    for p in range(n):
        assert np.array_equal(sp[p], sp_ref[p]), p
    for k in ("e_mean", "absm_mean", "final_e"):
        assert max_abs_diff(got[k], ref[k]) < 1e-5, k


def test_fp32_split_batch_equals_device_memory_batch():
    """A batch of L = 24, 30 and 32 instances (ragged path counts) on each split batch variant
    and on the device-memory batch kernel: identical accept counts, final energies equal to
    FP32 rounding."""
    from paper_1305_6758_amd import mmc
    insts = [(24, 1.3, 1.0, 3, 4, 3), (30, 1.4, 1.0, 2, 3, 4), (30, 1.45, 1.0, 3, 2, 2), (32, 1.44, 1.0, 2, 3, 3)]
    # (pinned in order: a later pin takes every instance it fits, so the colour split, which
    # does not fit L = 32, comes after the generic x/y split)
    runs = [("f32-hbm-any-g512",), ("f32-splitxy-any-g1024", "f32-split-any-g1024"),
            ("f32-split-L24-g1024", "f32-split-L30-g1024", "f32-splitxy-L32-g1024")]
    got = []
    for pins in runs:
        say(f"case batch split {pins}")
        ctx = mmc.mmc_batch_create(insts, 1234, mmc.config(precision=mmc.MMC_FP32))
        try:
            for v in pins:
                mmc.mmc_set_variant(ctx, v)
            plan = mmc.mmc_plan(ctx)
            for v in pins:
                assert v in plan, plan
            mmc.mmc_batch_run(ctx)
            got.append([mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)])
        finally:
            mmc.mmc_destroy(ctx)
    for g in got[1:]:
        for i in range(len(insts)):
            assert np.array_equal(g[i]["n_accept"], got[0][i]["n_accept"]), i
            assert max_abs_diff(g[i]["final_e"], got[0][i]["final_e"]) < 1e-5, i


def test_fp64_mixed_batch_with_split_matches_oracle():
    """One FP64 batch running an LDS kernel (L = 8), the split kernel (L = 20) and the
    device-memory kernel (L = 32) side by side: every path matches the oracle run with
    instance id = batch index."""
    from paper_1305_6758_amd import mmc
    insts = [(8, 1.5, 1.0, 5, 3, 4), (20, 1.3, 1.0, 3, 2, 3), (32, 1.2, 1.0, 1, 1, 1), (8, 1.1, 1.0, 2, 4, 2)]
    say("case fp64 batch lds + split + device memory")
    ctx = mmc.mmc_batch_create(insts, 1234, mmc.config(precision=mmc.MMC_FP64))
    try:
        mmc.mmc_set_variant(ctx, "f64-split-any-g512")  # L = 8 and 20
        mmc.mmc_set_variant(ctx, "f64-lds-L8-g128")     # L = 8 back to the LDS kernel
        mmc.mmc_set_variant(ctx, "f64-hbm-L32-g512")
        plan = mmc.mmc_plan(ctx)
        say("plan", plan)
        assert "launches=3" in plan and "L20:f64-split-any-g512" in plan and "L8:f64-lds-L8-g128" in plan
        mmc.mmc_batch_run(ctx)
        for i, (L, T, J, n, nt, nm) in enumerate(insts):
            eng = mmc.mmc_batch_results(ctx, i, n)
            ora = oracle_run(L, T, n, nt, nm, J=J, instance_id=i)
            assert_results_close(eng, ora, TOL64)
    finally:
        mmc.mmc_destroy(ctx)


@pytest.mark.parametrize("variant", ["f64-split-any-g512-b512", "f64-splitxy-any-g512-b512"])
def test_fp64_split_edge_cases_match_oracle(variant):
    """The split placements at the edges: negative J, infinite temperature (every move
    accepted), no measured sweeps (NaN means) and a nonzero instance id with a 64-bit seed,
    each against the oracle to 1e-12."""
    import math
    say(f"case split edges {variant} J<0")
    ora = oracle_run(6, 0.9, 3, 4, 4, J=-1.0)
    eng, *_ = engine_run(6, 0.9, 3, 4, 4, J=-1.0, variant=variant)
    assert_results_close(eng, ora, TOL64)
    say(f"case split edges {variant} T=inf")
    ora = oracle_run(8, math.inf, 3, 2, 3)
    eng, *_ = engine_run(8, math.inf, 3, 2, 3, variant=variant)
    assert_results_close(eng, ora, TOL64)
    assert np.all(eng["n_accept"] == 512 * 5)
    say(f"case split edges {variant} n_meas=0")
    ora = oracle_run(8, 1.1, 3, 5, 0)
    eng, *_ = engine_run(8, 1.1, 3, 5, 0, variant=variant)
    assert np.all(np.isnan(eng["e_mean"]))
    assert_results_close(eng, ora, TOL64)
    say(f"case split edges {variant} instance/seed")
    ora = oracle_run(8, 1.4, 3, 2, 2, seed=0xDEADBEEF12345, instance_id=77)
    eng, *_ = engine_run(8, 1.4, 3, 2, 2, seed=0xDEADBEEF12345, instance_id=77, variant=variant)
    assert_results_close(eng, ora, TOL64)
