"""Parity of the z-pipelined window kernels (spins in device memory, swept in passes over
z-planes): the plane rings (both colours' planes in LDS with one sweep per pass, "ring", or two,
"ring2"; colour 0's only, "hring"), and the multi-sweep windows, with the planes staged through
a sliding window in LDS ("win") or left in device memory ("gwin").

  - FP64 (L = 12, 16, 24): trajectories, traces, accept counts and final spins match the
    oracle to 1e-12 -- odd sweep counts (a last pass shorter than the others), every start,
    runs split at arbitrary sweeps and a nonzero instance id;
  - FP32 (L = 24 ... 64): final spins and accept counts equal those of the device-memory
    kernels bit for bit (same per-site arithmetic and neighbour values, renormalisation
    boundaries included), energies and magnetisations to FP32 rounding of the sums.
"""
import numpy as np
import pytest

from helpers import assert_results_close, engine_run, max_abs_diff, oracle_run

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
PLACE_HBM, PLACE_WINDOW = 2, 4


def say(*a):
    print(*a, flush=True)


FP64_VARIANTS = [(12, "f64-win-L12-d1-b256"), (16, "f64-win-L16-d2-b256"), (16, "f64-gwin-L16-d2-b256"),
                 (24, "f64-gwin-L24-d3-b512"), (12, "f64-ring-L12-b256"), (16, "f64-ring-L16-b256"),
                 (16, "f64-hring-L16-b256"), (16, "f64-ring2-L16-b128")]


@pytest.mark.parametrize("L,variant", FP64_VARIANTS)
def test_window_fp64_matches_oracle(L, variant):
    for (n, nt, nm, init, inst) in [(5, 3, 4, 0, 0), (4, 0, 7, 2, 3), (3, 5, 0, 3, 1)]:
        if L > 16:
            n = 2
        say(f"case window fp64 {variant} n={n} sweeps={nt}+{nm} init={init} instance={inst}")
        ora = oracle_run(L, 1.3, n, nt, nm, init=["sphere", "angles", "ordered", "mixed"][init], trace=nt + nm,
                         instance_id=inst, want_spins=True)
        eng, tr, sp, plan, _ = engine_run(L, 1.3, n, nt, nm, placement=PLACE_WINDOW, init=init, trace=nt + nm,
                                          instance_id=inst, spins_of=range(n), variant=variant)
        assert plan.startswith(variant), plan
        assert_results_close(eng, ora, TOL64)
        assert max_abs_diff(tr, ora["trace"]) <= TOL64
        for p in range(n):
            assert max_abs_diff(sp[p], ora["spins"][p]) <= TOL64


@pytest.mark.parametrize("variant", ["f64-win-L16-d2-b256", "f64-gwin-L16-d2-b256", "f64-ring-L16-b256",
                                     "f64-hring-L16-b256", "f64-ring2-L16-b128"])
def test_window_fp64_split_runs(variant):
    """Sweeps run in chunks of 3, 1, 4 and the rest equal one uninterrupted run."""
    from paper_1305_6758_amd import mmc
    L, n, nt, nm = 16, 4, 5, 6
    say(f"case window fp64 split {variant}")
    full, _, sp_full, _, _ = engine_run(L, 0.9, n, nt, nm, placement=PLACE_WINDOW, spins_of=range(n), variant=variant)
    ctx = mmc.mmc_create_ex(L, 0.9, 1.0, n, nt, nm, 1234, mmc.config(precision=mmc.MMC_FP64, placement=PLACE_WINDOW))
    try:
        mmc.mmc_set_variant(ctx, variant)
        for k in (3, 1, 4):
            mmc.mmc_run_sweeps(ctx, k)
        mmc.mmc_run(ctx)
        res = mmc.mmc_results(ctx, n)
        assert np.array_equal(res["n_accept"], full["n_accept"])
        for k in ("e_mean", "m2_mean", "final_e"):
            assert max_abs_diff(res[k], full[k]) <= 1e-14
        for p in range(n):
            assert np.array_equal(mmc.mmc_get_spins(ctx, p, L), sp_full[p])
    finally:
        mmc.mmc_destroy(ctx)


FP32_VARIANTS = [(24, "f32-win-L24-d2-b512"), (24, "f32-win-L24-d3-b1024"), (30, "f32-win-L30-d2-b1024"),
                 (32, "f32-win-L32-d2-b512"), (32, "f32-win-L32-d2-b1024"), (32, "f32-gwin-L32-d2-b1024"),
                 (48, "f32-gwin-L48-d1-b1024"), (64, "f32-gwin-L64-d1-b1024"), (16, "f32-ring-L16-b256"),
                 (32, "f32-ring-L32-b512"), (48, "f32-ring-L48-b1024"), (48, "f32-ring-L48-b768"),
                 (16, "f32-hring-L16-b256"), (48, "f32-hring-L48-b1024"), (64, "f32-hring-L64-b1024"),
                 (64, "f32-hring-L64-b768"), (16, "f32-ring2-L16-b128"), (32, "f32-ring2-L32-b512"),
                 (48, "f32-ring2-L48-b768"), (48, "f32-ring2-L48-b1024")]


@pytest.mark.parametrize("L,variant", FP32_VARIANTS)
def test_window_fp32_equals_device_memory_kernels(L, variant):
    n, nt, nm = 3, 7, 6
    for renorm in (5, 0):
        say(f"case window fp32 {variant} renorm_every={renorm}")
        ref, _, sp_ref, plan_ref, _ = engine_run(L, 1.2, n, nt, nm, fp64=False, placement=PLACE_HBM, block=512,
                                                 lanes=512, renorm_every=renorm, spins_of=range(n))
        eng, _, sp, plan, _ = engine_run(L, 1.2, n, nt, nm, fp64=False, placement=PLACE_WINDOW,
                                         renorm_every=renorm, spins_of=range(n), variant=variant)
        assert plan.startswith(variant), plan
        assert np.array_equal(eng["n_accept"], ref["n_accept"]), (plan, plan_ref)
        for p in range(n):
            assert np.array_equal(sp[p], sp_ref[p]), (plan, plan_ref, p)
        for k in ("e_mean", "absm_mean", "m4_mean", "final_e"):
            assert max_abs_diff(eng[k], ref[k]) < 1e-5, (plan, k)


def test_set_variant_rejects_what_does_not_fit():
    from paper_1305_6758_amd import mmc
    ctx = mmc.mmc_create_ex(32, 1.2, 1.0, 2, 1, 1, 1234, mmc.config(precision=mmc.MMC_FP32))
    try:
        for bad in ("f32-gwin-L64-d1-b1024", "f64-gwin-L16-d2-b256", "no-such-variant"):
            with pytest.raises(mmc.MMCError):
                mmc.mmc_set_variant(ctx, bad)
        mmc.mmc_set_variant(ctx, "f32-gwin-L32-d2-b1024")
        mmc.mmc_run(ctx)
        assert mmc.mmc_plan(ctx).startswith("f32-gwin-L32-d2-b1024")
        with pytest.raises(mmc.MMCError):
            mmc.mmc_set_variant(ctx, "f32-hbm-L32-g512-b512")
    finally:
        mmc.mmc_destroy(ctx)


def test_ring_batch_equals_device_memory_batch():
    """The plane-ring batch kernels (L = 48: one sweep per pass with 1024 and 768 lanes, two
    sweeps per pass with 768 and 1024) against the device-memory batch kernel on the same
    instances, ragged path counts, odd sweep counts, renormalisation every 5 sweeps: identical
    accept counts (the spins are identical), energies and magnetisations to FP32 rounding."""
    from paper_1305_6758_amd import mmc
    insts = [(48, 1.3, 1.0, 3, 6, 5), (48, 1.45, 1.0, 2, 5, 6), (48, 2.0, -1.0, 1, 3, 3)]
    got = []
    for pin in ("f32-hbm-L48-g512", "f32-ring-L48-g1024", "f32-ring-L48-g768", "f32-ring2-L48-g768",
                "f32-ring2-L48-g1024"):
        say(f"case ring batch {pin}")
        ctx = mmc.mmc_batch_create(insts, 1234, mmc.config(precision=mmc.MMC_FP32, renorm_every=5))
        try:
            mmc.mmc_set_variant(ctx, pin)
            assert pin in mmc.mmc_plan(ctx)
            mmc.mmc_batch_run(ctx)
            got.append([mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)])
        finally:
            mmc.mmc_destroy(ctx)
    for g in got[1:]:
        for i in range(len(insts)):
            assert np.array_equal(g[i]["n_accept"], got[0][i]["n_accept"]), i
            for k in ("e_mean", "absm_mean", "final_e"):
                assert max_abs_diff(g[i][k], got[0][i][k]) < 1e-5, (i, k)


def test_half_ring_batch_equals_device_memory_batch():
    """The half-ring batch kernel (L = 64, 1024 lanes) against the device-memory batch kernel on
    the same instances, ragged path counts, renormalisation every 3 sweeps: identical accept
    counts (the spins are identical), energies and magnetisations to FP32 rounding."""
    from paper_1305_6758_amd import mmc
    insts = [(64, 1.3, 1.0, 2, 4, 3), (64, 1.45, -1.0, 1, 3, 4)]
    got = []
    for pin in ("f32-hbm-L64-g512", "f32-hring-L64-g1024"):
        say(f"case half-ring batch {pin}")
        ctx = mmc.mmc_batch_create(insts, 1234, mmc.config(precision=mmc.MMC_FP32, renorm_every=3))
        try:
            mmc.mmc_set_variant(ctx, pin)
            assert pin in mmc.mmc_plan(ctx)
            mmc.mmc_batch_run(ctx)
            got.append([mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)])
        finally:
            mmc.mmc_destroy(ctx)
    for i in range(len(insts)):
        assert np.array_equal(got[1][i]["n_accept"], got[0][i]["n_accept"]), i
        for k in ("e_mean", "absm_mean", "final_e"):
            assert max_abs_diff(got[1][i][k], got[0][i][k]) < 1e-5, (i, k)


def test_two_sweep_ring_batch_L32_equals_device_memory_batch():
    """The two-sweep ring's L = 32 batch kernel (two workgroups per CU) against the device-memory
    batch kernel: even and odd sweep counts, renormalisation every 4 sweeps (a one-sweep pass
    before each boundary), identical accept counts, energies and magnetisations to FP32
    rounding."""
    from paper_1305_6758_amd import mmc
    insts = [(32, 1.44, 1.0, 3, 4, 6), (32, 1.2, 1.0, 2, 3, 4), (32, 3.0, -1.0, 2, 1, 2)]
    got = []
    for pin in ("f32-hbm-L32-g512", "f32-ring2-L32-g512"):
        say(f"case two-sweep ring batch {pin}")
        ctx = mmc.mmc_batch_create(insts, 77, mmc.config(precision=mmc.MMC_FP32, renorm_every=4))
        try:
            mmc.mmc_set_variant(ctx, pin)
            assert pin in mmc.mmc_plan(ctx)
            mmc.mmc_batch_run(ctx)
            got.append([mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)])
        finally:
            mmc.mmc_destroy(ctx)
    for i in range(len(insts)):
        assert np.array_equal(got[1][i]["n_accept"], got[0][i]["n_accept"]), i
        for k in ("e_mean", "absm_mean", "final_e"):
            assert max_abs_diff(got[1][i][k], got[0][i][k]) < 1e-5, (i, k)


def test_two_sweep_ring_fp64_edge_cases():
    """The FP64 two-sweep ring at the edges, against the oracle to 1e-12: negative J, infinite
    temperature (every move accepted), no measured sweeps (NaN means), a nonzero instance id
    with a 64-bit seed; odd and even sweep counts (a last one-sweep pass or none)."""
    import math
    v = "f64-ring2-L16-b128"
    say("case two-sweep ring edges J<0")
    ora = oracle_run(16, 0.9, 3, 4, 4, J=-1.0)
    eng, _, _, plan, _ = engine_run(16, 0.9, 3, 4, 4, J=-1.0, placement=PLACE_WINDOW, variant=v)
    assert plan.startswith(v), plan
    assert_results_close(eng, ora, TOL64)
    say("case two-sweep ring edges T=inf")
    ora = oracle_run(16, math.inf, 3, 2, 3)
    eng, *_ = engine_run(16, math.inf, 3, 2, 3, placement=PLACE_WINDOW, variant=v)
    assert_results_close(eng, ora, TOL64)
    assert np.all(eng["n_accept"] == 16 ** 3 * 5)
    say("case two-sweep ring edges n_meas=0")
    ora = oracle_run(16, 1.1, 3, 5, 0)
    eng, *_ = engine_run(16, 1.1, 3, 5, 0, placement=PLACE_WINDOW, variant=v)
    assert np.all(np.isnan(eng["e_mean"]))
    assert_results_close(eng, ora, TOL64)
    say("case two-sweep ring edges instance/seed")
    ora = oracle_run(16, 1.4, 3, 2, 2, seed=0xDEADBEEF12345, instance_id=77)
    eng, *_ = engine_run(16, 1.4, 3, 2, 2, seed=0xDEADBEEF12345, instance_id=77, placement=PLACE_WINDOW,
                         variant=v)
    assert_results_close(eng, ora, TOL64)
