"""The fused batch kernel (asked for with MMC_BATCH_FUSED): one persistent launch for a batch
that mixes lattice sides, every item in one queue, largest first, each run with its instance's
member code. Against the per-variant launches on the same batch (same variants pinned), every
per-path result is identical bit for bit: a member computes a path exactly as the batch variant
it is named after. AUTO runs the per-variant launches."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MEMBERS = ["f32-lds-L8-g64", "f32-lds-L12-g256", "f32-lds-L16-g512", "f32-lds-L20-g1024", "f32-split-L24-g1024",
           "f32-split-L30-g1024", "f32-splitxy-L32-g1024", "f32-ring-L48-g1024"]
INSTS = [(8, 1.3, 1.0, 37, 4, 5), (12, 1.5, -1.0, 9, 3, 4), (16, 1.44, 1.0, 11, 5, 3), (20, 1.8, 1.0, 3, 3, 2),
         (24, 1.2, 1.0, 4, 4, 3), (30, 1.45, 1.0, 2, 3, 3), (32, 1.44, 1.0, 3, 2, 4), (48, 1.6, 1.0, 2, 3, 2),
         (16, math.inf, 1.0, 5, 2, 2), (8, 0.7, 1.0, 17, 6, 0)]


def say(*a):
    print(*a, flush=True)


def run(mode, pins=MEMBERS, insts=INSTS):
    from paper_1305_6758_amd import mmc
    ctx = mmc.mmc_batch_create(insts, 1234, mmc.config(precision=mmc.MMC_FP32, renorm_every=3, batch_launch=mode))
    try:
        for name in pins:
            mmc.mmc_set_variant(ctx, name)
        plan = mmc.mmc_plan(ctx)
        say("plan", plan[:160])
        mmc.mmc_batch_run(ctx)
        return plan, [mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)]
    finally:
        mmc.mmc_destroy(ctx)


def test_fused_batch_equals_per_variant_launches():
    from paper_1305_6758_amd import mmc
    say("case fused vs per-variant")
    p0, ref = run(mmc.MMC_BATCH_PER_VARIANT)
    assert "launches=8" in p0
    for mode in (mmc.MMC_BATCH_FUSED, mmc.MMC_BATCH_AUTO):
        p1, got = run(mode)
        # AUTO runs the per-variant launches
        assert ("launches=1 [fused:" in p1) if mode == mmc.MMC_BATCH_FUSED else p1 == p0, p1
        for i, (g, r) in enumerate(zip(got, ref)):
            assert np.array_equal(g["n_accept"], r["n_accept"]), i
            for k in ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e", "final_m"):
                assert np.array_equal(g[k], r[k], equal_nan=True), (i, k)


def test_fused_batch_refused_without_members():
    """An explicit fused request with a pinned variant that has no member (the device-memory
    kernel), or in FP64, makes the run fail with a message; AUTO falls back to per-variant
    launches."""
    from paper_1305_6758_amd import mmc
    insts = [(8, 1.3, 1.0, 5, 2, 2), (48, 1.5, 1.0, 1, 2, 2)]
    ctx = mmc.mmc_batch_create(insts, 1, mmc.config(batch_launch=mmc.MMC_BATCH_FUSED))
    try:
        mmc.mmc_set_variant(ctx, "f32-hbm-L48-g512")
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_batch_run(ctx)
        assert e.value.code == mmc.MMC_EUNSUPPORTED and "fused" in mmc.mmc_last_error()
    finally:
        mmc.mmc_destroy(ctx)
    ctx = mmc.mmc_batch_create(insts, 1, mmc.config(precision=mmc.MMC_FP64, batch_launch=mmc.MMC_BATCH_FUSED))
    try:
        with pytest.raises(mmc.MMCError):
            mmc.mmc_batch_run(ctx)
    finally:
        mmc.mmc_destroy(ctx)
    plan, _ = run(mmc.MMC_BATCH_AUTO, pins=["f32-lds-L8-g64", "f32-hbm-L48-g512"], insts=insts)
    assert "launches=2" in plan and "fused" not in plan


def test_per_variant_launches_on_fewer_graph_branches():
    """The per-variant launches of a batch run on at most GPU_MAX_HW_QUEUES graph branches (4
    when unset), the smallest launches one after another on the last branch: with 1, 2 and 4
    branches the eight launches of the batch give the same per-path results bit for bit."""
    import os
    from paper_1305_6758_amd import mmc
    say("case per-variant launches on 1, 2 and 4 graph branches")
    old = os.environ.get("GPU_MAX_HW_QUEUES")
    results = []
    try:
        for q in ("1", "2", "4"):
            os.environ["GPU_MAX_HW_QUEUES"] = q  # read by the library when it captures the batch's graph
            plan, res = run(mmc.MMC_BATCH_PER_VARIANT)
            assert "launches=8" in plan
            results.append(res)
    finally:
        if old is None:
            os.environ.pop("GPU_MAX_HW_QUEUES", None)
        else:
            os.environ["GPU_MAX_HW_QUEUES"] = old
    for res in results[1:]:
        for i, (g, r) in enumerate(zip(res, results[0])):
            assert np.array_equal(g["n_accept"], r["n_accept"]), i
            for k in ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e", "final_m"):
                assert np.array_equal(g[k], r[k], equal_nan=True), (i, k)
