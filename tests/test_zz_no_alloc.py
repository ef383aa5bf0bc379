"""The allocation-free batch entry point (mmc_batch_run_static) against the batch it mirrors:
mmc_batch_create + mmc_batch_run + mmc_batch_results with the same kernel variants pinned.
The same kernels run the same paths, so every per-path result is bit-identical (accept counts,
FP32 and FP64 sums alike). Two calls in a row on the same GPU, the second smaller than the
first (the scratch array keeps the first call's contents), in each precision."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# the default LDS batch variant of each side (the first compiled for that side, else the first
# generic one), as the static entry point picks them
DEFAULT_VARIANT = {False: {8: "f32-lds-L8-g64", 12: "f32-lds-L12-g256", 16: "f32-lds-L16-g512",
                           20: "f32-lds-L20-g512", 10: "f32-lds-any-g512", 6: "f32-lds-any-g512"},
                   True: {8: "f64-lds-L8-g128", 12: "f64-lds-L12-g512", 10: "f64-lds-any-g512",
                          16: "f64-lds-any-g512", 6: "f64-lds-any-g512"}}

CALLS = {
    False: [[(8, 1.3, 1.0, 70, 5, 7), (12, 1.5, -1.0, 33, 4, 6), (16, 1.44, 1.0, 50, 6, 3), (20, 2.0, 1.0, 9, 3, 3),
             (10, math.inf, 1.0, 17, 2, 2), (8, 0.9, 1.0, 130, 3, 0)],
            [(16, 1.2, 1.0, 5, 3, 4), (8, 1.8, 1.0, 3, 2, 2)]],
    True: [[(8, 1.3, 1.0, 40, 4, 5), (12, 1.5, -1.0, 21, 3, 4), (16, 1.44, 1.0, 9, 3, 2), (6, math.inf, 1.0, 11, 2, 3)],
           [(6, 1.1, 1.0, 4, 2, 2), (12, 2.2, 1.0, 2, 1, 3)]],
}


def say(*a):
    print(*a, flush=True)


def static_run(insts, fp64, seed=1234):
    import torch
    from paper_1305_6758_amd import mmc
    n = sum(x[3] for x in insts)
    out = torch.full((n * mmc.RESULT_DTYPE.itemsize,), 0xFF, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    cfg = mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32, renorm_every=3)
    mmc.mmc_batch_run_static(insts, seed, cfg, out.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    res = mmc.path_results_from_bytes(out.cpu().numpy(), n)
    per, o = [], 0
    for x in insts:
        per.append({k: v[o:o + x[3]] for k, v in res.items()})
        o += x[3]
    return per


def batch_run(insts, fp64, seed=1234):
    from paper_1305_6758_amd import mmc
    cfg = mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32, renorm_every=3)
    ctx = mmc.mmc_batch_create(insts, seed, cfg)
    try:
        for name in sorted({DEFAULT_VARIANT[fp64][x[0]] for x in insts}, key=lambda v: "any" not in v):
            mmc.mmc_set_variant(ctx, name)
        plan = mmc.mmc_plan(ctx)
        for x in insts:
            assert f"L{x[0]}:{DEFAULT_VARIANT[fp64][x[0]]}" in plan, plan
        mmc.mmc_batch_run(ctx)
        return [mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)]
    finally:
        mmc.mmc_destroy(ctx)


@pytest.mark.parametrize("fp64", [False, True], ids=["fp32", "fp64"])
def test_static_batch_equals_batch_run(fp64):
    import torch
    torch.cuda.set_device(0)
    for call, insts in enumerate(CALLS[fp64]):
        say(f"case static batch {'fp64' if fp64 else 'fp32'} call {call}: {len(insts)} instances, "
            f"{sum(x[3] for x in insts)} paths")
        got = static_run(insts, fp64)
        ref = batch_run(insts, fp64)
        for i, (g, r) in enumerate(zip(got, ref)):
            assert np.array_equal(g["n_accept"], r["n_accept"]), (call, i)
            for k in ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e", "final_m"):
                assert np.array_equal(g[k], r[k], equal_nan=True), (call, i, k)


def test_static_batch_rejects_what_it_cannot_hold():
    """Sizes beyond the static array, lattices that need device-memory spins and bad
    arguments are refused with a message, before any work is queued."""
    import torch
    from paper_1305_6758_amd import mmc
    out = torch.empty(80 * 16, dtype=torch.uint8, device="cuda")
    cases = [([(8, 1.0, 1.0, mmc.MMC_STATIC_MAX_PATHS + 1, 1, 1)], mmc.MMC_EINVAL, "paths"),
             ([(24, 1.0, 1.0, 4, 1, 1)], mmc.MMC_EUNSUPPORTED, "LDS"),
             ([(7, 1.0, 1.0, 4, 1, 1)], mmc.MMC_EINVAL, "even"),
             ([(8, 1.0, 1.0, 4, 1, 1)] * (mmc.MMC_STATIC_MAX_INSTANCES + 1), mmc.MMC_EINVAL, "instances")]
    for insts, code, word in cases:
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_batch_run_static(insts, 1, None, out.data_ptr(), 0)
        assert e.value.code == code and word in mmc.mmc_last_error(), mmc.mmc_last_error()
