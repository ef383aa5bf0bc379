"""Checkpoint and resume on the engines beyond the default ones (2-D Ising, LDS and
device-memory windows, the split placement, the two-sweep ring): a run of a few sweeps, saved
to a file, loaded into a new context and finished equals an uninterrupted run with the same
kernel variant (the checkpoint records the variant's name). Spins and accept counts are
exact everywhere; per-path sums are exact where the reduction order does not depend on where
a run is split (the 2-D Ising model's integer sums; the split placement's per-sweep sums),
else equal to rounding (the window kernels and the rings sum a pass's partials in an order set
by the pass length)."""
import numpy as np
import pytest

from helpers import engine_run, max_abs_diff

pytestmark = pytest.mark.gpu

KEYS = ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e")


def say(*a):
    print(*a, flush=True)


CASES = [
    # (name, L, T, n_paths, n_therm, n_meas, precision, model, variant, renorm, split, sum tolerance)
    ("ising", 20, 2.3, 6, 4, 7, "fp32", 1, None, 0, 5, 0.0),
    ("window-fp32", 24, 1.2, 3, 5, 6, "fp32", 0, "f32-win-L24-d2-b512", 5, 7, 1e-5),
    ("gwindow-fp64", 16, 1.3, 3, 4, 5, "fp64", 0, "f64-gwin-L16-d2-b256", 0, 3, 1e-14),
    ("split-fp32", 24, 1.2, 2, 5, 6, "fp32", 0, "f32-split-L24-g1024-b1024", 5, 7, 0.0),
    ("split-fp64", 10, 1.3, 3, 4, 5, "fp64", 0, "f64-split-any-g512-b512", 0, 3, 0.0),
    ("splitxy-fp32", 32, 1.4, 2, 3, 4, "fp32", 0, "f32-splitxy-L32-g1024-b1024", 3, 4, 0.0),
    # the two-sweep ring, resumed at an odd sweep (its passes pair other sweeps than the
    # uninterrupted run's)
    ("ring2-fp32", 32, 1.4, 2, 4, 5, "fp32", 0, "f32-ring2-L32-b512", 4, 3, 1e-5),
    ("ring2-fp64", 16, 1.3, 3, 4, 5, "fp64", 0, "f64-ring2-L16-b128", 0, 5, 1e-14),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_checkpoint_resume(case, tmp_path):
    from paper_1305_6758_amd import mmc
    name, L, T, n, nt, nm, prec, model, variant, renorm, split, tol = case
    dim = 2 if model == 1 else 3
    say(f"case checkpoint {name}")
    full, _, sp_full, plan_full, _ = engine_run(L, T, n, nt, nm, fp64=prec == "fp64", model=model,
                                                renorm_every=renorm, spins_of=range(n), variant=variant)
    cfg = mmc.config(precision=mmc.MMC_FP64 if prec == "fp64" else mmc.MMC_FP32, model=model, renorm_every=renorm)
    ctx = mmc.mmc_create_ex(L, T, 1.0, n, nt, nm, 1234, cfg)
    f = str(tmp_path / f"{name}.ck")
    try:
        if variant:
            mmc.mmc_set_variant(ctx, variant)
        mmc.mmc_run_sweeps(ctx, split)
        mmc.mmc_save(ctx, f)
    finally:
        mmc.mmc_destroy(ctx)
    ctx = mmc.mmc_load(f)
    try:
        assert mmc.mmc_sweeps_done(ctx) == split
        mmc.mmc_run(ctx)
        assert mmc.mmc_plan(ctx).split()[0] == plan_full.split()[0]
        res = mmc.mmc_results(ctx, n)
        assert np.array_equal(res["n_accept"], full["n_accept"])
        for p in range(n):
            assert np.array_equal(mmc.mmc_get_spins(ctx, p, L, dim), sp_full[p]), p
        for k in KEYS:
            if tol == 0.0:
                assert np.array_equal(res[k], full[k]), k
            else:
                assert max_abs_diff(res[k], full[k]) <= tol, k
    finally:
        mmc.mmc_destroy(ctx)
