"""Shared helpers of the tests: run the engine through the C ABI binding, compare with the oracle."""
import math

import numpy as np

RESULT_KEYS = ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e")


def engine_run(L, T, n_paths, n_therm, n_meas, *, J=1.0, seed=1234, fp64=True, placement=0, block=0,
               lanes=0, init=0, trace=0, instance_id=0, renorm_every=0, spins_of=(), torch_ws=False, proposal=0,
               model=0, variant=None):
    """Runs one instance on the GPU engine; returns (results dict, trace or None, {path: spins},
    plan string, ms)."""
    from paper_1305_6758_amd import mmc
    cfg = mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32, init=init, placement=placement,
                     block=block, lanes_per_path=lanes, renorm_every=renorm_every, instance_id=instance_id,
                     trace_sweeps=trace, proposal=proposal, model=model)
    ctx = mmc.mmc_create_ex(L, T, J, n_paths, n_therm, n_meas, seed, cfg)
    ws = None
    try:
        if torch_ws:
            ws = mmc.Workspace(ctx)
        if variant is not None:
            mmc.mmc_set_variant(ctx, variant)
        mmc.mmc_run(ctx)
        res = mmc.mmc_results(ctx, n_paths)
        tr = mmc.mmc_trace(ctx, n_paths, trace) if trace else None
        spins = {p: mmc.mmc_get_spins(ctx, p, L, 2 if model == 1 else 3) for p in spins_of}
        plan = mmc.mmc_plan(ctx)
        ms = mmc.mmc_last_timing_ms(ctx)
        if ws is not None:
            ws.stream.synchronize()
    finally:
        mmc.mmc_destroy(ctx)
    return res, tr, spins, plan, ms


def oracle_run(L, T, n_paths, n_therm, n_meas, *, J=1.0, seed=1234, init="sphere", trace=0, instance_id=0,
               path_begin=0, want_spins=False, threads=0, proposal="sphere"):
    from oracle import oracle as O
    return O.run_paths(L, T, J=J, n_therm=n_therm, n_meas=n_meas, seed=seed, path_begin=path_begin,
                       path_end=path_begin + n_paths, instance=instance_id, init=init,
                       trace_sweeps=trace, want_spins=want_spins, n_threads=threads, proposal=proposal)


def max_abs_diff(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    both_nan = np.isnan(a) & np.isnan(b)
    d = np.abs(a - b)
    d[both_nan] = 0.0
    return float(np.nanmax(np.where(np.isnan(d), np.inf, d))) if d.size else 0.0


def assert_results_close(eng, ora, tol, n=None, accept_exact=True):
    """Per-path results of engine and oracle agree elementwise within tol (absolute)."""
    sl = slice(0, n)
    for k in RESULT_KEYS:
        d = max_abs_diff(eng[k][sl], ora[k][sl])
        assert d <= tol, f"{k}: max |diff| = {d:.3e} > {tol:.1e}"
    d = max_abs_diff(eng["final_m"][sl], ora["final_m"][sl])
    assert d <= tol, f"final_m: max |diff| = {d:.3e}"
    if accept_exact:
        assert np.array_equal(eng["n_accept"][sl], ora["n_accept"][sl]), "accept counts differ"


def mean_se(x):
    x = np.asarray(x, dtype=np.float64)
    return float(x.mean()), float(x.std(ddof=1) / math.sqrt(x.size))


def four_sigma(a, b, key):
    """|mean_a - mean_b| <= 4 sqrt(SE_a^2 + SE_b^2); returns (diff, bound)."""
    ma, sa = mean_se(a[key])
    mb, sb = mean_se(b[key])
    return abs(ma - mb), 4.0 * math.hypot(sa, sb)
