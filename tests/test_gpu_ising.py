"""Parity of the 2-D Ising engine (appendix model) with the oracle: integer spins and integer
decisions, so every path's spins and accept counts are bit-exact and the FP64 accumulators
and traces equal the oracle's (same integer sums, same floating-point operations)."""
import math

import numpy as np
import pytest

from helpers import engine_run
from oracle import oracle as O

pytestmark = pytest.mark.gpu

ISING = 1


def say(*a):
    print(*a, flush=True)


def ising_oracle(L, T, n, nt, nm, J=1.0, init="sphere", trace=0, instance=0, seed=1234, path_begin=0):
    return O.ising_run_paths(L, T, J=J, n_therm=nt, n_meas=nm, seed=seed, path_begin=path_begin,
                             path_end=path_begin + n, instance=instance, init=init, trace_sweeps=trace,
                             want_spins=True)


def assert_exact(eng, ora, sp, n, L):
    for k in ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e"):
        a, b = np.asarray(eng[k]), np.asarray(ora[k])
        assert np.array_equal(np.isnan(a), np.isnan(b)), k
        assert np.max(np.abs(np.nan_to_num(a) - np.nan_to_num(b)), initial=0.0) <= 1e-15, k
    assert np.array_equal(eng["n_accept"], ora["n_accept"])
    assert np.max(np.abs(eng["final_m"] - ora["final_m"])) <= 1e-15
    for p in range(n):
        assert np.array_equal(sp[p][:, 2].astype(np.int8), ora["spins"][p]), p
        assert np.all(sp[p][:, :2] == 0.0)


@pytest.mark.parametrize("L", [4, 6, 10, 20, 50])
def test_ising_trajectories_bit_exact(L):
    """Several lattice sizes (full and partial last quads per row), both signs of J, every
    start, a traced run, a nonzero instance id and a path count that leaves waves idle."""
    cases = [(1.6, 1.0, "sphere", 0, 6), (2.3, 1.0, "ordered", 3, 5), (3.0, -1.0, "mixed", 1, 7), (math.inf, 1.0, "sphere", 2, 3)]
    for T, J, init, inst, n in cases:
        nt, nm = 4, 5
        say(f"case ising L={L} T={T} J={J} init={init} instance={inst} paths={n}")
        ora = ising_oracle(L, T, n, nt, nm, J=J, init=init, trace=nt + nm, instance=inst)
        code = {"sphere": 0, "ordered": 2, "mixed": 3}[init]
        eng, tr, sp, plan, _ = engine_run(L, T, n, nt, nm, J=J, init=code, trace=nt + nm, instance_id=inst,
                                          spins_of=range(n), model=ISING)
        assert plan.startswith("ising2d-"), plan
        assert_exact(eng, ora, sp, n, L)
        assert np.max(np.abs(tr - ora["trace"])) <= 1e-15
        if T == math.inf:
            assert np.all(eng["n_accept"] == L * L * (nt + nm))


def test_ising_resume_and_stats():
    """Sweeps run in chunks equal one uninterrupted run; the host statistics use N = L^2."""
    from paper_1305_6758_amd import mmc
    L, T, n, nt, nm = 20, 2.2, 9, 6, 10
    say("case ising resume")
    ora = ising_oracle(L, T, n, nt, nm)
    ctx = mmc.mmc_create_ex(L, T, 1.0, n, nt, nm, 1234, mmc.config(model=ISING))
    try:
        for k in (1, 4, 2):
            mmc.mmc_run_sweeps(ctx, k)
        mmc.mmc_run(ctx)
        res = mmc.mmc_results(ctx, n)
        sp = {p: mmc.mmc_get_spins(ctx, p, L, 2) for p in range(n)}
        assert_exact(res, ora, sp, n, L)
        st = mmc.mmc_stats(ctx)
        N = L * L
        chi = N / T * (np.mean(ora["m2_mean"]) - np.mean(ora["absm_mean"]) ** 2)
        assert abs(st["chi"] - chi) <= 1e-12 * max(1.0, abs(chi))
        assert abs(st["accept_rate"] - np.sum(ora["n_accept"]) / (n * N * (nt + nm))) < 1e-15
    finally:
        mmc.mmc_destroy(ctx)


def test_ising_rejects_unsupported_configurations():
    from paper_1305_6758_amd import mmc
    for cfg in (mmc.config(model=ISING, placement=mmc.MMC_PLACE_HBM),):
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_create_ex(10, 2.0, 1.0, 4, 1, 1, 1, cfg)
        assert e.value.code == mmc.MMC_EUNSUPPORTED
    for cfg in (mmc.config(model=ISING, init=mmc.MMC_INIT_ANGLES), mmc.config(model=2)):
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_create_ex(10, 2.0, 1.0, 4, 1, 1, 1, cfg)
        assert e.value.code == mmc.MMC_EINVAL
    with pytest.raises(mmc.MMCError) as e:
        mmc.mmc_batch_create([(10, 2.0, 1.0, 4, 1, 1)], 1, mmc.config(model=ISING))
    assert e.value.code == mmc.MMC_EUNSUPPORTED


def test_ising_experiment_drivers_match_oracle():
    """The appendix drivers (order parameter per (L, T), cumulant crossing, traced
    thermalisation) on small lattices equal the oracle's statistics of the oracle's paths."""
    from oracle import stats as S
    from paper_1305_6758_amd import experiments as X
    say("case ising magnetisation driver")
    out = X.ising_magnetisation(Ls=(4, 6), Ts=(2.0, 3.0), n_paths=32, sweeps=20)
    for i, row in enumerate(out["rows"]):
        o = ising_oracle(row["L"], row["T"], 32, 19, 1, instance=i)
        am = np.abs(o["final_m"][:, 0])
        assert abs(row["m"] - am.mean()) < 1e-15 and abs(row["se"] - am.std(ddof=1) / math.sqrt(32)) < 1e-15
    say("case ising binder driver")
    out = X.ising_binder(Ls=(6, 4), Ts=(2.2, 2.4), n_paths=40, sweeps=15)
    us, ses = [], []
    for i, c in enumerate(out["cumulants"]):
        o = ising_oracle(c["L"], c["T"], 40, 14, 1, instance=i)
        U, se = S.binder_cumulant(o["m2_mean"], o["m4_mean"])
        assert abs(c["U"] - U) < 1e-13 and abs(c["se"] - se) < 1e-13
        us.append(U)
        ses.append(se)
    Tc, sTc, *_ = S.cumulant_crossing(2.2, 2.4, us, ses)
    assert abs(out["tc"] - Tc) < 1e-12 and abs(out["se_tc"] - sTc) < 1e-12
    say("case ising thermalisation driver")
    out = X.thermalisation(L=8, T=2.5, n_paths=24, sweeps=16, init="mixed", model=ISING, instance_id=2)
    o = ising_oracle(8, 2.5, 24, 16, 0, init="mixed", trace=16, instance=2)
    for name, (b, st) in (("all", (0, 1)), ("random_half", (0, 2)), ("ordered_half", (1, 2))):
        ref = S.trace_statistics(o["trace"], b, st)
        for row in out[name]:
            k = row["sweeps"] - 1
            got = np.array([row["m"], row["se_m"], row["cv_m"], row["e"], row["se_e"]])
            assert np.max(np.abs(got - ref[k])) < 1e-12, (name, k)
