"""Parity of the HIP engine (through the C ABI) with the FP64 CPU oracle, small sizes.

FP64 mode reproduces the oracle's trajectories: same Philox words, same operation order, no
contraction. The only differences are the last-bit rounding of sin/cos/exp between the GPU
math library and glibc, which never accumulate (accepted spins are fresh proposals), so
per-path results agree to 1e-12 absolute. FP32 mode is compared statistically (4 standard
errors) because FP32 trajectories leave the FP64 ones at the first flipped decision.
"""
import math

import numpy as np
import pytest

from helpers import (assert_results_close, engine_run, four_sigma, max_abs_diff, mean_se, oracle_run)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
PLACE_AUTO, PLACE_LDS, PLACE_HBM, PLACE_PLAIN = 0, 1, 2, 3


def say(*a):
    print(*a, flush=True)


# (placement, block, lanes) forced variants covering every FP64 kernel shape
FP64_SHAPES = [(PLACE_LDS, 256, 64), (PLACE_LDS, 256, 256), (PLACE_LDS, 512, 512), (PLACE_HBM, 512, 512),
               (PLACE_HBM, 1024, 1024), (PLACE_PLAIN, 0, 0)]


@pytest.mark.parametrize("L", [2, 4, 6, 8, 10, 12, 16])
def test_fp64_small_lattices_every_shape(L):
    """Every FP64 kernel shape the engine has for L (LDS or device-memory spins, 1..8 paths
    per workgroup, column or flat site maps, the plain engine) against the oracle: results,
    accept counts, per-sweep trace and final spins. 5 paths (ragged against paths per
    workgroup), 3 + 4 sweeps."""
    from paper_1305_6758_amd import mmc
    n_paths, nt, nm, T = 5, 3, 4, 1.3
    ora = oracle_run(L, T, n_paths, nt, nm, trace=nt + nm, want_spins=True)
    ran = 0
    for place, block, lanes in FP64_SHAPES:
        say(f"case L={L} place={place} block={block} lanes={lanes}")
        try:
            eng, tr, sp, plan, _ = engine_run(L, T, n_paths, nt, nm, placement=place, block=block, lanes=lanes,
                                              trace=nt + nm, spins_of=range(n_paths))
        except mmc.MMCError as e:
            assert e.code == mmc.MMC_EUNSUPPORTED, str(e)
            continue
        ran += 1
        assert_results_close(eng, ora, TOL64)
        assert max_abs_diff(tr, ora["trace"]) <= TOL64, plan
        for p in range(n_paths):
            assert max_abs_diff(sp[p], ora["spins"][p]) <= TOL64, (plan, p)
    assert ran >= 2


def test_fp64_trajectory_L8_full_length():
    """L = 8, T = 1.5, 64 paths, 1000 + 1000 sweeps, FP64, seed 1234: every per-path output
    within 1e-12 of the oracle; per-sweep energy and magnetisation of the first 100 sweeps
    within 1e-12; all spins after sweep 100 within 1e-12."""
    L, T, n, nt, nm = 8, 1.5, 64, 1000, 1000
    say("case L8 full FP64 trajectory")
    ora = oracle_run(L, T, n, nt, nm, trace=100)
    eng, tr, _, plan, _ = engine_run(L, T, n, nt, nm, trace=100)
    assert_results_close(eng, ora, TOL64)
    assert max_abs_diff(tr, ora["trace"]) <= TOL64
    # spins after 100 sweeps
    ora100 = oracle_run(L, T, n, 100, 0, want_spins=True)
    from paper_1305_6758_amd import mmc
    ctx = mmc.mmc_create_ex(L, T, 1.0, n, nt, nm, 1234, mmc.config(precision=mmc.MMC_FP64))
    try:
        mmc.mmc_run_sweeps(ctx, 100)
        for p in range(n):
            assert max_abs_diff(mmc.mmc_get_spins(ctx, p, L), ora100["spins"][p]) <= TOL64
    finally:
        mmc.mmc_destroy(ctx)


def test_fp64_plain_engine_L8():
    """The plain FP64 engine (one launch per half-sweep) reproduces the oracle too."""
    L, T, n, nt, nm = 8, 1.5, 16, 50, 50
    say("case plain L8")
    ora = oracle_run(L, T, n, nt, nm, trace=20)
    eng, tr, _, _, _ = engine_run(L, T, n, nt, nm, placement=PLACE_PLAIN, trace=20)
    assert_results_close(eng, ora, TOL64)
    assert max_abs_diff(tr, ora["trace"]) <= TOL64


@pytest.mark.parametrize("init", ["sphere", "angles", "ordered"])
def test_initial_states(init):
    """The three initial states of the paper's comparison of starts (random on the sphere,
    random angles, ordered along +z) match the oracle."""
    code = {"sphere": 0, "angles": 1, "ordered": 2}[init]
    say(f"case init={init}")
    ora = oracle_run(8, 1.0, 6, 2, 3, init=init, trace=5)
    eng, tr, _, _, _ = engine_run(8, 1.0, 6, 2, 3, init=code, trace=5)
    assert_results_close(eng, ora, TOL64)
    assert max_abs_diff(tr, ora["trace"]) <= TOL64


def test_edge_cases_fp64():
    """Negative J, infinite temperature (every move accepted), no measured sweeps (NaN means),
    a nonzero instance id and a 64-bit seed all match the oracle."""
    say("case J<0")
    ora = oracle_run(6, 0.9, 3, 4, 4, J=-1.0)
    eng, *_ = engine_run(6, 0.9, 3, 4, 4, J=-1.0)
    assert_results_close(eng, ora, TOL64)
    say("case T=inf")
    ora = oracle_run(8, math.inf, 3, 2, 3)
    eng, *_ = engine_run(8, math.inf, 3, 2, 3)
    assert_results_close(eng, ora, TOL64)
    assert np.all(eng["n_accept"] == 512 * 5)
    say("case n_meas=0")
    ora = oracle_run(8, 1.1, 3, 5, 0)
    eng, *_ = engine_run(8, 1.1, 3, 5, 0)
    assert np.all(np.isnan(eng["e_mean"]))
    assert_results_close(eng, ora, TOL64)
    say("case instance/seed")
    ora = oracle_run(8, 1.4, 3, 2, 2, seed=0xDEADBEEF12345, instance_id=77)
    eng, *_ = engine_run(8, 1.4, 3, 2, 2, seed=0xDEADBEEF12345, instance_id=77)
    assert_results_close(eng, ora, TOL64)


@pytest.mark.parametrize("L", [100, 128])
def test_large_lattices_fp64(L):
    """Sides beyond the workloads' (generic device-memory variant, L = 100 with 50-site rows of a
    colour and L = 128 with 2^21 sites): two paths, three sweeps, match the oracle to 1e-12."""
    say(f"case large lattice L={L}")
    ora = oracle_run(L, 1.3, 2, 2, 1, want_spins=True)
    eng, _, sp, plan, _ = engine_run(L, 1.3, 2, 2, 1, placement=PLACE_HBM, spins_of=(0, 1))
    say("plan", plan)
    assert_results_close(eng, ora, TOL64)
    for p in (0, 1):
        assert max_abs_diff(sp[p], ora["spins"][p]) <= TOL64


def test_fp32_statistics_L8():
    """FP32 engine against the FP64 oracle, L = 8, T = 1.5: <e> and <|m|> within 4 standard
    errors; |S| stays 1 to FP32 accuracy."""
    L, T, nt, nm = 8, 1.5, 300, 300
    say("case fp32 L8 stats")
    ora = oracle_run(L, T, 128, nt, nm)
    eng, _, sp, plan, _ = engine_run(L, T, 2048, nt, nm, fp64=False, spins_of=[0, 1])
    for key in ("e_mean", "absm_mean", "e2_mean", "m2_mean"):
        d, bound = four_sigma(eng, ora, key)
        assert d <= bound, f"{key}: |diff| {d:.3e} > 4 sigma {bound:.3e} ({plan})"
    for s in sp.values():
        assert np.max(np.abs(np.linalg.norm(s, axis=1) - 1.0)) < 2e-6


def test_fp32_kernel_shapes_agree_bitwise():
    """Every FP32 kernel shape for L = 16 (64 to 1024 lanes per path, LDS or device-memory
    spins) produces the same final spins and accept counts bit for bit: the update of a site
    does not depend on which lane does it. Energies agree to FP32 rounding of the sums."""
    from paper_1305_6758_amd import mmc
    L, T, n, nt, nm = 16, 1.443, 6, 10, 10
    ref = None
    for place, block, lanes in [(PLACE_LDS, 256, 256), (PLACE_LDS, 512, 512), (PLACE_LDS, 1024, 1024),
                                (PLACE_HBM, 512, 512)]:
        say(f"case fp32 L16 place={place} block={block} lanes={lanes}")
        try:
            eng, _, sp, plan, _ = engine_run(L, T, n, nt, nm, fp64=False, placement=place, block=block,
                                             lanes=lanes, spins_of=range(n))
        except mmc.MMCError as e:
            assert e.code == mmc.MMC_EUNSUPPORTED
            continue
        if ref is None:
            ref = (eng, sp)
            continue
        assert np.array_equal(eng["n_accept"], ref[0]["n_accept"]), plan
        for p in range(n):
            assert np.array_equal(sp[p], ref[1][p]), (plan, p)
        for k in ("e_mean", "absm_mean", "final_e"):
            assert max_abs_diff(eng[k], ref[0][k]) < 1e-5, (plan, k)


def test_compiled_side_variants_equal_generic_ones():
    """Variants compiled for one side (L = 10 single-instance; L = 20 batch, 512 lanes on the
    flat map and 1024 on the column map) and the generic any-L variants give the same spins
    and accept counts bit for bit (final energies equal to rounding: lane sums in another
    order)."""
    from paper_1305_6758_amd import mmc
    for name, generic in (("f32-lds-L10-g256-b256", "f32-lds-any-g256-b256"),):
        say(f"case {name} vs {generic}")
        a, _, sa, _, _ = engine_run(10, 1.1, 7, 6, 6, fp64=False, spins_of=range(7), variant=name)
        b, _, sb, _, _ = engine_run(10, 1.1, 7, 6, 6, fp64=False, spins_of=range(7), variant=generic)
        assert np.array_equal(a["n_accept"], b["n_accept"])
        for p in range(7):
            assert np.array_equal(sa[p], sb[p]), p
    say("case batch f32-lds-L20-g512 and f32-lds-L20-g1024 vs f32-lds-any-g512")
    got = []
    for v in ("f32-lds-any-g512", "f32-lds-L20-g512", "f32-lds-L20-g1024"):
        ctx = mmc.mmc_batch_create([(20, 1.44, 1.0, 5, 4, 3), (20, 1.45, 1.0, 3, 2, 5)], 1234,
                                   mmc.config(precision=mmc.MMC_FP32))
        try:
            mmc.mmc_set_variant(ctx, v)
            assert v in mmc.mmc_plan(ctx)
            mmc.mmc_batch_run(ctx)
            got.append([mmc.mmc_batch_results(ctx, i, n) for i, n in enumerate((5, 3))])
        finally:
            mmc.mmc_destroy(ctx)
    for g in got[1:]:
        for i in range(2):
            assert np.array_equal(got[0][i]["n_accept"], g[i]["n_accept"])
            assert max_abs_diff(got[0][i]["final_e"], g[i]["final_e"]) < 1e-5


def test_resume_and_checkpoint_bit_identical(tmp_path):
    """Counter-based random numbers: 7 sweeps + save + load + the rest equals one
    uninterrupted run bit for bit (FP32 and FP64)."""
    from paper_1305_6758_amd import mmc
    for fp64 in (True, False):
        say(f"case resume fp64={fp64}")
        L, T, n, nt, nm = 8, 1.2, 4, 6, 9
        full, _, sp_full, _, _ = engine_run(L, T, n, nt, nm, fp64=fp64, spins_of=range(n))
        cfg = mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32)
        ctx = mmc.mmc_create_ex(L, T, 1.0, n, nt, nm, 1234, cfg)
        f = str(tmp_path / f"ck{int(fp64)}.bin")
        try:
            mmc.mmc_run_sweeps(ctx, 7)
            mmc.mmc_save(ctx, f)
        finally:
            mmc.mmc_destroy(ctx)
        ctx = mmc.mmc_load(f)
        try:
            assert mmc.mmc_sweeps_done(ctx) == 7
            mmc.mmc_run(ctx)
            res = mmc.mmc_results(ctx, n)
            for k in ("e_mean", "e2_mean", "absm_mean", "m4_mean", "final_e"):
                assert np.array_equal(res[k], full[k]), k
            assert np.array_equal(res["n_accept"], full["n_accept"])
            for p in range(n):
                assert np.array_equal(mmc.mmc_get_spins(ctx, p, L), sp_full[p])
        finally:
            mmc.mmc_destroy(ctx)


def test_torch_workspace_binding():
    """Device memory and stream from torch (mmc_bind) give the same results as the
    library's own allocation."""
    say("case torch workspace")
    a, *_ = engine_run(8, 1.5, 9, 5, 5, torch_ws=True)
    b, *_ = engine_run(8, 1.5, 9, 5, 5)
    for k in ("e_mean", "final_e"):
        assert np.array_equal(a[k], b[k])


def test_batch_fp64_matches_oracle():
    """An uneven FP64 batch (L from 4 to 24, different T, path counts and sweep counts) in one
    persistent launch: every path matches the oracle run with instance id = batch index."""
    from paper_1305_6758_amd import mmc
    insts = [(8, 1.5, 1.0, 5, 3, 4), (12, 1.2, 1.0, 3, 2, 3), (10, 2.0, 1.0, 2, 4, 1),
             (16, 1.443, 1.0, 2, 2, 2), (24, 1.1, 1.0, 1, 1, 2), (4, math.inf, 1.0, 3, 1, 1),
             (6, 0.7, -1.0, 2, 2, 2)]
    say("case batch fp64")
    ctx = mmc.mmc_batch_create(insts, 1234, mmc.config(precision=mmc.MMC_FP64))
    try:
        mmc.mmc_batch_run(ctx)
        say("plan", mmc.mmc_plan(ctx))
        for i, (L, T, J, n, nt, nm) in enumerate(insts):
            eng = mmc.mmc_batch_results(ctx, i, n)
            ora = oracle_run(L, T, n, nt, nm, J=J, instance_id=i)
            assert_results_close(eng, ora, TOL64)
    finally:
        mmc.mmc_destroy(ctx)


def test_batch_fp32_equals_single_instance_runs():
    """The persistent batch kernel and the single-instance kernels with the same site map give
    bit-identical FP32 results (L = 8: 64 lanes per path; L = 16: 512 lanes per path)."""
    from paper_1305_6758_amd import mmc
    insts = [(8, 1.5, 1.0, 11, 5, 5), (16, 1.443, 1.0, 3, 4, 4)]
    say("case batch fp32 vs single")
    ctx = mmc.mmc_batch_create(insts, 1234, mmc.config(precision=mmc.MMC_FP32))
    try:
        for name in ("f32-lds-L8-g64", "f32-lds-L16-g512"):
            mmc.mmc_set_variant(ctx, name)
        mmc.mmc_batch_run(ctx)
        got = [mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)]
    finally:
        mmc.mmc_destroy(ctx)
    shapes = [(PLACE_LDS, 256, 64), (PLACE_LDS, 512, 512)]
    for i, ((L, T, J, n, nt, nm), (pl, b, g)) in enumerate(zip(insts, shapes)):
        one, *_ = engine_run(L, T, n, nt, nm, fp64=False, placement=pl, block=b, lanes=g, instance_id=i)
        for k in ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e", "n_accept"):
            assert np.array_equal(got[i][k], one[k]), (L, k)


def test_batch_autotuner_and_pinned_variants():
    """The batch autotuner times the batch variants that fit each L at creation; whatever it
    picks, and with every instance pinned to the generic device-memory variant instead, FP64
    paths match the oracle and spins and accept counts agree between the two plans."""
    from paper_1305_6758_amd import mmc
    insts = [(8, 1.4, 1.0, 6, 2, 3), (16, 1.2, 1.0, 3, 2, 2), (6, 2.0, -1.0, 4, 3, 1), (12, 1.0, 1.0, 2, 1, 3)]
    plans, res = [], []
    for pin in (None, "f64-hbm-any-g512"):
        say(f"case batch autotuner, pin {pin}")
        ctx = mmc.mmc_batch_create(insts, 77, mmc.config(precision=mmc.MMC_FP64))
        try:
            if pin:
                mmc.mmc_set_variant(ctx, pin)
            plans.append(mmc.mmc_plan(ctx))
            mmc.mmc_batch_run(ctx)
            res.append([mmc.mmc_batch_results(ctx, i, x[3]) for i, x in enumerate(insts)])
            with pytest.raises(mmc.MMCError):
                mmc.mmc_set_variant(ctx, "f64-hbm-any-g512")  # after the first run
        finally:
            mmc.mmc_destroy(ctx)
        say("plan", plans[-1])
    assert plans[1].split(";", 1)[1].count("f64-hbm-any-g512") == len(insts), plans[1]
    for i, (L, T, J, n, nt, nm) in enumerate(insts):
        ora = oracle_run(L, T, n, nt, nm, J=J, seed=77, instance_id=i)
        assert_results_close(res[0][i], ora, TOL64)
        assert_results_close(res[1][i], ora, TOL64)
        assert np.array_equal(res[0][i]["n_accept"], res[1][i]["n_accept"])
    ctx = mmc.mmc_batch_create(insts, 77, mmc.config(precision=mmc.MMC_FP64))
    try:
        with pytest.raises(mmc.MMCError):
            mmc.mmc_set_variant(ctx, "f64-lds-L8-g128-no-such")
        with pytest.raises(mmc.MMCError):
            mmc.mmc_set_variant(ctx, "f32-lds-L16-g512")  # an FP32 variant in an FP64 batch
    finally:
        mmc.mmc_destroy(ctx)


def test_invalid_arguments_rejected():
    from paper_1305_6758_amd import mmc
    for args in [(7, 1.0, 1.0, 4, 1, 1, 1), (8, 0.0, 1.0, 4, 1, 1, 1), (8, -1.0, 1.0, 4, 1, 1, 1),
                 (8, float("nan"), 1.0, 4, 1, 1, 1), (8, 1.0, float("inf"), 4, 1, 1, 1), (8, 1.0, 1.0, 0, 1, 1, 1),
                 (8, 1.0, 1.0, 4, -1, 1, 1), (0, 1.0, 1.0, 4, 1, 1, 1)]:
        with pytest.raises(mmc.MMCError) as e:
            mmc.mmc_create(*args)
        assert e.value.code == mmc.MMC_EINVAL
    with pytest.raises(mmc.MMCError):
        mmc.mmc_create_ex(8, 1.0, 1.0, 4, 1, 1, 1, mmc.config(precision=0, placement=PLACE_PLAIN))


def test_mixed_start_every_engine():
    """The mixed start of Sec. 3 (even paths random, odd paths ordered) on the LDS, device-memory
    and plain FP64 engines and in a batch: trajectories and traces match the oracle."""
    from paper_1305_6758_amd import mmc
    ora = oracle_run(6, 1.1, 8, 3, 4, init="mixed", trace=7)
    for place in (mmc.MMC_PLACE_LDS, mmc.MMC_PLACE_HBM, mmc.MMC_PLACE_PLAIN):
        say(f"case mixed start, placement {place}")
        eng, tr, _, plan, _ = engine_run(6, 1.1, 8, 3, 4, init=mmc.MMC_INIT_MIXED, trace=7, placement=place)
        assert_results_close(eng, ora, TOL64)
        assert max_abs_diff(tr, ora["trace"]) <= TOL64
    say("case mixed start, batch")
    ctx = mmc.mmc_batch_create([(6, 1.1, 1.0, 8, 3, 4)], 1234, mmc.config(precision=mmc.MMC_FP64, init=mmc.MMC_INIT_MIXED))
    try:
        mmc.mmc_batch_run(ctx)
        assert_results_close(mmc.mmc_batch_results(ctx, 0, 8), ora, TOL64)
    finally:
        mmc.mmc_destroy(ctx)


def test_angle_proposal_plain_engine():
    """Moves with both angles uniform (plain FP64 engine) match the oracle's angle proposal;
    other engines refuse the proposal."""
    from paper_1305_6758_amd import mmc
    say("case angle proposal, plain engine")
    for init in ("sphere", "angles"):
        ora = oracle_run(6, 0.8, 5, 4, 6, init=init, trace=10, proposal="angles", instance_id=3)
        eng, tr, _, plan, _ = engine_run(6, 0.8, 5, 4, 6, init={"sphere": 0, "angles": 1}[init], trace=10,
                                         placement=mmc.MMC_PLACE_PLAIN, proposal=mmc.MMC_PROPOSAL_ANGLES, instance_id=3)
        assert_results_close(eng, ora, TOL64)
        assert max_abs_diff(tr, ora["trace"]) <= TOL64
    with pytest.raises(mmc.MMCError) as e:
        mmc.mmc_create_ex(6, 1.0, 1.0, 2, 1, 1, 1, mmc.config(precision=mmc.MMC_FP64, proposal=mmc.MMC_PROPOSAL_ANGLES))
    assert e.value.code == mmc.MMC_EUNSUPPORTED


def test_thermalisation_and_table_drivers_fp64():
    """The thermalisation (traced mixed start) and Table-1 drivers on the FP64 engine: per-sweep
    <m>, cv and <e> of each half, and the distribution coefficients of the final states, equal
    the oracle's statistics of the oracle's paths."""
    from oracle import stats as S
    from paper_1305_6758_amd.experiments import distribution_table, thermalisation
    say("case thermalisation driver")
    out = thermalisation(L=6, T=1.0, n_paths=40, sweeps=24, init="mixed", fp64=True, instance_id=5)
    ora = oracle_run(6, 1.0, 40, 24, 0, init="mixed", trace=24, instance_id=5)
    for name, (b, st) in (("all", (0, 1)), ("random_half", (0, 2)), ("ordered_half", (1, 2))):
        ref = S.trace_statistics(ora["trace"], b, st)
        for row in out[name]:
            k = row["sweeps"] - 1
            got = [row["m"], row["se_m"], row["cv_m"], row["e"], row["se_e"]]
            assert np.max(np.abs(np.array(got) - ref[k])) < 1e-10, (name, k)
    say("case distribution table driver, both proposals")
    for prop in ("sphere", "angles"):
        tab = distribution_table(L=4, Ts=(0.9, 1.5), n_paths=48, sweeps=20, proposal=prop, fp64=True)
        for i, row in enumerate(tab["rows"]):
            o = oracle_run(4, row["T"], 48, 19, 1, instance_id=i, proposal=prop)
            fm = o["final_m"]
            for key, x in (("r_H", o["final_e"]), ("r_Mx", fm[:, 0]), ("r_My", fm[:, 1]), ("r_Mz", fm[:, 2]),
                           ("r_absMz", np.abs(fm[:, 2]))):
                assert abs(row[key] - S.distribution_coefficient(x)) < 1e-9, (prop, i, key)


def test_spin_norm_diagnostic_and_renormalisation(tmp_path):
    """Failure detection: a spin whose length is corrupted in a checkpoint is flagged by
    mmc_spin_norm_deviation after loading; FP32 renormalisation at the next boundary repairs
    it; an untouched run stays within FP32 rounding of unit length."""
    import ctypes
    from paper_1305_6758_amd import mmc
    L, n = 8, 2
    cfg = mmc.config(precision=mmc.MMC_FP32, renorm_every=4)
    ctx = mmc.mmc_create_ex(L, 1.2, 1.0, n, 3, 10, 1234, cfg)
    f = tmp_path / "ck.bin"
    try:
        mmc.mmc_run_sweeps(ctx, 3)
        assert mmc.mmc_spin_norm_deviation(ctx) < 1e-6
        mmc.mmc_save(ctx, str(f))
    finally:
        mmc.mmc_destroy(ctx)
    raw = bytearray(f.read_bytes())
    head = 8 + 4 + 8 + 8 + 4 + 4 + 4 + 8 + ctypes.sizeof(mmc.mmc_config) + 4 + 64 + 8
    x = np.frombuffer(bytes(raw[head:head + 4]), dtype=np.float32)[0]
    raw[head:head + 4] = np.float32(3.0 * x + 0.5).tobytes()  # site 0 of path 0, x component
    f.write_bytes(bytes(raw))
    ctx = mmc.mmc_load(str(f))
    try:
        say("case corrupted spin")
        assert mmc.mmc_spin_norm_deviation(ctx) > 0.1
        mmc.mmc_run_sweeps(ctx, 2)  # sweeps 3 and 4: renormalisation at the start of sweep 4
        assert mmc.mmc_spin_norm_deviation(ctx) < 1e-6
    finally:
        mmc.mmc_destroy(ctx)
