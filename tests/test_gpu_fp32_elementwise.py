"""Element-by-element parity of the FP32 engine with the FP64 oracle run on the FP32 engine's
uniform grid (the oracle's uniforms="fp32" option: the same Philox words and the same
uniforms ((w >> 8) | 1) 2^-24, FP64 arithmetic).

Tolerances (FP32 unit roundoff u = 2^-24):
  - proposal step: z = 2 u0 - 1 is exact in FP32 (an integer over 2^23), so the z components
    agree bit for bit; x and y carry the rounding of 1 - z^2 (one fma, u/2 relative), the
    hardware square root, the hardware sine and cosine of the angle in revolutions and the
    rounding of the product (u/2). TOL_PROP = 8 u bounds their combined absolute error:
    test_proposal_step_exhaustive checks it over every one of the 2^23 FP32 uniforms for u0
    and for u1 (one MI355X measured 3.2 u at most, a margin of 2.5).
  - at T = inf every move is accepted, so after sweep k every spin is its sweep-(k-1)
    proposal: the spins agree within TOL_PROP (z bit for bit) and the accept counts exactly.
  - per-path sums in FP32: a lane adds up its n_lane sites' terms in turn, then a tree of at
    most 16 levels combines the lanes; each addition's rounding is at most u times the sum
    of the magnitudes, so |d m_a| <= (n_lane + 16) u + TOL_PROP with |S_a| <= 1 and
    |d e| <= 6 (n_lane + 16) u + 40 TOL_PROP with |S . h| <= 6 per site.
"""
import math
import re

import numpy as np
import pytest

U32 = 2.0 ** -24
TOL_PROP = 8 * U32  # absolute error bound of an FP32 proposal's x and y components

# FP32 single-instance variants by lattice side (every compiled FP32 kernel form: LDS,
# colour split, x/y split, device memory, LDS window, device-memory window, plane rings of
# one and two sweeps per pass, half ring, generic maps)
SINGLE_VARIANTS = [
    (8, "f32-lds-L8-g64-b256"), (8, "f32-lds-L8-g128-b256"), (8, "f32-lds-L8-g256-b256"),
    (10, "f32-lds-L10-g256-b256"), (12, "f32-lds-L12-g128-b256"), (12, "f32-lds-L12-g256-b256"),
    (16, "f32-lds-L16-g256-b256"), (16, "f32-lds-L16-g512-b512"), (16, "f32-lds-L16-g1024-b1024"),
    (6, "f32-lds-any-g256-b256"),
    (24, "f32-split-L24-g1024-b1024"), (30, "f32-split-L30-g1024-b1024"), (22, "f32-split-any-g512-b512"),
    (32, "f32-splitxy-L32-g1024-b1024"), (34, "f32-splitxy-any-g512-b512"),
    (24, "f32-hbm-L24-g512-b512"), (32, "f32-hbm-L32-g512-b512"), (32, "f32-hbm-L32-g1024-b1024"),
    (48, "f32-hbm-L48-g512-b512"), (64, "f32-hbm-L64-g1024-b1024"), (14, "f32-hbm-any-g512-b512"),
    (24, "f32-win-L24-d2-b512"), (24, "f32-win-L24-d3-b1024"), (30, "f32-win-L30-d2-b1024"),
    (32, "f32-win-L32-d2-b1024"), (32, "f32-gwin-L32-d2-b1024"), (48, "f32-gwin-L48-d1-b1024"),
    (16, "f32-ring-L16-b256"), (32, "f32-ring-L32-b512"), (48, "f32-ring-L48-b1024"), (48, "f32-ring-L48-b768"),
    (16, "f32-hring-L16-b256"), (48, "f32-hring-L48-b1024"), (64, "f32-hring-L64-b1024"), (64, "f32-hring-L64-b768"),
    (16, "f32-ring2-L16-b128"), (32, "f32-ring2-L32-b512"), (48, "f32-ring2-L48-b768"), (48, "f32-ring2-L48-b1024"),
]

# the batch variants the uneven batch of lattice sides 8 ... 48 runs on
BATCH_VARIANTS = {8: "f32-lds-L8-g64", 12: "f32-lds-L12-g256", 16: "f32-lds-L16-g512",
                  24: "f32-split-L24-g1024", 32: "f32-splitxy-L32-g1024", 48: "f32-hbm-L48-g512"}
BATCH_SETS = [BATCH_VARIANTS, {**BATCH_VARIANTS, 48: "f32-ring-L48-g1024"}, {**BATCH_VARIANTS, 48: "f32-ring-L48-g768"},
              {**BATCH_VARIANTS, 32: "f32-ring2-L32-g512", 48: "f32-ring2-L48-g1024"}]


def lanes_of(name):
    """Lanes that share one path in a variant (g<lanes>, or the whole block of a window)."""
    m = re.search(r"-g(\d+)", name) or re.search(r"-b(\d+)", name)
    return int(m.group(1))


def sum_tolerances(L, lanes):
    n_lane = L ** 3 / lanes + 16
    return n_lane * U32 + TOL_PROP, 6.0 * n_lane * U32 + 40.0 * TOL_PROP


def oracle32(L, T, n_paths, sweeps, instance=0, path_begin=0):
    from oracle import oracle as O
    return O.run_paths(L, T, n_therm=sweeps, n_meas=0, seed=1234, path_begin=path_begin,
                       path_end=path_begin + n_paths, instance=instance, want_spins=True, uniforms="fp32")


def check_spins(g, o, what):
    """g, o: [N, 3] spins of one path (site-id order)."""
    assert np.array_equal(g[:, 2], o[:, 2]), f"{what}: z components differ (max {np.max(np.abs(g[:, 2] - o[:, 2])):.3e})"
    d = float(np.max(np.abs(g[:, :2] - o[:, :2])))
    assert d <= TOL_PROP, f"{what}: max |dx|, |dy| = {d:.3e} > {TOL_PROP:.3e}"
    return d


@pytest.mark.gpu
def test_proposal_step_exhaustive():
    """Every FP32 uniform (2^23 values) as u0 and as u1: the engine's FP32 proposal against the
    oracle's unit vector on the same grid -- z bit for bit, x and y within TOL_PROP; and the
    FP64 proposal against the oracle's FP64 unit vector on a million random word pairs within
    4 ulp (the GPU's and the host's library sine and cosine may differ in the last bit)."""
    from oracle import oracle as O
    from paper_1305_6758_amd import mmc
    k = np.arange(1 << 23, dtype=np.uint64)
    w = np.empty((k.size, 2), dtype=np.uint32)
    w[:, 0] = (k << np.uint64(9)).astype(np.uint32)  # ((w >> 8) | 1) = 2k + 1: every odd numerator
    w[:, 1] = (((k * np.uint64(0x2F0B1D)) & np.uint64((1 << 23) - 1)) << np.uint64(9)).astype(np.uint32)
    g = mmc.mmc_proposal_vectors(mmc.MMC_FP32, mmc.MMC_PROPOSAL_SPHERE, w)
    o = O.unit_vectors(w, uniforms="fp32")
    d = check_spins(g, o, "FP32 proposals")
    dn = float(np.max(np.abs(np.sqrt((g * g).sum(axis=1)) - 1.0)))
    print(f"\nFP32 proposal: max |dx|,|dy| = {d:.3e} ({d / U32:.1f} u), max ||S| - 1| = {dn:.3e}", flush=True)
    assert dn <= 2 * TOL_PROP
    rng = np.random.default_rng(11)
    w64 = rng.integers(0, 2 ** 32, size=(1 << 20, 2), dtype=np.uint64).astype(np.uint32)
    g64 = mmc.mmc_proposal_vectors(mmc.MMC_FP64, mmc.MMC_PROPOSAL_SPHERE, w64)
    o64 = O.unit_vectors(w64)
    d64 = float(np.max(np.abs(g64 - o64)))
    print(f"FP64 proposal: max |d| = {d64:.3e}", flush=True)
    assert d64 <= 4 * 2.0 ** -53


@pytest.mark.gpu
@pytest.mark.parametrize("L,variant", SINGLE_VARIANTS, ids=[v for _, v in SINGLE_VARIANTS])
def test_infinite_temperature_spins_elementwise(L, variant):
    """T = inf, FP32, one and three sweeps: every spin of every path equals the oracle's (its
    last sweep's proposal) within TOL_PROP, z bit for bit; accept counts exact; the final
    magnetisation and energy within the FP32 summation bounds."""
    from helpers import engine_run
    n_paths = 2
    tol_m, tol_e = sum_tolerances(L, lanes_of(variant))
    for sweeps in (1, 3):
        res, _, spins, plan, _ = engine_run(L, math.inf, n_paths, sweeps, 0, fp64=False, variant=variant,
                                            spins_of=range(n_paths), instance_id=5)
        assert plan == variant
        ora = oracle32(L, math.inf, n_paths, sweeps, instance=5)
        for p in range(n_paths):
            check_spins(spins[p], ora["spins"][p], f"{variant} sweeps={sweeps} path={p}")
        assert np.array_equal(res["n_accept"], np.full(n_paths, sweeps * L ** 3, dtype=np.uint64))
        assert np.max(np.abs(res["final_m"] - ora["final_m"])) <= tol_m
        assert np.max(np.abs(res["final_e"] - ora["final_e"])) <= tol_e


@pytest.mark.gpu
@pytest.mark.parametrize("variants", BATCH_SETS, ids=["hbm48", "ring48-g1024", "ring48-g768", "ring2-32-48"])
def test_infinite_temperature_batch_elementwise(variants):
    """The batch kernels of the uneven batch's lattice sides (8, 12, 16 in LDS, 24 colour
    split, 32 x/y split or two-sweep ring, 48 device memory, plane ring or two-sweep ring),
    pinned by name: at T = inf after one
    and three sweeps the accept counts are exact and every path's final magnetisation and
    energy equal the oracle's (same instance ids) within the FP32 summation bounds."""
    from paper_1305_6758_amd import mmc
    n_paths = 3
    for sweeps in (1, 3):
        inst = [(L, math.inf, 1.0, n_paths, sweeps, 0) for L in variants]
        ctx = mmc.mmc_batch_create(inst, 1234, mmc.config(precision=mmc.MMC_FP32))
        try:
            for name in variants.values():
                mmc.mmc_set_variant(ctx, name)
            plan = mmc.mmc_plan(ctx)
            mmc.mmc_batch_run(ctx)
            for i, (L, name) in enumerate(variants.items()):
                assert f"L{L}:{name}" in plan, plan
                res = mmc.mmc_batch_results(ctx, i, n_paths)
                ora = oracle32(L, math.inf, n_paths, sweeps, instance=i)
                tol_m, tol_e = sum_tolerances(L, lanes_of(name))
                assert np.array_equal(res["n_accept"], np.full(n_paths, sweeps * L ** 3, dtype=np.uint64)), name
                dm = float(np.max(np.abs(res["final_m"] - ora["final_m"])))
                de = float(np.max(np.abs(res["final_e"] - ora["final_e"])))
                assert dm <= tol_m and de <= tol_e, (name, sweeps, dm, de)
        finally:
            mmc.mmc_destroy(ctx)


# variants of the uneven batch's sides with a single-instance form whose spins can be read
FLIP_VARIANTS = [(8, "f32-lds-L8-g64-b256", 48), (12, "f32-lds-L12-g256-b256", 16), (16, "f32-lds-L16-g512-b512", 8),
                 (24, "f32-split-L24-g1024-b1024", 4), (32, "f32-splitxy-L32-g1024-b1024", 2),
                 (48, "f32-hbm-L48-g512-b512", 1), (48, "f32-ring-L48-b1024", 1), (32, "f32-ring2-L32-b512", 2),
                 (48, "f32-ring2-L48-b1024", 1)]


@pytest.mark.gpu
def test_one_sweep_decisions_at_finite_temperature():
    """T = 1.443, one sweep from the random start: each site's FP32 spin must be its proposal
    or its start spin (within TOL_PROP), and its decision is compared with the oracle's on the
    same grid. A decision flips only when u lies within |dp| of p = exp(-beta dE), so a flip
    has probability at most E|dp| per update. With the proposal errors above,
    |d((S' - S) . h)| <= sqrt(3) (24 TOL_PROP + 48 u) + 36 u for |S' - S| <= 2 and |h| <= 6,
    hence E|dp| <= beta |J| (that + 2^-20) (the hardware exp2 within 8 ulp): P_MAX below.
    Counted: colour-0 sites that differ (their inputs are the start spins) and colour-1 sites
    that differ while all six neighbours agree (a flipped neighbour changes a site's field by
    O(1), which is not a rounding flip). The total must stay within the Poisson 1e-6 tail of
    P_MAX times the updates; it is printed."""
    from oracle import oracle as O
    from oracle import philox_np as P
    from helpers import engine_run
    T, J = 1.443, 1.0
    P_MAX = (1.0 / T) * abs(J) * (math.sqrt(3.0) * (24 * TOL_PROP + 48 * U32) + 36 * U32 + 2.0 ** -20)
    flips = updates = 0
    for L, variant, n_paths in FLIP_VARIANTS:
        N = L ** 3
        res, _, spins, plan, _ = engine_run(L, T, n_paths, 1, 0, J=J, fp64=False, variant=variant,
                                            spins_of=range(n_paths))
        ora = oracle32(L, T, n_paths, 1)
        ids = np.arange(N)
        x, y, z = ids % L, (ids // L) % L, ids // (L * L)
        colour = (x + y + z) & 1
        nb = np.stack([((x + dx) % L) + L * (((y + dy) % L) + L * ((z + dz) % L))
                       for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))], axis=1)
        key = np.array([1234, 0], dtype=np.uint32)
        params = O.make_params(L, T, J, seed=1234, uniforms="fp32")
        for p in range(n_paths):
            start = O.PathState(params, p).spins
            w = P.philox4x32_10(np.stack([ids, np.zeros(N), np.full(N, p), np.ones(N)], axis=1).astype(np.uint32), key)
            prop = O.unit_vectors(w[:, :2], uniforms="fp32")
            g, o = spins[p], ora["spins"][p]
            close = lambda a, b: np.max(np.abs(a - b), axis=1) <= TOL_PROP
            g_acc, g_rej = close(g, prop), close(g, start)
            assert np.all(g_acc | g_rej), f"{variant}: a spin is neither its proposal nor its start"
            o_acc = np.max(np.abs(o - prop), axis=1) == 0.0
            same = (g_acc == o_acc) | (g_acc & g_rej)  # (a proposal equal to the start decides nothing)
            primary = ~same & ((colour == 0) | np.all(same[nb], axis=1))
            flips += int(primary.sum())
            updates += N
        assert res["n_accept"].sum() > 0
    mean = P_MAX * updates
    bound = mean + 5.0 * math.sqrt(mean) + 12.0
    print(f"\nflipped decisions: {flips} in {updates} updates (worst-case rate {P_MAX:.2e}, bound {bound:.1f})", flush=True)
    assert flips <= bound
