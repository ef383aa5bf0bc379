"""Pins of the FP64 CPU oracle against facts fixed outside the oracle itself.

Each test names what it pins and which plausible mistake it would catch. Paper =
arXiv:1305.6758. None of these tests touches the GPU.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.stats as ss

from oracle import oracle as O
from oracle import philox_np as P
from oracle import stats as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def langevin(K):
    """<S1.S2> of one bond with coupling K = beta J: coth K - 1/K (classical spin chain,
    Fisher 1964)."""
    return 1.0 / math.tanh(K) - 1.0 / K


def within_4sigma(a, se_a, b, se_b=0.0, extra=0.0):
    return abs(a - b) <= 4.0 * math.hypot(se_a, se_b) + extra


def jackknife(f, *cols):
    """Delete-one jackknife estimate and standard error of f(mean(col1), mean(col2), ...)."""
    cols = [np.asarray(c, dtype=np.float64) for c in cols]
    n = cols[0].size
    sums = [c.sum() for c in cols]
    full = f(*[s / n for s in sums])
    loo = np.array([f(*[(s - c[i]) / (n - 1) for s, c in zip(sums, cols)]) for i in range(n)])
    se = math.sqrt((n - 1) / n * ((loo - loo.mean()) ** 2).sum())
    return full, se


# ---------------------------------------------------------------- random numbers

def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Random123, Salmon et al. SC'11) for
    both oracle-side generators. Catches a wrong multiplier, Weyl constant, round count,
    word permutation or key schedule."""
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        ctr, key, want = np.array([r[:4]]), np.array(r[4:6]), r[6:10]
        assert list(O.philox(ctr, key)[0]) == want
        assert list(P.philox4x32_10(ctr.astype(np.uint32), key.astype(np.uint32))[0]) == want


def test_philox_c_equals_numpy():
    """The two oracle-side generators agree bit for bit on 10^5 random counters/keys."""
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2 ** 32, size=(100000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(100000, 2), dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(O.philox(ctr, key), P.philox4x32_10(ctr, key))


def test_uniform_exact_open_interval():
    """u = (w + 1/2) 2^-32 is exact, strictly inside (0,1), and symmetric."""
    lib = O.lib()
    for w in [0, 1, 12345, 2 ** 31, 2 ** 32 - 2, 2 ** 32 - 1]:
        u = lib.mmco_uniform(w)
        assert 0.0 < u < 1.0
        assert u * 2.0 ** 33 == 2 * w + 1
    assert lib.mmco_uniform(0) + lib.mmco_uniform(2 ** 32 - 1) == 1.0


# ---------------------------------------------------------------- proposal

def test_fp32_uniform_grid_exact():
    """The FP32 engine's uniforms (the oracle's FP32-grid option): u = ((w >> 8) | 1) / 2^24
    exactly, an odd multiple of 2^-24 inside (0, 1), checked with integer arithmetic; the grid
    reaches the sweep: at beta = 0 the spins after one sweep are the FP32-grid unit vectors of
    the sweep-0 words, whose z = 2u - 1 is exact, and they differ from the FP64-grid spins by
    no more than the grids do (|du| < 2^-24, so |dz| < 2^-23 and a turn of phi below 2 pi 2^-24)."""
    from fractions import Fraction
    rng = np.random.default_rng(3)
    words = [0, 1, 255, 256, 511, 0x7FFFFFFF, 0x80000000, 0xFFFFFEFF, 0xFFFFFFFF] + list(rng.integers(0, 2 ** 32, 2000))
    for w in words:
        w = int(w)
        want = Fraction((w >> 8) | 1, 2 ** 24)
        got = O.uniform_fp32(w)
        assert Fraction(got) == want and 0 < got < 1
        assert abs(Fraction(got) - Fraction(O.lib().mmco_uniform(w))) < Fraction(1, 2 ** 24)
    L, N, path = 4, 64, 2
    r32 = O.run_paths(L, math.inf, n_therm=1, path_begin=path, path_end=path + 1, want_spins=True, uniforms="fp32")
    r64 = O.run_paths(L, math.inf, n_therm=1, path_begin=path, path_end=path + 1, want_spins=True)
    key = np.array([1234, 0], dtype=np.uint32)
    w = P.philox4x32_10(np.array([[i, 0, path, 1] for i in range(N)], dtype=np.uint32), key)
    want = O.unit_vectors(w[:, :2], uniforms="fp32")
    assert np.array_equal(r32["spins"][0], want)
    z_exact = np.array([2.0 * float(Fraction((int(a) >> 8) | 1, 2 ** 24)) - 1.0 for a in w[:, 0]])
    assert np.array_equal(r32["spins"][0][:, 2], z_exact)
    assert np.max(np.abs(r32["spins"][0][:, 2] - r64["spins"][0][:, 2])) < 2.0 ** -23
    assert np.max(np.abs(r32["spins"][0] - r64["spins"][0])) < 1e-3  # near the poles r moves by sqrt(|dz|)
    assert not np.array_equal(r32["spins"][0], r64["spins"][0])


def test_fp32_grid_two_spin_stationary_law():
    """The FP32-grid oracle is still a correct sampler: the two-spin law (density proportional
    to exp(beta J c)) holds with uniforms at 2^-24 resolution."""
    K, J = 2.0, 1.0
    T = J / K
    r = O.run_paths(2, T, J=J, n_therm=60, n_meas=0, path_end=4000, dim=1, periodic=False, uniforms="fp32")
    c = -2.0 * r["final_e"] / J
    cdf = lambda x: (np.exp(K * x) - math.exp(-K)) / (math.exp(K) - math.exp(-K))
    assert ss.kstest(c, cdf).pvalue > 1e-3
    m, se = S.mean_se(c)
    assert within_4sigma(m, se, langevin(K))


def test_proposal_uniform_on_sphere():
    """Proposal of the uniform-sphere reading: |S| = 1, E[S] = 0, E[S_a S_b] = delta_ab/3,
    z uniform on (-1,1), phi uniform on [0, 2 pi). Catches z = u instead of 2u - 1, a
    missing sqrt(1 - z^2), or angle-uniform sampling (which is not isotropic)."""
    n = 1_000_000
    s = O.proposals(n, seed=99)
    assert np.max(np.abs(np.linalg.norm(s, axis=1) - 1.0)) < 4e-16
    for a in range(3):
        assert abs(s[:, a].mean()) < 4.0 * math.sqrt(1.0 / 3.0 / n)
        assert abs((s[:, a] ** 2).mean() - 1.0 / 3.0) < 4.0 * math.sqrt(4.0 / 45.0 / n)
    for a, b in itertools.combinations(range(3), 2):
        assert abs((s[:, a] * s[:, b]).mean()) < 4.0 * math.sqrt(1.0 / 15.0 / n)
    assert ss.kstest(s[:, 2], ss.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    phi = np.mod(np.arctan2(s[:, 1], s[:, 0]), 2 * math.pi)
    assert ss.kstest(phi, ss.uniform(loc=0, scale=2 * math.pi).cdf).pvalue > 1e-3


def test_acceptance_rule_brute_force():
    """Metropolis acceptance min(1, exp(-beta dE)): over a fine uniform grid of u the
    accepted fraction equals min(1, exp(-beta dE)) to the grid spacing. Catches a wrong
    sign of dE, a wrong beta or a '>' test."""
    lib = O.lib()
    K = 20000
    us = (np.arange(K) + 0.5) / K
    for beta in [0.0, 0.3, 1.0, 2.5]:
        for dE in [-3.0, -0.1, 0.0, 0.2, 1.0, 4.0]:
            frac = np.mean([lib.mmco_accept(u, dE, beta) for u in us])
            assert abs(frac - min(1.0, math.exp(-beta * dE))) <= 1.0 / K + 1e-12


# ---------------------------------------------------------------- geometry and energy

def _brute_neighbors(L, dim, periodic, i):
    coords = np.array(np.unravel_index(np.arange(L ** dim), (L,) * dim, order="F")).T
    me = coords[i]
    d = np.abs(coords - me)
    if periodic:
        d = np.minimum(d, L - d)
    return sorted(np.nonzero(d.sum(axis=1) == 1)[0].tolist())


@pytest.mark.parametrize("L,dim,periodic", [(3, 3, True), (4, 3, True), (5, 3, True),
                                            (4, 3, False), (6, 2, True), (5, 1, False),
                                            (7, 1, True)])
def test_neighbors_brute_force(L, dim, periodic):
    """Nearest neighbours equal the sites at lattice distance 1 (brute force over all
    sites). Catches a wrong stride, a wrong wrap or x/y/z mixed up."""
    p = O.make_params(L, 1.0, dim=dim, periodic=periodic)
    for i in range(L ** dim):
        nb = sorted(j for j in O.neighbors(p, i) if j >= 0)
        assert nb == _brute_neighbors(L, dim, periodic, i)


def test_neighbors_L2_counted_twice():
    """With L = 2 and periodic boundaries the literal neighbour sum of eq. (ham) reaches the
    same site from both sides: every axis neighbour appears twice."""
    p = O.make_params(2, 1.0)
    for i in range(8):
        nb = O.neighbors(p, i)
        assert len(nb) == 6 and all(nb.count(j) == 2 for j in set(nb))


def _brute_energy(L, dim, periodic, J, spins):
    """-J sum over unordered pairs of sites at lattice distance 1 (each bond once)."""
    N = L ** dim
    E = 0.0
    for i in range(N):
        for j in _brute_neighbors(L, dim, periodic, i):
            if j > i:
                E += float(spins[i] @ spins[j])
    return -J * E


@pytest.mark.parametrize("L,dim,periodic,J", [(3, 3, True, 1.0), (4, 3, True, -0.7),
                                              (4, 3, False, 1.3), (5, 2, True, 1.0),
                                              (6, 1, False, 2.0)])
def test_energy_and_delta_e_brute_force(L, dim, periodic, J):
    """eq. (ham), -(J/2) sum_n sum_lambda S_n.S_n+lambda, equals -J sum over bonds (brute
    force), and dE of one replacement equals E(after) - E(before). Catches a missing 1/2,
    a dropped neighbour, and a wrong sign in dE."""
    rng = np.random.default_rng(L * 10 + dim)
    N = L ** dim
    s = rng.standard_normal((N, 3))
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    p = O.make_params(L, 1.0, J=J, dim=dim, periodic=periodic)
    E = O.energy(p, s)
    assert abs(E - _brute_energy(L, dim, periodic, J, s)) < 1e-12 * N
    for i in rng.integers(0, N, size=5):
        snew = rng.standard_normal(3)
        snew /= np.linalg.norm(snew)
        s2 = s.copy()
        s2[i] = snew
        dE = O.delta_e(p, s, int(i), snew)
        assert abs(dE - (_brute_energy(L, dim, periodic, J, s2) - E)) < 1e-12 * N


# ---------------------------------------------------------------- closed forms

def test_infinite_temperature_closed_forms():
    """beta = 0: every move is accepted, so after sweep 0 each spin is its own proposal
    Philox((i, 0, path, 1)), and each sweep yields independent uniform spins:
    <e> = 0, <e^2> = 1/N (3N bonds of variance 1/3), <m^2> = 1/N and
    <m^4> = (N^2 + 2N(N-1)/3)/N^4 exactly. Catches a missed accept, a wrong proposal
    counter, and wrong m^2/m^4 accumulators."""
    L, N, n_paths, n_meas = 4, 64, 1000, 20
    r = O.run_paths(L, math.inf, n_therm=0, n_meas=n_meas, path_end=n_paths)
    assert np.all(r["n_accept"] == N * n_meas)
    e, se = S.mean_se(r["e_mean"])
    assert within_4sigma(e, se, 0.0)
    for key, exact in [("e2_mean", 1.0 / N), ("m2_mean", 1.0 / N),
                       ("m4_mean", (N * N + 2.0 * N * (N - 1) / 3.0) / N ** 4)]:
        v, se = S.mean_se(r[key])
        assert within_4sigma(v, se, exact), key
    # one sweep at beta = 0: spins are exactly the proposals of sweep 0
    r1 = O.run_paths(L, math.inf, n_therm=1, n_meas=0, path_begin=3, path_end=4, want_spins=True)
    key = np.array([1234 & 0xFFFFFFFF, 1234 >> 32], dtype=np.uint32)
    ctr = np.array([[i, 0, 3, 1] for i in range(N)], dtype=np.uint32)
    w = P.philox4x32_10(ctr, key)
    want = np.array([O.unit_vector(int(a), int(b)) for a, b, _, _ in w])
    assert np.array_equal(r1["spins"][0], want)


@pytest.mark.parametrize("K,J", [(0.5, 1.0), (2.0, 1.0), (2.0, -1.0)])
def test_two_spin_stationary_law(K, J):
    """Two spins, one bond (open chain of N = 2): the stationary law of c = S1.S2 has density
    proportional to exp(beta J c) on [-1, 1]; <c> = coth(beta J) - 1/(beta J). KS test on
    final states plus 4 sigma on the mean. Detailed balance of the whole sampler."""
    T = abs(J) / K
    n_paths = 4000
    r = O.run_paths(2, T, J=J, n_therm=60, n_meas=0, path_end=n_paths, dim=1, periodic=False)
    c = -2.0 * r["final_e"] / J  # E = -J c, e = E / 2
    bJ = J / T
    cdf = lambda x: (np.exp(bJ * x) - math.exp(-bJ)) / (math.exp(bJ) - math.exp(-bJ))
    assert ss.kstest(c, cdf).pvalue > 1e-3
    m, se = S.mean_se(c)
    assert within_4sigma(m, se, langevin(bJ))


@pytest.mark.parametrize("K", [0.5, 1.0, 2.0])
def test_open_chain_closed_forms(K):
    """Open classical Heisenberg chain of N spins (exact: independent bonds):
    <E> = -(N-1) J u, u = coth K - 1/K; C_V per site = (N-1)/N (1 - K^2/sinh^2 K);
    <|sum S|^2> = N + 2 sum_r (N-r) u^r. Pins energy sign and scale, acceptance, the
    E^2 and m^2 accumulators and the heat-capacity formula of eq. (cv)."""
    N, J = 16, 1.0
    T = J / K
    r = O.run_paths(N, T, J=J, n_therm=200, n_meas=1000, path_end=384, dim=1, periodic=False)
    u = langevin(K)
    e, se = S.mean_se(r["e_mean"])
    assert within_4sigma(e, se, -(N - 1) * J * u / N)
    m2, se = S.mean_se(r["m2_mean"])
    exact_m2 = (N + 2.0 * sum((N - k) * u ** k for k in range(1, N))) / N ** 2
    assert within_4sigma(m2, se, exact_m2)
    # the heat capacity as oracle.stats.path_statistics computes it (eq. (cv)), not a retyped
    # formula: a dropped N or T instead of T^2 (K != 1) fails here
    cvh, se = path_statistic_jackknife(r, N, T, "cv_heat", dim=1)
    assert within_4sigma(cvh, se, (N - 1) / N * (1.0 - K * K / math.sinh(K) ** 2))


def path_statistic_jackknife(res, L, T, key, dim=3, blocks=32):
    """S.path_statistics(res)[key] over all paths and its delete-one-block jackknife standard
    error (paths are independent; `blocks` contiguous groups of paths)."""
    n = res["e_mean"].size
    cols = ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean")
    full = S.path_statistics({k: res[k] for k in cols}, L, T, dim=dim)[key]
    edges = np.linspace(0, n, blocks + 1).astype(int)
    loo = []
    for b in range(blocks):
        keep = np.r_[0:edges[b], edges[b + 1]:n]
        loo.append(S.path_statistics({k: res[k][keep] for k in cols}, L, T, dim=dim)[key])
    loo = np.asarray(loo)
    return full, math.sqrt((blocks - 1) / blocks * ((loo - loo.mean()) ** 2).sum())


def _two_spin_m_moments(K):
    """<m> and <m^2> of two coupled spins, m = |S1 + S2| / 2 = sqrt(2 + 2c) / 2 with c = S1.S2
    distributed with density proportional to exp(K c) on [-1, 1] (the joint law of two unit
    vectors with weight exp(K S1.S2): S2's angle to S1 is uniform in cos, tilted by exp(K c))."""
    import scipy.integrate as si
    z = si.quad(lambda c: math.exp(K * c), -1.0, 1.0)[0]
    m1 = si.quad(lambda c: 0.5 * math.sqrt(2.0 + 2.0 * c) * math.exp(K * c), -1.0, 1.0)[0] / z
    m2 = si.quad(lambda c: 0.25 * (2.0 + 2.0 * c) * math.exp(K * c), -1.0, 1.0)[0] / z
    return m1, m2


@pytest.mark.parametrize("K", [0.5, 2.0])
def test_susceptibility_two_spin_exact(K):
    """chi of eq. (cv), chi = (N/T)(<m^2> - <m>^2) with m = |M| per site, as
    oracle.stats.path_statistics computes it from oracle runs of two coupled spins (open chain,
    N = 2), against the exact moments from one-dimensional quadrature. T = 1/K = 2 and 0.5,
    so T^2 in place of T, or a dropped N, changes chi by a factor of 2 and fails; so does the
    mean of m^2 taken in place of the mean of m (or the reverse)."""
    T = 1.0 / K
    r = O.run_paths(2, T, J=1.0, n_therm=40, n_meas=400, path_end=3000, dim=1, periodic=False)
    m1, m2 = _two_spin_m_moments(K)
    chi_exact = 2.0 / T * (m2 - m1 * m1)
    chi, se = path_statistic_jackknife(r, 2, T, "chi", dim=1)
    assert within_4sigma(chi, se, chi_exact), (chi, se, chi_exact)
    # the factor-of-two alternatives lie far outside the bound
    assert 4.0 * se < 0.25 * chi_exact


@pytest.mark.parametrize("L,path,inst,seed,init", [(4, 0, 0, 1234, "sphere"), (6, 5, 3, 0x123456789ABCDEF, "sphere"),
                                                   (4, 2, 1, 99, "angles")])
def test_initial_state_stream(L, path, inst, seed, init):
    """The random start of Sec. 2.2: every site's spin is the unit vector of words 0 and 1 of
    Philox4x32-10 at counter (site id, 0, path, 0 | instance << 8) with key (seed_lo, seed_hi),
    the words recomputed here with the independent numpy Philox. A start drawn from tag 1 (the
    sweep-0 proposals), with the path and site words swapped, or without the instance or the
    seed's high word fails."""
    p = O.make_params(L, 1.5, seed=seed, instance=inst, init=init)
    st = O.PathState(p, path)
    N = L ** 3
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)
    ctr = np.array([[i, 0, path, inst << 8] for i in range(N)], dtype=np.uint32)
    w = P.philox4x32_10(ctr, key)
    want = np.array([O.unit_vector(int(a), int(b), init) for a, b, _, _ in w])
    assert np.array_equal(st.spins, want)


def test_low_temperature_limit_3d():
    """3-D ferromagnet from the ordered start at T -> 0: ground state -3J per spin plus
    harmonic equipartition of the 2N - 2 transverse modes, e = -3J + T (N-1)/N + O(T^2).
    Catches a dropped neighbour (ground state -2.5J) and a wrong sign of J or dE."""
    L, T = 4, 0.05
    N = L ** 3
    r = O.run_paths(L, T, n_therm=2000, n_meas=2000, path_end=64, init="ordered")
    e, se = S.mean_se(r["e_mean"])
    assert within_4sigma(e, se, -3.0 + T * (N - 1) / N, extra=T * T)


def test_coupling_sign_invariance():
    """J -> -J leaves the energy distribution unchanged on the bipartite lattice (the paper
    states the sign of J makes no difference classically). Catches J entering dE with the
    wrong power or only in part of the update."""
    a = O.run_paths(4, 1.5, J=1.0, n_therm=200, n_meas=300, path_end=256)
    b = O.run_paths(4, 1.5, J=-1.0, n_therm=200, n_meas=300, path_end=256)
    ea, sa = S.mean_se(a["e_mean"])
    eb, sb = S.mean_se(b["e_mean"])
    assert within_4sigma(ea, sa, eb, sb)


def test_isotropy():
    """Finite lattice, no field: <M_a> = 0 and <M_a^2> equal for a = x, y, z (the paper's
    discussion of the magnetisation components). Catches an anisotropic proposal such as
    angle-uniform sampling."""
    r = O.run_paths(4, 1.0, n_therm=300, n_meas=0, path_end=768)
    m = r["final_m"]
    for a in range(3):
        v, se = S.mean_se(m[:, a])
        assert within_4sigma(v, se, 0.0)
    sq = [S.mean_se(m[:, a] ** 2) for a in range(3)]
    for (va, sa), (vb, sb) in itertools.combinations(sq, 2):
        assert within_4sigma(va, sa, vb, sb)


def test_sweep_orders_agree_at_equilibrium():
    """Checkerboard, the paper's random-site sweep and a typewriter sweep share one
    stationary law: equilibrium <e> and <|m|> agree within 4 sigma."""
    runs = {s: O.run_paths(4, 1.5, n_therm=300, n_meas=400, path_end=256, sweep=s)
            for s in ("checkerboard", "random_site", "typewriter")}
    for key in ("e_mean", "absm_mean"):
        vals = [S.mean_se(r[key]) for r in runs.values()]
        for (va, sa), (vb, sb) in itertools.combinations(vals, 2):
            assert within_4sigma(va, sa, vb, sb), key


def test_checkerboard_order_within_colour_is_irrelevant():
    """All neighbours of a site lie in the other colour, so visiting a colour in reverse
    changes no bit. Catches a colour rule that lets a site see a same-colour neighbour."""
    kw = dict(n_therm=20, n_meas=30, path_end=4, trace_sweeps=50, want_spins=True)
    a = O.run_paths(4, 1.2, sweep="checkerboard", **kw)
    b = O.run_paths(4, 1.2, sweep="checkerboard_reversed", **kw)
    for k in ("spins", "trace", "e_mean", "m4_mean", "n_accept"):
        assert np.array_equal(a[k], b[k]), k


def test_resume_is_bit_identical():
    """Counter-based random numbers carry no state: running 25 sweeps, stopping and going on
    to 60 equals running 60 at once."""
    p = O.make_params(4, 1.3, n_therm=20, n_meas=40, seed=77)
    a = O.PathState(p, 5)
    a.advance(25)
    a.advance(60)
    b = O.PathState(p, 5)
    b.advance(60)
    assert np.array_equal(a.spins, b.spins)
    ra, rb = a.result(), b.result()
    for f in ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e", "n_accept"):
        assert getattr(ra, f) == getattr(rb, f)


def test_outputs_match_brute_force_of_final_state():
    """The per-path output of Sec. 2.2 is computed from the final state: final_e is the
    brute-force energy per site of the returned spins, final_m their mean, and the last
    trace row is that same snapshot."""
    L, n = 4, 3
    r = O.run_paths(L, 1.4, J=0.9, n_therm=5, n_meas=7, path_end=n, want_spins=True,
                    trace_sweeps=12)
    for t in range(n):
        s = r["spins"][t]
        assert abs(r["final_e"][t] - _brute_energy(L, 3, True, 0.9, s) / L ** 3) < 1e-13
        assert np.allclose(r["final_m"][t], s.mean(axis=0), atol=1e-15, rtol=0)
        assert np.allclose(r["trace"][t, -1], [r["final_e"][t], *r["final_m"][t]], atol=1e-15)
        # measured sweeps are the last n_meas trace rows
        tr = r["trace"][t, 5:12]
        assert abs(r["e_mean"][t] - tr[:, 0].mean()) < 1e-14
        assert abs(r["absm_mean"][t] - np.linalg.norm(tr[:, 1:], axis=1).mean()) < 1e-14


def test_instance_and_seed_select_distinct_streams():
    """Instance id and seed enter the counter/key: different values give different paths,
    equal values identical ones."""
    base = dict(n_therm=3, n_meas=2, path_end=2, want_spins=True)
    a = O.run_paths(4, 1.5, **base)
    assert np.array_equal(a["spins"], O.run_paths(4, 1.5, **base)["spins"])
    assert not np.array_equal(a["spins"], O.run_paths(4, 1.5, instance=1, **base)["spins"])
    assert not np.array_equal(a["spins"], O.run_paths(4, 1.5, seed=1235, **base)["spins"])
    assert not np.array_equal(a["spins"][0], a["spins"][1])


# ---------------------------------------------------------------- statistics

def test_distribution_coefficient_matches_probplot_and_correlation():
    """eq. (dist-coefficient) with an OLS line is the coefficient of determination of the
    Q-Q fit: equal to scipy.stats.probplot's r squared and to the squared correlation of
    sorted data and normal quantiles; exactly 1 for points on a line."""
    rng = np.random.default_rng(3)
    for n in (20, 200, 5000):
        for x in (rng.standard_normal(n) * 0.3 - 1.2, rng.exponential(size=n)):
            r = S.distribution_coefficient(x)
            assert abs(r - ss.probplot(x)[1][2] ** 2) < 1e-12
            from scipy.special import ndtri
            q = ndtri(S.filliben_medians(n))
            assert abs(r - np.corrcoef(np.sort(x), q)[0, 1] ** 2) < 1e-12
    q = ndtri(S.filliben_medians(50))
    assert abs(S.distribution_coefficient(3.0 + 2.0 * q) - 1.0) < 1e-14


def test_normality_k2_matches_library():
    rng = np.random.default_rng(4)
    for n in (20, 100, 4096):
        for x in (rng.standard_normal(n), rng.exponential(size=n), rng.uniform(size=n)):
            k2, p = S.normality_k2(x)
            ref = ss.normaltest(x)
            assert abs(k2 - ref.statistic) < 1e-9 * max(1.0, ref.statistic)
            assert abs(p - ref.pvalue) < 1e-9


def test_binder_and_cv_definitions():
    """Binder cumulant at beta = 0 (independent unit spins, exact moments):
    U = 2/3 - 2(N-1)/(9N); coefficient of variation eq. (eq:cv) against scipy."""
    N = 64
    m2 = 1.0 / N
    m4 = (N * N + 2.0 * N * (N - 1) / 3.0) / N ** 4
    st = S.path_statistics({"e_mean": np.arange(5.0), "absm_mean": np.arange(1.0, 6.0),
                            "e2_mean": np.ones(5), "m2_mean": np.full(5, m2),
                            "m4_mean": np.full(5, m4)}, L=4, T=1.0)
    assert abs(st["binder"] - (2.0 / 3.0 - 2.0 * (N - 1) / (9.0 * N))) < 1e-14
    x = np.random.default_rng(5).uniform(1, 2, size=300)
    assert abs(S.coeff_variation(x) - ss.variation(x, ddof=1) / math.sqrt(x.size)) < 1e-15


def test_binder_cumulant_error_by_repetition():
    """eq. (kum) with its delta-method error, pinned two ways on paths whose total spin is an
    isotropic Gaussian vector (the high-temperature limit of M): U -> 1 - 15/(3*9) = 4/9
    (E|g|^2 = 3, E|g|^4 = 15 for g ~ N(0, I_3)), and the reported standard error equals the
    spread of U over independent repetitions (a dropped covariance term would overstate it
    about 11-fold, a wrong sign in dU/d<M^2> about 21-fold)."""
    rng = np.random.default_rng(21)
    reps, n = 300, 4000
    g = rng.standard_normal((reps, n, 3))
    m2 = (g * g).sum(axis=2)
    m4 = m2 * m2
    us, ses = np.empty(reps), np.empty(reps)
    for k in range(reps):
        us[k], ses[k] = S.binder_cumulant(m2[k], m4[k])
    assert abs(us.mean() - 4.0 / 9.0) < 4.0 * us.std(ddof=1) / math.sqrt(reps)
    assert abs(us.std(ddof=1) / ses.mean() - 1.0) < 0.12
    # leave-one-out jackknife on one sample agrees with the first-order error
    a, b = m4[0], m2[0]
    A, B = a.sum(), b.sum()
    jk = 1.0 - ((A - a) / (n - 1)) / (3.0 * ((B - b) / (n - 1)) ** 2)
    se_jk = math.sqrt((n - 1) / n * ((jk - jk.mean()) ** 2).sum())
    assert abs(se_jk / ses[0] - 1.0) < 0.03


def test_binder_cumulant_of_oracle_runs_at_infinite_temperature():
    """Snapshot output (n_meas = 1) at beta ~ 0 on L = 2 (N = 8 independent unit spins once
    every site has been redrawn): U = 2/3 - 2(N-1)/(9N) within 4 standard errors."""
    N = 8
    r = O.run_paths(2, 1e12, n_therm=1, n_meas=1, path_end=6000, seed=77)
    U, se = S.binder_cumulant(r["m2_mean"], r["m4_mean"])
    exact = 2.0 / 3.0 - 2.0 * (N - 1) / (9.0 * N)
    assert 0 < se < 0.01
    assert abs(U - exact) < 4.0 * se


def test_cumulant_crossing_exact_and_error():
    """Sec. 4 crossing: a ratio linear in T through 1 at Tc gives Tc to rounding; the
    propagated error matches the spread of Tc under independent noise on the four cumulants."""
    Tc0, k = 1.442, -3.7
    T1, T2 = 1.44, 1.45
    v1, v2 = 0.61, 0.58
    u = np.array([(1 + k * (T1 - Tc0)) * v1, v1, (1 + k * (T2 - Tc0)) * v2, v2])
    se = np.array([1e-4, 2e-4, 1.5e-4, 0.5e-4])
    Tc, sTc, R1, s1, R2, s2 = S.cumulant_crossing(T1, T2, u, se)
    assert abs(Tc - Tc0) < 1e-13
    assert abs(R1 - (1 + k * (T1 - Tc0))) < 1e-15 and abs(R2 - (1 + k * (T2 - Tc0))) < 1e-15
    rng = np.random.default_rng(8)
    draws = u + rng.standard_normal((20000, 4)) * se
    tcs = np.array([S.cumulant_crossing(T1, T2, d, se)[0] for d in draws])
    assert abs(tcs.std(ddof=1) / sTc - 1.0) < 0.04
    assert abs(tcs.mean() - Tc0) < 4.0 * sTc / math.sqrt(draws.shape[0]) + 1e-6


def _angle_proposal_two_spin_moments(K, n=96):
    """<S1.S2> and <cos^2 theta_1> for two coupled spins under the both-angles-uniform proposal.
    Its stationary law is the Boltzmann weight times prod 1/sin(theta_i) on the sphere, i.e.
    exp(K c) times the flat measure d theta1 d phi1 d theta2 d phi2; integrated over (theta1,
    theta2, phi1 - phi2) by Gauss-Legendre in the polar angles and the trapezoid rule in phi."""
    x, w = np.polynomial.legendre.leggauss(n)
    th, wt = (x + 1) * math.pi / 2, w * math.pi / 2
    m = 2 * n
    ph = np.arange(m) * 2 * math.pi / m
    T1, T2, P = np.meshgrid(th, th, ph, indexing="ij")
    W = wt[:, None, None] * wt[None, :, None]
    c = np.cos(T1) * np.cos(T2) + np.sin(T1) * np.sin(T2) * np.cos(P)
    b = W * np.exp(K * c)
    return (c * b).sum() / b.sum(), (np.cos(T1) ** 2 * b).sum() / b.sum()


@pytest.mark.parametrize("K", [1.0, 2.0])
def test_angle_proposal_two_spin_law(K):
    """The both-angles-uniform proposal (Sec. 2.2's random-start parametrisation used for the
    moves) leaves Metropolis without a Hastings correction: its stationary law is anisotropic.
    Two spins on one bond: <S1.S2> and <(S1^z)^2> against the quadrature of that law (they
    differ from the isotropic coth K - 1/K and 1/3 by many standard errors); the sphere
    proposal on the same chain keeps <(S1^z)^2> = 1/3."""
    T = 1.0 / K
    c_ref, z2_ref = _angle_proposal_two_spin_moments(K)
    n = 16000
    r = O.run_paths(2, T, n_therm=60, n_meas=0, path_end=n, dim=1, periodic=False, proposal="angles",
                    want_spins=True)
    c = -2.0 * r["final_e"]
    m, se = S.mean_se(c)
    assert within_4sigma(m, se, c_ref)
    assert abs(c_ref - langevin(K)) > 8 * se
    z2 = r["spins"][:, 0, 2] ** 2
    m, se = S.mean_se(z2)
    assert within_4sigma(m, se, z2_ref)
    r = O.run_paths(2, T, n_therm=60, n_meas=0, path_end=n, dim=1, periodic=False, want_spins=True)
    m, se = S.mean_se(r["spins"][:, 0, 2] ** 2)
    assert within_4sigma(m, se, 1.0 / 3.0)


def test_mixed_start_is_sphere_and_ordered_by_path_parity():
    """The mixed start of Sec. 3 (half of the paths random, half ordered): even paths are the
    random-start (sphere) paths and odd paths the ordered-start paths, bit for bit."""
    kw = dict(n_therm=3, n_meas=4, path_end=6, seed=9, instance=2)
    mix = O.run_paths(4, 1.2, init="mixed", want_spins=True, **kw)
    sph = O.run_paths(4, 1.2, init="sphere", want_spins=True, **kw)
    ordr = O.run_paths(4, 1.2, init="ordered", want_spins=True, **kw)
    for k in ("e_mean", "absm_mean", "m4_mean", "final_e", "final_m", "n_accept", "spins"):
        assert np.array_equal(mix[k][0::2], sph[k][0::2]), k
        assert np.array_equal(mix[k][1::2], ordr[k][1::2]), k
    st = O.run_paths(4, 1.2, init="mixed", n_therm=0, n_meas=0, path_end=2, want_spins=True)
    assert np.all(st["spins"][1] == np.array([0.0, 0.0, 1.0]))
    assert np.std(st["spins"][0][:, 2]) > 0.3


def test_trace_statistics_against_scipy():
    """Per-sweep statistics of a trace (Sec. 3: <m> and the coefficient of variation of the
    mean, eq. (eq:cv)) against scipy's sem and variation of |M_k| computed directly."""
    r = O.run_paths(4, 1.2, n_therm=12, n_meas=0, path_end=30, init="mixed", trace_sweeps=12, seed=3)
    t = r["trace"]
    for b, st in ((0, 1), (1, 2)):
        rows = S.trace_statistics(t, b, st)
        for k in range(12):
            m = np.linalg.norm(t[b::st, k, 1:4], axis=1)
            assert abs(rows[k, 0] - m.mean()) < 1e-15
            assert abs(rows[k, 1] - ss.sem(m)) < 1e-15
            assert abs(rows[k, 2] - ss.variation(m, ddof=1) / math.sqrt(m.size)) < 1e-14
            assert abs(rows[k, 3] - t[b::st, k, 0].mean()) < 1e-15
            assert abs(rows[k, 4] - ss.sem(t[b::st, k, 0])) < 1e-15
    # the ordered half starts at |m| = 1 exactly, the random half far below
    rows = S.trace_statistics(O.run_paths(4, 1.2, n_therm=1, n_meas=0, path_end=30, init="mixed", trace_sweeps=1,
                                          seed=3)["trace"], 1, 2)
    assert rows[0, 0] > 0.9


@pytest.mark.parametrize("N,K,sweep", [(4, 1.0, "checkerboard"), (4, 2.0, "checkerboard"), (3, 2.0, "typewriter"),
                                       (6, 2.0, "random_site")])
def test_periodic_ring_exact(N, K, sweep):
    """Periodic classical Heisenberg ring of N spins, solvable at any N: expanding each bond's
    weight exp(K S.S') in Legendre polynomials with modified spherical Bessel coefficients
    i_l(K), Z = sum_l (2l + 1) i_l(K)^N and <S_i . S_i+1> = sum_l (2l+1) i_l^(N-1) i_l' / Z.
    Pins the periodic wrap with the loop it closes (the value differs from the open chain's
    coth K - 1/K by many standard errors at these N); odd N with a sequential sweep."""
    from scipy.special import spherical_in
    l = np.arange(80)
    i, d = spherical_in(l, K), spherical_in(l, K, derivative=True)
    exact = ((2 * l + 1) * i ** (N - 1) * d).sum() / ((2 * l + 1) * i ** N).sum()
    r = O.run_paths(N, 1.0 / K, n_therm=100, n_meas=600, path_end=3000, dim=1, periodic=True, sweep=sweep, seed=31)
    m, se = S.mean_se(-np.asarray(r["e_mean"]))  # e = -J <S_i . S_i+1> per site, J = 1
    assert within_4sigma(m, se, exact)
    if N <= 4:
        assert abs(exact - langevin(K)) > 10 * se
