"""Pins of the FP64 CPU oracle's 2-D Ising model (appendix "2D Ising model" of
arXiv:1305.6758) against facts fixed outside the oracle: the counter-based random stream
recomputed with the independent numpy Philox, exact enumeration of the 4 x 4 lattice, a
transfer-matrix solution of the 6 x 6 lattice (with the full magnetisation distribution),
the infinite-temperature moments, Onsager's exact energy and the Onsager-Yang spontaneous
magnetisation. None of these tests touches the GPU."""
import itertools
import math

import numpy as np
import pytest
from scipy.special import ellipk

from oracle import oracle as O
from oracle import philox_np as P
from oracle import stats as S

SEED = 1234


def within(m, se, exact, extra=0.0):
    return abs(m - exact) <= 4.0 * se + extra


# ---------------------------------------------------------------- random stream

def _quad_words(L, x, y, k, path, tag, inst, seed):
    Q = (L // 2 + 3) // 4
    c, j = (x + y) & 1, x >> 1
    q = c * L * Q + y * Q + (j >> 2)
    ctr = np.array([[q, k, path, tag | (inst << 8)]], dtype=np.uint32)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)
    return int(P.philox4x32_10(ctr, key)[0][j & 3])


@pytest.mark.parametrize("L,inst,seed", [(10, 0, SEED), (6, 5, 2 ** 40 + 7), (8, 1, 3)])
def test_start_and_acceptance_words_from_the_stream_definition(L, inst, seed):
    """The random start and the acceptance uniforms follow the quad mapping (one Philox call
    per four sites of a row of one colour, word j mod 4), recomputed here with the numpy
    Philox. Catches a wrong quad index, word, tag or counter word."""
    r = O.ising_run_paths(L, 2.0, n_therm=0, n_meas=0, seed=seed, instance=inst, path_begin=3, path_end=5,
                          want_spins=True)
    lib = O.lib()
    for t, path in enumerate((3, 4)):
        for y in range(L):
            for x in range(L):
                w = _quad_words(L, x, y, 0, path, 4, inst, seed)
                assert r["spins"][t][x + L * y] == (1 if w < 2 ** 31 else -1)
    beta, J = 0.45, 1.0
    for (x, y, k, a) in [(0, 0, 0, 2), (L - 1, 3, 7, 4), (3, L - 1, 2, -2), (1, 1, 11, 0), (L - 2, 2, 5, 4)]:
        u = (_quad_words(L, x, y, k, 9, 3, inst, seed) + 0.5) / 2 ** 32
        assert lib.mmco_ising_accept(L, x, y, k, 9, inst, seed, beta, J, a) == int(u < math.exp(-beta * 2 * J * a))


# ---------------------------------------------------------------- exact small lattices

def _enumerate(L):
    """(E, M) of every configuration of the L x L periodic lattice (bonds counted once)."""
    N = L * L
    idx = np.arange(2 ** N, dtype=np.int64)
    s = 1 - 2 * ((idx[:, None] >> np.arange(N)) & 1).astype(np.int64)
    s = s.reshape(-1, L, L)  # [config, y, x]
    E = -(s * np.roll(s, 1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, 1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    return E, M


def _moments(E, M, N, T, weights=None):
    w = np.exp(-(E - E.min()) / T) * (1 if weights is None else weights)
    Z = w.sum()
    e, m = E / N, M / N
    return {"e": (w * e).sum() / Z, "absm": (w * np.abs(m)).sum() / Z, "m2": (w * m ** 2).sum() / Z,
            "m4": (w * m ** 4).sum() / Z}


@pytest.mark.parametrize("T", [1.8, 3.0])
def test_L4_against_exact_enumeration(T):
    """4 x 4 periodic lattice, all 2^16 states: per-path time means of e, |m|, m^2, m^4 over
    independent paths agree with the exact canonical averages (4 standard errors)."""
    E, M = _enumerate(4)
    ex = _moments(E.astype(float), M.astype(float), 16, T)
    r = O.ising_run_paths(4, T, n_therm=100, n_meas=400, path_end=2000)
    for key, col in (("e", "e_mean"), ("absm", "absm_mean"), ("m2", "m2_mean"), ("m4", "m4_mean")):
        m, se = S.mean_se(r[col])
        assert within(m, se, ex[key]), (key, m, se, ex[key])


def _transfer_matrix_L6(T):
    """6 x 6 periodic lattice by the row transfer matrix: Z(theta) = Tr (T D(theta))^6 with
    D(theta) = diag(exp(i theta M_row)); the distribution of the total M follows from the
    discrete Fourier transform over the 37 possible values, <E> from the exact energy
    derivative of ln Z (energy-weighted transfer matrix)."""
    L, N = 6, 36
    rows = np.array(list(itertools.product([1, -1], repeat=L)))           # [64, 6]
    horiz = (rows * np.roll(rows, 1, axis=1)).sum(axis=1)                  # bonds within a row
    vert = rows @ rows.T                                                   # bonds between rows
    Mrow = rows.sum(axis=1)
    K = 1.0 / T
    A = np.exp(K * (vert + horiz[None, :]))                                # A[a, b]: row b after a
    thetas = 2 * np.pi * np.arange(37) / 37
    Zt = np.array([np.trace(np.linalg.matrix_power(A * np.exp(1j * th * Mrow)[None, :], L)) for th in thetas])
    Ms = np.arange(-N, N + 1, 2)
    PM = np.array([(Zt * np.exp(-1j * thetas * Mv)).sum().real / 37 for Mv in Ms])
    PM /= PM.sum()
    # <E>: derivative of Tr A^L in K, A' = A * (vert + horiz)
    Ad = A * (vert + horiz[None, :])
    Z = np.trace(np.linalg.matrix_power(A, L))
    dZ = L * np.trace(np.linalg.matrix_power(A, L - 1) @ Ad)
    mean_bonds = dZ / Z
    return {"e": -mean_bonds / N, "absm": (PM * np.abs(Ms / N)).sum(), "m2": (PM * (Ms / N) ** 2).sum()}


def test_transfer_matrix_matches_enumeration_on_L4():
    """The transfer-matrix construction itself, checked where enumeration is possible (4 x 4)."""
    L, N, T = 4, 16, 2.3
    E, M = _enumerate(4)
    ex = _moments(E.astype(float), M.astype(float), N, T)
    rows = np.array(list(itertools.product([1, -1], repeat=L)))
    horiz = (rows * np.roll(rows, 1, axis=1)).sum(axis=1)
    A = np.exp((rows @ rows.T + horiz[None, :]) / T)
    Ad = A * (rows @ rows.T + horiz[None, :])
    Z = np.trace(np.linalg.matrix_power(A, L))
    e = -(L * np.trace(np.linalg.matrix_power(A, L - 1) @ Ad) / Z) / N
    assert abs(e - ex["e"]) < 1e-12


@pytest.mark.parametrize("T", [2.2, 2.6])
def test_L6_against_transfer_matrix(T):
    """6 x 6 lattice (2^36 states, out of reach of enumeration) near and above T_c."""
    ex = _transfer_matrix_L6(T)
    r = O.ising_run_paths(6, T, n_therm=200, n_meas=600, path_end=1200)
    for key, col in (("e", "e_mean"), ("absm", "absm_mean"), ("m2", "m2_mean")):
        m, se = S.mean_se(r[col])
        assert within(m, se, ex[key]), (key, m, se, ex[key])


def test_infinite_temperature_moments():
    """beta ~ 0: every flip is taken, spins independent and +-1 after the random start:
    <e> = 0, <m^2> = 1/N, <m^4> = (3N^2 - 2N)/N^4 over single-output paths."""
    L, N = 6, 36
    r = O.ising_run_paths(L, 1e12, n_therm=3, n_meas=1, path_end=20000)
    m, se = S.mean_se(r["final_e"])
    assert within(m, se, 0.0)
    m, se = S.mean_se(r["m2_mean"])
    assert within(m, se, 1.0 / N)
    m, se = S.mean_se(r["m4_mean"])
    assert within(m, se, (3.0 * N * N - 2.0 * N) / N ** 4)
    assert np.all(r["n_accept"] == 4 * N)


# ---------------------------------------------------------------- Onsager

def onsager_energy(T, J=1.0):
    """Energy per site of the infinite square lattice (Onsager 1944):
    u = -J coth(2K) [1 + (2/pi)(2 tanh^2(2K) - 1) K(k)], k = 2 sinh(2K)/cosh^2(2K)."""
    K = J / T
    k = 2.0 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    return -J / math.tanh(2 * K) * (1.0 + 2.0 / math.pi * (2.0 * math.tanh(2 * K) ** 2 - 1.0) * ellipk(k * k))


def onsager_yang_m(T, J=1.0):
    """Spontaneous magnetisation (Onsager; Yang 1952): (1 - sinh^-4(2K))^(1/8) below T_c."""
    x = 1.0 - math.sinh(2.0 * J / T) ** -4
    return x ** 0.125 if x > 0 else 0.0


@pytest.mark.parametrize("T", [1.5, 2.0, 3.5])
def test_onsager_energy_and_magnetisation_L32(T):
    """32 x 32 lattice away from T_c (finite-size corrections exponentially small): <e> equals
    Onsager's energy and, below T_c, <|m|> the Onsager-Yang magnetisation (4 standard errors
    plus 2e-4 for the finite lattice)."""
    r = O.ising_run_paths(32, T, n_therm=300, n_meas=300, path_end=64)
    m, se = S.mean_se(r["e_mean"])
    assert within(m, se, onsager_energy(T), 2e-4), (m, se, onsager_energy(T))
    if T < 2.2:
        m, se = S.mean_se(r["absm_mean"])
        assert within(m, se, onsager_yang_m(T), 2e-4), (m, se, onsager_yang_m(T))


def test_critical_temperature_constants():
    """T_c = 2/ln(1 + sqrt 2) is where sinh(2K) = 1: the magnetisation vanishes there and the
    energy equals -sqrt(2) J (Onsager's value at T_c)."""
    Tc = 2.0 / math.log(1.0 + math.sqrt(2.0))
    assert abs(math.sinh(2.0 / Tc) - 1.0) < 1e-15
    assert onsager_yang_m(Tc * (1 + 1e-9)) == 0.0 and onsager_yang_m(Tc * 0.999) > 0.3
    assert abs(onsager_energy(Tc * (1 + 1e-6)) + math.sqrt(2.0)) < 1e-4
    assert abs(onsager_energy(Tc * (1 - 1e-6)) + math.sqrt(2.0)) < 1e-4
