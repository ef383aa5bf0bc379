"""The two-sweep plane ring's pass schedule (placement PL_RING2 of the sweep kernels), replayed
on the CPU at the granularity of half-planes (one colour of one z-plane) against the sequential
checkerboard order (every site of colour 0, then colour 1, sweep after sweep).

The replay follows the kernel's pass: stage j (colour j mod 2 of sweep ks + j // 2) updates
virtual plane tau - lag_j at step tau, over virtual planes j .. j + L - 1; stages 0 and 2 share
phase 1 of a step, stages 1 and 3 phase 2; five colour-0 and six colour-1 slots; stage 0's own
spins staged from device memory a step ahead, stage 3's own spins copied from their slot in
phase 1 and its neighbours below in phase 2 of the step before; colour 0 written back four steps
after its plane's first update; colour 1 written by stage 3, and by stage 1 for virtual planes 1
and 2; one-sweep passes run stages 0 and 1 alone, both writing to device memory.

The spins are integers and the update an exact hash of the site, the sweep, the own spin and
the six neighbours in order, so any neighbour read at the wrong time, from the wrong slot or in
the wrong state changes the outcome. Every update must see exactly the values of the sequential
order (checked per half-plane and sweep), the stages of one phase must touch disjoint
half-planes, and no device-memory half-plane loaded at the start of a step may be written
during it. Planted schedule mistakes must fail.
"""
import random

import pytest

MOD = (1 << 61) - 1
KS = 5  # first sweep of the pass


class ScheduleError(Exception):
    pass


def neighbours(L, c, z, s):
    """Site id and in-plane neighbour half-indices (-x, +x, -y, +y; the other colour) of
    half-index s of colour c in plane z."""
    HL = L // 2
    j, y = s % HL, s // HL
    p = (y + z + c) & 1
    x = 2 * j + p
    row = s - j
    jm = HL - 1 if j == 0 else j - 1
    jp = 0 if j == HL - 1 else j + 1
    nb = (row + (j if p else jm), row + (jp if p else j),
          s + ((L - 1) * HL if y == 0 else -HL), s + (-(L - 1) * HL if y == L - 1 else HL))
    return x + L * (y + L * z), nb


def update(sid, k, own, nbr):
    v = own * 1000003 + sid * 7919 + k * 104729
    for i, n in enumerate(nbr):
        v = v * 31 + n * (i + 3)
    return v % MOD


def half_plane(L, c, z, k, own, oth, below, above):
    out = []
    for s in range(L * L // 2):
        sid, nb = neighbours(L, c, z, s)
        out.append(update(sid, k, own[s], tuple(oth[n] for n in nb) + (below[s], above[s])))
    return out


def sequential(L, G, sweeps):
    G = [[list(p) for p in G[c]] for c in range(2)]
    seen = {}
    for k in range(KS, KS + sweeps):
        for c in (0, 1):
            G[c] = [half_plane(L, c, z, k, G[c][z], G[1 - c][z], G[1 - c][(z - 1) % L], G[1 - c][(z + 1) % L])
                    for z in range(L)]
            for z in range(L):
                seen[(k, c, z)] = G[c][z]
    return G, seen


def replay(L, G, two, lag=(0, 1, 3, 4), slots1=6, early_c1=(1, 2), wb_after=4):
    """One pass of the ring from device-memory state G; returns the final state and every
    half-plane update (sweep, colour, plane) -> values."""
    G = [[list(p) for p in G[c]] for c in range(2)]
    S0, S1 = {}, {}
    sl0 = lambda v: v % 5
    sl1 = lambda v: v % slots1
    done = {}
    S1[sl1(-1)], S1[sl1(0)], S1[sl1(1)] = list(G[1][L - 1]), list(G[1][0]), list(G[1][1 % L])
    own0 = list(G[0][0])
    own3 = zm3 = zm3_next = None
    nsteps = L + 7 if two else L + 2
    c1_last, c0_last = (L + 2, L + 3) if two else (L, L + 1)

    def active(j, tau):
        return (two or j < 2) and j + lag[j] <= tau < j + lag[j] + L

    for tau in range(nsteps):
        loads = []
        r1 = own0n = None
        if tau + 2 <= c1_last:
            r1 = list(G[1][(tau + 2) % L])
            loads.append(("G1", (tau + 2) % L))
        if tau + 1 <= c0_last:
            own0n = list(G[0][(tau + 1) % L])
            loads.append(("G0", (tau + 1) % L))
        written = set()
        for phase in (1, 2):
            ops = []  # (name, reads, writes, action)
            if phase == 1:
                if active(0, tau):
                    v = tau - lag[0]

                    def st0(v=v, own=own0):
                        new = half_plane(L, 0, v % L, KS, own, S1[sl1(v)], S1[sl1(v - 1)], S1[sl1(v + 1)])
                        done[(KS, 0, v % L)] = new
                        S0[sl0(v)] = new
                        if not two:
                            G[0][v % L] = list(new)
                    ops.append(("stage 0", {("S1", sl1(v)), ("S1", sl1(v - 1)), ("S1", sl1(v + 1))},
                                {("S0", sl0(v))} | (set() if two else {("G0", v % L)}), st0))
                elif L <= tau <= c0_last:
                    def copy(t=tau, own=own0):
                        S0[sl0(t)] = list(own)
                    ops.append(("copy", set(), {("S0", sl0(tau))}, copy))
                if active(2, tau):
                    v = tau - lag[2]

                    def st2(v=v):
                        new = half_plane(L, 0, v % L, KS + 1, S0[sl0(v)], S1[sl1(v)], S1[sl1(v - 1)], S1[sl1(v + 1)])
                        done[(KS + 1, 0, v % L)] = new
                        S0[sl0(v)] = new
                    ops.append(("stage 2", {("S0", sl0(v)), ("S1", sl1(v)), ("S1", sl1(v - 1)), ("S1", sl1(v + 1))},
                                {("S0", sl0(v))}, st2))
                if active(3, tau):
                    v3 = tau - lag[3]

                    def stage3_own(v=v3):
                        nonlocal own3
                        own3 = list(S1[sl1(v)])
                    ops.append(("stage 3 own", {("S1", sl1(v3))}, set(), stage3_own))
                if two and wb_after <= tau <= L + 1 + wb_after:
                    v = tau - wb_after

                    def writeback(v=v):
                        G[0][v % L] = list(S0[sl0(v)])
                    ops.append(("write-back", {("S0", sl0(v))}, {("G0", v % L)}, writeback))
            else:
                if active(1, tau):
                    v = tau - lag[1]
                    wg = not two or v in early_c1

                    def st1(v=v, wg=wg):
                        new = half_plane(L, 1, v % L, KS, S1[sl1(v)], S0[sl0(v)], S0[sl0(v - 1)], S0[sl0(v + 1)])
                        done[(KS, 1, v % L)] = new
                        S1[sl1(v)] = new
                        if wg:
                            G[1][v % L] = list(new)
                    ops.append(("stage 1", {("S1", sl1(v)), ("S0", sl0(v)), ("S0", sl0(v - 1)), ("S0", sl0(v + 1))},
                                {("S1", sl1(v))} | ({("G1", v % L)} if wg else set()), st1))
                if active(3, tau):
                    v = tau - lag[3]

                    def st3(v=v, own=own3, zm=zm3):
                        new = half_plane(L, 1, v % L, KS + 1, own, S0[sl0(v)], zm, S0[sl0(v + 1)])
                        done[(KS + 1, 1, v % L)] = new
                        G[1][v % L] = new
                    ops.append(("stage 3", {("S0", sl0(v)), ("S0", sl0(v + 1))}, {("G1", v % L)}, st3))
                if r1 is not None:
                    def store1(t=tau, r=r1):
                        S1[sl1(t + 2)] = r
                    ops.append(("colour-1 store", set(), {("S1", sl1(tau + 2))}, store1))
                if active(3, tau + 1):
                    v = tau + 1 - lag[3] - 1  # the next step's stage-3 plane, less one

                    def stage3_below(v=v):
                        nonlocal zm3_next
                        zm3_next = list(S0[sl0(v)])
                    ops.append(("stage 3 below", {("S0", sl0(v))}, set(), stage3_below))
            for a in ops:
                for b in ops:
                    if a is not b and a[2] & (b[1] | b[2]):
                        raise ScheduleError(f"step {tau} phase {phase}: {a[0]} writes {a[2] & (b[1] | b[2])} "
                                            f"which {b[0]} touches")
            for op in ops:
                op[3]()
                written |= {w for w in op[2] if w[0] in ("G0", "G1")}
        for ld in loads:
            if ld in written:
                raise ScheduleError(f"step {tau}: {ld} loaded at the step's start and written during it")
        own0 = own0n
        zm3, zm3_next = zm3_next, None
    return G, done


def state(L, seed):
    rng = random.Random(seed)
    return [[[rng.randrange(MOD) for _ in range(L * L // 2)] for _ in range(L)] for _ in range(2)]


def check(L, two, **mistake):
    G = state(L, 7 * L + two)
    ref, seen = sequential(L, G, 2 if two else 1)
    got, done = replay(L, G, two, **mistake)
    assert sorted(done) == sorted(seen), "every half-plane of every sweep updated exactly once"
    for key, vals in seen.items():
        assert done[key] == vals, f"half-plane {key} differs from the sequential order"
    assert got == ref, "final state"


@pytest.mark.parametrize("L", [6, 8, 10, 16])
@pytest.mark.parametrize("two", [False, True])
def test_pass_equals_sequential_order(L, two):
    check(L, two)


@pytest.mark.parametrize("mistake", [
    dict(lag=(0, 1, 2, 3)),   # stage 2 one plane closer: reads colour 1 before stage 1 is done
    dict(slots1=5),           # five colour-1 slots: the stored plane overwrites a live one
    dict(early_c1=(1,)),      # plane 2's sweep-ks colour 1 not written for its reload
    dict(wb_after=3),         # colour 0 written back in the step stage 2 updates it
])
def test_planted_mistakes_fail(mistake):
    with pytest.raises((AssertionError, ScheduleError)):
        for L in (8, 10):
            check(L, True, **mistake)
