"""Seeded synthetic workloads of the benchmark and the parity tests.

Input recipes only -- no simulation arithmetic. The paper uses no dataset: every input is a
lattice size, temperatures, path and sweep counts, a seed and an instance id; the random
starts and moves come from the counter-based generator inside the engine and inside the
oracle. All use J = 1 (the paper's energy scale, Sec. 2.1) and seed 1234.

Instance ids: a workload with several (L, T) instances numbers them 0, 1, ... in the order
listed here; the id enters the random-number counter, so instance i of a batch and a
single-instance run with instance_id = i draw the same numbers.
"""
import numpy as np

SEED = 1234
J = 1.0

# One-GPU workloads. "instances": list of (L, T, n_paths, n_therm, n_meas).
WORKLOADS = {
    # L = 8, FP64, the trajectory-parity case.
    "L8-T1.5-p64-fp64": dict(precision="fp64", instances=[(8, 1.5, 64, 1000, 1000)]),
    # L = 16 at three temperatures around T_c, 4096 paths each, FP32 spins in LDS.
    "L16-T3-p4096-fp32": dict(precision="fp32", instances=[(16, T, 4096, 2000, 8000) for T in (1.2, 1.443, 1.7)]),
    # L = 32 at T = 1.443, 1024 paths, device-memory spins, run in FP32 and in FP64.
    "L32-T1.443-p1024": dict(precision="both", instances=[(32, 1.443, 1024, 5000, 5000)]),
    # L = 64 at T = 1.443, 256 paths, device-memory spins, FP32.
    "L64-T1.443-p256-fp32": dict(precision="fp32", instances=[(64, 1.443, 256, 10000, 10000)]),
    # Critical temperature from the Binder-cumulant ratio U_30/U_20 (Sec. 4): L = 30 and 20 at
    # T = 1.44 and 1.45, 10^6 single-output paths each (random start, 200 sweeps, the final
    # state measured: 199 thermalisation sweeps + 1 measured sweep), FP32.
    "binder-L30-L20-p1e6-fp32": dict(precision="fp32", instances=[(L, T, 10 ** 6, 199, 1)
                                                                   for T in (1.44, 1.45) for L in (30, 20)]),
    # The 200-sweep protocol from the other starts the paper's set-up allows: every spin along
    # +z, or half of the paths random and half ordered (init applies to the whole batch).
    "binder-L30-L20-p1e6-ordered-fp32": dict(precision="fp32", init="ordered",
                                             instances=[(L, T, 10 ** 6, 199, 1) for T in (1.44, 1.45) for L in (30, 20)]),
    "binder-L30-L20-p1e6-mixed-fp32": dict(precision="fp32", init="mixed",
                                           instances=[(L, T, 10 ** 6, 199, 1) for T in (1.44, 1.45) for L in (30, 20)]),
    # The same crossing at equilibrium: 4000 thermalisation sweeps, then the cumulant from the
    # per-path time means of M^2 and M^4 over 4000 measured sweeps, 10^4 paths per (L, T).
    "binder-L30-L20-p1e4-s8000-fp32": dict(precision="fp32", instances=[(L, T, 10 ** 4, 4000, 4000)
                                                                         for T in (1.44, 1.45) for L in (30, 20)]),
}

BATCH_LS = (8, 12, 16, 24, 32, 48)
BATCH_TS = tuple(float(t) for t in np.linspace(1.0, 2.0, 16))


def uneven_batch():
    """The uneven batch: L in {8, 12, 16, 24, 32, 48} x 16 temperatures evenly spaced on
    [1, 2] (both ends included), paths per instance drawn uniformly from [64, 2048] with
    numpy's default_rng(1234) in (L, T) order, 2000 thermalisation + 2000 measured sweeps."""
    rng = np.random.default_rng(SEED)
    paths = rng.integers(64, 2049, size=len(BATCH_LS) * len(BATCH_TS))
    out = []
    k = 0
    for L in BATCH_LS:
        for T in BATCH_TS:
            out.append((L, T, int(paths[k]), 2000, 2000))
            k += 1
    return out


WORKLOADS["uneven-batch-96-fp32"] = dict(precision="fp32", instances=uneven_batch())


# Experiments of Sec. 3 run through paper_1305_6758_amd.experiments (single-instance
# contexts: traced sweeps, or the plain FP64 engine for the both-angles proposal).
TABLE1_TS = (0.6, 0.8, 1.0, 1.2, 1.4, 1.6)
ISING_TS = (1.0, 1.5, 2.0, 2.1, 2.2, 2.269, 2.3, 2.4, 2.5, 3.0)
EXPERIMENTS = {
    # Sec. 3: L = 10, T = 1, 10^4 paths, half from a random start and half ordered, every one of
    # 5000 sweeps traced; <m> and its cv per sweep for each half.
    "thermalisation-L10-T1-mixed-p1e4-fp32": dict(kind="thermalisation", L=10, T=1.0, n_paths=10 ** 4,
                                                  sweeps=5000, init="mixed", fp64=False),
    # Sec. 3, Table 1: L = 10 at six temperatures, 10^4 single-output paths after 5000 sweeps;
    # isotropic proposal on the FP32 engine, both-angles proposal on the plain FP64 engine.
    "table1-L10-sphere-p1e4-fp32": dict(kind="table", L=10, Ts=TABLE1_TS, n_paths=10 ** 4, sweeps=5000,
                                        proposal="sphere", init="sphere", fp64=False),
    "table1-L10-angles-p1e4-fp64": dict(kind="table", L=10, Ts=TABLE1_TS, n_paths=10 ** 4, sweeps=5000,
                                        proposal="angles", init="angles", fp64=True),
    # Appendix, 2-D Ising model: <|m|> of 10^4 single-output paths after 3 10^4 sweeps for
    # L = 20, 40, 50, 60 at ten temperatures; T_c from U_60/U_50 at T = 2.264 and 2.268 with
    # 5 10^4 paths; the thermalisation of <|m|> and its cv at T = 3 and T = 1 (L = 50).
    "ising-magnetisation-L20-60-p1e4": dict(kind="ising_m", Ls=(20, 40, 50, 60), Ts=ISING_TS, n_paths=10 ** 4,
                                            sweeps=3 * 10 ** 4, init="sphere", fp64=False),
    "ising-binder-L60-L50-p5e4": dict(kind="ising_binder", Ls=(60, 50), Ts=(2.264, 2.268), n_paths=5 * 10 ** 4,
                                      sweeps=3 * 10 ** 4, init="sphere", fp64=False),
    "ising-thermalisation-L50-T3-p1e4": dict(kind="thermalisation", model=1, L=50, T=3.0, n_paths=10 ** 4,
                                             sweeps=3000, init="sphere", fp64=False),
    "ising-thermalisation-L50-T1-p1e4": dict(kind="thermalisation", model=1, L=50, T=1.0, n_paths=10 ** 4,
                                             sweeps=3000, init="sphere", fp64=False),
}


def experiment_instances(spec):
    """(L, T, n_paths, n_therm, n_meas) per context an experiment runs (instance id = index)."""
    if spec["kind"] == "thermalisation":
        return [(spec["L"], spec["T"], spec["n_paths"], spec["sweeps"], 0)]
    if spec["kind"] == "ising_m":
        return [(L, T, spec["n_paths"], spec["sweeps"] - 1, 1) for L in spec["Ls"] for T in spec["Ts"]]
    if spec["kind"] == "ising_binder":
        return [(L, T, spec["n_paths"], spec["sweeps"] - 1, 1) for T in spec["Ts"] for L in spec["Ls"]]
    return [(spec["L"], T, spec["n_paths"], spec["sweeps"] - 1, 1) for T in spec["Ts"]]


def site_count(spec, L):
    """Sites of one lattice of side L in an experiment's model."""
    return L * L if spec.get("model", 0) == 1 or spec["kind"].startswith("ising") else L ** 3


def updates(instances):
    """Metropolis attempts of a workload: sum over instances of paths * L^3 * sweeps."""
    return sum(p * L ** 3 * (nt + nm) for (L, T, p, nt, nm) in instances)
