"""Drivers for the paper's multipath experiments on top of the engine's C ABI.

Each driver only builds the instance list, calls the library (batched sweeps on the GPU,
statistics in the library's host code) and arranges the outputs; no simulation arithmetic
happens here.

  - binder_crossing: the O(3) critical temperature from the ratio of fourth-order cumulants
    U_30/U_20 at two temperatures, 10^6 single-output paths per (L, T) and 200 sweeps
    (Sec. 4, eq. (kum));
  - thermalisation: the order parameter <|M|> and the coefficient of variation of its mean
    against the number of sweeps from one traced run, for any start (random, both-angles,
    ordered, or the mixed half-and-half set-up with each half reported separately) (Sec. 3);
  - distribution_table: the distribution coefficient r of the single-output paths' H, M^x,
    M^y, M^z and |M^z| per temperature (Sec. 3, Table 1), for either proposal;
  - ising_magnetisation / ising_binder: the appendix's 2-D Ising runs -- the order parameter
    <|m|> of single-output paths against temperature beside the exact spontaneous
    magnetisation, and the critical temperature from the cumulant ratio of two lattices.

Usage: python -m paper_1305_6758_amd.experiments {binder,thermalisation,table,ising-m,ising-binder} [options]
"""
import argparse
import json
import math
import sys
import time

from . import mmc
from .workloads import SEED


def binder_crossing(Ls=(30, 20), Ts=(1.44, 1.45), n_paths=10 ** 6, sweeps=200, seed=SEED, fp64=False,
                    keep_results=False):
    """One batched launch of the four (L, T) instances, ordered (Ls[0], Ts[0]), (Ls[1], Ts[0]),
    (Ls[0], Ts[1]), (Ls[1], Ts[1]) -- instance ids 0..3 -- each n_paths paths from a random start
    through `sweeps` sweeps with the final state measured (n_therm = sweeps - 1, n_meas = 1).
    Returns the cumulants with their errors, the ratio U_L/U_L' at each T and the crossing."""
    if len(Ls) != 2 or len(Ts) != 2 or sweeps < 1:
        raise ValueError("need two lattice sizes, two temperatures and at least one sweep")
    instances = [(L, T, 1.0, n_paths, sweeps - 1, 1) for T in Ts for L in Ls]
    ctx = mmc.mmc_batch_create(instances, seed, mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32))
    try:
        t0 = time.perf_counter()
        mmc.mmc_batch_run(ctx)
        wall = time.perf_counter() - t0
        kernel_ms = mmc.mmc_last_timing_ms(ctx)
        plan = mmc.mmc_plan(ctx)
        results = [mmc.mmc_batch_results(ctx, i, n_paths) for i in range(len(instances))]
    finally:
        mmc.mmc_destroy(ctx)
    cum = [mmc.mmc_binder_cumulant(r) for r in results]
    cross = mmc.mmc_cumulant_crossing(Ts[0], Ts[1], [c[0] for c in cum], [c[1] for c in cum])
    updates = sum(p * L ** 3 * (nt + nm) for (L, T, _, p, nt, nm) in instances)
    out = {
        "Ls": list(Ls), "Ts": list(Ts), "n_paths": n_paths, "sweeps": sweeps, "seed": seed,
        "precision": "fp64" if fp64 else "fp32", "plan": plan,
        "cumulants": [{"L": L, "T": T, "U": c[0], "se": c[1]}
                      for (L, T, *_), c in zip(instances, cum)],
        "ratio": [{"T": Ts[0], "R": cross["r_t1"], "se": cross["se_r_t1"]},
                  {"T": Ts[1], "R": cross["r_t2"], "se": cross["se_r_t2"]}],
        "tc": cross["tc"], "se_tc": cross["se_tc"],
        "updates": updates, "kernel_ms": kernel_ms, "wall_s": wall,
        "updates_per_s": updates / (kernel_ms * 1e-3),
    }
    if keep_results:
        out["results"] = results
    return out


INITS = {"sphere": mmc.MMC_INIT_SPHERE, "angles": mmc.MMC_INIT_ANGLES, "ordered": mmc.MMC_INIT_ORDERED,
         "mixed": mmc.MMC_INIT_MIXED}


def doubling_sweeps(n):
    """Sweep counts 1, 2, 4, ... up to n, and n itself (the paper doubles the number of sweeps
    from one simulation to the next)."""
    out, k = [], 1
    while k < n:
        out.append(k)
        k *= 2
    return out + [n]


def thermalisation(L=10, T=1.0, n_paths=1000, sweeps=5000, init="sphere", fp64=False, seed=SEED, instance_id=0,
                   report=None, model=mmc.MMC_MODEL_HEISENBERG3D):
    """One run of n_paths paths through `sweeps` sweeps with every sweep traced. Row k of the
    trace is the output a path would give if it stopped after k + 1 sweeps, so the paper's
    series of simulations with growing sweep counts come from one run. Returns, at the sweep
    counts `report` (default: doubling), <m> with its standard error and the coefficient of
    variation of the mean, and <e>, over all paths and -- for the mixed start -- over the
    random-start (even) and ordered-start (odd) halves separately."""
    cfg = mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32, init=INITS[init], trace_sweeps=sweeps,
                     instance_id=instance_id, model=model)
    ctx = mmc.mmc_create_ex(L, T, 1.0, n_paths, sweeps, 0, seed, cfg)
    try:
        mmc.mmc_run(ctx)
        kernel_ms = mmc.mmc_last_timing_ms(ctx)
        plan = mmc.mmc_plan(ctx)
        trace = mmc.mmc_trace(ctx, n_paths, sweeps)
    finally:
        mmc.mmc_destroy(ctx)
    report = report or doubling_sweeps(sweeps)
    sets = {"all": (0, 1)}
    if init == "mixed":
        sets.update({"random_half": (0, 2), "ordered_half": (1, 2)})
    dim = 2 if model == mmc.MMC_MODEL_ISING2D else 3
    out = {"L": L, "T": T, "n_paths": n_paths, "sweeps": sweeps, "init": init, "model": model,
           "precision": "fp64" if fp64 else "fp32", "plan": plan, "kernel_ms": kernel_ms,
           "updates_per_s": n_paths * L ** dim * sweeps / (kernel_ms * 1e-3), "report_sweeps": report}
    for name, (b, st) in sets.items():
        rows = mmc.mmc_trace_stats(trace, b, st)
        out[name] = [{"sweeps": k, "m": rows[k - 1, 0], "se_m": rows[k - 1, 1], "cv_m": rows[k - 1, 2],
                      "e": rows[k - 1, 3], "se_e": rows[k - 1, 4]} for k in report]
    return out


def distribution_table(L=10, Ts=(0.6, 0.8, 1.0, 1.2, 1.4, 1.6), n_paths=10 ** 4, sweeps=5000, proposal="sphere",
                       init="sphere", seed=SEED, fp64=False):
    """Table 1 of Sec. 3: for each T, n_paths single-output paths (random start, `sweeps`
    sweeps, the final state measured) and the distribution coefficient r, eq.
    (dist-coefficient), of H/N, M^x, M^y, M^z and |M^z| over the paths. The paper leaves out
    r(M^z) in the ordered phase (two accumulation points) and r(|M^z|) in the disordered one;
    both are reported here. proposal 'angles' (both angles uniform) runs on the plain FP64
    engine; 'sphere' on the FP32 engine (FP64 with fp64=True). Instance id = index of T."""
    rows = []
    for i, T in enumerate(Ts):
        if proposal == "angles":
            cfg = mmc.config(precision=mmc.MMC_FP64, placement=mmc.MMC_PLACE_PLAIN, proposal=mmc.MMC_PROPOSAL_ANGLES,
                             init=INITS[init], instance_id=i)
        else:
            cfg = mmc.config(precision=mmc.MMC_FP64 if fp64 else mmc.MMC_FP32, init=INITS[init], instance_id=i)
        ctx = mmc.mmc_create_ex(L, T, 1.0, n_paths, sweeps - 1, 1, seed, cfg)
        try:
            mmc.mmc_run(ctx)
            ms = mmc.mmc_last_timing_ms(ctx)
            plan = mmc.mmc_plan(ctx)
            r = mmc.mmc_results(ctx, n_paths)
        finally:
            mmc.mmc_destroy(ctx)
        fm = r["final_m"]
        rows.append({"T": T, "plan": plan, "kernel_ms": ms,
                     "updates_per_s": n_paths * L ** 3 * sweeps / (ms * 1e-3),
                     "r_H": mmc.mmc_distribution_coefficient(r["final_e"]),
                     "r_Mx": mmc.mmc_distribution_coefficient(fm[:, 0]),
                     "r_My": mmc.mmc_distribution_coefficient(fm[:, 1]),
                     "r_Mz": mmc.mmc_distribution_coefficient(fm[:, 2]),
                     "r_absMz": mmc.mmc_distribution_coefficient(abs(fm[:, 2])),
                     "mean_absMz": float(abs(fm[:, 2]).mean()),
                     "mean_m": float(((fm ** 2).sum(axis=1) ** 0.5).mean())})
    return {"L": L, "n_paths": n_paths, "sweeps": sweeps, "proposal": proposal, "init": init, "rows": rows}


def onsager_yang(T, J=1.0):
    """Exact spontaneous magnetisation of the square-lattice Ising model (Onsager; Yang 1952):
    (1 - sinh(2J/T)^-4)^(1/8) below T_c = 2J/ln(1 + sqrt 2), zero above."""
    x = 1.0 - math.sinh(2.0 * J / T) ** -4
    return x ** 0.125 if x > 0 else 0.0


def _ising_single_output(L, T, n_paths, sweeps, seed, instance_id):
    cfg = mmc.config(model=mmc.MMC_MODEL_ISING2D, instance_id=instance_id)
    ctx = mmc.mmc_create_ex(L, T, 1.0, n_paths, sweeps - 1, 1, seed, cfg)
    try:
        mmc.mmc_run(ctx)
        ms = mmc.mmc_last_timing_ms(ctx)
        plan = mmc.mmc_plan(ctx)
        r = mmc.mmc_results(ctx, n_paths)
    finally:
        mmc.mmc_destroy(ctx)
    return r, ms, plan


def ising_magnetisation(Ls=(20, 40, 50, 60), Ts=(1.0, 1.5, 2.0, 2.1, 2.2, 2.269, 2.3, 2.4, 2.5, 3.0),
                        n_paths=10 ** 4, sweeps=3 * 10 ** 4, seed=SEED):
    """Appendix, Fig. Izing a): n_paths single-output paths per (L, T) from random starts through
    `sweeps` sweeps; <|m|> of the final states with its standard error, beside the exact
    spontaneous magnetisation. Instance id = index of (L, T) in L-major order."""
    rows, total_ms, upd = [], 0.0, 0
    for a, L in enumerate(Ls):
        for b, T in enumerate(Ts):
            r, ms, plan = _ising_single_output(L, T, n_paths, sweeps, seed, a * len(Ts) + b)
            am = abs(r["final_m"][:, 0])
            se = float(am.std(ddof=1) / math.sqrt(am.size))
            rows.append({"L": L, "T": T, "m": float(am.mean()), "se": se, "exact": onsager_yang(T),
                         "e": float(r["final_e"].mean()), "plan": plan, "kernel_ms": ms})
            total_ms += ms
            upd += n_paths * L * L * sweeps
    return {"n_paths": n_paths, "sweeps": sweeps, "rows": rows, "kernel_ms": total_ms, "updates": upd,
            "updates_per_s": upd / (total_ms * 1e-3)}


def ising_binder(Ls=(60, 50), Ts=(2.264, 2.268), n_paths=5 * 10 ** 4, sweeps=3 * 10 ** 4, seed=SEED):
    """Appendix: T_c of the square-lattice Ising model from U_L/U_L' = 1 between two
    temperatures, single-output paths (instance id = index of (L, T) in T-major order, as in
    binder_crossing)."""
    cum, total_ms, upd, plans = [], 0.0, 0, []
    i = 0
    for T in Ts:
        for L in Ls:
            r, ms, plan = _ising_single_output(L, T, n_paths, sweeps, seed, i)
            U, se = mmc.mmc_binder_cumulant(r)
            cum.append({"L": L, "T": T, "U": U, "se": se})
            total_ms += ms
            upd += n_paths * L * L * sweeps
            plans.append(plan)
            i += 1
    cross = mmc.mmc_cumulant_crossing(Ts[0], Ts[1], [c["U"] for c in cum], [c["se"] for c in cum])
    return {"Ls": list(Ls), "Ts": list(Ts), "n_paths": n_paths, "sweeps": sweeps, "cumulants": cum,
            "ratio": [{"T": Ts[0], "R": cross["r_t1"], "se": cross["se_r_t1"]},
                      {"T": Ts[1], "R": cross["r_t2"], "se": cross["se_r_t2"]}],
            "tc": cross["tc"], "se_tc": cross["se_tc"], "tc_exact": 2.0 / math.log(1.0 + math.sqrt(2.0)),
            "plan": " ".join(plans), "kernel_ms": total_ms, "updates": upd, "updates_per_s": upd / (total_ms * 1e-3)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment", choices=["binder", "thermalisation", "table", "ising-m", "ising-binder"])
    ap.add_argument("--paths", type=int, default=None)
    ap.add_argument("--sweeps", type=int, default=None)
    ap.add_argument("--L", type=int, default=10)
    ap.add_argument("--T", type=float, default=1.0)
    ap.add_argument("--init", default="sphere", choices=sorted(INITS))
    ap.add_argument("--proposal", default="sphere", choices=["sphere", "angles"])
    ap.add_argument("--fp64", action="store_true")
    a = ap.parse_args(argv)
    if a.experiment == "binder":
        out = binder_crossing(n_paths=a.paths or 10 ** 6, sweeps=a.sweeps or 200, fp64=a.fp64)
    elif a.experiment == "thermalisation":
        out = thermalisation(L=a.L, T=a.T, n_paths=a.paths or 1000, sweeps=a.sweeps or 5000, init=a.init, fp64=a.fp64)
    elif a.experiment == "table":
        out = distribution_table(L=a.L, n_paths=a.paths or 10 ** 4, sweeps=a.sweeps or 5000, proposal=a.proposal,
                                 init=a.init)
    elif a.experiment == "ising-m":
        out = ising_magnetisation(n_paths=a.paths or 10 ** 4, sweeps=a.sweeps or 3 * 10 ** 4)
    else:
        out = ising_binder(n_paths=a.paths or 5 * 10 ** 4, sweeps=a.sweeps or 3 * 10 ** 4)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
