"""Drivers for the paper's multipath experiments on top of the engine's C ABI.

Each driver only builds the instance list, calls the library (batched sweeps on the GPU,
statistics in the library's host code) and arranges the outputs; no simulation arithmetic
happens here.

  - binder_crossing: the O(3) critical temperature from the ratio of fourth-order cumulants
    U_30/U_20 at two temperatures, 10^6 single-output paths per (L, T) and 200 sweeps
    (Sec. 5, eq. (kum)).

Usage: python -m paper_1305_6758_amd.experiments binder [--paths N] [--fp64]
"""
import argparse
import json
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment", choices=["binder"])
    ap.add_argument("--paths", type=int, default=10 ** 6)
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--fp64", action="store_true")
    a = ap.parse_args(argv)
    out = binder_crossing(n_paths=a.paths, sweeps=a.sweeps, fp64=a.fp64)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
