"""Writes the oracle's per-path results for sampled paths of the full-size workloads.

Calls only the FP64 CPU oracle (oracle/) and the input recipes; the GPU engine is never
involved. The full-size parity tests compare the engine's paths with these files, so the
parity tests do not rerun hours of oracle work. Paths sampled: the first K of each instance
(same counter streams on both sides: path index and instance id select the stream).

Usage: python tests/golden/make_oracle_golden.py [workload ...] [--threads N]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1305_6758_amd.workloads import J, SEED, WORKLOADS  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# paths sampled per instance
SAMPLE = {
    "L16-T3-p4096-fp32": 32,
    "L32-T1.443-p1024": 16,
    "L64-T1.443-p256-fp32": 8,
    "uneven-batch-96-fp32": 8,
    "binder-L30-L20-p1e6-fp32": 256,
    "binder-L30-L20-p1e4-s8000-fp32": 64,
}


def run(name, threads):
    spec = WORKLOADS[name]
    K = SAMPLE[name]
    out = {"workload": name, "seed": SEED, "J": J, "paths_per_instance": K, "instances": []}
    t0 = time.time()
    for inst_id, (L, T, n_paths, n_therm, n_meas) in enumerate(spec["instances"]):
        r = O.run_paths(L, T, J=J, n_therm=n_therm, n_meas=n_meas, seed=SEED, path_begin=0,
                        path_end=min(K, n_paths), instance=inst_id, n_threads=threads)
        out["instances"].append({
            "L": L, "T": T, "n_paths": n_paths, "n_therm": n_therm, "n_meas": n_meas,
            "instance_id": inst_id,
            **{k: [float(x) for x in r[k]] for k in ("e_mean", "e2_mean", "absm_mean", "m2_mean",
                                                      "m4_mean", "final_e")},
            "final_m": [[float(x) for x in row] for row in r["final_m"]],
            "n_accept": [int(x) for x in r["n_accept"]],
        })
        print(f"{name}: instance {inst_id} (L={L}, T={T:.4g}) done at {time.time() - t0:.0f} s", flush=True)
    out["oracle_seconds"] = time.time() - t0
    out["oracle_threads"] = threads
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=0)
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", default=list(SAMPLE))
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    a = ap.parse_args()
    for w in a.workloads:
        run(w, a.threads)
