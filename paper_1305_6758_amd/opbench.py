"""Measures gfx950 VALU instruction throughput (libmmc_opbench.so) and prints the issue cost
of each instruction class in full-rate lane slots (v_add_f32 = 1), the unit of the engine's
VALU roofline. With --copy-bytes B it instead runs one plain device-to-device copy of B bytes
(torch), the calibration kernel for the HBM byte counters; with --copy-reps R as well it then
times R more copies (HIP events on torch's stream), and R launches each of hand-written
16-byte streaming kernels (copy, read only, write only; plain or nontemporal accesses) over
192 launch shapes, and prints the bytes moved per second of the best shapes: the streaming
rates a memory-bound kernel can reach in practice.

Usage: python -m paper_1305_6758_amd.opbench [--ms MS] [--copy-bytes B [--copy-reps R]]
"""
import argparse
import ctypes as C
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ms", type=float, default=50.0, help="target run time per instruction class")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--copy-reps", type=int, default=0)
    a = ap.parse_args()
    import torch
    if a.copy_bytes:
        x = torch.ones(a.copy_bytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        out = {"copy_bytes": a.copy_bytes}
        if a.copy_reps > 0:
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(a.copy_reps):
                y.copy_(x)
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / a.copy_reps
            out.update({"copy_reps": a.copy_reps, "ms_per_copy": ms,
                        "read_plus_write_TBps": 2 * a.copy_bytes / (ms * 1e-3) / 1e12})
            # hand-written streaming kernels (copy, read only, write only; plain or nontemporal
            # accesses) over launch shapes: the best rate of each is the practical ceiling of
            # that access pattern
            lib = C.CDLL(os.path.join(HERE, "libmmc_opbench.so"))
            lib.mmc_opbench_stream.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_int, C.c_int,
                                               C.c_int, C.c_int, C.POINTER(C.c_double)]
            nb = a.copy_bytes // 16 * 16
            best = {}
            for kind, name, moved in ((0, "copy", 2 * nb), (1, "read", nb), (2, "write", nb)):
                rates = {}
                for nt in (0, 1):
                    for threads, bpcs in ((256, (1, 2, 4, 8, 16, 32)), (1024, (1, 2))):
                        for bpc in bpcs:
                            for unroll in (1, 2, 4, 8):
                                t = C.c_double()
                                rc = lib.mmc_opbench_stream(x.data_ptr(), y.data_ptr(), nb, a.copy_reps, kind, nt,
                                                            threads, bpc, unroll, C.byref(t))
                                if rc != 0:
                                    raise RuntimeError(f"mmc_opbench_stream failed ({rc})")
                                rates[f"{'nt' if nt else 'plain'}-t{threads}-b{bpc}-u{unroll}"] = moved / (t.value * 1e-3) / 1e12
                top = sorted(rates, key=rates.get, reverse=True)[:5]
                best[name] = {"best": top[0], "best_TBps": rates[top[0]], "top5": {k: rates[k] for k in top},
                              "shapes": len(rates)}
            out["hand_stream_TBps"] = best
        print(json.dumps(out))
        return
    lib = C.CDLL(os.path.join(HERE, "libmmc_opbench.so"))
    lib.mmc_opbench_name.restype = C.c_char_p
    lib.mmc_opbench_run.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    rows = {}
    for i in range(lib.mmc_opbench_count()):
        rate, ms = C.c_double(), C.c_double()
        iters = 1024
        for _ in range(8):  # grow the run until it lasts about --ms (sustained clocks)
            rc = lib.mmc_opbench_run(i, iters, C.byref(rate), C.byref(ms))
            if rc != 0:
                raise RuntimeError(f"opbench op {i} failed ({rc})")
            if ms.value >= a.ms:
                break
            iters = int(iters * min(64.0, max(2.0, 1.2 * a.ms / max(ms.value, 1e-3))))
        rows[lib.mmc_opbench_name(i).decode()] = (rate.value, ms.value)
    mix = rows.pop("update_mix")
    base = rows["v_add_f32"][0]
    props = torch.cuda.get_device_properties(0)
    print(f"device: {props.name} {props.gcnArchName}, {props.multi_processor_count} CUs")
    print(f"v_add_f32: {base:.4e} lane-ops/s = {base / (props.multi_processor_count * 64) / 1e9:.3f} G issue/s per lane-slot "
          "(effective VALU clock, 64 lanes per CU per clock)")
    print(f"{'instruction':16s} {'lane-ops/s':>12s} {'slots':>7s} {'ms':>8s}")
    for k, (r, ms) in rows.items():
        print(f"{k:16s} {r:12.4e} {base / r:7.2f} {ms:8.2f}")
    peak = 7.86432e13  # published FP32 vector rate / 2 FLOP per lane operation
    print(f"update mix (81.5 algorithmic VALU instructions per FP32 update): {mix[0]:.4e} updates/s "
          f"({mix[1]:.2f} ms) = {peak / mix[0]:.1f} lane-slots of the {peak:.4g} lane-op/s peak per update")
    out = {k: {"lane_ops_per_s": r, "slots": base / r} for k, (r, _) in rows.items()}
    out["update_mix"] = {"updates_per_s": mix[0], "lane_slots_per_update": peak / mix[0]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
