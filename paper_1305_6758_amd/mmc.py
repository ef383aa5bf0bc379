"""Python binding of libmmc.so: the C ABI of include/mmc.h with the same names.

Argument marshalling only -- every step of the simulation runs in the HIP kernels of the
library. PyTorch supplies device memory and the stream (mmc_bind); it does no computation.
Loading fails loudly if the library has not been built.
"""
import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmc.so")

MMC_OK, MMC_EINVAL, MMC_ENOMEM, MMC_EHIP, MMC_ESTATE, MMC_EUNSUPPORTED, MMC_EIO = 0, -1, -2, -3, -4, -5, -6
MMC_FP32, MMC_FP64 = 0, 1
MMC_INIT_SPHERE, MMC_INIT_ANGLES, MMC_INIT_ORDERED, MMC_INIT_MIXED = 0, 1, 2, 3
MMC_PROPOSAL_SPHERE, MMC_PROPOSAL_ANGLES = 0, 1
MMC_MODEL_HEISENBERG3D, MMC_MODEL_ISING2D = 0, 1
MMC_PLACE_AUTO, MMC_PLACE_LDS, MMC_PLACE_HBM, MMC_PLACE_PLAIN, MMC_PLACE_WINDOW = 0, 1, 2, 3, 4
MMC_BATCH_AUTO, MMC_BATCH_FUSED, MMC_BATCH_PER_VARIANT = 0, 1, 2
MMC_STATIC_SCRATCH_BYTES, MMC_STATIC_MAX_INSTANCES, MMC_STATIC_MAX_PATHS = 18 << 20, 256, 131072


class mmc_config(C.Structure):
    _fields_ = [("precision", C.c_int), ("init", C.c_int), ("placement", C.c_int), ("block", C.c_int),
                ("lanes_per_path", C.c_int), ("renorm_every", C.c_int), ("instance_id", C.c_uint32),
                ("trace_sweeps", C.c_int), ("async_", C.c_int), ("proposal", C.c_int), ("model", C.c_int),
                ("batch_launch", C.c_int)]


class mmc_path_result(C.Structure):
    _fields_ = [("e_mean", C.c_double), ("e2_mean", C.c_double), ("absm_mean", C.c_double),
                ("m2_mean", C.c_double), ("m4_mean", C.c_double), ("final_m", C.c_double * 3),
                ("final_e", C.c_double), ("n_accept", C.c_uint64)]


class mmc_stats_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean_e", C.c_double), ("se_e", C.c_double), ("mean_absm", C.c_double),
                ("se_absm", C.c_double), ("e2", C.c_double), ("m2", C.c_double), ("m4", C.c_double),
                ("chi", C.c_double), ("cv_heat", C.c_double), ("binder", C.c_double), ("cv_absm", C.c_double),
                ("r_e", C.c_double), ("r_absm", C.c_double), ("p_norm_e", C.c_double),
                ("p_norm_absm", C.c_double), ("accept_rate", C.c_double)]


class mmc_crossing_t(C.Structure):
    _fields_ = [("tc", C.c_double), ("se_tc", C.c_double), ("r_t1", C.c_double), ("se_r_t1", C.c_double),
                ("r_t2", C.c_double), ("se_r_t2", C.c_double)]


class mmc_instance(C.Structure):
    _fields_ = [("L", C.c_int), ("T", C.c_double), ("J", C.c_double), ("n_paths", C.c_int),
                ("n_therm", C.c_int), ("n_meas", C.c_int)]


class MMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mmc error {code}: {msg}")
        self.code = code


# (name, restype, argtypes) of every exported function of include/mmc.h
_P = C.c_void_p
_SIGNATURES = [
    ("mmc_create", _P, [C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_uint64]),
    ("mmc_create_ex", _P, [C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_uint64,
                           C.POINTER(mmc_config)]),
    ("mmc_last_error", C.c_char_p, []),
    ("mmc_last_status", C.c_int, []),
    ("mmc_workspace_bytes", C.c_size_t, [_P]),
    ("mmc_bind", C.c_int, [_P, _P, C.c_size_t, _P]),
    ("mmc_tune", C.c_int, [_P]),
    ("mmc_set_variant", C.c_int, [_P, C.c_char_p]),
    ("mmc_run", C.c_int, [_P]),
    ("mmc_run_sweeps", C.c_int, [_P, C.c_int]),
    ("mmc_sync", C.c_int, [_P]),
    ("mmc_reset", C.c_int, [_P]),
    ("mmc_sweeps_done", C.c_int, [_P]),
    ("mmc_results", C.c_int, [_P, C.POINTER(mmc_path_result), C.c_int]),
    ("mmc_trace", C.c_int, [_P, C.POINTER(C.c_double), C.c_size_t]),
    ("mmc_get_spins", C.c_int, [_P, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
    ("mmc_spin_norm_deviation", C.c_int, [_P, C.POINTER(C.c_double)]),
    ("mmc_stats", C.c_int, [_P, C.POINTER(mmc_stats_t)]),
    ("mmc_stats_from_results", C.c_int, [C.POINTER(mmc_path_result), C.c_int, C.c_int, C.c_double,
                                         C.POINTER(mmc_stats_t)]),
    ("mmc_binder_cumulant", C.c_int, [C.POINTER(mmc_path_result), C.c_int, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
    ("mmc_cumulant_crossing", C.c_int, [C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(mmc_crossing_t)]),
    ("mmc_distribution_coefficient", C.c_int, [C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double)]),
    ("mmc_trace_stats", C.c_int, [C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    ("mmc_save", C.c_int, [_P, C.c_char_p]),
    ("mmc_load", _P, [C.c_char_p]),
    ("mmc_last_timing_ms", C.c_double, [_P]),
    ("mmc_proposal_vectors", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_uint32), C.c_int64, C.POINTER(C.c_double)]),
    ("mmc_plan", C.c_int, [_P, C.c_char_p, C.c_size_t]),
    ("mmc_destroy", None, [_P]),
    ("mmc_batch_create", _P, [C.POINTER(mmc_instance), C.c_int, C.c_uint64, C.POINTER(mmc_config)]),
    ("mmc_batch_run", C.c_int, [_P]),
    ("mmc_batch_results", C.c_int, [_P, C.c_int, C.POINTER(mmc_path_result), C.c_int]),
    ("mmc_batch_stats", C.c_int, [_P, C.c_int, C.POINTER(mmc_stats_t)]),
    ("mmc_batch_run_static", C.c_int, [C.POINTER(mmc_instance), C.c_int, C.c_uint64, C.POINTER(mmc_config), _P, _P]),
]
EXPORTED = [s[0] for s in _SIGNATURES]

_lib = None


def lib():
    """The loaded libmmc.so. Raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one libmmc binds
        # to, so the process holds a single HIP/HSA runtime and torch's device pointers and
        # streams are valid inside the library.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1305_6758_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != MMC_OK:
        raise MMCError(rc, lib().mmc_last_error().decode())
    return rc


def _ptr(h):
    if not h:
        raise MMCError(lib().mmc_last_status(), lib().mmc_last_error().decode())
    return h


def config(precision=MMC_FP32, init=MMC_INIT_SPHERE, placement=MMC_PLACE_AUTO, block=0, lanes_per_path=0,
           renorm_every=0, instance_id=0, trace_sweeps=0, async_=0, proposal=MMC_PROPOSAL_SPHERE,
           model=MMC_MODEL_HEISENBERG3D, batch_launch=0):
    return mmc_config(precision, init, placement, block, lanes_per_path, renorm_every, instance_id,
                      trace_sweeps, async_, proposal, model, batch_launch)


# ---------------------------------------------------------------- same names as the C ABI
def mmc_create(L, T, J, n_paths, n_therm, n_meas, seed):
    return _ptr(lib().mmc_create(L, T, J, n_paths, n_therm, n_meas, seed))


def mmc_create_ex(L, T, J, n_paths, n_therm, n_meas, seed, cfg=None):
    return _ptr(lib().mmc_create_ex(L, T, J, n_paths, n_therm, n_meas, seed, C.byref(cfg) if cfg else None))


def mmc_last_error():
    return lib().mmc_last_error().decode()


def mmc_last_status():
    return lib().mmc_last_status()


def mmc_workspace_bytes(ctx):
    return lib().mmc_workspace_bytes(ctx)


def mmc_bind(ctx, dev_ptr, nbytes, stream_handle):
    return _check(lib().mmc_bind(ctx, dev_ptr, nbytes, stream_handle))


def mmc_tune(ctx):
    return _check(lib().mmc_tune(ctx))


def mmc_set_variant(ctx, name):
    return _check(lib().mmc_set_variant(ctx, name.encode()))


def mmc_run(ctx):
    return _check(lib().mmc_run(ctx))


def mmc_run_sweeps(ctx, k):
    return _check(lib().mmc_run_sweeps(ctx, k))


def mmc_sync(ctx):
    return _check(lib().mmc_sync(ctx))


def mmc_reset(ctx):
    return _check(lib().mmc_reset(ctx))


def mmc_sweeps_done(ctx):
    return lib().mmc_sweeps_done(ctx)


# numpy view of mmc_path_result (same field order, 80 bytes, no padding)
RESULT_DTYPE = np.dtype([("e_mean", "<f8"), ("e2_mean", "<f8"), ("absm_mean", "<f8"), ("m2_mean", "<f8"),
                         ("m4_mean", "<f8"), ("final_m", "<f8", (3,)), ("final_e", "<f8"), ("n_accept", "<u8")])
assert RESULT_DTYPE.itemsize == C.sizeof(mmc_path_result)


def _result_buffer(n):
    buf = np.zeros(n, dtype=RESULT_DTYPE)
    return buf, buf.ctypes.data_as(C.POINTER(mmc_path_result))


def _results_to_numpy(buf):
    return {k: np.array(buf[k]) for k in RESULT_DTYPE.names}


def _results_array(results):
    """dict of per-path arrays (as returned by mmc_results) -> C array of mmc_path_result."""
    n = len(results["e_mean"])
    buf, ptr = _result_buffer(n)
    for k in RESULT_DTYPE.names:
        if k in results:
            buf[k] = np.asarray(results[k]).reshape(buf[k].shape)
    return buf, ptr, n


def mmc_results(ctx, n_paths):
    buf, ptr = _result_buffer(n_paths)
    _check(lib().mmc_results(ctx, ptr, n_paths))
    return _results_to_numpy(buf)


def mmc_trace(ctx, n_paths, trace_sweeps):
    out = np.empty((n_paths, trace_sweeps, 4))
    _check(lib().mmc_trace(ctx, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
    return out


def mmc_spin_norm_deviation(ctx):
    d = C.c_double()
    _check(lib().mmc_spin_norm_deviation(ctx, C.byref(d)))
    return d.value


def mmc_get_spins(ctx, path, L, dim=3):
    """[L^dim, 3] spins of one path (dim = 2 for the Ising model: s in the z component)."""
    out = np.empty((L ** dim, 3))
    _check(lib().mmc_get_spins(ctx, path, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
    return out


def _stats_dict(s):
    return {name: getattr(s, name) for name, _ in mmc_stats_t._fields_}


def mmc_stats(ctx):
    s = mmc_stats_t()
    _check(lib().mmc_stats(ctx, C.byref(s)))
    return _stats_dict(s)


def mmc_stats_from_results(results, L, T):
    """results: dict of arrays as returned by mmc_results."""
    buf, ptr, n = _results_array(results)
    s = mmc_stats_t()
    _check(lib().mmc_stats_from_results(ptr, n, L, T, C.byref(s)))
    return _stats_dict(s)


def mmc_binder_cumulant(results):
    """(U, se) of eq. (kum) over the paths of results (dict of arrays)."""
    buf, ptr, n = _results_array(results)
    U, se = C.c_double(), C.c_double()
    _check(lib().mmc_binder_cumulant(ptr, n, C.byref(U), C.byref(se)))
    return U.value, se.value


def mmc_cumulant_crossing(T1, T2, u, se):
    """u, se: (U_L(T1), U_L'(T1), U_L(T2), U_L'(T2)) and their errors -> dict of mmc_crossing_t."""
    cu = (C.c_double * 4)(*[float(x) for x in u])
    cs = (C.c_double * 4)(*[float(x) for x in se])
    out = mmc_crossing_t()
    _check(lib().mmc_cumulant_crossing(float(T1), float(T2), cu, cs, C.byref(out)))
    return {name: getattr(out, name) for name, _ in mmc_crossing_t._fields_}


def mmc_trace_stats(trace, path_begin=0, path_stride=1):
    """trace: [n_paths, n_sweeps, 4] as returned by mmc_trace -> [n_sweeps, 5] array of
    (<m>, se, cv of the mean, <e>, se) over the selected paths."""
    t = np.ascontiguousarray(trace, dtype=np.float64)
    n_paths, n_sweeps = t.shape[0], t.shape[1]
    out = np.empty((n_sweeps, 5))
    dp = C.POINTER(C.c_double)
    _check(lib().mmc_trace_stats(t.ctypes.data_as(dp), n_paths, n_sweeps, path_begin, path_stride,
                                 out.ctypes.data_as(dp)))
    return out


def mmc_distribution_coefficient(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = C.c_double()
    _check(lib().mmc_distribution_coefficient(x.ctypes.data_as(C.POINTER(C.c_double)), x.size, C.byref(r)))
    return r.value


def mmc_save(ctx, path):
    return _check(lib().mmc_save(ctx, path.encode()))


def mmc_load(path):
    return _ptr(lib().mmc_load(path.encode()))


def mmc_last_timing_ms(ctx):
    return lib().mmc_last_timing_ms(ctx)


def mmc_proposal_vectors(precision, proposal, words):
    """words: uint32 [n, 2] -> float64 [n, 3], the engine's proposed unit vectors."""
    import numpy as np
    w = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1, 2)
    out = np.empty((w.shape[0], 3))
    _check(lib().mmc_proposal_vectors(precision, proposal, w.ctypes.data_as(C.POINTER(C.c_uint32)), w.shape[0],
                                      out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def mmc_plan(ctx):
    buf = C.create_string_buffer(4096)
    _check(lib().mmc_plan(ctx, buf, 4096))
    return buf.value.decode()


def mmc_destroy(ctx):
    lib().mmc_destroy(ctx)


def mmc_batch_create(instances, seed, cfg=None):
    """instances: list of (L, T, J, n_paths, n_therm, n_meas)."""
    arr = (mmc_instance * len(instances))(*[mmc_instance(*x) for x in instances])
    return _ptr(lib().mmc_batch_create(arr, len(instances), seed, C.byref(cfg) if cfg else None))


def mmc_batch_run(ctx):
    return _check(lib().mmc_batch_run(ctx))


def mmc_batch_results(ctx, inst, n_paths):
    buf, ptr = _result_buffer(n_paths)
    _check(lib().mmc_batch_results(ctx, inst, ptr, n_paths))
    return _results_to_numpy(buf)


def mmc_batch_stats(ctx, inst):
    s = mmc_stats_t()
    _check(lib().mmc_batch_stats(ctx, inst, C.byref(s)))
    return _stats_dict(s)


def mmc_batch_run_static(instances, seed, cfg, out_dev, stream):
    """instances: list of (L, T, J, n_paths, n_therm, n_meas); out_dev: device address of
    sum(n_paths) mmc_path_result records; stream: HIP stream handle (0: null stream). Enqueues
    the run and returns."""
    arr = (mmc_instance * len(instances))(*[mmc_instance(*x) for x in instances])
    return _check(lib().mmc_batch_run_static(arr, len(instances), seed, C.byref(cfg) if cfg else None, out_dev,
                                             stream))


def path_results_from_bytes(raw, n):
    """n mmc_path_result records from a bytes-like host copy of device memory -> dict of arrays."""
    buf = np.frombuffer(bytes(raw[:n * RESULT_DTYPE.itemsize]), dtype=RESULT_DTYPE, count=n)
    return _results_to_numpy(buf)


# ---------------------------------------------------------------- torch-backed workspace
class Workspace:
    """Binds torch-owned device memory and the current torch stream to a context."""

    def __init__(self, ctx, device="cuda"):
        import torch
        nbytes = mmc_workspace_bytes(ctx)
        self.buf = torch.empty(max(nbytes, 256) + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.buf.device)
        mmc_bind(ctx, aligned, nbytes, self.stream.cuda_stream)
