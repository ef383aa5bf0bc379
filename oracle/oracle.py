"""Python face of the FP64 CPU oracle (ctypes over oracle/liboracle.so).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. It shares no code with the HIP engine.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

SWEEPS = {"checkerboard": 0, "random_site": 1, "typewriter": 2, "checkerboard_reversed": 3}
INITS = {"sphere": 0, "angles": 1, "ordered": 2, "mixed": 3}
PROPOSALS = {"sphere": 0, "angles": 1}
UNIFORMS = {"fp64": 0, "fp32": 1}  # (w + 1/2) 2^-32, or the FP32 engine's ((w >> 8) | 1) 2^-24


class Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("L", C.c_int), ("periodic", C.c_int), ("T", C.c_double),
                ("J", C.c_double), ("n_therm", C.c_int), ("n_meas", C.c_int),
                ("seed", C.c_uint64), ("instance", C.c_uint32), ("sweep", C.c_int),
                ("init", C.c_int), ("trace_sweeps", C.c_int), ("proposal", C.c_int), ("uniforms", C.c_int)]


class PathResult(C.Structure):
    _fields_ = [("e_mean", C.c_double), ("e2_mean", C.c_double), ("absm_mean", C.c_double),
                ("m2_mean", C.c_double), ("m4_mean", C.c_double), ("final_m", C.c_double * 3),
                ("final_e", C.c_double), ("n_accept", C.c_uint64)]


class State(C.Structure):
    _fields_ = [("spins", C.POINTER(C.c_double)), ("sweeps_done", C.c_int),
                ("sum_e", C.c_double), ("sum_e2", C.c_double), ("sum_m", C.c_double),
                ("sum_m2", C.c_double), ("sum_m4", C.c_double), ("n_accept", C.c_uint64)]


_lib = None


def lib():
    """Loads liboracle.so, building it first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        u32p = C.POINTER(C.c_uint32)
        i64p = C.POINTER(C.c_int64)
        L.mmco_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.mmco_philox_many.argtypes = [C.c_int64, u32p, u32p, u32p]
        L.mmco_uniform.argtypes = [C.c_uint32]
        L.mmco_uniform.restype = C.c_double
        L.mmco_uniform_fp32.argtypes = [C.c_uint32]
        L.mmco_uniform_fp32.restype = C.c_double
        L.mmco_unit_vectors.argtypes = [C.c_int64, u32p, C.c_int, C.c_int, dp]
        L.mmco_n_sites.argtypes = [C.POINTER(Params)]
        L.mmco_n_sites.restype = C.c_int64
        L.mmco_neighbors.argtypes = [C.POINTER(Params), C.c_int64, i64p]
        L.mmco_neighbors.restype = C.c_int
        L.mmco_colour.argtypes = [C.POINTER(Params), C.c_int64]
        L.mmco_colour.restype = C.c_int
        L.mmco_local_field.argtypes = [C.POINTER(Params), dp, C.c_int64, dp]
        L.mmco_energy.argtypes = [C.POINTER(Params), dp]
        L.mmco_energy.restype = C.c_double
        L.mmco_delta_e.argtypes = [C.POINTER(Params), dp, C.c_int64, dp]
        L.mmco_delta_e.restype = C.c_double
        L.mmco_unit_vector.argtypes = [C.c_uint32, C.c_uint32, C.c_int, dp]
        L.mmco_proposals.argtypes = [C.c_int64, C.c_uint64, dp]
        L.mmco_accept.argtypes = [C.c_double, C.c_double, C.c_double]
        L.mmco_accept.restype = C.c_int
        L.mmco_init_state.argtypes = [C.POINTER(Params), C.c_uint32, C.POINTER(State)]
        L.mmco_advance.argtypes = [C.POINTER(Params), C.c_uint32, C.c_int, C.POINTER(State), dp]
        L.mmco_finish.argtypes = [C.POINTER(Params), C.POINTER(State), C.POINTER(PathResult)]
        L.mmco_observe.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.mmco_run_paths.argtypes = [C.POINTER(Params), C.c_int, C.c_int, C.POINTER(PathResult),
                                     dp, dp, C.c_int]
        L.mmco_run_paths.restype = C.c_int
        L.mmco_max_threads.restype = C.c_int
        L.mmco_ising_init_spin.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint32, C.c_uint32, C.c_uint64]
        L.mmco_ising_init_spin.restype = C.c_int
        L.mmco_ising_accept.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                        C.c_double, C.c_double, C.c_int]
        L.mmco_ising_accept.restype = C.c_int
        L.mmco_ising_run_paths.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_uint64,
                                           C.c_uint32, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(PathResult),
                                           dp, C.POINTER(C.c_int8), C.c_int]
        L.mmco_ising_run_paths.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(L, T, J=1.0, n_therm=0, n_meas=0, seed=1234, instance=0, dim=3, periodic=True,
                sweep="checkerboard", init="sphere", trace_sweeps=0, proposal="sphere", uniforms="fp64"):
    return Params(dim, L, 1 if periodic else 0, float(T), float(J), n_therm, n_meas, seed,
                  instance, SWEEPS[sweep], INITS[init], trace_sweeps, PROPOSALS[proposal], UNIFORMS[uniforms])


def philox(ctr, key):
    """ctr uint32 [n,4], key uint32 [n,2] -> uint32 [n,4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(np.broadcast_to(np.asarray(key, dtype=np.uint32), (ctr.shape[0], 2)))
    out = np.empty_like(ctr)
    P = C.POINTER(C.c_uint32)
    lib().mmco_philox_many(ctr.shape[0], ctr.ctypes.data_as(P), key.ctypes.data_as(P),
                           out.ctypes.data_as(P))
    return out


def run_paths(L, T, J=1.0, n_therm=0, n_meas=0, seed=1234, path_begin=0, path_end=1, instance=0,
              dim=3, periodic=True, sweep="checkerboard", init="sphere", trace_sweeps=0,
              want_spins=False, n_threads=0, proposal="sphere", uniforms="fp64"):
    """Runs paths [path_begin, path_end) (uniforms "fp32": the FP32 engine's uniform grid, same
    words, FP64 arithmetic). Returns a dict of numpy arrays:
    e_mean, e2_mean, absm_mean, m2_mean, m4_mean [n]; final_m [n,3]; final_e [n];
    n_accept [n]; trace [n, trace_sweeps, 4] (e_k, Mx_k, My_k, Mz_k); spins [n, N, 3]."""
    p = make_params(L, T, J, n_therm, n_meas, seed, instance, dim, periodic, sweep, init,
                    trace_sweeps, proposal, uniforms)
    n = path_end - path_begin
    N = L ** dim
    res = (PathResult * n)()
    trace = np.zeros((n, trace_sweeps, 4)) if trace_sweeps > 0 else None
    spins = np.zeros((n, N, 3)) if want_spins else None
    rc = lib().mmco_run_paths(C.byref(p), path_begin, path_end, res,
                              _dp(trace) if trace is not None else None,
                              _dp(spins) if spins is not None else None, n_threads)
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    out = {k: np.array([getattr(r, k) for r in res]) for k in
           ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e", "n_accept")}
    out["final_m"] = np.array([list(r.final_m) for r in res]).reshape(n, 3)
    out["n_accept"] = out["n_accept"].astype(np.uint64)
    if trace is not None:
        out["trace"] = trace
    if spins is not None:
        out["spins"] = spins
    return out


def ising_run_paths(L, T, J=1.0, n_therm=0, n_meas=0, seed=1234, path_begin=0, path_end=1, instance=0,
                    init="sphere", trace_sweeps=0, want_spins=False, n_threads=0):
    """2-D Ising paths [path_begin, path_end) (init 'sphere' = random start). Same result keys as
    run_paths; final_m[:, 0] = M/N; trace [n, trace_sweeps, 4] = (e_k, m_k, 0, 0); spins [n, L*L]
    int8 in site-id order (x fastest)."""
    n = path_end - path_begin
    res = (PathResult * n)()
    trace = np.zeros((n, trace_sweeps, 4)) if trace_sweeps > 0 else None
    spins = np.zeros((n, L * L), dtype=np.int8) if want_spins else None
    rc = lib().mmco_ising_run_paths(L, float(T), float(J), n_therm, n_meas, seed, instance, INITS[init], path_begin,
                                    path_end, trace_sweeps, res, _dp(trace) if trace is not None else None,
                                    spins.ctypes.data_as(C.POINTER(C.c_int8)) if spins is not None else None,
                                    n_threads)
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    out = {k: np.array([getattr(r, k) for r in res]) for k in
           ("e_mean", "e2_mean", "absm_mean", "m2_mean", "m4_mean", "final_e", "n_accept")}
    out["final_m"] = np.array([list(r.final_m) for r in res]).reshape(n, 3)
    out["n_accept"] = out["n_accept"].astype(np.uint64)
    if trace is not None:
        out["trace"] = trace
    if spins is not None:
        out["spins"] = spins
    return out


class PathState:
    """Stepwise path (init, advance to a sweep, finish) -- for resume checks."""

    def __init__(self, params, path):
        self.p = params
        self.path = path
        self.N = lib().mmco_n_sites(C.byref(params))
        self.spins = np.zeros((self.N, 3))
        self.st = State()
        self.st.spins = _dp(self.spins)
        lib().mmco_init_state(C.byref(self.p), path, C.byref(self.st))

    def advance(self, k_end, trace=None):
        lib().mmco_advance(C.byref(self.p), self.path, k_end, C.byref(self.st),
                           _dp(trace) if trace is not None else None)

    def result(self):
        r = PathResult()
        lib().mmco_finish(C.byref(self.p), C.byref(self.st), C.byref(r))
        return r


def neighbors(params, i):
    out = (C.c_int64 * 6)()
    k = lib().mmco_neighbors(C.byref(params), i, out)
    return list(out)[:k]


def energy(params, spins):
    s = np.ascontiguousarray(spins, dtype=np.float64)
    return lib().mmco_energy(C.byref(params), _dp(s))


def delta_e(params, spins, i, snew):
    s = np.ascontiguousarray(spins, dtype=np.float64)
    sn = np.ascontiguousarray(snew, dtype=np.float64)
    return lib().mmco_delta_e(C.byref(params), _dp(s), i, _dp(sn))


def proposals(n, seed):
    out = np.zeros((n, 3))
    lib().mmco_proposals(n, seed, _dp(out))
    return out


def unit_vector(w0, w1, mode="sphere"):
    out = np.zeros(3)
    lib().mmco_unit_vector(w0, w1, INITS[mode], _dp(out))
    return out


def unit_vectors(words, mode="sphere", uniforms="fp64"):
    """Unit vectors of word pairs words[t] = (w0, w1) -> [n, 3], on either uniform grid."""
    w = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros((w.shape[0], 3))
    lib().mmco_unit_vectors(w.shape[0], w.ctypes.data_as(C.POINTER(C.c_uint32)), INITS[mode], UNIFORMS[uniforms],
                            _dp(out))
    return out


def uniform_fp32(w):
    return lib().mmco_uniform_fp32(w)


def max_threads():
    return lib().mmco_max_threads()
