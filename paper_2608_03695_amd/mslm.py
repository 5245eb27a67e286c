"""Thin ctypes binding of libmslm.so (argument marshalling only; all work runs in HIP).

Names follow the C ABI in include/mslm.h.  The library must have been built in-tree
(``paper_2608_03695_amd/build.py``); importing this module on a machine without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from fractions import Fraction
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmslm.so")

MSLM_OK, MSLM_EINVAL, MSLM_ENOMEM, MSLM_EOVERFLOW, MSLM_EUNSUPPORTED, MSLM_EHIP, MSLM_EBUSY = \
    0, -1, -2, -3, -4, -5, -6
MSLM_INPUT_ON_DEVICE, MSLM_OUTPUT_ON_DEVICE, MSLM_PROFILE, MSLM_COUNT = 1, 2, 4, 8
MSLM_COUPLE_PRESENT = 16
MSLM_NULL_MULTISLICE, MSLM_NULL_GLOBAL, MSLM_NULL_CPM = 0, 1, 2

EXPORTED = ["mslm_create", "mslm_leiden", "mslm_destroy", "mslm_q_exact", "mslm_q_exact_global",
            "mslm_q_exact_variant", "mslm_footprint_bytes",
            "mslm_graph_info", "mslm_last_error", "mslm_set_allocator", "mslm_leiden_static",
            "mslm_batch_leiden", "mslm_get_tuning", "mslm_set_tuning", "mslm_autotune",
            "mslm_server_create", "mslm_server_submit", "mslm_server_wait",
            "mslm_server_memory", "mslm_server_destroy", "mslm_bethe_hessian", "mslm_bh_apply",
            "mslm_kmeans", "mslm_leiden_windowed"]


_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_RELEASE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_allocators = []   # every installed callback pair stays alive: buffers release through theirs


class MslmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mslm status {status}: {msg}")
        self.status = status


class GraphDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_slices", C.c_int32),
                ("slice_offsets", C.c_void_p), ("src", C.c_void_p), ("dst", C.c_void_p),
                ("weight", C.c_void_p), ("omega_num", C.c_int64), ("omega_den", C.c_int64),
                ("flags", C.c_uint32), ("coupling", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("gamma_num", C.c_int64), ("gamma_den", C.c_int64),
                ("omega_num", C.c_int64), ("omega_den", C.c_int64),
                ("max_levels", C.c_int32), ("max_iterations", C.c_int32),
                ("max_sweeps", C.c_int32), ("null_model", C.c_int32),
                ("seed", C.c_uint64), ("flags", C.c_uint32), ("reserved1", C.c_uint32),
                ("gamma_slices", C.c_void_p), ("initial_membership", C.c_void_p)]


class Tuning(C.Structure):
    """mslm_tuning: execution choices that never change a result."""
    _fields_ = [("graphs", C.c_int32), ("latency_units", C.c_int32),
                ("split_group_units", C.c_int32), ("copy_moves", C.c_int32),
                ("lat_parts_max", C.c_int32), ("batch_units", C.c_int32),
                ("reserved", C.c_int32 * 2)]
    KEYS = ["graphs", "latency_units", "split_group_units", "copy_moves", "lat_parts_max",
            "batch_units"]

    def as_dict(self):
        return {k: getattr(self, k) for k in self.KEYS}


class Result(C.Structure):
    _fields_ = [("q", C.c_double), ("n_communities", C.c_int32), ("levels_run", C.c_int32),
                ("iterations_run", C.c_int32), ("colours_level0", C.c_int32),
                ("sweeps", C.c_int64), ("moves", C.c_int64), ("sweep_cap_hits", C.c_int64),
                ("refine_rounds", C.c_int64), ("merges", C.c_int64), ("splits", C.c_int64),
                ("exact_fallbacks", C.c_int64), ("ms_total", C.c_double),
                ("ms_colour", C.c_double), ("ms_local_move", C.c_double),
                ("ms_refine", C.c_double), ("ms_aggregate", C.c_double),
                ("ms_finish", C.c_double), ("lm_kernel_ms", C.c_double),
                ("lm_launches", C.c_int64), ("lm_units", C.c_int64), ("lm_entries", C.c_int64),
                ("lm_candidates", C.c_int64), ("q_components", C.c_int64 * (3 * 64 + 1)),
                ("lm0_kernel_ms", C.c_double), ("lm0_launches", C.c_int64),
                ("lm0_units", C.c_int64), ("lm0_entries", C.c_int64),
                ("lm0_candidates", C.c_int64), ("coupling_total", C.c_int64)]

    def as_dict(self, n_slices):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "q_components"}
        d["q_components"] = np.array(self.q_components[:3 * n_slices + 1], dtype=np.int64)
        return d


class SpectralParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("lanczos_steps", C.c_int32),
                ("kmeans_iterations", C.c_int32), ("reserved", C.c_int32), ("r", C.c_double),
                ("omega_num", C.c_int64), ("omega_den", C.c_int64), ("seed", C.c_uint64)]


class SpectralResult(C.Structure):
    _fields_ = [("r", C.c_double), ("residual_max", C.c_double), ("lanczos_steps", C.c_int32),
                ("tridiagonal_steps", C.c_int32), ("kmeans_iterations", C.c_int32),
                ("second_passes", C.c_int32), ("spmv_ms", C.c_double), ("spmv_launches", C.c_int64),
                ("ms_total", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class WindowResult(C.Structure):
    _fields_ = [("windows", C.c_int32), ("n_communities", C.c_int32), ("ms_total", C.c_double)]


class Solve(C.Structure):
    _fields_ = [("graph", C.c_int32), ("reserved", C.c_int32), ("params", Params),
                ("membership", C.c_void_p), ("result", C.c_void_p)]


_lib = None


def load():
    """Load the in-tree HIP library; raise when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2608_03695_amd/build.py")
    # PyTorch carries its own HIP runtime beside the system one this library links; torch's
    # did not come up on a device the library's runtime had already brought up in the same
    # process, so torch is brought up first whenever it is importable and sees a GPU
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.mslm_create.argtypes = [C.POINTER(GraphDesc), P, C.POINTER(C.c_void_p)]
    lib.mslm_create.restype = C.c_int
    lib.mslm_leiden.argtypes = [P, C.POINTER(Params), P, C.POINTER(Result)]
    lib.mslm_leiden.restype = C.c_int
    lib.mslm_leiden_static.argtypes = [P, C.POINTER(Params), P, C.POINTER(Result)]
    lib.mslm_leiden_static.restype = C.c_int
    lib.mslm_destroy.argtypes = [P]
    lib.mslm_destroy.restype = None
    lib.mslm_q_exact.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.c_int64,
                                 C.c_int64, C.c_char_p, C.c_size_t, C.c_char_p, C.c_size_t]
    lib.mslm_q_exact.restype = C.c_int
    lib.mslm_q_exact_global.argtypes = lib.mslm_q_exact.argtypes
    lib.mslm_q_exact_global.restype = C.c_int
    lib.mslm_q_exact_variant.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, C.c_int64,
                                         C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_char_p,
                                         C.c_size_t, C.c_char_p, C.c_size_t]
    lib.mslm_q_exact_variant.restype = C.c_int
    lib.mslm_get_tuning.argtypes = [P, C.POINTER(Tuning)]
    lib.mslm_get_tuning.restype = C.c_int
    lib.mslm_set_tuning.argtypes = [P, C.POINTER(Tuning)]
    lib.mslm_set_tuning.restype = C.c_int
    lib.mslm_autotune.argtypes = [P, C.POINTER(Params), C.c_int32, C.POINTER(Tuning),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.mslm_autotune.restype = C.c_int
    lib.mslm_footprint_bytes.argtypes = [C.POINTER(GraphDesc)]
    lib.mslm_footprint_bytes.restype = C.c_size_t
    lib.mslm_graph_info.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]
    lib.mslm_graph_info.restype = C.c_int
    lib.mslm_last_error.restype = C.c_char_p
    lib.mslm_batch_leiden.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Solve),
                                      C.c_int32, P]
    lib.mslm_batch_leiden.restype = C.c_int
    lib.mslm_set_allocator.argtypes = [_ALLOC_T, _RELEASE_T, P]
    lib.mslm_set_allocator.restype = C.c_int
    lib.mslm_server_create.argtypes = [C.c_size_t, C.c_int32, P, C.POINTER(C.c_void_p)]
    lib.mslm_server_create.restype = C.c_int
    lib.mslm_server_submit.argtypes = [P, C.POINTER(GraphDesc), C.POINTER(Params),
                                       C.POINTER(C.c_uint64)]
    lib.mslm_server_submit.restype = C.c_int
    lib.mslm_server_wait.argtypes = [P, C.c_uint64, C.c_int32, P, C.POINTER(Result),
                                     C.POINTER(C.c_double)]
    lib.mslm_server_wait.restype = C.c_int
    lib.mslm_server_memory.argtypes = [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                       C.POINTER(C.c_size_t)]
    lib.mslm_server_memory.restype = C.c_int
    lib.mslm_server_destroy.argtypes = [P]
    lib.mslm_server_destroy.restype = None
    lib.mslm_bethe_hessian.argtypes = [P, C.POINTER(SpectralParams), P, P, P,
                                       C.POINTER(SpectralResult)]
    lib.mslm_bethe_hessian.restype = C.c_int
    lib.mslm_bh_apply.argtypes = [P, C.c_double, C.c_int64, C.c_int64, P, P]
    lib.mslm_bh_apply.restype = C.c_int
    lib.mslm_kmeans.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, P, P,
                                C.POINTER(C.c_int32), P]
    lib.mslm_kmeans.restype = C.c_int
    lib.mslm_leiden_windowed.argtypes = [C.POINTER(GraphDesc), C.POINTER(Params), C.c_int32,
                                         C.c_int32, P, P, C.POINTER(WindowResult)]
    lib.mslm_leiden_windowed.restype = C.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != MSLM_OK:
        raise MslmError(rc, load().mslm_last_error().decode())


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _desc(tg, omega, coupling=None, present_only=False):
    """mslm_graph_desc of a temporal graph; coupling: T x T integer matrix c_sr (omega^(sr) =
    omega * c_sr; None: ordinal); present_only: couple only copies with an edge."""
    omega = Fraction(omega)
    keep = [np.ascontiguousarray(tg.offsets, dtype=np.int64),
            np.ascontiguousarray(tg.src, dtype=np.int32),
            np.ascontiguousarray(tg.dst, dtype=np.int32),
            None if tg.weight is None else np.ascontiguousarray(tg.weight, dtype=np.int32),
            None if coupling is None else np.ascontiguousarray(coupling, dtype=np.int32)]
    d = GraphDesc(tg.n_nodes, tg.n_slices, keep[0].ctypes.data, keep[1].ctypes.data,
                  keep[2].ctypes.data, None if keep[3] is None else keep[3].ctypes.data,
                  omega.numerator, omega.denominator,
                  MSLM_COUPLE_PRESENT if present_only else 0,
                  None if keep[4] is None else keep[4].ctypes.data)
    return d, keep


def _slices_array(gamma_slices):
    if gamma_slices is None:
        return None
    return np.array([[Fraction(x).numerator, Fraction(x).denominator] for x in gamma_slices],
                    dtype=np.int64).ravel()


def params(gamma=Fraction(1), omega=None, max_levels=32, max_iterations=2, max_sweeps=0, seed=0,
           flags=0, null_model=MSLM_NULL_MULTISLICE, gamma_slices=None, initial=None):
    """(Params, arrays its pointers refer to): keep the second alive for the call."""
    gamma = Fraction(gamma)
    if omega is None:
        on, od = 0, 0
    else:
        omega = Fraction(omega)
        on, od = omega.numerator, omega.denominator
    keep = [_slices_array(gamma_slices),
            None if initial is None else np.ascontiguousarray(initial, dtype=np.int32)]
    p = Params(gamma.numerator, gamma.denominator, on, od, max_levels, max_iterations,
               max_sweeps, null_model, seed, flags, 0,
               None if keep[0] is None else keep[0].ctypes.data,
               None if keep[1] is None else keep[1].ctypes.data)
    return p, keep


def stream_handle(stream=None):
    """hipStream_t of a torch stream (torch.cuda.Stream on ROCm), or None for the default."""
    if stream is None:
        return None
    return C.c_void_p(int(stream.cuda_stream))


class Graph:
    """A temporal graph resident on the device (mslm_create / mslm_destroy)."""

    def __init__(self, tg, omega=Fraction(1), stream=None, coupling=None, present_only=False):
        lib = load()
        self.n_nodes, self.n_slices = tg.n_nodes, tg.n_slices
        self.omega = Fraction(omega)
        d, keep = _desc(tg, omega, coupling, present_only)
        h = C.c_void_p()
        _check(lib.mslm_create(C.byref(d), stream_handle(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().mslm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tuning(self):
        t = Tuning()
        _check(load().mslm_get_tuning(self._h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Change execution choices (mslm_tuning fields by name); results never change."""
        t = Tuning()
        _check(load().mslm_get_tuning(self._h, C.byref(t)))
        for k, v in kw.items():
            if k not in Tuning.KEYS:
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(load().mslm_set_tuning(self._h, C.byref(t)))

    def autotune(self, gamma=Fraction(1), omega=None, rounds=1, max_levels=32,
                 max_iterations=2, seed=0, null_model=MSLM_NULL_MULTISLICE):
        """mslm_autotune: returns (chosen tuning dict, ms with the starting tuning, ms tuned)."""
        p, keep = params(gamma, omega, max_levels, max_iterations, 0, seed, 0, null_model)
        t = Tuning()
        a, b = C.c_double(), C.c_double()
        _check(load().mslm_autotune(self._h, C.byref(p), int(rounds), C.byref(t), C.byref(a),
                                    C.byref(b)))
        return t.as_dict(), a.value, b.value

    def info(self):
        n, m, t = C.c_int64(), C.c_int64(), C.c_int64()
        _check(load().mslm_graph_info(self._h, C.byref(n), C.byref(m), C.byref(t)))
        return dict(n_supra=n.value, nnz=m.value, two_m=t.value)

    def leiden(self, gamma=Fraction(1), omega=None, max_levels=32, max_iterations=2, max_sweeps=0,
               seed=0, profile=False, count=False, out=None, no_alloc=False,
               null_model=MSLM_NULL_MULTISLICE, gamma_slices=None, initial=None):
        """Returns (membership int32[T*N], result dict).  `out` may be a device tensor
        (torch, int32, T*N elements) to receive the membership on the device.  no_alloc
        calls the allocation-free entry point (mslm_leiden_static).  null_model selects
        Q_MS (Eq. 6, the default), the global modularity of the supra-graph (Eq. 5) or the
        multislice CPM; gamma_slices gives T per-slice resolutions in place of gamma; initial
        is a start partition (T*N labels in [0, T*N))."""
        lib = load()
        flags = (MSLM_PROFILE if profile else 0) | (MSLM_COUNT if count else 0)
        if out is not None:
            flags |= MSLM_OUTPUT_ON_DEVICE
            dest = C.c_void_p(int(out.data_ptr()))
            memb = None
        else:
            memb = np.empty(self.n_nodes * self.n_slices, dtype=np.int32)
            dest = _ptr(memb)
        p, keep = params(gamma, omega, max_levels, max_iterations, max_sweeps, seed, flags,
                         null_model, gamma_slices, initial)
        res = Result()
        entry = lib.mslm_leiden_static if no_alloc else lib.mslm_leiden
        _check(entry(self._h, C.byref(p), dest, C.byref(res)))
        return memb, res.as_dict(self.n_slices)


def _graph_bethe_hessian(self, k, r=0.0, lanczos_steps=0, kmeans_iterations=0, omega=None,
                        seed=0, embedding=True, labels=True):
    """The Bethe-Hessian pathway (mslm_bethe_hessian): (eigenvalues[k], embedding n x k or
    None, labels n or None, result dict)."""
    n = self.n_nodes * self.n_slices
    if omega is None:
        on, od = 0, 0
    else:
        omega = Fraction(omega)
        on, od = omega.numerator, omega.denominator
    p = SpectralParams(int(k), int(lanczos_steps), int(kmeans_iterations), 0, float(r), on, od,
                       int(seed))
    ev = np.zeros(int(k), np.float64)
    emb = np.zeros((n, int(k)), np.float64) if embedding else None
    lab = np.zeros(n, np.int32) if labels else None
    res = SpectralResult()
    _check(load().mslm_bethe_hessian(self._h, C.byref(p), _ptr(ev), _ptr(emb), _ptr(lab),
                                     C.byref(res)))
    return ev, emb, lab, res.as_dict()


def _graph_bh_apply(self, x, r, omega=None):
    """y = H(r) x (mslm_bh_apply)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    on, od = (0, 0) if omega is None else (Fraction(omega).numerator, Fraction(omega).denominator)
    _check(load().mslm_bh_apply(self._h, float(r), on, od, _ptr(x), _ptr(y)))
    return y


Graph.bethe_hessian = _graph_bethe_hessian
Graph.bh_apply = _graph_bh_apply


def kmeans(points, k, max_iterations=0, stream=None):
    """The pathway's deterministic k-means (mslm_kmeans): (labels, centroids, iterations)."""
    P = np.ascontiguousarray(points, dtype=np.float64)
    n, dim = P.shape
    lab = np.zeros(n, np.int32)
    cen = np.zeros((int(k), dim), np.float64)
    it = C.c_int32()
    _check(load().mslm_kmeans(_ptr(P), n, dim, int(k), int(max_iterations), _ptr(lab), _ptr(cen),
                              C.byref(it), stream_handle(stream)))
    return lab, cen, it.value


def leiden_windowed(tg, omega, window, overlap, gamma=Fraction(1), max_levels=32,
                    max_iterations=2, seed=0, null_model=MSLM_NULL_MULTISLICE, gamma_slices=None,
                    present_only=False, stream=None):
    """Windowed optimisation of a sequence of any length (mslm_leiden_windowed):
    (membership int32[T*N], {"windows", "n_communities", "ms_total"})."""
    d, keep = _desc(tg, omega, None, present_only)
    p, pkeep = params(gamma, None, max_levels, max_iterations, 0, seed, 0, null_model,
                      gamma_slices)
    memb = np.empty(tg.n_nodes * tg.n_slices, dtype=np.int32)
    res = WindowResult()
    _check(load().mslm_leiden_windowed(C.byref(d), C.byref(p), int(window), int(overlap),
                                       stream_handle(stream), _ptr(memb), C.byref(res)))
    return memb, {k: getattr(res, k) for k, _ in res._fields_}


def q_exact(components, n_slices, n_nodes, gamma, omega) -> Fraction:
    """Exact Q (Eq. 6) from the 3T+1 integer components, via the library's reduction."""
    lib = load()
    gamma, omega = Fraction(gamma), Fraction(omega)
    comps = np.ascontiguousarray(components, dtype=np.int64)
    num = C.create_string_buffer(4096)
    den = C.create_string_buffer(4096)
    _check(lib.mslm_q_exact(_ptr(comps), n_slices, n_nodes, gamma.numerator, gamma.denominator,
                            omega.numerator, omega.denominator, num, 4096, den, 4096))
    return Fraction(int(num.value.decode()), int(den.value.decode()))


def q_exact_global(components, n_slices, n_nodes, gamma, omega) -> Fraction:
    """Exact global modularity of the supra-graph (Eq. 5) from a global-null-model solve's
    components, via the library's reduction."""
    lib = load()
    gamma, omega = Fraction(gamma), Fraction(omega)
    comps = np.ascontiguousarray(components, dtype=np.int64)
    num = C.create_string_buffer(4096)
    den = C.create_string_buffer(4096)
    _check(lib.mslm_q_exact_global(_ptr(comps), n_slices, n_nodes, gamma.numerator,
                                   gamma.denominator, omega.numerator, omega.denominator, num,
                                   4096, den, 4096))
    return Fraction(int(num.value.decode()), int(den.value.decode()))


def q_exact_variant(components, n_slices, n_nodes, gamma, omega, null_model=MSLM_NULL_MULTISLICE,
                    gamma_slices=None, coupling_total=None) -> Fraction:
    """Exact value of any objective (Eq. 6 with per-slice resolutions, the global null model,
    the multislice CPM) from a solve's components, via the library's reduction; coupling_total
    is the graph's (a result's "coupling_total"; None: the ordinal coupling of every copy)."""
    lib = load()
    gamma, omega = Fraction(gamma), Fraction(omega)
    comps = np.ascontiguousarray(components, dtype=np.int64)
    gs = _slices_array(gamma_slices)
    num = C.create_string_buffer(1 << 16)
    den = C.create_string_buffer(1 << 16)
    _check(lib.mslm_q_exact_variant(_ptr(comps), n_slices, n_nodes, null_model, _ptr(gs),
                                    gamma.numerator, gamma.denominator, omega.numerator,
                                    omega.denominator,
                                    -1 if coupling_total is None else int(coupling_total),
                                    num, 1 << 16, den, 1 << 16))
    return Fraction(int(num.value.decode()), int(den.value.decode()))


def footprint_bytes(tg, omega=Fraction(1), coupling=None) -> int:
    d, keep = _desc(tg, omega, coupling)
    return int(load().mslm_footprint_bytes(C.byref(d)))


def use_torch_allocator(device=None):
    """Route the library's device allocations through PyTorch's caching allocator
    (mslm_set_allocator with torch.cuda.caching_allocator_alloc / _delete)."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev)
        except RuntimeError:
            return None

    def release(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    pair = (_ALLOC_T(alloc), _RELEASE_T(release))
    _allocators.append(pair)
    _check(load().mslm_set_allocator(pair[0], pair[1], None))


def use_hip_allocator():
    """Back to hipMalloc / hipFree for new buffers."""
    _check(load().mslm_set_allocator(_ALLOC_T(), _RELEASE_T(), None))


class Server:
    """Continuous-batching request loop (mslm_server_*): submit() copies the graph and
    returns a ticket; wait() returns (membership, result dict, latency seconds)."""

    def __init__(self, hbm_budget_bytes, max_slots=4, stream=None):
        lib = load()
        h = C.c_void_p()
        _check(lib.mslm_server_create(int(hbm_budget_bytes), int(max_slots), stream_handle(stream),
                                      C.byref(h)))
        self._h = h
        self._shape = {}

    def submit(self, tg, gamma=Fraction(1), omega=Fraction(1), max_levels=32, max_iterations=2,
               seed=0, null_model=MSLM_NULL_MULTISLICE, gamma_slices=None, initial=None,
               coupling=None, present_only=False) -> int:
        d, keep = _desc(tg, omega, coupling, present_only)
        p, pkeep = params(gamma, None, max_levels, max_iterations, 0, seed, 0, null_model,
                          gamma_slices, initial)
        t = C.c_uint64()
        _check(load().mslm_server_submit(self._h, C.byref(d), C.byref(p), C.byref(t)))
        self._shape[t.value] = (tg.n_nodes, tg.n_slices)
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        n_nodes, n_slices = self._shape.get(ticket, (0, 1))   # unknown: the library says so
        memb = np.empty(n_nodes * n_slices, dtype=np.int32)
        res = Result()
        lat = C.c_double()
        _check(load().mslm_server_wait(self._h, C.c_uint64(ticket), int(timeout_ms), _ptr(memb),
                                       C.byref(res), C.byref(lat)))
        self._shape.pop(ticket, None)
        return memb, res.as_dict(n_slices), lat.value

    def memory(self):
        """(bytes the slots hold, peak held, peak charged against the budget)."""
        a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(load().mslm_server_memory(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None):
            load().mslm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_leiden(graphs: Sequence[Graph], solves, stream=None):
    """solves: list of (graph index, gamma, omega, max_levels, max_iterations, seed) with
    optional further items: the null model, the per-slice resolutions, a start partition.
    Returns a list of (membership, result dict), bit-identical to plain calls."""
    lib = load()
    arr = (C.c_void_p * len(graphs))(*[g._h for g in graphs])
    cs = (Solve * len(solves))()
    outs = []
    keep = []
    for i, sv in enumerate(solves):
        gi, gamma, omega, levels, iters, seed = sv[:6]
        null_model = sv[6] if len(sv) > 6 else MSLM_NULL_MULTISLICE
        gamma_slices = sv[7] if len(sv) > 7 else None
        initial = sv[8] if len(sv) > 8 else None
        g = graphs[gi]
        memb = np.empty(g.n_nodes * g.n_slices, dtype=np.int32)
        res = Result()
        outs.append((memb, res, g.n_slices))
        cs[i].graph = gi
        p, pkeep = params(gamma, omega, levels, iters, 0, seed, 0, null_model, gamma_slices,
                          initial)
        keep.append(pkeep)
        cs[i].params = p
        cs[i].membership = memb.ctypes.data
        cs[i].result = C.addressof(res)
    _check(lib.mslm_batch_leiden(arr, len(graphs), cs, len(solves), stream_handle(stream)))
    return [(m, r.as_dict(t)) for m, r, t in outs]
