"""Oracle for the multislice-modularity Leiden path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU baseline import this package.
It holds two tiers that share no code with the HIP library:

* ``oracle.definitional``: Eq. 6 and Eq. 3 written out in exact rationals for tiny inputs.
* ``mslm_oracle.c`` (wrapped here): the complete deterministic schedule in plain C with its
  own exact arithmetic, fast enough for the parity workloads.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mslm_oracle.c")
_LIB_PATH = os.environ.get("MSLM_ORACLE_LIB") or os.path.join(_HERE, "libmslm_oracle.so")
_SHA_PATH = _LIB_PATH + ".sha256"
_lib = None


def _source_sha() -> str:
    with open(_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP inside a colour batch; results do not depend on it).
    The sha256 of the source is written beside the library, so a stale build is detected."""
    if force or not _is_current():
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
        with open(_SHA_PATH, "w") as fh:
            fh.write(_source_sha() + "\n")
    return _LIB_PATH


def _is_current() -> bool:
    if not (os.path.exists(_LIB_PATH) and os.path.exists(_SHA_PATH)):
        return False
    with open(_SHA_PATH) as fh:
        return fh.read().strip() == _source_sha()


class Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("moves", C.c_int64), ("sweep_cap_hits", C.c_int64),
                ("refine_rounds", C.c_int64), ("merges", C.c_int64), ("splits", C.c_int64),
                ("levels_run", C.c_int32), ("iterations_run", C.c_int32),
                ("n_communities", C.c_int32), ("colours_first", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # never compiles here: a process that already drives the GPU must not start a compiler
    # (build() and the test session's start do that); a missing or stale library is an error
    if os.environ.get("MSLM_ORACLE_LIB") is None and not _is_current():
        raise RuntimeError(f"oracle library {_LIB_PATH} is missing or older than its source; "
                           "run oracle.build() (or __graft_entry__.build()) first")
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    lib.orc_create.argtypes = [C.c_int32, C.c_int32, P, P, P, P, C.c_int64, C.c_int64, P,
                               C.c_int32, C.POINTER(C.c_void_p)]
    lib.orc_create.restype = C.c_int
    lib.orc_destroy.argtypes = [P]
    lib.orc_nnz.argtypes = [P]
    lib.orc_nnz.restype = C.c_int64
    lib.orc_coupling_total.argtypes = [P]
    lib.orc_coupling_total.restype = C.c_int64
    lib.orc_csr.argtypes = [P, P, P, P, P, P]
    lib.orc_leiden.argtypes = [P, C.c_int64, C.c_int64, P, P, C.c_int32, C.c_int32, C.c_int32,
                               C.c_uint64, C.c_int32, P, P, C.POINTER(Stats)]
    lib.orc_leiden.restype = C.c_int
    lib.orc_q_components.argtypes = [P, P, P]
    lib.orc_q_components_global.argtypes = [P, P, P]
    lib.orc_q_components_cpm.argtypes = [P, P, P]
    lib.orc_mix64.argtypes = [C.c_uint64]
    lib.orc_mix64.restype = C.c_uint64
    lib.orc_priority.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_uint32]
    lib.orc_priority.restype = C.c_uint64
    lib.orc_gain_sign.argtypes = [C.c_int64, C.c_int64, C.c_int64, P, C.c_int64, C.c_int, P, P, P]
    lib.orc_gain_sign.restype = C.c_int
    lib.orc_trace_enable.argtypes = [C.c_int]
    lib.orc_trace_count.restype = C.c_int
    lib.orc_trace_info.argtypes = [C.c_int, P]
    lib.orc_trace_get.argtypes = [C.c_int] + [P] * 11 + [C.c_int64]
    lib.orc_trace_refine.argtypes = [C.c_int, P, P]
    lib.orc_num_threads.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def mix64(z: int) -> int:
    return int(_load().orc_mix64(C.c_uint64(z & (2 ** 64 - 1))))


def priority(seed, it, lvl, phase, v) -> int:
    return int(_load().orc_priority(seed, it, lvl, phase, v))


def gain_sign(p, q, b, S, W, slices, k, y) -> int:
    """Sign of q*W*Pi - p*b*sum_j k_j*y_j*Pi/S_{s_j}, Pi = prod_j S_{s_j} (exact)."""
    S = np.ascontiguousarray(S, dtype=np.int64)
    sl = np.ascontiguousarray(slices, dtype=np.int32)
    kk = np.ascontiguousarray(k, dtype=np.int64)
    yy = np.ascontiguousarray(y, dtype=np.int64)
    return int(_load().orc_gain_sign(p, q, b, _ptr(S), W, len(sl), _ptr(sl), _ptr(kk), _ptr(yy)))


class OracleGraph:
    """Level-0 supra-graph held by the C oracle for one coupling omega: ordinal by default,
    else omega^(sr) = omega * coupling[s][r] (a T x T integer matrix), optionally only between
    copies present in both slices."""

    def __init__(self, g, omega, coupling=None, present_only=False):
        lib = _load()
        omega = Fraction(omega)
        self.g = g
        self.omega = omega
        self._keep = [np.ascontiguousarray(g.offsets, dtype=np.int64),
                      np.ascontiguousarray(g.src, dtype=np.int32),
                      np.ascontiguousarray(g.dst, dtype=np.int32),
                      None if g.weight is None else np.ascontiguousarray(g.weight, dtype=np.int32)]
        self._cm = None if coupling is None else np.ascontiguousarray(coupling, dtype=np.int32)
        h = C.c_void_p()
        rc = lib.orc_create(g.n_nodes, g.n_slices, *[_ptr(a) for a in self._keep],
                            omega.numerator, omega.denominator, _ptr(self._cm),
                            1 if present_only else 0, C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle create failed: {rc}")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            _load().orc_destroy(self._h)
            self._h = None

    def coupling_total(self) -> int:
        """Sum of c_sr over the ordered coupled copy pairs (2mu = sum 2m_s + omega * this)."""
        return int(_load().orc_coupling_total(self._h))

    def csr(self):
        lib = _load()
        n = self.g.n_supra
        m = int(lib.orc_nnz(self._h))
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(m, np.int32)
        w = np.zeros(m, np.int64)
        raw = np.zeros(m, np.int32)
        twom = np.zeros(self.g.n_slices, np.int64)
        lib.orc_csr(self._h, _ptr(rp), _ptr(col), _ptr(w), _ptr(raw), _ptr(twom))
        return rp, col, w, raw, twom

    def leiden(self, gamma=Fraction(1), max_levels=32, max_iterations=2, max_sweeps=0, seed=0,
               null_model=0, gamma_slices=None, initial=None):
        """null_model 0: the multislice modularity of Eq. 6 (per-slice null model);
        1: the global modularity of the supra-graph (Eq. 5 over all supra-nodes); 2: the
        multislice CPM.  gamma_slices: T per-slice resolutions gamma^(s) (> 0) in place of
        gamma; initial: the first iteration's start partition (N*T labels in [0, N*T))."""
        lib = _load()
        gamma = Fraction(gamma)
        memb = np.zeros(self.g.n_supra, np.int32)
        comps = np.zeros(3 * self.g.n_slices + 1, np.int64)
        st = Stats()
        gs = None
        if gamma_slices is not None:
            gs = np.array([[Fraction(x).numerator, Fraction(x).denominator]
                           for x in gamma_slices], dtype=np.int64).ravel()
        ini = None if initial is None else np.ascontiguousarray(initial, dtype=np.int32)
        rc = lib.orc_leiden(self._h, gamma.numerator, gamma.denominator, _ptr(gs), _ptr(ini),
                            max_levels, max_iterations, max_sweeps, seed, null_model, _ptr(memb),
                            _ptr(comps), C.byref(st))
        if rc != 0:
            raise ValueError(f"oracle leiden failed: {rc}")
        return memb, comps, st.as_dict()

    def q_components(self, membership, null_model=0):
        memb = np.ascontiguousarray(membership, dtype=np.int32)
        comps = np.zeros(3 * self.g.n_slices + 1, np.int64)
        lib = _load()
        fn = {0: lib.orc_q_components, 1: lib.orc_q_components_global,
              2: lib.orc_q_components_cpm}[null_model]
        fn(self._h, _ptr(memb), _ptr(comps))
        return comps


def _per_slice(gamma, T):
    if isinstance(gamma, (list, tuple, np.ndarray)):
        assert len(gamma) == T
        return [Fraction(x) for x in gamma]
    return [Fraction(gamma)] * T


def _coupled(n_nodes, n_slices, coupling_total):
    return 2 * n_nodes * (n_slices - 1) if coupling_total is None else int(coupling_total)


def q_from_components(comps, n_nodes, n_slices, gamma, omega, coupling_total=None) -> Fraction:
    """Q = (sum_s [W_s - gamma^(s) SS_s / 2m_s] + omega I) / (sum_s 2m_s + omega Ctot);
    gamma: one resolution or T per-slice resolutions; Ctot: the coupling total of the graph
    (None: 2 N (T-1), every copy coupled ordinally)."""
    T = n_slices
    gam, omega = _per_slice(gamma, T), Fraction(omega)
    W, SS, tm, I = comps[:T], comps[T:2 * T], comps[2 * T:3 * T], comps[3 * T]
    num = Fraction(0)
    for s in range(T):
        num += int(W[s])
        if int(tm[s]):
            num -= gam[s] * int(SS[s]) / Fraction(int(tm[s]))
    num += omega * int(I)
    den = sum(int(x) for x in tm) + omega * _coupled(n_nodes, T, coupling_total)
    return num / den if den else Fraction(0)


def q_cpm_from_components(comps, n_nodes, n_slices, gamma, omega,
                          coupling_total=None) -> Fraction:
    """The multislice CPM from its components (SS_s = sum over communities of the squared
    number of their slice-s supra-nodes): (sum_s [W_s - gamma^(s) SS_s] + omega I) / 2mu, the
    normalisation 2mu = sum_s 2m_s + omega Ctot of Eq. 6."""
    T = n_slices
    gam, omega = _per_slice(gamma, T), Fraction(omega)
    W, SS, tm, I = comps[:T], comps[T:2 * T], comps[2 * T:3 * T], comps[3 * T]
    num = sum(int(W[s]) - gam[s] * int(SS[s]) for s in range(T)) + omega * int(I)
    den = sum(int(x) for x in tm) + omega * _coupled(n_nodes, T, coupling_total)
    return num / den if den else Fraction(0)


def q_global_from_components(comps, n_nodes, n_slices, gamma, omega,
                             coupling_total=None) -> Fraction:
    """Global modularity of the supra-graph from its components: with 2mu = sum_s 2m_s +
    omega Ctot (Ctot = 2 N (T-1) for the ordinal coupling of every copy), Q = (sum_s W_s + omega I - gamma (comps[T] / b^2) / 2mu) / 2mu, where
    comps[T] = sum_C (sum_v kappa'_v)^2 in units scaled by the coupling denominator b."""
    T = n_slices
    gamma, omega = Fraction(gamma), Fraction(omega)
    b = omega.denominator
    W, SS, tm, I = comps[:T], int(comps[T]), comps[2 * T:3 * T], comps[3 * T]
    two_mu = sum(int(x) for x in tm) + omega * _coupled(n_nodes, T, coupling_total)
    if two_mu == 0:
        return Fraction(0)
    num = sum(int(x) for x in W) + omega * int(I) - gamma * Fraction(SS, b * b) / two_mu
    return num / two_mu


def trace_enable(on: bool = True):
    _load().orc_trace_enable(1 if on else 0)


def trace_levels(n0):
    """Per-level records of the last traced run(s): graph, colours, partitions, refinement."""
    lib = _load()
    out = []
    for i in range(lib.orc_trace_count()):
        info = np.zeros(8, np.int64)
        lib.orc_trace_info(i, _ptr(info))
        it, lvl, n, nnz, ncol, sweeps, npf, has_r = (int(x) for x in info)
        rec = dict(it=it, lvl=lvl, n=n, nnz=nnz, ncol=ncol, sweeps=sweeps,
                   rp=np.zeros(n + 1, np.int64), col=np.zeros(nnz, np.int32),
                   w=np.zeros(nnz, np.int64), pp=np.zeros(n + 1, np.int64),
                   ps=np.zeros(npf, np.int32), pk=np.zeros(npf, np.int64),
                   colour=np.zeros(n, np.int32), p_in=np.zeros(n, np.uint32),
                   p_lm=np.zeros(n, np.uint32), r=np.zeros(n, np.uint32) if has_r else None,
                   map0=np.zeros(n0, np.int64))
        lib.orc_trace_get(i, *[_ptr(rec[k]) for k in ("rp", "col", "w", "pp", "ps", "pk",
                                                     "colour", "p_in", "p_lm")],
                          _ptr(rec["r"]) if has_r else None, _ptr(rec["map0"]), n0)
        rec["ext"] = rec["wc"] = None
        if has_r:
            rec["ext"] = np.zeros(n, np.int64)
            rec["wc"] = np.zeros(n, np.int8)
            lib.orc_trace_refine(i, _ptr(rec["ext"]), _ptr(rec["wc"]))
        out.append(rec)
    return out
