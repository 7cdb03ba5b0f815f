"""CPU oracle for the H0 barcode -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links
or executes anything here; the two share no code.

``ph0_oracle.cpp`` is a plain, single-threaded C++ implementation of the
barcode algorithm of Section 2 of the paper (distances, sort, dedupe to
grades, dense F2 column reduction, read-off).  This wrapper builds it with
g++ on first use and exposes it on numpy arrays.

``ph0_omp.cpp`` is the paper's multi-core CPU scheme (Section 3: OpenMP
work-sharing loops inside the sequential column loop), a CPU timing baseline
beside the GPU; ``omp_barcode`` runs it.  It is written apart from the oracle
and checked against it in the tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ph0_oracle.cpp")
_LIB = os.path.join(_HERE, "libph0_oracle.so")
_OMP_SRC = os.path.join(_HERE, "ph0_omp.cpp")
_OMP_LIB = os.path.join(_HERE, "libph0_omp.so")

INF = 0xFFFFFFFF


class _Stats(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_int64),
        ("E_eff", ctypes.c_int64),
        ("distinct", ctypes.c_int64),
        ("additions", ctypes.c_int64),
        ("pivots", ctypes.c_int64),
        ("columns", ctypes.c_int64),
        ("late_nonzero", ctypes.c_int64),
        ("not_two_sparse", ctypes.c_int64),
        ("s_dist", ctypes.c_double),
        ("s_sort", ctypes.c_double),
        ("s_rank", ctypes.c_double),
        ("s_reduce", ctypes.c_double),
        ("s_emit", ctypes.c_double),
    ]


def _compile(src: str, lib: str, flags: list, force: bool) -> str:
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", *flags,
                               "-o", tmp, src])
        os.replace(tmp, lib)
    return lib


def build(force: bool = False) -> str:
    """Compile the oracle shared library (single-threaded, -O3) and the
    OpenMP baseline with g++; returns the oracle library's path."""
    _compile(_OMP_SRC, _OMP_LIB, ["-fopenmp"], force)
    return _compile(_SRC, _LIB, [], force)


class _H1Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("E", "T", "T_eff", "additions", "pivots", "zero_length", "columns")]


_lib = None


def _bind(lib):
    P = ctypes.c_void_p
    lib.ph0o_barcode.argtypes = [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int, P, P, P, P, ctypes.POINTER(_Stats)]
    lib.ph0o_barcode.restype = ctypes.c_int
    lib.ph0o_sorted_edges.argtypes = [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int32,
                                      P, P, P, P, P, ctypes.POINTER(ctypes.c_int64)]
    lib.ph0o_sorted_edges.restype = ctypes.c_int
    lib.ph0o_h1.argtypes = [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                            P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(_H1Stats)]
    lib.ph0o_h1.restype = ctypes.c_int
    return lib


def build_planted(define: str, out_dir: str):
    """The oracle compiled with one PH0O_PLANT_* switch (a known mistake),
    loaded from out_dir: only for the tests that show a pin catches it."""
    lib = os.path.join(out_dir, "libph0_oracle_%s.so" % define.lower())
    _compile(_SRC, lib, ["-D" + define], True)
    return _bind(ctypes.CDLL(lib))


def build_native(out_dir: str):
    """The oracle compiled with -O3 -march=native for the host it runs on,
    loaded from out_dir: for timing it as the CPU baseline (the source is the
    same; only the instruction set the compiler may use differs)."""
    lib = os.path.join(out_dir, "libph0_oracle_native.so")
    _compile(_SRC, lib, ["-march=native"], True)
    return _bind(ctypes.CDLL(lib))


def _load():
    global _lib
    if _lib is None:
        _lib = _bind(ctypes.CDLL(build()))
    return _lib


def _points(points: np.ndarray) -> tuple[np.ndarray, int]:
    x = np.ascontiguousarray(points)
    if x.ndim != 2:
        raise ValueError("points must be N x d")
    if x.dtype == np.int8:
        return x, 1
    if x.dtype == np.int16:
        return x, 2
    raise TypeError("points must be int8 or int16")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class OracleResult:
    canonical: np.ndarray        # n uint32 deaths ascending, INF last
    death_by_vertex: np.ndarray  # n uint32
    killer_pos: np.ndarray       # n int64 sorted position of the killing column
    partner: np.ndarray          # n int32 other row of the stored column
    E: int
    E_eff: int
    distinct: int
    additions: int
    pivots: int
    columns: int
    late_nonzero: int
    not_two_sparse: int
    seconds: dict

    def bars(self) -> np.ndarray:
        """n x 2 uint32 (birth, death) in canonical order."""
        out = np.zeros((self.canonical.size, 2), dtype=np.uint32)
        out[:, 1] = self.canonical
        return out


def barcode(points: np.ndarray, early_exit: bool = True, lib=None) -> OracleResult:
    """Run the full oracle on an N x d int8/int16 cloud (`lib`: a build from
    build_native, else the portable one)."""
    x, eb = _points(points)
    n, d = x.shape
    if n < 1 or d < 1:
        raise ValueError("need N >= 1 and d >= 1")
    lib = lib or _load()
    dv = np.empty(n, np.uint32)
    can = np.empty(n, np.uint32)
    kp = np.empty(n, np.int64)
    par = np.empty(n, np.int32)
    st = _Stats()
    rc = lib.ph0o_barcode(_ptr(x), eb, n, d, 1 if early_exit else 0, _ptr(dv), _ptr(can),
                          _ptr(kp), _ptr(par), ctypes.byref(st))
    if rc != 0:
        raise RuntimeError("oracle rejected its arguments")
    return OracleResult(
        canonical=can, death_by_vertex=dv, killer_pos=kp, partner=par,
        E=st.E, E_eff=st.E_eff, distinct=st.distinct, additions=st.additions,
        pivots=st.pivots, columns=st.columns, late_nonzero=st.late_nonzero,
        not_two_sparse=st.not_two_sparse,
        seconds=dict(dist=st.s_dist, sort=st.s_sort, rank=st.s_rank,
                     reduce=st.s_reduce, emit=st.s_emit),
    )


@dataclass
class H1Result:
    bars: np.ndarray         # m x 2 uint32 (birth, death) grades, birth < death, sorted
    tri_of_edge: np.ndarray  # E int64: triangle (in triangle order) paired with the edge at
                             # each sorted position, -1 if none
    E: int
    T: int
    T_eff: int
    additions: int
    pivots: int
    zero_length: int
    columns: int


def h1_barcode(points: np.ndarray, early_exit: bool = True, lib=None) -> H1Result:
    """H1 of the same filtration: dense F2 reduction of the edge-by-triangle
    boundary matrix (readings in ph0_oracle.cpp).  `lib` selects a planted
    build (build_planted) in the pin tests."""
    x, eb = _points(points)
    n, d = x.shape
    if n < 1 or d < 1:
        raise ValueError("need N >= 1 and d >= 1")
    E = n * (n - 1) // 2
    cap = max(E - n + 1, 0)
    lib = lib or _load()
    toe = np.empty(E, np.int64)
    b = np.empty(max(cap, 1), np.uint32)
    dd = np.empty(max(cap, 1), np.uint32)
    nb = ctypes.c_int64(0)
    st = _H1Stats()
    rc = lib.ph0o_h1(_ptr(x), eb, n, d, 1 if early_exit else 0, _ptr(toe), _ptr(b), _ptr(dd),
                     cap, ctypes.byref(nb), ctypes.byref(st))
    if rc != 0:
        raise RuntimeError("oracle rejected its arguments (%d)" % rc)
    m = int(nb.value)
    return H1Result(bars=np.stack([b[:m], dd[:m]], axis=1), tri_of_edge=toe, E=st.E, T=st.T,
                    T_eff=st.T_eff, additions=st.additions, pivots=st.pivots,
                    zero_length=st.zero_length, columns=st.columns)


@dataclass
class SortedEdges:
    colex_delta: np.ndarray  # E int64, squared distance of edge (i, j) at j(j-1)/2 + i
    delta: np.ndarray        # E int64 sorted
    j: np.ndarray            # E int32
    i: np.ndarray            # E int32
    grade: np.ndarray        # E uint32, 1-based index in D
    distinct: int


def sorted_edges(points: np.ndarray) -> SortedEdges:
    """Steps 1-3 of the oracle: colex distances, the sorted list, the grades."""
    x, eb = _points(points)
    n, d = x.shape
    E = n * (n - 1) // 2
    lib = _load()
    cd = np.empty(E, np.int64)
    de = np.empty(E, np.int64)
    jj = np.empty(E, np.int32)
    ii = np.empty(E, np.int32)
    gg = np.empty(E, np.uint32)
    nd = ctypes.c_int64(0)
    rc = lib.ph0o_sorted_edges(_ptr(x), eb, n, d, _ptr(cd), _ptr(de), _ptr(jj), _ptr(ii),
                               _ptr(gg), ctypes.byref(nd))
    if rc != 0:
        raise RuntimeError("oracle rejected its arguments")
    return SortedEdges(cd, de, jj, ii, gg, int(nd.value))


class _OmpStats(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_int64),
        ("E_eff", ctypes.c_int64),
        ("distinct", ctypes.c_int64),
        ("additions", ctypes.c_int64),
        ("pivots", ctypes.c_int64),
        ("threads", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("s_dist", ctypes.c_double),
        ("s_sort", ctypes.c_double),
        ("s_rank", ctypes.c_double),
        ("s_reduce", ctypes.c_double),
        ("s_emit", ctypes.c_double),
    ]


_omp = None


def _load_omp():
    global _omp
    if _omp is None:
        build()
        lib = ctypes.CDLL(_OMP_LIB)
        P = ctypes.c_void_p
        lib.ph0p_barcode.argtypes = [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                     ctypes.c_int, P, P, ctypes.POINTER(_OmpStats)]
        lib.ph0p_barcode.restype = ctypes.c_int
        _omp = lib
    return _omp


@dataclass
class OmpResult:
    canonical: np.ndarray        # n uint32 deaths ascending, INF last
    death_by_vertex: np.ndarray  # n uint32
    E: int
    E_eff: int
    distinct: int
    additions: int
    pivots: int
    threads: int
    seconds: dict


def omp_barcode(points: np.ndarray, threads: int, early_exit: bool = True) -> OmpResult:
    """The paper's multi-core CPU scheme (Section 3) with `threads` OpenMP
    threads: a timing baseline, not the oracle."""
    x, eb = _points(points)
    n, d = x.shape
    if n < 1 or d < 1 or threads < 1:
        raise ValueError("need N >= 1, d >= 1, threads >= 1")
    lib = _load_omp()
    dv = np.empty(n, np.uint32)
    can = np.empty(n, np.uint32)
    st = _OmpStats()
    rc = lib.ph0p_barcode(_ptr(x), eb, n, d, int(threads), 1 if early_exit else 0, _ptr(dv),
                          _ptr(can), ctypes.byref(st))
    if rc != 0:
        raise RuntimeError("OpenMP baseline rejected its arguments")
    return OmpResult(
        canonical=can, death_by_vertex=dv, E=st.E, E_eff=st.E_eff, distinct=st.distinct,
        additions=st.additions, pivots=st.pivots, threads=st.threads,
        seconds=dict(dist=st.s_dist, sort=st.s_sort, rank=st.s_rank,
                     reduce=st.s_reduce, emit=st.s_emit),
    )
