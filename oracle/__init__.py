"""CPU oracle for the directed triad census. TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (``libtriad.so`` and
its Python binding) never imports, links or calls it, and the two share no
code, headers or tables; they meet only at the seeded inputs.

Functions (all plain C in ``liboracle.so``, wrapped with ctypes):

* :func:`census`        Batagelj-Mrvar sweep of Fig. 5 (two-pointer union walk of
                        Fig. 8), single thread; 003 in 128-bit arithmetic.
* :func:`census_mt`     the same task routine over dynamically claimed CSR-entry
                        chunks on T threads (exact integer sum of partials).
* :func:`census_tasks`  partial census (no 003) over a given list of tasks.
* :func:`brute`         O(n^3) definition: every triple, classified by an
                        independent isomorphism invariant; reads raw arcs.
* :func:`wedge_census`  wedge/triangle decomposition, a second exact algorithm.
* :func:`lut`           the 64-state -> 16-class table of the sweep.
* :func:`exhaustive`    every labelled digraph on n <= 5 vertices, sweep and
                        decomposition against the brute force.
* :func:`labelled_census` the 64-state census (states of triples a < b < c by
                        id order, Sec. 3), by the same sweep.
* :func:`brute64`       the 64-state census by its definition, every triple.

``oracle.checkpoint`` runs the census in chunks of CSR entries with a JSON
checkpoint after each, so that a long run can stop and resume exactly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["census_oracle.c", "brute.c", "wedge.c", "selftest.c", "labelled.c"]
TYPES = ["003", "012", "102", "021D", "021U", "021C", "111D", "111U",
         "030T", "030C", "201", "120D", "120U", "120C", "210", "300"]

_LIB = None


def lib_path():
    return os.path.join(HERE, "liboracle.so")


def build():
    """Compile the oracle with gcc (plain C11, -O2)."""
    out = lib_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           *[os.path.join(HERE, s) for s in SOURCES], "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + r.stderr)
    os.replace(tmp, out)
    return out


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path()):
            build()
        L = ctypes.CDLL(lib_path())
        i64, vp, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        L.oracle_census.argtypes = [i64, vp, vp, vp, vp, vp]
        L.oracle_census.restype = i32
        L.oracle_census_mt.argtypes = [i64, vp, vp, vp, i32, vp, vp]
        L.oracle_census_mt.restype = i32
        L.oracle_census_entries.argtypes = [i64, vp, vp, vp, i64, i64, vp]
        L.oracle_census_entries.restype = None
        L.oracle_census_tasks.argtypes = [i64, vp, vp, vp, i64, vp, vp]
        L.oracle_census_tasks.restype = None
        L.oracle_census_tasks_mt.argtypes = [i64, vp, vp, vp, i64, vp, i32, vp]
        L.oracle_census_tasks_mt.restype = None
        L.oracle_brute.argtypes = [i64, i64, vp, vp, vp, vp]
        L.oracle_brute.restype = i32
        L.oracle_brute_classify.argtypes = [i32, i32, i32]
        L.oracle_brute_classify.restype = i32
        L.oracle_wedge_census.argtypes = [i64, vp, vp, vp, i32, vp, vp]
        L.oracle_wedge_census.restype = i32
        L.oracle_build_lut.argtypes = [vp]
        L.oracle_build_lut.restype = None
        L.oracle_choose3.argtypes = [i64, vp, vp]
        L.oracle_choose3.restype = None
        L.oracle_exhaustive.argtypes = [i32, vp]
        L.oracle_exhaustive.restype = i64
        L.oracle_labelled_census.argtypes = [i64, vp, vp, vp, vp, vp]
        L.oracle_labelled_census.restype = i32
        L.oracle_brute64.argtypes = [i64, i64, vp, vp, vp, vp]
        L.oracle_brute64.restype = i32
        _LIB = L
    return _LIB


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _csr_args(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    nb = np.ascontiguousarray(g.nbrs, dtype=np.int32)
    fl = np.ascontiguousarray(g.flags, dtype=np.uint8)
    return off, nb, fl


def _result(out, hi):
    """Census as a list of Python ints; 003 carries its high word."""
    res = [int(x) for x in out]
    res[0] += int(hi[0]) << 64
    return res


def census(g):
    off, nb, fl = _csr_args(g)
    out = np.zeros(16, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    lib().oracle_census(g.n, _p(off), _p(nb), _p(fl), _p(out), _p(hi))
    return _result(out, hi)


def census_mt(g, nthreads=None):
    off, nb, fl = _csr_args(g)
    out = np.zeros(16, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    t = nthreads or max(1, len(os.sched_getaffinity(0)))
    lib().oracle_census_mt(g.n, _p(off), _p(nb), _p(fl), t, _p(out), _p(hi))
    return _result(out, hi)


def census_tasks(g, tasks, nthreads=1):
    """Partial census over tasks given as CSR entry indices j (row < nbrs[j])."""
    off, nb, fl = _csr_args(g)
    tk = np.ascontiguousarray(tasks, dtype=np.int64)
    out = np.zeros(16, dtype=np.uint64)
    if nthreads > 1:
        lib().oracle_census_tasks_mt(g.n, _p(off), _p(nb), _p(fl), tk.size, _p(tk), nthreads, _p(out))
    else:
        lib().oracle_census_tasks(g.n, _p(off), _p(nb), _p(fl), tk.size, _p(tk), _p(out))
    return [int(x) for x in out]


def brute(n, src, dst):
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    out = np.zeros(16, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    r = lib().oracle_brute(n, s.size, _p(s), _p(d), _p(out), _p(hi))
    if r < 0:
        raise MemoryError("brute force adjacency allocation failed")
    return _result(out, hi)


def brute_classify(sab, sac, sbc):
    return int(lib().oracle_brute_classify(sab, sac, sbc))


def wedge_census(g, nthreads=None):
    off, nb, fl = _csr_args(g)
    out = np.zeros(16, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    t = nthreads or max(1, len(os.sched_getaffinity(0)))
    lib().oracle_wedge_census(g.n, _p(off), _p(nb), _p(fl), t, _p(out), _p(hi))
    return _result(out, hi)


def lut():
    t = np.zeros(64, dtype=np.uint8)
    lib().oracle_build_lut(_p(t))
    return t


def choose3(n):
    lo = np.zeros(1, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    lib().oracle_choose3(n, _p(lo), _p(hi))
    return int(lo[0]) + (int(hi[0]) << 64)


def exhaustive(n):
    m = np.zeros(2, dtype=np.int64)
    total = lib().oracle_exhaustive(n, _p(m))
    return int(total), int(m[0]), int(m[1])


def labelled_census(g):
    """64 counts: state f_ab | f_ac << 2 | f_bc << 4 of the triples a < b < c
    (state 0 with its high word)."""
    off, nb, fl = _csr_args(g)
    out = np.zeros(64, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    lib().oracle_labelled_census(g.n, _p(off), _p(nb), _p(fl), _p(out), _p(hi))
    return _result(out, hi)


def brute64(n, src, dst):
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    out = np.zeros(64, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    if lib().oracle_brute64(n, s.size, _p(s), _p(d), _p(out), _p(hi)) < 0:
        raise MemoryError("brute force adjacency allocation failed")
    return _result(out, hi)

