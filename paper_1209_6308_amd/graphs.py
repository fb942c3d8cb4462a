"""Seeded synthetic inputs for the triad census: generators and the CSR builder.

This module holds no census arithmetic. It wraps ``libtriadgen.so`` (built from
``gen/graphgen.cpp``) and emits the compact symmetric CSR of Sec. 6 / Fig. 7 of
the paper: ``offsets`` int64[n+1], ``nbrs`` int32[nnz] (rows strictly
increasing, no self-loops, symmetric) and ``flags`` uint8[ceil(nnz/4)] with two
direction bits per entry (bit0 = row->neighbour, bit1 = neighbour->row).

The named workloads reproduce the paper's graph shapes (Sec. 5) with synthetic
generators, because the patents, Orkut and .uk graphs are not available:

* ``rmat10``  R-MAT scale 10, edge factor 8 (a tiny graph the brute force covers)
* ``rmat20``  R-MAT scale 20, edge factor 16, 10% of asymmetric pairs reciprocated
  (arc count of the patents network)
* ``rmat24``  R-MAT scale 24, edge factor 16 (arc count of the Orkut network)
* ``cl22``    Chung-Lu, n = 2^22, exponent 2.1 (Orkut's out-degree exponent 2.127)
* ``nullens`` an ensemble of 4,096 small Erdos-Renyi / Chung-Lu null models with
  degree-preserving swaps
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.gen_lib_path()
        if not os.path.exists(path):
            _build.build_gen()
        L = ctypes.CDLL(path)
        i64, u64, i32, dbl, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.tg_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, vp, vp, i32]
        L.tg_rmat.restype = i64
        L.tg_chung_lu.argtypes = [i64, dbl, dbl, dbl, i64, u64, vp, vp, i32]
        L.tg_chung_lu.restype = i64
        L.tg_erdos_renyi.argtypes = [i64, i64, u64, vp, vp]
        L.tg_erdos_renyi.restype = i64
        L.tg_swap.argtypes = [i64, vp, vp, i64, u64]
        L.tg_swap.restype = i64
        L.tg_swap_ensemble.argtypes = [i64, vp, vp, ctypes.c_int32, i64, u64, vp, vp, i32]
        L.tg_swap_ensemble.restype = i64
        L.tg_csr_build.argtypes = [i64, i64, vp, vp, dbl, u64, i32]
        L.tg_csr_build.restype = vp
        L.tg_csr_nnz.argtypes = [vp]
        L.tg_csr_nnz.restype = i64
        L.tg_csr_fetch.argtypes = [vp, vp, vp, vp]
        L.tg_csr_fetch.restype = None
        L.tg_csr_free.argtypes = [vp]
        L.tg_csr_free.restype = None
        L.tg_batch_build.argtypes = [ctypes.c_int32, u64, i64, i64, dbl, dbl, dbl, dbl, i32]
        L.tg_batch_build.restype = vp
        L.tg_batch_nv.argtypes = [vp]
        L.tg_batch_nv.restype = i64
        L.tg_batch_nnz.argtypes = [vp]
        L.tg_batch_nnz.restype = i64
        L.tg_batch_fetch.argtypes = [vp, vp, vp, vp, vp, vp]
        L.tg_batch_fetch.restype = None
        L.tg_batch_free.argtypes = [vp]
        L.tg_batch_free.restype = None
        L.tg_hash.argtypes = [vp, i64, u64]
        L.tg_hash.restype = u64
        _LIB = L
    return _LIB


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def nthreads():
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, len(os.sched_getaffinity(0)))


@dataclass
class CSR:
    """Symmetric CSR with packed 2-bit direction flags (see module docstring)."""

    n: int
    offsets: np.ndarray  # int64 [n+1]
    nbrs: np.ndarray  # int32 [nnz]
    flags: np.ndarray  # uint8 [ceil(nnz/4)]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.nbrs.size)

    def flag_array(self) -> np.ndarray:
        """Per-entry 2-bit flags as uint8[nnz]."""
        j = np.arange(self.nnz, dtype=np.int64)
        return ((self.flags[j >> 2] >> (2 * (j & 3)).astype(np.uint8)) & 3).astype(np.uint8)

    def content_hash(self) -> str:
        L = lib()
        h = L.tg_hash(_p(self.offsets), self.offsets.nbytes, ctypes.c_uint64(self.n))
        h = L.tg_hash(_p(self.nbrs), self.nbrs.nbytes, ctypes.c_uint64(h))
        h = L.tg_hash(_p(self.flags), self.flags.nbytes, ctypes.c_uint64(h))
        return f"{h:016x}"

    def arcs(self):
        """Directed arcs (src, dst) recovered from the CSR (each arc once)."""
        f = self.flag_array()
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.offsets))
        out = (f & 1) != 0
        return rows[out].astype(np.int32), self.nbrs[out].copy()

    def stats(self) -> dict:
        d = np.diff(self.offsets).astype(np.int64)
        f = self.flag_array()
        m_sym = self.nnz // 2
        mutual = int(np.count_nonzero(f == 3)) // 2
        return {
            "n": int(self.n),
            "nnz": int(self.nnz),
            "m_sym": int(m_sym),
            "arcs": int(m_sym + mutual),
            "mutual_pairs": mutual,
            "d_max": int(d.max()) if d.size else 0,
            "sum_d2": int(np.dot(d, d)),
            "isolated": int(np.count_nonzero(d == 0)),
        }


def build_csr(n: int, src: np.ndarray, dst: np.ndarray, recip_p: float = 0.0, recip_seed: int = 2,
              name: str = "") -> CSR:
    """Arc list -> symmetric CSR (self-loops and duplicate arcs dropped)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("arc endpoint out of range")
    L = lib()
    h = L.tg_csr_build(n, src.size, _p(src), _p(dst), float(recip_p), recip_seed, nthreads())
    try:
        nnz = L.tg_csr_nnz(h)
        off = np.empty(n + 1, dtype=np.int64)
        nb = np.empty(nnz, dtype=np.int32)
        fl = np.empty((nnz + 3) // 4, dtype=np.uint8)
        L.tg_csr_fetch(h, _p(off), _p(nb), _p(fl))
    finally:
        L.tg_csr_free(h)
    return CSR(n, off, nb, fl, name=name)


def rmat_arcs(scale: int, narcs: int, a=0.57, b=0.19, c=0.19, seed=1):
    src = np.empty(narcs, dtype=np.int32)
    dst = np.empty(narcs, dtype=np.int32)
    lib().tg_rmat(scale, narcs, a, b, c, seed, _p(src), _p(dst), nthreads())
    return src, dst


def chung_lu_arcs(n: int, gamma: float, mean: float, w0: float, narcs: int, seed=1):
    src = np.empty(narcs, dtype=np.int32)
    dst = np.empty(narcs, dtype=np.int32)
    lib().tg_chung_lu(n, gamma, mean, w0, narcs, seed, _p(src), _p(dst), nthreads())
    return src, dst


def erdos_renyi_arcs(n: int, narcs: int, seed=1):
    src = np.empty(narcs, dtype=np.int32)
    dst = np.empty(narcs, dtype=np.int32)
    lib().tg_erdos_renyi(n, narcs, seed, _p(src), _p(dst))
    return src, dst


def degree_preserving_swaps(src, dst, attempts: int, seed: int):
    """Double-edge swaps that keep in-, out- and mutual degrees (distinct arcs in)."""
    s = np.ascontiguousarray(src, dtype=np.int32).copy()
    d = np.ascontiguousarray(dst, dtype=np.int32).copy()
    acc = lib().tg_swap(s.size, _p(s), _p(d), attempts, seed)
    return s, d, int(acc)


def rmat(scale: int, edge_factor: int, seed: int = 1, recip_p: float = 0.0, recip_seed: int = 2,
         a=0.57, b=0.19, c=0.19) -> CSR:
    n = 1 << scale
    src, dst = rmat_arcs(scale, edge_factor * n, a, b, c, seed)
    g = build_csr(n, src, dst, recip_p, recip_seed, name=f"rmat{scale}")
    g.meta = {"gen": "rmat", "scale": scale, "edge_factor": edge_factor, "seed": seed,
              "recip_p": recip_p, "abcd": [a, b, c, round(1 - a - b - c, 6)]}
    return g


def chung_lu(n: int, gamma: float, mean: float, w0: float, seed: int = 1) -> CSR:
    narcs = int(round(mean * n))
    src, dst = chung_lu_arcs(n, gamma, mean, w0, narcs, seed)
    g = build_csr(n, src, dst, name=f"chunglu{n}")
    g.meta = {"gen": "chung_lu", "n": n, "gamma": gamma, "mean": mean, "w0": w0, "seed": seed}
    return g


def from_arcs(n: int, arcs) -> CSR:
    """Small helper: CSR from a Python list / array of (src, dst) arcs."""
    a = np.asarray(arcs, dtype=np.int64).reshape(-1, 2)
    return build_csr(n, a[:, 0], a[:, 1])


WORKLOADS = {
    "rmat10": dict(kind="rmat", scale=10, edge_factor=8, seed=1),
    "rmat20": dict(kind="rmat", scale=20, edge_factor=16, seed=1, recip_p=0.1, recip_seed=2),
    "rmat24": dict(kind="rmat", scale=24, edge_factor=16, seed=1),
    "cl22": dict(kind="chung_lu", n=1 << 22, gamma=2.1, mean=24.0, w0=float(1 << 18), seed=1),
}


def workload(name: str) -> CSR:
    """Build one of the named single-graph workloads (deterministic from its seed)."""
    w = dict(WORKLOADS[name])
    kind = w.pop("kind")
    if kind == "rmat":
        g = rmat(**w)
    else:
        g = chung_lu(**w)
    g.name = name
    return g


@dataclass
class BatchCSR:
    """G graphs in one concatenated CSR; graph g owns rows [vbase[g], vbase[g+1])
    and its neighbour ids are graph-local; offsets are global entry positions."""

    G: int
    vbase: np.ndarray  # int64 [G+1]
    offsets: np.ndarray  # int64 [vbase[G]+1]
    nbrs: np.ndarray  # int32 [nnz]
    flags: np.ndarray  # uint8 [ceil(nnz/4)]
    params: np.ndarray  # float64 [G,6]: kind, n, mean, recip, gamma, arcs

    @property
    def nnz(self):
        return int(self.nbrs.size)

    def graph(self, g: int) -> CSR:
        v0, v1 = int(self.vbase[g]), int(self.vbase[g + 1])
        e0, e1 = int(self.offsets[v0]), int(self.offsets[v1])
        off = (self.offsets[v0:v1 + 1] - e0).astype(np.int64)
        nb = self.nbrs[e0:e1].copy()
        j = np.arange(e0, e1, dtype=np.int64)
        f = (self.flags[j >> 2] >> (2 * (j & 3)).astype(np.uint8)) & 3
        k = np.arange(e1 - e0, dtype=np.int64)
        fl = np.zeros((e1 - e0 + 3) // 4, dtype=np.uint8)
        np.bitwise_or.at(fl, k >> 2, (f.astype(np.uint8) << (2 * (k & 3)).astype(np.uint8)))
        return CSR(v1 - v0, off, nb, fl, name=f"member{g}")

    def content_hash(self) -> str:
        L = lib()
        h = 0
        for a in (self.vbase, self.offsets, self.nbrs, self.flags):
            h = L.tg_hash(_p(a), a.nbytes, ctypes.c_uint64(h))
        return f"{h:016x}"

    def sum_d2(self) -> int:
        d = np.diff(self.offsets).astype(np.int64)
        return int(np.dot(d, d))


def null_ensemble(G: int = 4096, seed: int = 1, nmin: int = 64, nmax: int = 8192, dmin: float = 4.0,
                  dmax: float = 32.0, rmax: float = 0.3, swap_factor: float = 10.0) -> BatchCSR:
    """Degree-preserving randomisations of Erdos-Renyi (even g) and Chung-Lu (odd g) graphs."""
    L = lib()
    h = L.tg_batch_build(G, seed, nmin, nmax, dmin, dmax, rmax, swap_factor, nthreads())
    try:
        nv = L.tg_batch_nv(h)
        nnz = L.tg_batch_nnz(h)
        vb = np.empty(G + 1, dtype=np.int64)
        off = np.empty(nv + 1, dtype=np.int64)
        nb = np.empty(nnz, dtype=np.int32)
        fl = np.empty((nnz + 3) // 4, dtype=np.uint8)
        pr = np.empty((G, 6), dtype=np.float64)
        L.tg_batch_fetch(h, _p(vb), _p(off), _p(nb), _p(fl), _p(pr))
    finally:
        L.tg_batch_free(h)
    return BatchCSR(G, vb, off, nb, fl, pr)


def concat_csrs(members, params=None) -> BatchCSR:
    """One batch (graph-local ids, global entry offsets) from a list of CSRs."""
    vb = [0]
    offs, nbs, fls = [np.zeros(1, np.int64)], [], []
    e0 = 0
    for g in members:
        vb.append(vb[-1] + g.n)
        offs.append(g.offsets[1:] + e0)
        nbs.append(g.nbrs)
        fls.append(g.flag_array())
        e0 += g.nnz
    f = np.concatenate(fls) if fls else np.zeros(0, np.uint8)
    j = np.arange(f.size)
    packed = np.zeros((f.size + 3) // 4, np.uint8)
    np.bitwise_or.at(packed, j >> 2, (f << (2 * (j & 3))).astype(np.uint8))
    return BatchCSR(len(members), np.array(vb, np.int64), np.concatenate(offs).astype(np.int64),
                    np.concatenate(nbs).astype(np.int32) if nbs else np.zeros(0, np.int32), packed,
                    params if params is not None else np.zeros((len(members), 6)))


def randomised_ensemble(g: CSR, K: int, seed: int = 1, swap_factor: float = 10.0) -> BatchCSR:
    """K degree-preserving randomisations of g (double-edge swaps within
    asymmetric arcs and within mutual dyads, swap_factor x arcs attempts each;
    in-, out- and mutual degrees kept) as one batch: the null-model ensemble of
    a triad significance profile."""
    src, dst = g.arcs()
    m = src.size
    out_s = np.empty(K * m, dtype=np.int32)
    out_d = np.empty(K * m, dtype=np.int32)
    lib().tg_swap_ensemble(m, _p(src), _p(dst), K, int(swap_factor * m), seed, _p(out_s), _p(out_d), nthreads())
    members = [build_csr(g.n, out_s[k * m:(k + 1) * m], out_d[k * m:(k + 1) * m]) for k in range(K)]
    return concat_csrs(members)



def window_batches(n: int, src: np.ndarray, dst: np.ndarray, times: np.ndarray, width: float, step: float,
                   t_end: float):
    """Update batches that keep a census of a sliding time window over a stream
    of timestamped arcs (the census at fixed intervals of Sec. 3): the window
    [t, t + width) moves by `step` from t = 0 while t + width <= t_end. An arc
    is present while any of its occurrences lies in the window, so each step's
    batch is the difference of the two windows' arc sets: deletions of the arcs
    that left it, insertions of those that entered (self-loops never count).
    Yields (start time, src, dst, insert) per step, the first step the whole
    first window as insertions."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    times = np.asarray(times, dtype=np.float64)
    keep = src != dst
    src, dst, times = src[keep], dst[keep], times[keep]
    key = src * n + dst
    prev = np.zeros(0, dtype=np.int64)
    t = 0.0
    while t + width <= t_end:
        cur = np.unique(key[(times >= t) & (times < t + width)])
        gone = np.setdiff1d(prev, cur, assume_unique=True)
        came = np.setdiff1d(cur, prev, assume_unique=True)
        k = np.concatenate([gone, came])
        ins = np.concatenate([np.zeros(gone.size, np.uint8), np.ones(came.size, np.uint8)])
        yield t, (k // n).astype(np.int32), (k % n).astype(np.int32), ins
        prev = cur
        t += step
