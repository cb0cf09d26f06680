"""CPU oracle for the GPU filtering stage (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU search path never imports, links or calls it,
and the two share no code: this package has its own index-file reader and
its own plain C implementation (``ann_oracle.c``) of the online search steps
of the paper (Sec. 3, steps 1-8; Eq. 1), plus brute-force exact kNN.

Every float-valued selection uses float32 distances that are either exact
integers or float64 sums rounded once to float32, ordered by (distance, id).
"""
from __future__ import annotations

import ctypes
import os
import struct
import subprocess
import zlib
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ann_oracle.c")
LIB = os.path.join(HERE, "_ann_oracle.so")

_DTYPES = {0: np.float32, 1: np.uint8, 2: np.int8}
_KIND = {0: "f32", 1: "u8", 2: "i8"}


_CFLAGS = ["-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O3, OpenMP, no FP contraction, no
    fast-math (so no reassociation: every sum keeps the order of the source)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", *_CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


def use_native(directory: str | None = None) -> str:
    """Build a copy tuned for this host's CPU (-march=native, same flags
    otherwise, so the same results) in a scratch directory and make it the
    library this module calls.  For timing the oracle on the machine that runs
    it; the in-tree build stays portable."""
    global _lib
    import tempfile
    d = directory or tempfile.mkdtemp(prefix="ann_oracle_")
    out = os.path.join(d, "_ann_oracle_native.so")
    subprocess.run(["gcc", *_CFLAGS, "-march=native", SRC, "-o", out, "-lm"], check=True)
    _lib = None
    _load(out)
    return out


class _OrcIndex(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("dim", ctypes.c_int32), ("n", ctypes.c_int64),
        ("nlist", ctypes.c_int32), ("m", ctypes.c_int32), ("ksub", ctypes.c_int32),
        ("dsub", ctypes.c_int32), ("r", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("centroids", ctypes.c_void_p), ("codebooks", ctypes.c_void_p),
        ("codes", ctypes.c_void_p), ("vectors", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p), ("entries", ctypes.c_void_p),
    ]


class _OrcGraph(ctypes.Structure):
    _fields_ = [("adj", ctypes.c_void_p), ("deg", ctypes.c_int32), ("n_entry", ctypes.c_int32),
                ("entry", ctypes.c_void_p), ("beam", ctypes.c_int32), ("pad_", ctypes.c_int32)]


_lib = None


def _load(path: str | None = None):
    global _lib
    if _lib is None:
        if path is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            path = LIB
        lib = ctypes.CDLL(path)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.orc_probe.argtypes = [P, P, i64, P, i32, P, P, ctypes.c_int]
        lib.orc_lut.argtypes = [P, P, i64, P, P, ctypes.c_int]
        lib.orc_round_half.argtypes = [P, i64, P]
        lib.orc_gather_dedup.argtypes = [P, P, i32, P, P]
        lib.orc_gather_dedup.restype = i64
        lib.orc_adc.argtypes = [P, P, P, P, i64, P, P]
        lib.orc_exact.argtypes = [P, P, P, i64, P]
        lib.orc_search.argtypes = [P, P, i64, P, i32, i32, P, P, P, P, P, P, ctypes.c_int,
                                   ctypes.c_int, i32, ctypes.c_double, i32, P, P, P, P]
        lib.orc_graph_probe.argtypes = [P, P, P, i64, P, i32, P, P, P, ctypes.c_int]
        lib.orc_page_layout.argtypes = [P, i64, i32, i32, i32, P, P]
        lib.orc_page_layout.restype = i64
        lib.orc_bruteforce.argtypes = [P, P, i64, i32, P, P, ctypes.c_int]
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.flags.c_contiguous
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class Index:
    """An index file as the oracle reads it (external vector order)."""
    kind: str
    dim: int
    n: int
    nlist: int
    M: int
    ksub: int
    dsub: int
    R: int
    int_grid: bool
    eps: float
    centroids: np.ndarray
    codebooks: np.ndarray
    codes: np.ndarray
    vectors: np.ndarray
    offsets: np.ndarray
    entries: np.ndarray
    assign: np.ndarray
    _c: _OrcIndex = None

    def cstruct(self) -> _OrcIndex:
        if self._c is None:
            self._c = _OrcIndex(
                {"f32": 0, "u8": 1, "i8": 2}[self.kind], self.dim, self.n, self.nlist, self.M,
                self.ksub, self.dsub, self.R, 0,
                self.centroids.ctypes.data, self.codebooks.ctypes.data, self.codes.ctypes.data,
                self.vectors.ctypes.data, self.offsets.ctypes.data, self.entries.ctypes.data)
        return self._c


def read_index(path: str, verify: bool = True) -> Index:
    """Parse the index file (header, section table, CRC32 checks) into arrays."""
    with open(path, "rb") as f:
        hdr = f.read(512)
    if len(hdr) < 512 or hdr[:8] != b"FANNIDX1":
        raise ValueError("not an index file")
    (ver, hbytes, dtype, dim, n, nlist, M, ksub, dsub, R, flags, eps, nsec,
     E) = struct.unpack_from("<IIIIQIIIIIIfIQ", hdr, 8)
    if ver != 1 or hbytes != 512 or nsec != 7:
        raise ValueError("unsupported index version")
    if verify and zlib.crc32(hdr[:508]) & 0xFFFFFFFF != struct.unpack_from("<I", hdr, 508)[0]:
        raise ValueError("header checksum mismatch")
    secs = [struct.unpack_from("<QQII", hdr, 128 + 24 * i)[:3] for i in range(7)]
    mm = np.memmap(path, dtype=np.uint8, mode="r")
    shapes = [
        (np.float32, (nlist, dim)), (np.float32, (M, ksub, dsub)), (np.uint8, (n, M)),
        (_DTYPES[dtype], (n, dim)), (np.int64, (nlist + 1,)), (np.int32, (E,)),
        (np.int32, (n, R)),
    ]
    arrays = []
    for (off, nbytes, crc), (dt, shp) in zip(secs, shapes):
        raw = mm[off:off + nbytes]
        if verify and zlib.crc32(raw) & 0xFFFFFFFF != crc:
            raise ValueError("section checksum mismatch")
        arrays.append(np.ascontiguousarray(raw.view(dt).reshape(shp)))
    return Index(_KIND[dtype], dim, n, nlist, M, ksub, dsub, R, bool(flags & 1), eps, *arrays)


def _q(Q):
    return np.ascontiguousarray(Q, dtype=np.float32)


def _np(nprobe, nq):
    a = np.asarray(nprobe, dtype=np.int32)
    if a.ndim == 0:
        a = np.full(nq, int(a), dtype=np.int32)
    return np.ascontiguousarray(a)


def probe(ix: Index, Q, nprobe, threads: int = 0):
    """Step 2: (lists [nq, max nprobe] int32 -1 padded, float32 distances +inf padded)."""
    Q = _q(Q)
    nq = Q.shape[0]
    npr = _np(nprobe, nq)
    w = int(npr.max()) if nq else 0
    lists = np.empty((nq, w), dtype=np.int32)
    d = np.empty((nq, w), dtype=np.float32)
    _load().orc_probe(ctypes.byref(ix.cstruct()), _p(Q), nq, _p(npr), w, _p(lists), _p(d), threads)
    return lists, d


def lut(ix: Index, Q, f16: bool = False):
    """Step 1: float32 table [nq, M, ksub] and the float64 table it is rounded from
    (f16: the float32 entries rounded on to binary16, returned widened)."""
    Q = _q(Q)
    nq = Q.shape[0]
    l32 = np.empty((nq, ix.M, ix.ksub), dtype=np.float32)
    l64 = np.empty((nq, ix.M, ix.ksub), dtype=np.float64)
    _load().orc_lut(ctypes.byref(ix.cstruct()), _p(Q), nq, _p(l32), _p(l64), 1 if f16 else 0)
    return l32, l64


def round_half(x):
    """Nearest binary16 values (ties to even) of float32 values, as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    out = np.empty_like(x)
    _load().orc_round_half(_p(x), len(x), _p(out))
    return out


def gather_dedup(ix: Index, lists):
    """Steps 3 and 5 for one query: (distinct IDs ascending, multiset size)."""
    lists = np.ascontiguousarray(np.asarray(lists, dtype=np.int32))
    lists = lists[lists >= 0]
    cap = int(sum(int(ix.offsets[l + 1] - ix.offsets[l]) for l in lists)) + 1
    buf = np.empty(cap, dtype=np.int32)
    nu = ctypes.c_int64(0)
    g = _load().orc_gather_dedup(ctypes.byref(ix.cstruct()), _p(lists), len(lists), _p(buf),
                                 ctypes.byref(nu))
    return buf[:nu.value].copy(), int(g)


def adc(ix: Index, lut32, ids, lut64=None):
    """Eq. 1 for explicit IDs: float32 sums (and float64 sums when lut64 is given)."""
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int32))
    l32 = np.ascontiguousarray(lut32, dtype=np.float32)
    l64 = None if lut64 is None else np.ascontiguousarray(lut64, dtype=np.float64)
    a32 = np.empty(len(ids), dtype=np.float32)
    a64 = None if l64 is None else np.empty(len(ids), dtype=np.float64)
    _load().orc_adc(ctypes.byref(ix.cstruct()), _p(l32), _p(l64), _p(ids), len(ids), _p(a32),
                    _p(a64))
    return (a32, a64) if l64 is not None else a32


def exact(ix: Index, q, ids):
    """Exact squared distances (float32) of explicit IDs to one query."""
    q = _q(np.asarray(q).reshape(-1))
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int32))
    out = np.empty(len(ids), dtype=np.float32)
    _load().orc_exact(ctypes.byref(ix.cstruct()), _p(q), _p(ids), len(ids), _p(out))
    return out


@dataclass
class PageLayout:
    """Raw vectors on fixed-size pages, bucketed by nearest list (Sec. 4.3)."""
    page: np.ndarray      # [n] page of each vector
    slot: np.ndarray      # [n] slot of each vector inside its page
    pages: int
    per_page: int


def page_layout(bucket_of, nbuckets: int, row_bytes: int, page_bytes: int = 4096) -> PageLayout:
    """Buckets (one per list: the vectors whose nearest list it is, ascending
    ID) laid out on pages of page_bytes holding whole vectors of row_bytes:
    every bucket's full pages first, then the buckets' leftover tails combined
    onto shared pages, largest tail first and then the largest that still fits."""
    b = np.ascontiguousarray(np.asarray(bucket_of, dtype=np.int32))
    n = len(b)
    page = np.empty(n, dtype=np.int32)
    slot = np.empty(n, dtype=np.int32)
    np_ = _load().orc_page_layout(_p(b), n, int(nbuckets), int(row_bytes), int(page_bytes),
                                  _p(page), _p(slot))
    if np_ < 0:
        raise ValueError("a vector does not fit a page")
    return PageLayout(page, slot, int(np_), page_bytes // row_bytes)


def index_page_layout(ix: "Index", page_bytes: int = 4096) -> PageLayout:
    """The layout of an index's raw vectors: bucket = each vector's first (nearest) list."""
    row = ix.dim * (4 if ix.kind == "f32" else 1)
    return page_layout(ix.assign[:, 0], ix.nlist, row, page_bytes)


@dataclass
class NavGraph:
    """A navigation graph over the list centroids (Sec. 4.1): adj [nlist, deg]
    neighbour lists (-1 padded), the entry vertices, and the walk's beam width."""
    adj: np.ndarray
    entry: np.ndarray
    beam: int

    def cstruct(self) -> _OrcGraph:
        self.adj = np.ascontiguousarray(self.adj, dtype=np.int32)
        self.entry = np.ascontiguousarray(self.entry, dtype=np.int32)
        return _OrcGraph(self.adj.ctypes.data, self.adj.shape[1], len(self.entry),
                         self.entry.ctypes.data, int(self.beam), 0)


def graph_probe(ix: Index, g: NavGraph, Q, nprobe, threads: int = 0):
    """Step 2 by a best-first beam search of the navigation graph: (lists [nq,
    max nprobe] -1 padded, float32 distances +inf padded, distances computed
    per query)."""
    Q = _q(Q)
    nq = Q.shape[0]
    npr = _np(nprobe, nq)
    w = int(npr.max()) if nq else 0
    lists = np.empty((nq, w), dtype=np.int32)
    d = np.empty((nq, w), dtype=np.float32)
    nd = np.empty(nq, dtype=np.int64)
    gs = g.cstruct()
    _load().orc_graph_probe(ctypes.byref(ix.cstruct()), ctypes.byref(gs), _p(Q), nq, _p(npr), w,
                            _p(lists), _p(d), _p(nd), threads)
    return lists, d, nd


@dataclass
class SearchResult:
    ids: np.ndarray
    dists: np.ndarray
    topn_ids: np.ndarray
    topn_adc: np.ndarray
    ncand: np.ndarray
    nentries: np.ndarray
    reranked: np.ndarray = None
    page_reads: np.ndarray = None


def search(ix: Index, Q, nprobe, k: int, rerank_n: int, threads: int = 0,
           lut_f16: bool = False, heuristic=None, pages: PageLayout = None,
           graph: NavGraph = None) -> SearchResult:
    """Steps 1-8 for a batch of queries (lut_f16: half-precision table variant;
    heuristic = (batch_size, eps, beta): step 8 by the heuristic re-ranking;
    pages: a page layout of the raw vectors, whose page reads per query are
    then counted; graph: step 2 by the navigation-graph walk)."""
    Q = _q(Q)
    nq = Q.shape[0]
    npr = _np(nprobe, nq)
    ids = np.empty((nq, k), dtype=np.int64)
    dists = np.empty((nq, k), dtype=np.float32)
    tids = np.empty((nq, rerank_n), dtype=np.int32)
    tadc = np.empty((nq, rerank_n), dtype=np.float32)
    nc = np.empty(nq, dtype=np.int64)
    ne = np.empty(nq, dtype=np.int64)
    hb, he, hbeta = heuristic if heuristic else (0, 0.0, 1)
    rr = np.empty(nq, dtype=np.int64)
    pr = np.empty(nq, dtype=np.int64) if pages is not None else None
    _load().orc_search(ctypes.byref(ix.cstruct()), _p(Q), nq, _p(npr), k, rerank_n, _p(ids),
                       _p(dists), _p(tids), _p(tadc), _p(nc), _p(ne), threads,
                       1 if lut_f16 else 0, int(hb), float(he), int(hbeta), _p(rr),
                       _p(pages.page) if pages is not None else None, _p(pr),
                       ctypes.byref(graph.cstruct()) if graph is not None else None)
    return SearchResult(ids, dists, tids, tadc, nc, ne, rr, pr)


def bruteforce(ix: Index, Q, k: int, threads: int = 0):
    """Exact kNN over all vectors: (ids [nq, k] int64, squared distances float32)."""
    Q = _q(Q)
    nq = Q.shape[0]
    ids = np.empty((nq, k), dtype=np.int64)
    d = np.empty((nq, k), dtype=np.float32)
    _load().orc_bruteforce(ctypes.byref(ix.cstruct()), _p(Q), nq, k, _p(ids), _p(d), threads)
    return ids, d


def recall_at_k(found: np.ndarray, truth: np.ndarray, k: int) -> float:
    """Mean |found_q[:k] ∩ truth_q[:k]| / k over queries."""
    hits = 0
    for a, b in zip(found, truth):
        hits += len(set(int(x) for x in a[:k] if x >= 0) & set(int(x) for x in b[:k]))
    return hits / (k * len(found)) if len(found) else 1.0
