"""Offline IVF-PQ index construction and the index file writer.

The index follows the paper's offline processing (Sec. 3, Sec. 4.1): the
dataset is clustered into posting lists, boundary vectors are replicated into
neighbouring lists by the rule of Eq. 2 (at most R lists per vector), the
posting lists are reduced to vector IDs, and every vector gets one M-byte PQ
code (Sec. 2.2).  ``build_nav_graph`` builds the navigation graph over the
list centroids (Sec. 4.1) for the graph probe; without it the search probes
the centroids exactly.

Clustering is flat k-means for up to ``FLAT_MAX_LISTS`` lists and two-level
(hierarchical) k-means above that, following the paper's hierarchical
clustering of the dataset.  For uint8/int8 data the list centroids and the PQ
codebooks are rounded to the integer grid of the data type, so every distance
the search computes between a query and a centroid, a codeword or a vector is
an exact integer.

File layout (little-endian), as read by ``ann_load_index``:

======  ============  =====================================================
offset  type          field
======  ============  =====================================================
0       char[8]       magic ``FANNIDX1``
8       u32           version (1)
12      u32           header bytes (512)
16      u32           dtype: 0 float32, 1 uint8, 2 int8
20      u32           dimension D
24      u64           N vectors
32      u32           nlist
36      u32           M subspaces
40      u32           ksub (256)
44      u32           dsub = D / M
48      u32           R, max lists per vector
52      u32           flags: bit 0 = centroids and codebooks are integers
56      f32           eps of Eq. 2 used at build time
60      u32           number of sections (7)
64      u64           E, total posting-list entries
128     7 x 24 bytes  sections: u64 offset, u64 bytes, u32 crc32, u32 0
508     u32           crc32 of header bytes 0..507
======  ============  =====================================================

Sections, each starting on a 4096-byte boundary, all in external vector order:
0 centroids f32 [nlist, D]; 1 codebooks f32 [M, ksub, dsub]; 2 codes u8
[N, M]; 3 vectors [N, D] of dtype; 4 list offsets i64 [nlist + 1]; 5 list
entries i32 [E] (external IDs, ascending inside each list); 6 assignment i32
[N, R] (each vector's lists, nearest first, -1 padded).
"""
from __future__ import annotations

import ctypes
import os
import struct
import subprocess
import zlib
from dataclasses import dataclass

import numpy as np

from .. import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ivfpq_build.cpp")
LIB = os.path.join(HERE, "_ivfpq_build.so")

MAGIC = b"FANNIDX1"
HEADER_BYTES = 512
DTYPE_CODE = {"f32": 0, "u8": 1, "i8": 2}
NP_DTYPE = {"f32": np.float32, "u8": np.uint8, "i8": np.int8}
FLAT_MAX_LISTS = 4096
ROW_CHUNK = 1 << 20

_lib = None


def compile_builder(force: bool = False) -> str:
    """Compile the C++ helpers with g++ (OpenMP) into an in-tree shared object."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["g++", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-std=c++17", SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(compile_builder())
        P = ctypes.c_void_p
        i64, i32, f32 = ctypes.c_int64, ctypes.c_int, ctypes.c_float
        lib.bld_kmeans.argtypes = [P, i64, i32, P, i32, i32]
        lib.bld_nearest.argtypes = [P, i64, i32, P, i32, P, P]
        lib.bld_assign_flat.argtypes = [P, i64, i32, P, i32, i32, f32, P]
        lib.bld_assign_hier.argtypes = [P, i64, i32, P, i32, P, P, i32, i32, f32, P]
        lib.bld_pq_encode.argtypes = [P, i64, i32, P, i32, i32, i32, P]
        lib.bld_balanced_assign.argtypes = [P, i64, i32, P, i32, i64, i32, P]
        lib.bld_nav_graph.argtypes = [P, i32, i32, i32, P, i32, P, P, i32, i32, i32, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class BuildParams:
    nlist: int
    M: int
    R: int = 2
    eps: float = 0.1
    ksub: int = 256
    kmeans_iters: int = 10
    pq_iters: int = 20
    train_per_list: int = 40
    pq_train_rows: int = 65536
    hier_top_probe: int = 2
    balance: float = 0.0      # > 0: balanced clustering, at most (1 + balance) x the mean size
    balance_iters: int = 3
    seed: int = 0
    init_centroids: np.ndarray | None = None  # optional initial list centroids


def _rows_f32(X: np.ndarray, r0: int, r1: int) -> np.ndarray:
    return np.ascontiguousarray(X[r0:r1], dtype=np.float32)


def kmeans(Xs: np.ndarray, k: int, iters: int, seed: int, init: np.ndarray | None = None) -> np.ndarray:
    """Lloyd k-means on float32 rows, initialised from k distinct seeded rows."""
    lib = _load()
    Xs = np.ascontiguousarray(Xs, dtype=np.float32)
    n, d = Xs.shape
    if init is None:
        rng = np.random.default_rng(seed)
        if n >= k:
            pick = rng.choice(n, size=k, replace=False)
        else:
            pick = rng.choice(n, size=k, replace=True)
        C = np.ascontiguousarray(Xs[pick])
        if n < k:  # duplicate rows: separate them slightly so all clusters can be used
            C = C + rng.standard_normal(C.shape).astype(np.float32) * 1e-3
    else:
        C = np.ascontiguousarray(init, dtype=np.float32).copy()
    lib.bld_kmeans(_ptr(Xs), n, d, _ptr(C), k, iters)
    return C


def balanced_kmeans(Xs: np.ndarray, C: np.ndarray, slack: float, iters: int) -> np.ndarray:
    """Lloyd iterations whose assignment step is capacity-constrained: each
    cluster holds at most ceil((1 + slack) n / k) rows (bld_balanced_assign);
    starts from centroids C, returns the new centroids."""
    lib = _load()
    Xs = np.ascontiguousarray(Xs, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32).copy()
    n, d = Xs.shape
    k = C.shape[0]
    cap = int(np.ceil((1.0 + slack) * n / k))
    lab = np.empty(n, dtype=np.int32)
    for _ in range(max(1, iters)):
        lib.bld_balanced_assign(_ptr(Xs), n, d, _ptr(C), k, cap, 8, _ptr(lab))
        sums = np.zeros((k, d), dtype=np.float64)
        np.add.at(sums, lab, Xs)
        cnt = np.bincount(lab, minlength=k)
        nz = cnt > 0
        C[nz] = (sums[nz] / cnt[nz, None]).astype(np.float32)
    return C


def _grid(a: np.ndarray, kind: str) -> np.ndarray:
    if kind == "u8":
        return np.clip(np.rint(a), 0, 255).astype(np.float32)
    if kind == "i8":
        return np.clip(np.rint(a), -128, 127).astype(np.float32)
    return a.astype(np.float32)


def train_ivf(X: np.ndarray, kind: str, p: BuildParams):
    """Return (centroids [nlist, D] f32, hierarchy or None)."""
    n, d = X.shape
    ns = min(n, max(p.nlist * p.train_per_list, 1))
    rows = inputs.sample_rows(p.seed, n, ns)
    Xs = np.ascontiguousarray(X[rows], dtype=np.float32)
    if p.init_centroids is not None or p.nlist <= FLAT_MAX_LISTS:
        C = kmeans(Xs, p.nlist, p.kmeans_iters, p.seed + 1, init=p.init_centroids)
        if p.balance > 0:
            C = balanced_kmeans(Xs, C, p.balance, p.balance_iters)
        return _grid(C, kind), None
    # Two-level: ktop clusters, then each split into sub-lists proportional to its size.
    ktop = 1 << int(np.ceil(np.log2(np.sqrt(p.nlist))))
    ktop = min(ktop, p.nlist)
    Ctop = kmeans(Xs, ktop, p.kmeans_iters, p.seed + 2)
    if p.balance > 0:  # hierarchical balanced clustering: every level balanced
        Ctop = balanced_kmeans(Xs, Ctop, p.balance, p.balance_iters)
    lib = _load()
    lab = np.empty(ns, dtype=np.int32)
    lib.bld_nearest(_ptr(Xs), ns, d, _ptr(Ctop), ktop, _ptr(lab), None)
    sizes = np.bincount(lab, minlength=ktop).astype(np.float64)
    share = sizes / sizes.sum() * p.nlist
    cnt = np.maximum(np.floor(share).astype(np.int64), 1)
    while cnt.sum() > p.nlist:
        j = int(np.argmax(cnt - share))
        cnt[j] -= 1
    rem = share - cnt
    order = np.argsort(-rem, kind="stable")
    i = 0
    while cnt.sum() < p.nlist:
        cnt[order[i % ktop]] += 1
        i += 1
    subs = []
    for a in range(ktop):
        Xa = Xs[lab == a]
        if len(Xa) == 0:
            Xa = Ctop[a:a + 1]
        Ca = kmeans(Xa, int(cnt[a]), p.kmeans_iters, p.seed + 1000 + a)
        if p.balance > 0 and len(Xa) >= cnt[a]:
            Ca = balanced_kmeans(Xa, Ca, p.balance, p.balance_iters)
        subs.append(Ca)
    Csub = np.ascontiguousarray(np.concatenate(subs, axis=0))
    off = np.zeros(ktop + 1, dtype=np.int32)
    off[1:] = np.cumsum(cnt)
    return _grid(Csub, kind), (_grid(Ctop, kind) if kind != "f32" else Ctop.astype(np.float32), off)


def assign_lists(X: np.ndarray, C: np.ndarray, hier, p: BuildParams, progress=None) -> np.ndarray:
    lib = _load()
    n, d = X.shape
    A = np.empty((n, p.R), dtype=np.int32)
    for r0 in range(0, n, ROW_CHUNK):
        if progress and r0 and r0 % (16 * ROW_CHUNK) == 0:
            progress(f"assigned {r0} of {n} vectors")
        r1 = min(n, r0 + ROW_CHUNK)
        Xc = _rows_f32(X, r0, r1)
        out = np.empty((r1 - r0, p.R), dtype=np.int32)
        if hier is None:
            lib.bld_assign_flat(_ptr(Xc), r1 - r0, d, _ptr(C), C.shape[0], p.R, p.eps, _ptr(out))
        else:
            Ctop, off = hier
            Ctop = np.ascontiguousarray(Ctop, dtype=np.float32)
            lib.bld_assign_hier(_ptr(Xc), r1 - r0, d, _ptr(Ctop), Ctop.shape[0], _ptr(C),
                                _ptr(off), p.hier_top_probe, p.R, p.eps, _ptr(out))
        A[r0:r1] = out
    return A


def assign_lists_gpu(X: np.ndarray, C: np.ndarray, kind: str, R: int, eps: float,
                     device: int = 0, chunk: int = 65536, progress=None) -> np.ndarray:
    """Eq. 2 assignment on the GPU, by the search library's exact probe: the R
    nearest lists of every row over all centroids (exact distances: integers
    on the integer grid, float64 sums otherwise; ties to the lower list), list
    i kept iff its squared distance is at most (1 + eps)^2 times the nearest
    one's.  The centroids are loaded as a small index of their own (one
    vector per list).  Returns [n, R] int32, nearest first, -1 padded."""
    import tempfile

    import torch

    from .. import ann
    C = np.ascontiguousarray(C, dtype=np.float32)
    nlist, d = C.shape
    dsub = next(s_ for s_ in range(1, d + 1) if d % s_ == 0 and d // s_ <= 64)
    M = d // dsub
    own = np.stack([np.arange(nlist), -np.ones(nlist, dtype=np.int64)], axis=1).astype(np.int32)
    off, ent = lists_from_assignment(own, nlist)
    cix = IndexArrays(kind, C, np.zeros((M, 256, dsub), np.float32), np.zeros((nlist, M), np.uint8),
                      C.astype(NP_DTYPE[kind]), off, ent, own, 0.0, kind != "f32")
    n = X.shape[0]
    A = np.full((n, R), -1, dtype=np.int32)
    lim = (1.0 + float(eps)) ** 2
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "centroids.fidx")
        write_index(path, cix)
        g = ann.Index(path, device)
        try:
            for r0 in range(0, n, chunk):
                r1 = min(n, r0 + chunk)
                q = torch.from_numpy(np.ascontiguousarray(X[r0:r1], dtype=np.float32)).cuda(device)
                lists, dist = g.probe(q, min(R, nlist))
                lists, dist = lists.cpu().numpy(), dist.cpu().numpy().astype(np.float64)
                keep = dist <= lim * dist[:, :1]  # ascending, so the kept lists are a prefix
                A[r0:r1, :lists.shape[1]] = np.where(keep, lists, -1)
                if progress and r0 and r0 % (16 * chunk) == 0:
                    progress(f"assigned {r0} of {n} vectors on the GPU")
        finally:
            g.close()
    return A


def train_pq(X: np.ndarray, kind: str, p: BuildParams) -> np.ndarray:
    n, d = X.shape
    dsub = d // p.M
    rows = inputs.sample_rows(p.seed + 5, n, p.pq_train_rows)
    Xs = np.ascontiguousarray(X[rows], dtype=np.float32)
    CB = np.empty((p.M, p.ksub, dsub), dtype=np.float32)
    for m in range(p.M):
        sub = np.ascontiguousarray(Xs[:, m * dsub:(m + 1) * dsub])
        CB[m] = kmeans(sub, p.ksub, p.pq_iters, p.seed + 7000 + m)
    return _grid(CB, kind).reshape(p.M, p.ksub, dsub)


def encode_pq(X: np.ndarray, CB: np.ndarray) -> np.ndarray:
    lib = _load()
    n, d = X.shape
    M, ksub, dsub = CB.shape
    CBc = np.ascontiguousarray(CB, dtype=np.float32)
    codes = np.empty((n, M), dtype=np.uint8)
    for r0 in range(0, n, ROW_CHUNK):
        r1 = min(n, r0 + ROW_CHUNK)
        Xc = _rows_f32(X, r0, r1)
        out = np.empty((r1 - r0, M), dtype=np.uint8)
        lib.bld_pq_encode(_ptr(Xc), r1 - r0, d, _ptr(CBc), M, ksub, dsub, _ptr(out))
        codes[r0:r1] = out
    return codes


def lists_from_assignment(A: np.ndarray, nlist: int):
    """CSR posting lists (external IDs ascending inside each list) from [N, R] assignment."""
    n, R = A.shape
    ids = np.repeat(np.arange(n, dtype=np.int64), R)
    lst = A.reshape(-1).astype(np.int64)
    keep = lst >= 0
    ids, lst = ids[keep], lst[keep]
    order = np.lexsort((ids, lst))
    entries = ids[order].astype(np.int32)
    counts = np.bincount(lst, minlength=nlist)
    offsets = np.zeros(nlist + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return offsets, entries


@dataclass
class IndexArrays:
    kind: str
    centroids: np.ndarray
    codebooks: np.ndarray
    codes: np.ndarray
    vectors: np.ndarray
    offsets: np.ndarray
    entries: np.ndarray
    assign: np.ndarray
    eps: float
    int_grid: bool


def build_arrays(X: np.ndarray, kind: str, p: BuildParams, progress=None) -> IndexArrays:
    """progress: optional callable taking a message per finished stage."""
    assert X.dtype == NP_DTYPE[kind] and X.ndim == 2
    n, d = X.shape
    if d % p.M:
        raise ValueError(f"D={d} is not a multiple of M={p.M}")
    say = progress or (lambda _m: None)
    C, hier = train_ivf(X, kind, p)
    say("list centroids trained")
    A = assign_lists(X, C, hier, p, progress)
    say("vectors assigned to lists")
    CB = train_pq(X, kind, p)
    say("PQ codebooks trained")
    codes = encode_pq(X, CB)
    say("vectors encoded")
    offsets, entries = lists_from_assignment(A, p.nlist)
    return IndexArrays(kind, C, CB, codes, X, offsets, entries, A, p.eps, kind != "f32")


def write_index(path: str, ix: IndexArrays) -> None:
    n, d = ix.vectors.shape
    nlist = ix.centroids.shape[0]
    M, ksub, dsub = ix.codebooks.shape
    R = ix.assign.shape[1]
    secs = [
        np.ascontiguousarray(ix.centroids, dtype=np.float32),
        np.ascontiguousarray(ix.codebooks, dtype=np.float32),
        np.ascontiguousarray(ix.codes, dtype=np.uint8),
        np.ascontiguousarray(ix.vectors, dtype=NP_DTYPE[ix.kind]),
        np.ascontiguousarray(ix.offsets, dtype=np.int64),
        np.ascontiguousarray(ix.entries, dtype=np.int32),
        np.ascontiguousarray(ix.assign, dtype=np.int32),
    ]
    table = []
    off = HEADER_BYTES
    for s in secs:
        off = (off + 4095) // 4096 * 4096
        mv = memoryview(s).cast("B")
        table.append((off, s.nbytes, zlib.crc32(mv) & 0xFFFFFFFF))
        off += s.nbytes
    hdr = bytearray(HEADER_BYTES)
    struct.pack_into("<8sIIIIQIIIIIIfIQ", hdr, 0, MAGIC, 1, HEADER_BYTES, DTYPE_CODE[ix.kind], d,
                     n, nlist, M, ksub, dsub, R, 1 if ix.int_grid else 0, float(ix.eps),
                     len(secs), int(ix.entries.shape[0]))
    for i, (o, b, c) in enumerate(table):
        struct.pack_into("<QQII", hdr, 128 + 24 * i, o, b, c, 0)
    struct.pack_into("<I", hdr, 508, zlib.crc32(bytes(hdr[:508])) & 0xFFFFFFFF)
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        f.write(hdr)
        for (o, b, c), s in zip(table, secs):
            f.seek(o)
            f.write(memoryview(s).cast("B"))
    os.replace(tmp, path)


def build_index(path: str, X: np.ndarray, kind: str, p: BuildParams, progress=None) -> IndexArrays:
    ix = build_arrays(X, kind, p, progress)
    write_index(path, ix)
    return ix


def read_centroids(path: str) -> np.ndarray:
    """The list centroids [nlist, D] float32 of an index file."""
    with open(path, "rb") as f:
        hdr = f.read(HEADER_BYTES)
        if hdr[:8] != MAGIC:
            raise ValueError("not an index file")
        dim, nlist = struct.unpack_from("<I", hdr, 20)[0], struct.unpack_from("<I", hdr, 32)[0]
        off, nbytes = struct.unpack_from("<QQ", hdr, 128)
        if nbytes != nlist * dim * 4:
            raise ValueError("centroid section size")
        f.seek(off)
        return np.frombuffer(f.read(nbytes), dtype=np.float32).reshape(nlist, dim).copy()


def read_list_meta(path: str):
    """(list sizes, first-list member counts) of an index file, without the big sections."""
    with open(path, "rb") as f:
        hdr = f.read(HEADER_BYTES)
        if hdr[:8] != MAGIC:
            raise ValueError("not an index file")
        n, nlist = struct.unpack_from("<Q", hdr, 24)[0], struct.unpack_from("<I", hdr, 32)[0]
        R = struct.unpack_from("<I", hdr, 48)[0]
        offs_off, offs_bytes = struct.unpack_from("<QQ", hdr, 128 + 24 * 4)
        asg_off, asg_bytes = struct.unpack_from("<QQ", hdr, 128 + 24 * 6)
        f.seek(offs_off)
        offsets = np.frombuffer(f.read(offs_bytes), dtype=np.int64)
        f.seek(asg_off)
        first = np.frombuffer(f.read(asg_bytes), dtype=np.int32).reshape(n, R)[:, 0]
    sizes = np.diff(offsets)
    primary = np.bincount(first, minlength=nlist).astype(np.int64)
    return sizes, primary


def build_nav_graph(C: np.ndarray, deg: int = 32, seed: int = 0, gprobe: int = 8,
                    rng: bool = True, pool: int = 0):
    """Navigation graph over list centroids C [nlist, D] (Sec. 4.1).

    Candidates of a centroid: the ``pool`` (default 4 deg) nearest members of
    its ``gprobe`` nearest centroid groups (a k-means of the centroids into
    about sqrt(nlist) groups).  Its edges: with ``rng``, first the candidates
    that pass the relative neighbourhood rule (no edge already taken is nearer
    to the candidate than the centroid itself), then the nearest candidates
    left, up to ``deg``; without, the ``deg`` nearest.  A centroid chosen by
    another is offered that one as a candidate too (reverse edges) and its
    edges are chosen again.  Entry vertices: the member nearest to each
    group's centre, plus one vertex of every part of the graph those do not
    reach, so every centroid is reachable from the entries.

    Returns (adj [nlist, deg] int32, -1 padded; entry int32).
    """
    lib = _load()
    C = np.ascontiguousarray(C, dtype=np.float32)
    k, d = C.shape
    deg = max(1, min(int(deg), max(k - 1, 1)))
    ng = max(1, min(k, int(round(np.sqrt(k)))))
    G = kmeans(C, ng, 5, seed + 31)
    gof = np.empty(k, dtype=np.int32)
    gd = np.empty(k, dtype=np.float32)
    lib.bld_nearest(_ptr(C), k, d, _ptr(G), ng, _ptr(gof), _ptr(gd))
    order = np.lexsort((np.arange(k), gof))
    gmem = np.ascontiguousarray(order.astype(np.int32))
    goff = np.zeros(ng + 1, dtype=np.int32)
    goff[1:] = np.cumsum(np.bincount(gof, minlength=ng))
    adj = np.empty((k, deg), dtype=np.int32)
    lib.bld_nav_graph(_ptr(C), k, d, deg, _ptr(G), ng, _ptr(goff), _ptr(gmem), int(gprobe),
                      int(pool or 4 * deg), 1 if rng else 0, _ptr(adj))
    entry = []
    for g in range(ng):
        mem = gmem[goff[g]:goff[g + 1]]
        if len(mem):
            dd = ((C[mem] - G[g]) ** 2).sum(1)
            entry.append(int(mem[np.lexsort((mem, dd))[0]]))
    # reachability from the entries (breadth first); unreached parts get an entry
    seen = np.zeros(k, dtype=bool)

    def reach(starts):
        front = np.array(starts, dtype=np.int64)
        seen[front] = True
        while len(front):
            nb = adj[front].reshape(-1)
            nb = np.unique(nb[nb >= 0])
            nb = nb[~seen[nb]]
            seen[nb] = True
            front = nb

    reach(entry)
    while not seen.all():
        v = int(np.argmin(seen))
        entry.append(v)
        reach([v])
    return adj, np.asarray(entry, dtype=np.int32)
