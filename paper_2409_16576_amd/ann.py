"""Thin ctypes binding of the C ABI in include/ann.h.

Argument marshalling only: every step of the search runs in the HIP kernels
of ``libann.so``.  Torch tensors provide device memory and the current HIP
stream; outputs are allocated here with torch and filled by the library.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBANN = os.path.join(HERE, "libann.so")

ANN_OK = 0
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EIO", 4: "EFORMAT", 5: "EDEVICE", 6: "EUNSUPPORTED"}


class AnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ann {_STATUS.get(status, status)}: {msg}")
        self.status = status


class IndexDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("nlist", ctypes.c_int32), ("m", ctypes.c_int32), ("ksub", ctypes.c_int32),
        ("dsub", ctypes.c_int32), ("r", ctypes.c_int32), ("int_grid", ctypes.c_int32),
        ("entries", ctypes.c_int64), ("replica_entries", ctypes.c_int64),
        ("max_list", ctypes.c_int64), ("hbm_bytes", ctypes.c_int64), ("device", ctypes.c_int32),
        ("max_rerank_n", ctypes.c_int32), ("raw_tier", ctypes.c_int32),
        ("page_bytes", ctypes.c_int32), ("pages", ctypes.c_int64), ("host_bytes", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class LoadCfg(ctypes.Structure):
    _fields_ = [("raw_tier", ctypes.c_int32), ("page_bytes", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 6), ("launches", ctypes.c_int64 * 6)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int64), ("split", ctypes.c_int32), ("tried", ctypes.c_int32),
                ("ms", ctypes.c_double), ("list_major", ctypes.c_int32),
                ("lm_alpha", ctypes.c_int32), ("lm_tile", ctypes.c_int32),
                ("lm_blocks", ctypes.c_int32), ("lm_min_rows", ctypes.c_int32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_nprobe", ctypes.c_int32),
                ("max_k", ctypes.c_int32), ("max_rerank_n", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_int64), ("queries_done", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("max_in_flight", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("budget_bytes", ctypes.c_int64),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


STAGES = ("probe", "lut", "scan", "merge_rerank", "list_major", "lm_worklist")

_lib = None


def lib():
    """The loaded libann.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBANN):
            raise RuntimeError(f"{LIBANN} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIBANN)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.ann_last_error.restype = ctypes.c_char_p
        L.ann_load_index.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(P)]
        L.ann_load_index_ex.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(LoadCfg),
                                        ctypes.POINTER(P)]
        L.ann_search_pages.argtypes = [P, P, i64, P, i32, i32, i32, i32, ctypes.c_double, i32,
                                       P, P, P, P, P]
        L.ann_index_info.argtypes = [P, ctypes.POINTER(IndexDesc)]
        L.ann_free_index.argtypes = [P]
        L.ann_free_index.restype = None
        L.ann_search.argtypes = [P, P, i64, P, i32, i32, i32, P, P, P]
        L.ann_search_noalloc.argtypes = [P, P, i64, P, i32, i32, i32, P, P, P]
        L.ann_noalloc_scratch_bytes.argtypes = []
        L.ann_noalloc_scratch_bytes.restype = ctypes.c_size_t
        L.ann_search_topn.argtypes = [P, P, i64, P, i32, i32, P, P, P, P, P]
        L.ann_probe.argtypes = [P, P, i64, P, i32, P, P, P]
        L.ann_lut.argtypes = [P, P, i64, P, P]
        L.ann_scan_trace.argtypes = [P, P, i64, i32, P, i64, P, P, P, P]
        L.ann_rerank.argtypes = [P, P, i64, P, i32, i32, P, P, P]
        L.ann_set_profiling.argtypes = [P, ctypes.c_int]
        L.ann_get_profile.argtypes = [P, ctypes.POINTER(Profile), ctypes.c_int]
        L.ann_set_option.argtypes = [P, ctypes.c_int, i64]
        L.ann_set_nav_graph.argtypes = [P, P, i32, P, i32]
        L.ann_get_option.argtypes = [P, ctypes.c_int, ctypes.POINTER(i64)]
        L.ann_adc_forward.argtypes = [P, i64, P, i32, i32, P, i64, P, P]
        L.ann_exact_sq.argtypes = [P, i64, P, i64, i32, P, P]
        L.ann_exact_sq.restype = ctypes.c_int
        L.ann_adc_forward.restype = ctypes.c_int
        L.ann_adc_backward_workspace.argtypes = [i64, i64, i32, i32]
        L.ann_adc_backward_workspace.restype = ctypes.c_size_t
        L.ann_adc_backward.argtypes = [P, i64, P, i32, i32, P, i64, P, P, P, P, ctypes.c_size_t, P]
        L.ann_adc_backward.restype = ctypes.c_int
        L.ann_search_heuristic.argtypes = [P, P, i64, P, i32, i32, i32, i32, ctypes.c_double, i32,
                                           P, P, P, P]
        L.ann_graph_create.argtypes = [P, P, i64, P, i32, i32, i32, P, P, ctypes.POINTER(P)]
        L.ann_graph_launch.argtypes = [P, P]
        L.ann_graph_free.argtypes = [P]
        L.ann_graph_free.restype = None
        L.ann_autotune.argtypes = [P, P, i64, P, i32, i32, i32, i32, ctypes.POINTER(TuneResult)]
        L.ann_server_start.argtypes = [P, ctypes.POINTER(ServerCfg), ctypes.POINTER(P)]
        L.ann_server_submit.argtypes = [P, P, i32, P, i32, i32, i32,
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.ann_server_poll.argtypes = [P, ctypes.c_uint64, P, P, ctypes.POINTER(i32), i32]
        L.ann_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats), ctypes.c_int]
        L.ann_server_stop.argtypes = [P]
        for f in ("ann_load_index", "ann_index_info", "ann_search", "ann_search_topn", "ann_probe",
                  "ann_lut", "ann_scan_trace", "ann_rerank", "ann_set_profiling",
                  "ann_get_profile", "ann_set_option", "ann_get_option", "ann_server_start",
                  "ann_server_submit", "ann_server_poll", "ann_server_get_stats",
                  "ann_server_stop", "ann_graph_create", "ann_graph_launch", "ann_autotune",
                  "ann_search_heuristic", "ann_search_noalloc", "ann_load_index_ex",
                  "ann_search_pages", "ann_set_nav_graph"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != ANN_OK:
        raise AnnError(status, lib().ann_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device, stream):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


class Index:
    """A loaded index on one GPU (see ann_load_index)."""

    def __init__(self, path: str, device: int = 0, raw_tier: int = 0, page_bytes: int = 0):
        """raw_tier 1: raw vectors on pages of page_bytes in pinned host memory."""
        h = ctypes.c_void_p()
        cfg = LoadCfg(int(raw_tier), int(page_bytes))
        _check(lib().ann_load_index_ex(path.encode(), int(device), ctypes.byref(cfg),
                                       ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", int(device))
        d = IndexDesc()
        _check(lib().ann_index_info(self._h, ctypes.byref(d)))
        self.desc = d.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().ann_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------------
    def _queries(self, q):
        if not (q.is_cuda and q.device == self.device and q.dtype == torch.float32
                and q.dim() == 2 and q.shape[1] == self.desc["dim"]):
            raise ValueError("queries must be a float32 [nq, dim] tensor on the index device")
        return q.contiguous()

    def _nprobe(self, nprobe, nq):
        if isinstance(nprobe, int):
            return None, int(nprobe)
        t = nprobe.to(device=self.device, dtype=torch.int32).contiguous()
        if t.numel() != nq:
            raise ValueError("nprobe tensor must have one entry per query")
        mx = int(t.max().item()) if nq else 1
        return t, max(1, mx)

    # -- entry points ------------------------------------------------------------
    def search(self, queries, nprobe, k: int, rerank_n: int, stream=None):
        """Steps 1-8: (ids int64 [nq, k], squared distances float32 [nq, k])."""
        q = self._queries(queries)
        nq = q.shape[0]
        npt, npmax = self._nprobe(nprobe, nq)
        ids = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        d = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        _check(lib().ann_search(self._h, _ptr(q), nq, _ptr(npt), npmax, k, rerank_n, _ptr(ids),
                                _ptr(d), _stream(self.device, stream)))
        return ids, d

    def search_noalloc(self, queries, nprobe, k: int, rerank_n: int, out=None, stream=None):
        """ann_search_noalloc: the same search on the library's fixed per-device
        scratch array (no device allocation in the library).  `out` may give
        preallocated (ids, dists) tensors."""
        q = self._queries(queries)
        nq = q.shape[0]
        npt, npmax = self._nprobe(nprobe, nq)
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int64, device=self.device),
                   torch.empty((nq, k), dtype=torch.float32, device=self.device))
        ids, d = out
        _check(lib().ann_search_noalloc(self._h, _ptr(q), nq, _ptr(npt), npmax, k, rerank_n,
                                        _ptr(ids), _ptr(d), _stream(self.device, stream)))
        return ids, d

    def search_heuristic(self, queries, nprobe, k: int, rerank_n: int, batch_size: int,
                         eps: float, beta: int, stream=None):
        """Steps 1-8 with the heuristic re-ranking (Alg. 1): (ids, dists, re-ranked counts)."""
        q = self._queries(queries)
        nq = q.shape[0]
        npt, npmax = self._nprobe(nprobe, nq)
        ids = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        d = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        rr = torch.empty((nq,), dtype=torch.int32, device=self.device)
        _check(lib().ann_search_heuristic(self._h, _ptr(q), nq, _ptr(npt), npmax, k, rerank_n,
                                          int(batch_size), float(eps), int(beta), _ptr(ids),
                                          _ptr(d), _ptr(rr), _stream(self.device, stream)))
        return ids, d, rr

    def search_pages(self, queries, nprobe, k: int, rerank_n: int, batch_size: int = 0,
                     eps: float = 0.0, beta: int = 1, stream=None):
        """Steps 1-8 from host-memory pages (raw_tier 1): (ids, dists, re-ranked
        counts int32 [nq], pages read int32 [nq]).  batch_size 0: fixed re-rank,
        else Alg. 1 with (batch_size, eps, beta)."""
        q = self._queries(queries)
        nq = q.shape[0]
        npt, npmax = self._nprobe(nprobe, nq)
        ids = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        d = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        rr = torch.empty((nq,), dtype=torch.int32, device=self.device)
        pr = torch.empty((nq,), dtype=torch.int32, device=self.device)
        _check(lib().ann_search_pages(self._h, _ptr(q), nq, _ptr(npt), npmax, k, rerank_n,
                                      int(batch_size), float(eps), int(beta), _ptr(ids), _ptr(d),
                                      _ptr(rr), _ptr(pr), _stream(self.device, stream)))
        return ids, d, rr, pr

    def search_topn(self, queries, nprobe, rerank_n: int, stream=None, walked: bool = False):
        """Steps 1-7: (ids int32 [nq, n], ADC distances float32 [nq, n], candidates int64 [nq]),
        plus the list entries walked per query (int64 [nq]) when walked=True."""
        q = self._queries(queries)
        nq = q.shape[0]
        npt, npmax = self._nprobe(nprobe, nq)
        ids = torch.empty((nq, rerank_n), dtype=torch.int32, device=self.device)
        adc = torch.empty((nq, rerank_n), dtype=torch.float32, device=self.device)
        nc = torch.empty((nq,), dtype=torch.int64, device=self.device)
        nw = torch.empty((nq,), dtype=torch.int64, device=self.device) if walked else None
        _check(lib().ann_search_topn(self._h, _ptr(q), nq, _ptr(npt), npmax, rerank_n, _ptr(ids),
                                     _ptr(adc), _ptr(nc), _ptr(nw), _stream(self.device, stream)))
        return (ids, adc, nc, nw) if walked else (ids, adc, nc)

    def probe(self, queries, nprobe, with_dists: bool = True, stream=None):
        q = self._queries(queries)
        nq = q.shape[0]
        npt, npmax = self._nprobe(nprobe, nq)
        lists = torch.empty((nq, npmax), dtype=torch.int32, device=self.device)
        d = torch.empty((nq, npmax), dtype=torch.float32, device=self.device) if with_dists else None
        _check(lib().ann_probe(self._h, _ptr(q), nq, _ptr(npt), npmax, _ptr(lists), _ptr(d),
                               _stream(self.device, stream)))
        return lists, d

    def lut(self, queries, stream=None):
        q = self._queries(queries)
        nq = q.shape[0]
        out = torch.empty((nq, self.desc["m"], self.desc["ksub"]), dtype=torch.float32,
                          device=self.device)
        _check(lib().ann_lut(self._h, _ptr(q), nq, _ptr(out), _stream(self.device, stream)))
        return out

    def scan_trace(self, lists, lut, capacity: int, stream=None):
        lists = lists.to(device=self.device, dtype=torch.int32).contiguous()
        lut = lut.to(device=self.device, dtype=torch.float32).contiguous()
        nq, npmax = lists.shape
        ids = torch.empty((nq, capacity), dtype=torch.int32, device=self.device)
        adc = torch.empty((nq, capacity), dtype=torch.float32, device=self.device)
        cnt = torch.empty((nq,), dtype=torch.int64, device=self.device)
        _check(lib().ann_scan_trace(self._h, _ptr(lists), nq, npmax, _ptr(lut), capacity, _ptr(ids),
                                    _ptr(adc), _ptr(cnt), _stream(self.device, stream)))
        return ids, adc, cnt

    def rerank(self, queries, cand_ids, k: int, stream=None):
        q = self._queries(queries)
        cand = cand_ids.to(device=self.device, dtype=torch.int32).contiguous()
        nq, n = cand.shape
        ids = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        d = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        _check(lib().ann_rerank(self._h, _ptr(q), nq, _ptr(cand), n, k, _ptr(ids), _ptr(d),
                                _stream(self.device, stream)))
        return ids, d

    # -- measurement -------------------------------------------------------------
    def set_profiling(self, enable: bool):
        _check(lib().ann_set_profiling(self._h, 1 if enable else 0))

    def get_profile(self, reset: bool = True) -> dict:
        p = Profile()
        _check(lib().ann_get_profile(self._h, ctypes.byref(p), 1 if reset else 0))
        return {s: {"ms": p.ms[i], "launches": p.launches[i]} for i, s in enumerate(STAGES)}

    # -- tuning --------------------------------------------------------------------
    OPT_SCAN_TILE = 1
    OPT_SCAN_SPLIT = 2
    OPT_LUT_F16 = 3
    OPT_SCAN_ORDER = 4
    OPT_LIST_MAJOR = 5
    OPT_LM_ALPHA = 6
    OPT_LM_TILE = 7
    OPT_LM_BLOCKS = 8
    OPT_LM_CAP = 9
    OPT_LM_MIN_ROWS = 10
    OPT_PROBE_BEAM = 11

    def set_nav_graph(self, adj, entry):
        """Navigation graph over the list centroids (host arrays: adj [nlist,
        deg] int32 -1 padded, entry int32); None removes it.  The probe walks
        it once OPT_PROBE_BEAM is set."""
        if adj is None:
            _check(lib().ann_set_nav_graph(self._h, None, 0, None, 0))
            return
        a = np.ascontiguousarray(adj, dtype=np.int32)
        e = np.ascontiguousarray(entry, dtype=np.int32)
        _check(lib().ann_set_nav_graph(self._h, a.ctypes.data, a.shape[1], e.ctypes.data, len(e)))

    def set_option(self, option: int, value: int):
        _check(lib().ann_set_option(self._h, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64()
        _check(lib().ann_get_option(self._h, int(option), ctypes.byref(v)))
        return v.value


# -- batched form (ann_graph_*, ann_autotune) -------------------------------------------

def _nprobe_args(index, Q, nprobe):
    if isinstance(nprobe, int):
        return None, int(nprobe)
    t = nprobe.to(device=index.device, dtype=torch.int32).contiguous()
    return t, int(t.max().item()) if t.numel() else 1


class Graph:
    """A batch search captured into a HIP graph (see ann_graph_create).  Holds the
    query/nprobe/output tensors; launch() replays the search on them."""

    def __init__(self, index, Q, nprobe, k: int, rerank_n: int):
        self.index = index
        self.Q = Q.contiguous()
        self.np_t, self.np_max = _nprobe_args(index, Q, nprobe)
        nq = self.Q.shape[0]
        self.ids = torch.empty((nq, k), dtype=torch.int64, device=index.device)
        self.dists = torch.empty((nq, k), dtype=torch.float32, device=index.device)
        h = ctypes.c_void_p()
        _check(lib().ann_graph_create(index._h, _ptr(self.Q), nq, _ptr(self.np_t), self.np_max,
                                      int(k), int(rerank_n), _ptr(self.ids), _ptr(self.dists),
                                      ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().ann_graph_launch(self._h, _stream(self.index.device, stream)))
        return self.ids, self.dists

    def close(self):
        if getattr(self, "_h", None):
            lib().ann_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(index, Q, nprobe, k: int, rerank_n: int, reps: int = 3) -> dict:
    """Pick and set the batched form's options for this batch (ann_autotune): the
    per-query scan's work split and, on integer-grid indexes, whether to run
    list-major and with which alpha / rows per item / persistent blocks."""
    Q = Q.contiguous()
    np_t, np_max = _nprobe_args(index, Q, nprobe)
    r = TuneResult()
    _check(lib().ann_autotune(index._h, _ptr(Q), Q.shape[0], _ptr(np_t), np_max, int(k),
                              int(rerank_n), int(reps), ctypes.byref(r)))
    out = {"tile": r.tile, "split": r.split, "tried": r.tried, "ms": r.ms,
           "list_major": r.list_major}
    if r.list_major:
        out.update(lm_alpha=r.lm_alpha, lm_tile=r.lm_tile, lm_blocks=r.lm_blocks,
                   lm_min_rows=r.lm_min_rows)
    return out


# -- served form (ann_server_*) ---------------------------------------------------------

class Server:
    """Continuous-batching server over a loaded Index (see ann_server_start).
    Requests are numpy arrays in host memory; results come back as numpy."""

    def __init__(self, index: Index, hbm_budget_bytes: int = 0, max_slots: int = 0,
                 max_batch: int = 0, max_nprobe: int = 0, max_k: int = 0, max_rerank_n: int = 0):
        import numpy as np  # noqa: F401  (results are numpy arrays)
        cfg = ServerCfg(int(hbm_budget_bytes), int(max_slots), int(max_batch), int(max_nprobe),
                        int(max_k), int(max_rerank_n))
        h = ctypes.c_void_p()
        _check(lib().ann_server_start(index._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.index = index
        self._k = {}

    def submit(self, queries, nprobe, k: int, rerank_n: int) -> int:
        """queries: float32 [nq, dim] numpy; nprobe: int or int32 [nq] numpy."""
        import numpy as np
        q = np.ascontiguousarray(queries, dtype=np.float32)
        if isinstance(nprobe, (int, np.integer)):
            npp, npmax = None, int(nprobe)
        else:
            npp = np.ascontiguousarray(nprobe, dtype=np.int32)
            npmax = int(npp.max()) if npp.size else 1
        t = ctypes.c_uint64()
        _check(lib().ann_server_submit(self._h, q.ctypes.data_as(ctypes.c_void_p), q.shape[0],
                                       None if npp is None else npp.ctypes.data_as(ctypes.c_void_p),
                                       npmax, int(k), int(rerank_n), ctypes.byref(t)))
        self._k[t.value] = (q.shape[0], int(k))
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """(ids int64 [nq, k], dists float32 [nq, k]) once done, else None."""
        import numpy as np
        done = ctypes.c_int32()
        if ticket not in self._k:  # not issued here, or already collected: the library says so
            _check(lib().ann_server_poll(self._h, ctypes.c_uint64(ticket), None, None,
                                         ctypes.byref(done), 1 if wait else 0))
            return None
        nq, k = self._k[ticket]
        ids = np.empty((nq, k), dtype=np.int64)
        d = np.empty((nq, k), dtype=np.float32)
        _check(lib().ann_server_poll(self._h, ctypes.c_uint64(ticket),
                                     ids.ctypes.data_as(ctypes.c_void_p),
                                     d.ctypes.data_as(ctypes.c_void_p), ctypes.byref(done),
                                     1 if wait else 0))
        if not done.value:
            return None
        del self._k[ticket]
        return ids, d

    def stats(self, reset: bool = False) -> dict:
        s = ServerStats()
        _check(lib().ann_server_get_stats(self._h, ctypes.byref(s), 1 if reset else 0))
        return s.as_dict()

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(lib().ann_server_stop(h))

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


# -- differentiable PQ distance (ann_adc_forward / ann_adc_backward) ------------------

def _adc_args(Q, CB, codes):
    if not (Q.is_cuda and Q.dtype == torch.float32 and Q.dim() == 2):
        raise ValueError("queries must be a float32 CUDA tensor [B, D]")
    if not (CB.is_cuda and CB.dtype == torch.float32 and CB.dim() == 3 and CB.shape[1] == 256):
        raise ValueError("codebooks must be a float32 CUDA tensor [M, 256, dsub]")
    if not (codes.is_cuda and codes.dtype == torch.uint8 and codes.dim() == 2
            and codes.shape[1] == CB.shape[0]):
        raise ValueError("codes must be a uint8 CUDA tensor [C, M]")
    if Q.shape[1] != CB.shape[0] * CB.shape[2]:
        raise ValueError("query dimension must equal M * dsub")
    return Q.contiguous(), CB.contiguous(), codes.contiguous()


class ADCDistance(torch.autograd.Function):
    """Dhat[b, c] = sum_m ||Q[b, m-block] - CB[m, codes[c, m]]||^2 with codes fixed;
    forward and backward run in the library's kernels."""

    @staticmethod
    def forward(ctx, Q, CB, codes):
        Q, CB, codes = _adc_args(Q, CB, codes)
        B, C = Q.shape[0], codes.shape[0]
        M, dsub = CB.shape[0], CB.shape[2]
        out = torch.empty((B, C), dtype=torch.float32, device=Q.device)
        _check(lib().ann_adc_forward(_ptr(Q), B, _ptr(CB), M, dsub, _ptr(codes), C, _ptr(out),
                                     _stream(Q.device, None)))
        ctx.save_for_backward(Q, CB, codes)
        return out

    @staticmethod
    def backward(ctx, grad):
        Q, CB, codes = ctx.saved_tensors
        G = grad.contiguous().to(torch.float32)
        B, C = Q.shape[0], codes.shape[0]
        M, dsub = CB.shape[0], CB.shape[2]
        nbytes = lib().ann_adc_backward_workspace(B, C, M, dsub)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=Q.device)
        dQ = torch.empty_like(Q) if ctx.needs_input_grad[0] else None
        dCB = torch.empty_like(CB) if ctx.needs_input_grad[1] else None
        _check(lib().ann_adc_backward(_ptr(Q), B, _ptr(CB), M, dsub, _ptr(codes), C, _ptr(G),
                                      _ptr(dQ), _ptr(dCB), _ptr(ws), nbytes,
                                      _stream(Q.device, None)))
        return dQ, dCB, None


def _exact_sq_fwd(Q, X):
    Q = Q.detach().contiguous()
    X = X.detach().contiguous()
    if not (Q.is_cuda and X.is_cuda and Q.dtype == torch.float32 and X.dtype == torch.float32
            and Q.dim() == 2 and X.dim() == 2 and Q.shape[1] == X.shape[1]):
        raise ValueError("exact_sq: float32 [B, D] and [C, D] tensors on the GPU")
    out = torch.empty((Q.shape[0], X.shape[0]), dtype=torch.float32, device=Q.device)
    _check(lib().ann_exact_sq(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], Q.shape[1], _ptr(out),
                              _stream(Q.device, None)))
    return out


class ExactSq(torch.autograd.Function):
    """E[b, c] = ||q_b - x_c||^2 by ann_exact_sq (direct form); its gradient
    dE/dq_b = 2 sum_c G[b, c] (q_b - x_c) (and likewise for x_c) is a plain
    product with the incoming gradient."""

    @staticmethod
    def forward(ctx, Q, X):
        ctx.save_for_backward(Q, X)
        return _exact_sq_fwd(Q, X)

    @staticmethod
    def backward(ctx, G):
        Q, X = ctx.saved_tensors
        G = G.contiguous()
        dQ = dX = None
        if ctx.needs_input_grad[0]:
            dQ = 2.0 * (G.sum(1, keepdim=True) * Q - G @ X)
        if ctx.needs_input_grad[1]:
            dX = 2.0 * (G.sum(0)[:, None] * X - G.t().contiguous() @ Q)
        return dQ, dX


def exact_sq(Q, X):
    """Exact squared distances [B, C] (ann_exact_sq: direct form, float64 sums
    rounded once), differentiable in Q and X."""
    return ExactSq.apply(Q, X)


def adc_distance(Q, CB, codes):
    """Differentiable PQ distance (see ADCDistance)."""
    return ADCDistance.apply(Q, CB, codes)

