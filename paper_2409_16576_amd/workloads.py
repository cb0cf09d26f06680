"""Named synthetic workloads and the recipe that turns each into an index file.

Each workload fixes the dataset recipe (a seeded Gaussian mixture of the
paper's dataset shapes, Table 1), the IVF-PQ build parameters and the search
knobs (nprobe = the paper's top-m, rerank_n = its top-n, k).  ``scaled``
derives a smaller copy for tests.
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from dataclasses import dataclass

import numpy as np

from . import inputs


@dataclass(frozen=True)
class Workload:
    name: str
    wid: int                # seed namespace
    n: int
    dim: int
    kind: str               # "f32" | "u8" | "i8"
    n_centres: int
    centre_low: float
    centre_high: float
    sigma: float
    nlist: int
    M: int
    nq: int
    nprobe: int | tuple     # scalar, or (low, high) for per-query U{low..high}
    rerank_n: int
    k: int = 10
    R: int = 2
    eps: float = 0.1
    unit_norm: bool = False
    zipf_s: float = 0.0     # > 0: mixture weights 1/rank^s (skewed list lengths)
    sub_centres: int = 1    # > 1: each centre spawns this many sub-centres
    sub_sigma: float = 0.0
    kmeans_iters: int = 10
    rerank_n_op: int = 0    # smallest swept rerank_n with oracle recall@10 >= 0.9 (0: rerank_n)

    def describe(self) -> dict:
        return {"workload": self.name, "n": self.n, "dim": self.dim, "dtype": self.kind,
                "nlist": self.nlist, "M": self.M, "nq": self.nq,
                "nprobe": self.nprobe if isinstance(self.nprobe, int) else list(self.nprobe),
                "rerank_n": self.rerank_n, "k": self.k, "R": self.R, "eps": self.eps}


# 100k x 128-d float32, 256 centres U[0,100], sigma 5; 1024 lists; PQ 16 x 256.
IVF_F32_100K = Workload("ivf_f32_100k", 1, 100_000, 128, "f32", 256, 0.0, 100.0, 5.0,
                        1024, 16, 1000, 32, 100, rerank_n_op=400)
# 10M x 128-d uint8, 4096 centres; 16384 lists; PQ 32 x 256.
IVF_U8_10M = Workload("ivf_u8_10m", 2, 10_000_000, 128, "u8", 4096, 0.0, 255.0, 10.0,
                      16384, 32, 10_000, 64, 200, rerank_n_op=1400)
# 5M x 96-d unit-norm float32, 2048 centres x 4 sub-centres, Zipf(1.1) weights;
# 8192 lists; PQ 24 x 256; per-query nprobe U{8..128}.
ZIPF_F32_5M = Workload("zipf_f32_5m", 3, 5_000_000, 96, "f32", 2048, 0.0, 0.0, 0.3,
                       8192, 24, 16_384, (8, 128), 100, unit_norm=True, zipf_s=1.1,
                       sub_centres=4, sub_sigma=0.5, kmeans_iters=5, rerank_n_op=2400)
# 100M x 100-d int8, 8192 centres U[-128,127]; 65536 lists; PQ 50 x 256.
SERVE_I8_100M = Workload("serve_i8_100m", 5, 100_000_000, 100, "i8", 8192, -128.0, 127.0,
                         10.0, 65536, 50, 10_000, 64, 100, rerank_n_op=200)

# 2M x 100-d int8, 8192 centres; 200,000 lists (0.1 N, the paper's list count,
# Sec. 4.1), where the probe walks a navigation graph; PQ 50 x 256.
NAV_I8_2M = Workload("nav_i8_2m", 6, 2_000_000, 100, "i8", 8192, -128.0, 127.0, 10.0,
                     200_000, 50, 10_000, 256, 200)

# 4M x 100-d int8, 4096 centres; 8192 lists; PQ 50 x 256: the replication study
# (Eq. 2 with R = 1..8) and balanced clustering.
REPL_I8_4M = Workload("repl_i8_4m", 7, 4_000_000, 100, "i8", 4096, -128.0, 127.0, 10.0,
                      8192, 50, 10_000, 32, 200)

ALL = {w.name: w for w in (IVF_F32_100K, IVF_U8_10M, ZIPF_F32_5M, SERVE_I8_100M, NAV_I8_2M,
                           REPL_I8_4M)}


def scaled(w: Workload, **kw) -> Workload:
    """A copy with some fields replaced (name suffixed with the changed sizes)."""
    tag = ",".join(f"{k}={v}" for k, v in sorted(kw.items()))
    return dataclasses.replace(w, name=f"{w.name}[{tag}]", **kw)


def _centres(w: Workload) -> np.ndarray:
    if w.unit_norm:
        rng = np.random.default_rng(inputs.seed_for(w.wid, 1))
        c = rng.standard_normal((w.n_centres, w.dim))
        c /= np.linalg.norm(c, axis=1, keepdims=True)
        if w.sub_centres > 1:
            s = rng.standard_normal((w.n_centres, w.sub_centres, w.dim)) * (w.sub_sigma / np.sqrt(w.dim))
            c = (c[:, None, :] + s).reshape(-1, w.dim)
            c /= np.linalg.norm(c, axis=1, keepdims=True)
        return c
    return inputs.mixture_centres(inputs.seed_for(w.wid, 1), w.n_centres, w.dim,
                                  w.centre_low, w.centre_high)


def _weights(w: Workload, n_centres: int):
    if w.zipf_s > 0:
        return inputs.zipf_weights(inputs.seed_for(w.wid, 1) + 17, n_centres, w.zipf_s)
    return None


def _noise(w: Workload):
    return w.sigma / np.sqrt(w.dim) if w.unit_norm else None


def base_vectors(w: Workload) -> np.ndarray:
    c = _centres(w)
    return inputs.mixture_points(inputs.seed_for(w.wid, 2), w.n, c, w.sigma, w.kind,
                                 weights=_weights(w, len(c)), unit_norm=w.unit_norm,
                                 noise_scale=_noise(w))


def queries(w: Workload, nq: int | None = None) -> np.ndarray:
    """Queries from the same mixture, as float32 (exact for the integer kinds)."""
    c = _centres(w)
    q = inputs.mixture_points(inputs.seed_for(w.wid, 3), w.nq if nq is None else nq, c,
                              w.sigma, w.kind, weights=_weights(w, len(c)),
                              unit_norm=w.unit_norm, noise_scale=_noise(w))
    return q.astype(np.float32)


def nprobe_per_query(w: Workload, nq: int | None = None) -> np.ndarray:
    nq = w.nq if nq is None else nq
    if isinstance(w.nprobe, int):
        return np.full(nq, w.nprobe, dtype=np.int32)
    lo, hi = w.nprobe
    return inputs.nprobe_draws(inputs.seed_for(w.wid, 6), nq, lo, hi)


def build_params(w: Workload):
    from .builder import BuildParams
    init = None
    if w.sub_centres > 1 and w.nlist == w.n_centres * w.sub_centres:
        init = _centres(w).astype(np.float32)  # k-means starts at the sub-centres
    return BuildParams(nlist=w.nlist, M=w.M, R=w.R, eps=w.eps, seed=inputs.seed_for(w.wid, 4),
                       kmeans_iters=w.kmeans_iters, init_centroids=init)


def cache_dir() -> str:
    d = os.environ.get("ANN_INDEX_CACHE", os.path.join("/tmp", "ann_index_cache"))
    os.makedirs(d, exist_ok=True)
    return d


_INDEX_FIELDS = ("wid", "n", "dim", "kind", "n_centres", "centre_low", "centre_high", "sigma",
                 "nlist", "M", "R", "eps", "unit_norm", "zipf_s", "sub_centres", "sub_sigma",
                 "kmeans_iters")


def index_path(w: Workload) -> str:
    """Cache path keyed by the fields that determine the index file's bytes."""
    key = repr(tuple(getattr(w, f) for f in _INDEX_FIELDS))
    h = hashlib.sha1(key.encode()).hexdigest()[:16]
    safe = "".join(ch if ch.isalnum() or ch in "_-" else "_" for ch in w.name)[:60]
    return os.path.join(cache_dir(), f"{safe}-{h}.fidx")


def ensure_index(w: Workload, verbose: bool = False) -> str:
    """Build the workload's index file once (cached under ANN_INDEX_CACHE)."""
    path = index_path(w)
    if not os.path.exists(path):
        from .builder import build_index
        import time
        t0 = time.time()
        X = base_vectors(w)
        t1 = time.time()
        import sys
        say = None
        if verbose:  # progress goes to stderr: stdout carries results only
            say = lambda m: print(f"[index] {w.name}: {m} ({time.time() - t0:.0f}s)",  # noqa: E731
                                  file=sys.stderr, flush=True)
        build_index(path, X, w.kind, build_params(w), progress=say)
        if verbose:
            print(f"[index] {w.name}: data {t1 - t0:.1f}s build {time.time() - t1:.1f}s -> {path}",
                  file=sys.stderr, flush=True)
    return path
