"""Seeded synthetic inputs.

This module is the only code shared by the oracle tests and the GPU path.  It
draws random numbers and shapes them into datasets, query sets and per-query
knobs; it holds none of the search method's arithmetic (no distances, no
clustering, no quantisation).  Every array is a pure function of its seed and
sizes: generation is split into fixed-size row chunks whose generators are
derived from (seed, chunk index), so the bytes do not depend on the number of
threads used to draw them.

Dataset shapes follow the paper's evaluation sets (Table 1): 128-d uint8,
100-d int8 and 96-d float32 vectors.  The public datasets themselves are not
used; Gaussian mixtures of the same dtypes and dimensions stand in for them.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

CHUNK_ROWS = 1 << 16


def seed_for(workload_id: int, stream: int) -> int:
    """Seed of random stream ``stream`` of workload ``workload_id``.

    Streams: 1 mixture centres, 2 base vectors, 3 queries, 4 IVF k-means,
    5 PQ training, 6 per-query nprobe, 7 arrivals / request sizes,
    8 gradient batches.
    """
    return 1_000_003 * int(workload_id) + int(stream)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunk_rng(seed: int, chunk: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(chunk)]))


def _fill_chunks(n: int, fn):
    """Run fn(chunk_index, row0, row1) over fixed row chunks, in parallel."""
    nchunks = (n + CHUNK_ROWS - 1) // CHUNK_ROWS
    jobs = [(c, c * CHUNK_ROWS, min(n, (c + 1) * CHUNK_ROWS)) for c in range(nchunks)]
    if nchunks <= 1:
        for j in jobs:
            fn(*j)
        return
    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda j: fn(*j), jobs))


def _to_kind(x: np.ndarray, kind: str) -> np.ndarray:
    if kind == "f32":
        return x.astype(np.float32)
    if kind == "u8":
        return np.clip(np.rint(x), 0, 255).astype(np.uint8)
    if kind == "i8":
        return np.clip(np.rint(x), -128, 127).astype(np.int8)
    raise ValueError(f"unknown kind {kind!r}")


_NP_DTYPE = {"f32": np.float32, "u8": np.uint8, "i8": np.int8}


def mixture_centres(seed: int, n_centres: int, dim: int, low: float, high: float) -> np.ndarray:
    """Centres drawn uniformly from [low, high]^dim (float64)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=(n_centres, dim))


def mixture_points(seed: int, n: int, centres: np.ndarray, sigma: float, kind: str,
                   weights: np.ndarray | None = None, unit_norm: bool = False,
                   noise_scale: float | None = None) -> np.ndarray:
    """n points x = centre + sigma * N(0, I), converted to ``kind``.

    Each point picks its centre independently, uniformly or by ``weights``.
    ``kind`` is "f32", "u8" (round half to even, clip to 0..255) or "i8"
    (round, clip to -128..127).  With ``unit_norm`` the float result is
    scaled to unit length (used for the unit-normalised 96-d workload).
    """
    n_centres, dim = centres.shape
    out = np.empty((n, dim), dtype=_NP_DTYPE[kind])
    cdf = None
    if weights is not None:
        w = np.asarray(weights, dtype=np.float64)
        cdf = np.cumsum(w / w.sum())
        cdf[-1] = 1.0
    scale = sigma if noise_scale is None else noise_scale

    def work(c, r0, r1):
        rng = _chunk_rng(seed, c)
        m = r1 - r0
        if cdf is None:
            lab = rng.integers(0, n_centres, size=m)
        else:
            lab = np.searchsorted(cdf, rng.random(m), side="right")
            lab = np.minimum(lab, n_centres - 1)
        x = centres[lab] + scale * rng.standard_normal((m, dim))
        if unit_norm:
            x /= np.maximum(np.linalg.norm(x, axis=1, keepdims=True), 1e-30)
        out[r0:r1] = _to_kind(x, kind)

    _fill_chunks(n, work)
    return out


def nprobe_draws(seed: int, nq: int, low: int, high: int) -> np.ndarray:
    """Per-query nprobe drawn uniformly from {low..high} (int32)."""
    rng = np.random.default_rng(seed)
    return rng.integers(low, high + 1, size=nq).astype(np.int32)


def sample_rows(seed: int, n: int, count: int) -> np.ndarray:
    """``count`` distinct row indices of 0..n-1 in ascending order."""
    rng = np.random.default_rng(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def zipf_weights(seed: int, n: int, s: float) -> np.ndarray:
    """Weights 1/rank^s assigned to a seeded permutation of n items."""
    rng = np.random.default_rng(seed)
    ranks = rng.permutation(n) + 1
    return 1.0 / np.power(ranks.astype(np.float64), s)


def poisson_arrivals(seed: int, rate_per_s: float, duration_s: float,
                     size_low: int, size_high: int):
    """Request arrival times (s) of a Poisson process and request sizes U{low..high}."""
    rng = np.random.default_rng(seed)
    times = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        times.append(t)
    times = np.asarray(times, dtype=np.float64)
    sizes = rng.integers(size_low, size_high + 1, size=len(times)).astype(np.int32)
    return times, sizes
