"""Small index fixtures for the tests (written with the index builder's writer)."""
from __future__ import annotations

import os

import numpy as np

from paper_2409_16576_amd import builder, inputs
from paper_2409_16576_amd.builder import BuildParams, IndexArrays


def mixture(seed, n, dim, kind, n_centres=8, lo=0.0, hi=100.0, sigma=5.0):
    c = inputs.mixture_centres(seed, n_centres, dim, lo, hi)
    return inputs.mixture_points(seed + 1, n, c, sigma, kind)


def built(tmpdir, name, X, kind, nlist, M, R=2, eps=0.1, seed=7, **kw):
    path = os.path.join(str(tmpdir), f"{name}.fidx")
    p = BuildParams(nlist=nlist, M=M, R=R, eps=eps, seed=seed, **kw)
    ix = builder.build_index(path, X, kind, p)
    return path, ix


def write_arrays(tmpdir, name, kind, centroids, codebooks, codes, vectors, assign, eps=0.0,
                 int_grid=None):
    """Write a hand-made index; posting lists are derived from ``assign``."""
    nlist = centroids.shape[0]
    offsets, entries = builder.lists_from_assignment(np.asarray(assign, dtype=np.int32), nlist)
    ix = IndexArrays(kind, np.asarray(centroids, np.float32), np.asarray(codebooks, np.float32),
                     np.asarray(codes, np.uint8), vectors, offsets, entries,
                     np.asarray(assign, np.int32), eps,
                     (kind != "f32") if int_grid is None else int_grid)
    path = os.path.join(str(tmpdir), f"{name}.fidx")
    builder.write_index(path, ix)
    return path, ix


def lossless_u8(tmpdir, name, n=300, dim=8, nlist=4, seed=11):
    """uint8 data with dsub = 1 and every byte value a codeword: decoding is exact."""
    rng = np.random.default_rng(seed)
    X = rng.integers(0, 256, size=(n, dim)).astype(np.uint8)
    cb = np.tile(np.arange(256, dtype=np.float32).reshape(1, 256, 1), (dim, 1, 1))
    cent = np.rint(rng.uniform(0, 255, size=(nlist, dim))).astype(np.float32)
    d = ((X[:, None, :].astype(np.int64) - cent[None].astype(np.int64)) ** 2).sum(-1)
    assign = np.stack([np.argmin(d, axis=1), -np.ones(n, dtype=np.int64)], axis=1)
    return write_arrays(tmpdir, name, "u8", cent, cb, X.copy(), X, assign)
