"""The library's page layout of raw vectors (ann_page_layout, host code)
against the oracle's, which its own pins fix (Sec. 4.3): bit-identical page
and slot of every vector, on random bucket sizes and page capacities."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2409_16576_amd", "libann.so")


@pytest.fixture(scope="module")
def lib():
    assert os.path.exists(LIB), "build libann.so first (__graft_entry__.build())"
    L = ctypes.CDLL(LIB)
    L.ann_page_layout.restype = ctypes.c_int64
    P = ctypes.c_void_p
    L.ann_page_layout.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, P, P]
    return L


def _lay(lib, b, nb, row, page):
    b = np.ascontiguousarray(b, dtype=np.int32)
    pg = np.empty(len(b), np.int32)
    sl = np.empty(len(b), np.int32)
    npg = lib.ann_page_layout(b.ctypes.data, len(b), nb, row, page, pg.ctypes.data, sl.ctypes.data)
    return npg, pg, sl


@pytest.mark.parametrize("seed", range(12))
def test_layout_equals_oracle(lib, orc, seed):
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(1, 200))
    row = int(rng.choice([100, 128, 384, 17]))
    page = int(rng.choice([256, 1024, 4096, row, 3 * row + 5]))
    sizes = rng.integers(0, 3 * (page // row) + 2, size=nb)
    b = rng.permutation(np.repeat(np.arange(nb), sizes)).astype(np.int32)
    npg, pg, sl = _lay(lib, b, nb, row, page)
    o = orc.page_layout(b, nb, row, page)
    assert npg == o.pages
    assert np.array_equal(pg, o.page) and np.array_equal(sl, o.slot)


def test_layout_rejects_bad_arguments(lib):
    assert _lay(lib, [0, 1], 2, 128, 64)[0] == -1       # a row larger than a page
    assert _lay(lib, [0, 5], 2, 128, 4096)[0] == -1     # bucket out of range
