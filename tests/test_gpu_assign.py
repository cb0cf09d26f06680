"""Eq. 2 assignment on the GPU (the index builder's use of the exact probe):
each row's lists are its R nearest centroids that are within (1 + eps) of
the nearest in Euclidean distance, nearest first; checked against the same
rule evaluated in float64 with numpy."""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("kind", ["u8", "i8", "f32"])
@pytest.mark.parametrize("R,eps", [(1, 0.1), (2, 0.1), (8, 0.3)])
def test_gpu_assignment_follows_eq2(kind, R, eps):
    from paper_2409_16576_amd import builder as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lo, hi = {"u8": (0, 255), "i8": (-128, 127), "f32": (0, 100)}[kind]
    X = fx.mixture(601, 5000, 40, kind, n_centres=12, lo=lo, hi=hi)
    C = fx.mixture(602, 96, 40, kind, n_centres=12, lo=lo, hi=hi).astype(np.float32)
    A = B.assign_lists_gpu(X, C, kind, R, eps, chunk=1024)
    d = ((X[:, None, :].astype(np.float64) - C[None].astype(np.float64)) ** 2).sum(-1)
    order = np.lexsort((np.broadcast_to(np.arange(len(C)), d.shape), d), axis=1)[:, :R]
    dd = np.take_along_axis(d, order, 1)
    keep = dd <= (1 + eps) ** 2 * dd[:, :1]
    ref = np.where(keep, order, -1).astype(np.int32)
    if kind == "f32":  # distances rounded once to float32 on the GPU: near-ties may differ
        assert (A[:, 0] == ref[:, 0]).mean() > 0.999
        assert (A == ref).mean() > 0.99
    else:  # exact integers on both sides
        assert np.array_equal(A, ref)
