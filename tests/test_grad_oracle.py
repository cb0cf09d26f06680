"""Pins of the float64 gradient oracle (differentiable PQ distance, codes fixed)."""
import numpy as np

from oracle import grad as og


def _setup(seed=0, B=6, C=11, M=3, dsub=2, K=256):
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(B, M * dsub)) * 3
    CB = rng.normal(size=(M, K, dsub)) * 3
    codes = rng.integers(0, 12, size=(C, M)).astype(np.uint8)  # few codewords used
    X = rng.normal(size=(C, M * dsub)) * 3
    return Q, CB, codes, X


def test_forward_is_distance_to_decoded_vector():
    """Eq. 1 identity: the table sum equals ||q - decode(code)||^2."""
    Q, CB, codes, _ = _setup(1)
    d1 = og.adc_forward(Q, CB, codes)
    d2 = og.exact_sq(Q, og.decode(CB, codes))
    np.testing.assert_allclose(d1, d2, rtol=1e-12)


def test_backward_matches_finite_differences():
    """dQ and dCB of sum(G * Dhat) against central differences at eps = 1e-3."""
    Q, CB, codes, _ = _setup(2)
    rng = np.random.default_rng(3)
    G = rng.normal(size=(Q.shape[0], codes.shape[0]))
    dQ, dCB = og.adc_backward(Q, CB, codes, G)
    f = lambda: float((G * og.adc_forward(Q, CB, codes)).sum())
    fq = og.finite_diff(f, Q, range(Q.size))
    np.testing.assert_allclose(fq, dQ.reshape(-1), rtol=1e-6, atol=1e-6)
    used = sorted({(m, int(j)) for m in range(CB.shape[0]) for j in codes[:, m]})
    idx = [(m * CB.shape[1] + j) * CB.shape[2] + t for m, j in used for t in range(CB.shape[2])]
    fcb = og.finite_diff(f, CB, idx)
    np.testing.assert_allclose(fcb, dCB.reshape(-1)[idx], rtol=1e-6, atol=1e-6)


def test_loss_gradients_match_finite_differences():
    Q, CB, codes, X = _setup(4)
    L, dQ, dCB = og.loss_grads(Q, CB, codes, X)
    assert abs(L - og.loss(Q, CB, codes, X)) < 1e-9 * max(1.0, L)
    f = lambda: og.loss(Q, CB, codes, X)
    np.testing.assert_allclose(og.finite_diff(f, Q, range(Q.size)), dQ.reshape(-1),
                               rtol=1e-5, atol=1e-6)
    idx = list(range(0, CB.size, 7))
    np.testing.assert_allclose(og.finite_diff(f, CB, idx), dCB.reshape(-1)[idx],
                               rtol=1e-5, atol=1e-6)


def test_unused_codewords_have_zero_gradient():
    Q, CB, codes, X = _setup(5)
    _, _, dCB = og.loss_grads(Q, CB, codes, X)
    for m in range(CB.shape[0]):
        unused = np.setdiff1d(np.arange(CB.shape[1]), codes[:, m])
        assert (dCB[m][unused] == 0.0).all()


def test_lossless_codebook_gives_zero_loss():
    """Vectors that are exactly their decoded codes: PQ distance = exact distance."""
    Q, CB, codes, _ = _setup(6)
    X = og.decode(CB, codes)
    L, dQ, dCB = og.loss_grads(Q, CB, codes, X)
    assert L < 1e-20
    assert np.abs(dQ).max() < 1e-9 and np.abs(dCB).max() < 1e-9
