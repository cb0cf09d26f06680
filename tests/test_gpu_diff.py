"""Differentiable PQ distance on the GPU against the float64 gradient oracle."""
import numpy as np
import pytest

from oracle import grad as og

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-diff]", *a, flush=True)


@pytest.fixture(scope="module")
def A():
    from paper_2409_16576_amd import ann
    assert torch.cuda.is_available()
    ann.lib()
    return ann


def _data(B, C, M, dsub, used=256, seed=0):
    rng = np.random.default_rng(seed)
    CB = (rng.normal(size=(M, 256, dsub)) * 4).astype(np.float32)
    codes = rng.integers(0, used, size=(C, M)).astype(np.uint8)
    Q = (og.decode(CB, codes[rng.integers(0, C, size=B)]) + rng.normal(size=(B, M * dsub))).astype(np.float32)
    X = (og.decode(CB, codes) + rng.normal(size=(C, M * dsub)) * 0.5).astype(np.float32)
    return Q, CB, codes, X


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _close(gpu, ref, S, rtol=1e-4, stol=1e-6):
    """Element-wise |g - r| <= rtol |r| + stol S, S the operand scale of each
    element (the sum of the magnitudes of the terms it adds up)."""
    g = gpu.astype(np.float64)
    err = np.abs(g - ref)
    bound = rtol * np.abs(ref) + stol * S
    worst = float((err / np.maximum(bound, 1e-300)).max())
    assert (err <= bound).all(), ("worst error / bound", worst)
    return worst


def _scales(Q, CB, codes, G):
    """Operand scales: forward ||q_b||^2 + ||dec_c||^2; dQ[b, t] 2 sum_c |G|
    (|q_bt| + |dec_ct|); dCB[m, j, t] 2 sum_{c: code = j} sum_b |G| (|q_b,mt| +
    |CB_mjt|)."""
    Q = Q.astype(np.float64)
    CB64 = CB.astype(np.float64)
    dec = og.decode(CB64, codes)
    sf = (Q * Q).sum(1)[:, None] + (dec * dec).sum(1)[None, :]
    aG = np.abs(G.astype(np.float64))
    sq = 2.0 * (aG.sum(1)[:, None] * np.abs(Q) + aG @ np.abs(dec))
    M, K, dsub = CB.shape
    T = aG.T @ np.abs(Q)   # [C, D]
    cs = aG.sum(0)         # [C]
    scb = np.zeros_like(CB64)
    for m in range(M):
        j = codes[:, m].astype(np.int64)
        np.add.at(scb[m], j, T[:, m * dsub:(m + 1) * dsub] + cs[:, None] * np.abs(CB64[m][j]))
    return sf, sq, 2.0 * scb


@pytest.mark.parametrize("B,C,M,dsub", [(5, 7, 3, 2), (64, 128, 24, 4), (4096, 2048, 24, 4),
                                        (33, 65, 8, 16)])
def test_forward_and_backward_match_oracle(A, B, C, M, dsub):
    _say("shape", B, C, M, dsub)
    Q, CB, codes, _ = _data(B, C, M, dsub, seed=B + C)
    rng = np.random.default_rng(7)
    G = rng.normal(size=(B, C)).astype(np.float32)
    sf, sq, scb = _scales(Q, CB, codes, G)
    Dg = A.adc_distance(_t(Q), _t(CB), _t(codes))
    Dr = og.adc_forward(Q, CB, codes)
    w = [_close(Dg.cpu().numpy(), Dr, sf)]
    Qt = _t(Q).requires_grad_(True)
    CBt = _t(CB).requires_grad_(True)
    out = A.adc_distance(Qt, CBt, _t(codes))
    out.backward(_t(G))
    dQ, dCB = og.adc_backward(Q, CB, codes, G)
    w.append(_close(Qt.grad.cpu().numpy(), dQ, sq))
    w.append(_close(CBt.grad.cpu().numpy(), dCB, scb))
    _say("worst error / bound (forward, dQ, dCB):", w)


def test_exact_term_direct_form(A):
    """ann_exact_sq: float64 sums rounded once, so equal to the float64 oracle
    rounded to float32, to one unit in the last place."""
    rng = np.random.default_rng(5)
    for B, C, D in ((37, 53, 96), (300, 200, 7), (64, 130, 200)):
        Q = (rng.normal(size=(B, D)) * 30 + 50).astype(np.float32)
        X = (rng.normal(size=(C, D)) * 30 + 50).astype(np.float32)
        g = A.exact_sq(_t(Q), _t(X)).cpu().numpy()
        r = og.exact_sq(Q, X).astype(np.float32)
        ulp = np.abs(g.view(np.int32).astype(np.int64) - r.view(np.int32).astype(np.int64))
        assert ulp.max() <= 1, (B, C, D, int(ulp.max()))


def test_unused_codewords_zero_and_deterministic(A):
    Q, CB, codes, _ = _data(200, 300, 6, 4, used=40, seed=3)
    G = _t(np.random.default_rng(1).normal(size=(200, 300)).astype(np.float32))
    grads = []
    for _ in range(2):
        CBt = _t(CB).requires_grad_(True)
        A.adc_distance(_t(Q), CBt, _t(codes)).backward(G)
        grads.append(CBt.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1])  # bitwise reproducible
    assert (grads[0][:, 40:, :] == 0.0).all()
    assert np.abs(grads[0][:, :40, :]).max() > 0


def _fd_close(g, fd, what):
    """GPU float32 gradient vs float64 central differences, element-wise:
    |g - fd| <= 1e-3 |fd| + 1e-4 rms(fd)."""
    g = np.asarray(g, np.float64)
    bound = 1e-3 * np.abs(fd) + 1e-4 * np.sqrt((fd * fd).mean())
    err = np.abs(g - fd)
    worst = float((err / bound).max())
    assert (err <= bound).all(), (what, "worst error / bound", worst)
    return worst


def test_loss_gradient_against_fp64_finite_differences(A):
    """dL/dCB and dL/dQ of L = mean (Dhat - ||q - x||^2)^2 through autograd (GPU
    kernels for Dhat and the exact term) against central differences of the
    float64 loss (toy shape, every coordinate of the used codewords)."""
    from paper_2409_16576_amd import finetune
    Q, CB, codes, X = _data(16, 24, 4, 2, used=8, seed=9)
    Qt, CBt = _t(Q).requires_grad_(True), _t(CB).requires_grad_(True)
    L = finetune.distortion_loss(Qt, CBt, _t(codes), _t(X))
    L.backward()
    Q64, CB64 = Q.astype(np.float64), CB.astype(np.float64)
    f = lambda: og.loss(Q64, CB64, codes, X)
    assert abs(float(L.detach()) - f()) <= 1e-4 * f()
    iq = list(range(0, Q.size, 5))
    fq = og.finite_diff(f, Q64, iq)
    _fd_close(Qt.grad.cpu().numpy().reshape(-1)[iq], fq, "dQ")
    used = [(m, j) for m in range(4) for j in range(8)]
    ic = [(m * 256 + j) * 2 + t for m, j in used for t in range(2)]
    fc = og.finite_diff(f, CB64, ic)
    _fd_close(CBt.grad.cpu().numpy().reshape(-1)[ic], fc, "dCB")


def test_loss_gradient_fd_at_the_workload_codebook_shape(A):
    """The same check at the differentiation workload's codebook shape (24
    subspaces x 256 codewords x 4 dimensions) on a 64 x 128 sub-batch: every
    coordinate of every codeword the candidates use, and every query
    coordinate, by float64 central differences (h = 1e-3).  A perturbation of
    CB[m, j, t] moves one table column (the candidates coded j in subspace
    m), one of q_b[d] moves row b; the loss is re-evaluated from the moved
    terms in float64."""
    from paper_2409_16576_amd import finetune
    B, C, M, dsub = 64, 128, 24, 4
    Q, CB, codes, X = _data(B, C, M, dsub, used=256, seed=21)
    Qt, CBt = _t(Q).requires_grad_(True), _t(CB).requires_grad_(True)
    finetune.distortion_loss(Qt, CBt, _t(codes), _t(X)).backward()
    gq, gcb = Qt.grad.cpu().numpy(), CBt.grad.cpu().numpy()
    Q64, CB64, X64 = Q.astype(np.float64), CB.astype(np.float64), X.astype(np.float64)
    cidx = codes.astype(np.int64)
    E = og.exact_sq(Q64, X64)
    Dh = og.adc_forward(Q64, CB64, codes)
    h = 1e-3
    loss = lambda D, Ex: float(((D - Ex) ** 2).mean())
    # codebooks: every (m, j) some candidate uses, every coordinate
    fd_cb, g_cb = [], []
    for m in range(M):
        qm = Q64[:, m * dsub:(m + 1) * dsub]
        for j in np.unique(cidx[:, m]):
            mask = (cidx[:, m] == j)[None, :]
            old = ((qm - CB64[m, j]) ** 2).sum(1)
            for t in range(dsub):
                vals = []
                for sgn in (1.0, -1.0):
                    c = CB64[m, j].copy()
                    c[t] += sgn * h
                    delta = ((qm - c) ** 2).sum(1) - old
                    vals.append(loss(Dh + delta[:, None] * mask, E))
                fd_cb.append((vals[0] - vals[1]) / (2 * h))
                g_cb.append(gcb[m, j, t])
    # queries: every coordinate
    fd_q, g_q = [], []
    for b in range(B):
        for d in range(M * dsub):
            m, t = divmod(d, dsub)
            vals = []
            for sgn in (1.0, -1.0):
                qb = Q64[b].copy()
                qb[d] += sgn * h
                D2, E2 = Dh.copy(), E.copy()
                cw = CB64[m][cidx[:, m]]                      # [C, dsub]
                D2[b] += ((qb[m * dsub:(m + 1) * dsub] - cw) ** 2).sum(1) - \
                    ((Q64[b, m * dsub:(m + 1) * dsub] - cw) ** 2).sum(1)
                E2[b] += (qb[d] - X64[:, d]) ** 2 - (Q64[b, d] - X64[:, d]) ** 2
                vals.append(loss(D2, E2))
            fd_q.append((vals[0] - vals[1]) / (2 * h))
            g_q.append(gq[b, d])
    w_cb = _fd_close(g_cb, np.array(fd_cb), "dCB")
    w_q = _fd_close(g_q, np.array(fd_q), "dQ")
    _say(f"FD at 24x256x4: {len(fd_cb)} codeword and {len(fd_q)} query coordinates; "
         f"worst error / bound {w_cb:.3f}, {w_q:.3f}")


def test_finetune_reduces_distortion(A):
    from paper_2409_16576_amd import finetune
    Q, CB, codes, X = _data(512, 1024, 8, 4, used=256, seed=11)
    CB0 = _t(CB + np.random.default_rng(2).normal(size=CB.shape).astype(np.float32))  # perturbed
    Qt, ct, Xt = _t(Q), _t(codes), _t(X)
    l0 = float(finetune.distortion_loss(Qt, CB0, ct, Xt))
    r0 = finetune.adc_recall(Qt, CB0, ct, Xt, k=10, n=50)
    CB1, hist = finetune.finetune_codebooks(CB0, ct, Xt, Qt, steps=60, batch_q=256, batch_c=512,
                                            lr=0.05)
    l1 = float(finetune.distortion_loss(Qt, CB1, ct, Xt))
    r1 = finetune.adc_recall(Qt, CB1, ct, Xt, k=10, n=50)
    _say("loss", l0, "->", l1, "recall", r0, "->", r1)
    assert l1 < 0.5 * l0
    assert r1 >= r0
