"""Float64 oracle of the differentiable PQ distance (test infrastructure only).

Eq. 1 with dist = squared L2 of sub-vectors, as a function of the queries Q
[B, D] and the codebooks CB [M, 256, dsub], codes [C, M] fixed:

    Dhat[b, c] = sum_m || Q[b, m-block] - CB[m, codes[c, m]] ||^2

and the fine-tuning loss L = mean_{b,c} (Dhat[b, c] - ||Q[b] - X[c]||^2)^2
(PQ distance against the exact squared distance).  Plain numpy, float64.
The closed-form gradients below are pinned by central finite differences in
tests/test_grad_oracle.py.
"""
from __future__ import annotations

import numpy as np


def decode(CB: np.ndarray, codes: np.ndarray) -> np.ndarray:
    """Decoded vectors [C, D]: concatenation of the codewords named by each code."""
    M = CB.shape[0]
    return np.concatenate([CB[m][codes[:, m].astype(np.int64)] for m in range(M)], axis=1)


def adc_forward(Q: np.ndarray, CB: np.ndarray, codes: np.ndarray) -> np.ndarray:
    """Dhat [B, C] through per-query tables: table[b, m, j] = ||q_b,m - CB[m, j]||^2."""
    Q = np.asarray(Q, np.float64)
    CB = np.asarray(CB, np.float64)
    M, K, dsub = CB.shape
    B = Q.shape[0]
    Qs = Q.reshape(B, M, 1, dsub)
    table = ((Qs - CB[None]) ** 2).sum(-1)  # [B, M, K]
    out = np.zeros((B, codes.shape[0]))
    for m in range(M):
        out += table[:, m, codes[:, m].astype(np.int64)]
    return out


def exact_sq(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    Q = np.asarray(Q, np.float64)
    X = np.asarray(X, np.float64)
    return ((Q[:, None, :] - X[None, :, :]) ** 2).sum(-1)


def adc_backward(Q: np.ndarray, CB: np.ndarray, codes: np.ndarray, G: np.ndarray):
    """(dQ, dCB) of sum_{b,c} G[b,c] * Dhat[b,c]:
    dQ[b]     = 2 sum_c G[b,c] (q_b - dec_c)
    dCB[m, j] = -2 sum_{c: codes[c,m] = j} sum_b G[b,c] (q_b,m - CB[m, j])."""
    Q = np.asarray(Q, np.float64)
    CB = np.asarray(CB, np.float64)
    G = np.asarray(G, np.float64)
    M, K, dsub = CB.shape
    dec = decode(CB, codes)
    dQ = 2.0 * (G.sum(1)[:, None] * Q - G @ dec)
    T = G.T @ Q                    # [C, D]
    cs = G.sum(0)                  # [C]
    dCB = np.zeros_like(CB)
    for m in range(M):
        j = codes[:, m].astype(np.int64)
        blk = T[:, m * dsub:(m + 1) * dsub]
        np.add.at(dCB[m], j, blk)
        w = np.bincount(j, weights=cs, minlength=K)
        dCB[m] -= w[:, None] * CB[m]
    return dQ, -2.0 * dCB


def loss(Q, CB, codes, X) -> float:
    r = adc_forward(Q, CB, codes) - exact_sq(Q, X)
    return float((r * r).mean())


def loss_grads(Q, CB, codes, X):
    """(L, dL/dQ, dL/dCB) for L = mean (Dhat - E)^2, E = ||Q - X||^2."""
    Q = np.asarray(Q, np.float64)
    X = np.asarray(X, np.float64)
    r = adc_forward(Q, CB, codes) - exact_sq(Q, X)
    G = 2.0 * r / r.size
    dQ_adc, dCB = adc_backward(Q, CB, codes, G)
    dQ_exact = 2.0 * (G.sum(1)[:, None] * Q - G @ X)
    return float((r * r).mean()), dQ_adc - dQ_exact, dCB


def finite_diff(f, x: np.ndarray, idx, eps: float = 1e-3) -> np.ndarray:
    """Central differences of scalar f at the flat indices idx of x (x is restored)."""
    out = np.empty(len(idx))
    flat = x.reshape(-1)
    for n, i in enumerate(idx):
        v = flat[i]
        flat[i] = v + eps
        fp = f()
        flat[i] = v - eps
        fm = f()
        flat[i] = v
        out[n] = (fp - fm) / (2 * eps)
    return out
