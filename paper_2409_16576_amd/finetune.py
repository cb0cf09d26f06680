"""Codebook fine-tuning through the differentiable PQ distance (codes fixed).

The loss is the PQ distance's distortion against the exact squared distance,
L = mean_{b,c} (Dhat[b, c] - ||q_b - x_c||^2)^2, over batches of queries and
candidate vectors; Dhat and its gradients come from the library's kernels
(ann.adc_distance), and so does the exact term (ann.exact_sq: direct form,
float64 sums rounded once -- no cancellation); the optimizer step is ordinary
torch code.  Used on float32 indexes (an integer-grid index would lose its
exactness with non-integer codebooks).
"""
from __future__ import annotations

import torch

from . import ann


def exact_sq(Q: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """||q_b - x_c||^2 [B, C] (library kernel; constant w.r.t. the codebooks)."""
    return ann.exact_sq(Q, X)


def distortion_loss(Q, CB, codes, X) -> torch.Tensor:
    r = ann.adc_distance(Q, CB, codes) - exact_sq(Q, X)
    return (r * r).mean()


@torch.no_grad()
def adc_recall(Q, CB, codes, X, k: int = 10, n: int = 100) -> float:
    """Mean fraction of each query's exact top-k (within the candidate set X)
    found among its n best candidates by PQ distance."""
    d_adc = ann.adc_distance(Q, CB, codes)
    d_ex = exact_sq(Q, X)
    top_ex = torch.topk(d_ex, k, dim=1, largest=False).indices
    top_adc = torch.topk(d_adc, n, dim=1, largest=False).indices
    hit = (top_ex[:, :, None] == top_adc[:, None, :]).any(-1).float()
    return float(hit.mean())


def finetune_codebooks(CB0: torch.Tensor, codes: torch.Tensor, X: torch.Tensor,
                       queries: torch.Tensor, steps: int = 50, batch_q: int = 4096,
                       batch_c: int = 2048, lr: float = 0.05, seed: int = 0):
    """Adam on the codebooks; returns (codebooks, per-step losses)."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    CB = CB0.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([CB], lr=lr)
    hist = []
    for _ in range(steps):
        qi = torch.randint(0, queries.shape[0], (min(batch_q, queries.shape[0]),), generator=gen)
        ci = torch.randint(0, X.shape[0], (min(batch_c, X.shape[0]),), generator=gen)
        qi, ci = qi.to(queries.device), ci.to(X.device)
        opt.zero_grad(set_to_none=True)
        loss = distortion_loss(queries[qi].contiguous(), CB, codes[ci].contiguous(),
                               X[ci].contiguous())
        loss.backward()
        opt.step()
        hist.append(float(loss.detach()))
    return CB.detach(), hist
