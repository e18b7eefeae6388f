"""Per-Jacobian choice of the perturbation size, built on top of the C ABI.

The expansion behind the method converges only while every node satisfies
|eps_k| rho(A^{-1} D) < 1 (Sec. II-B), and its truncation error is about
prod_k |eps_k| rho^K, so one node set for a whole batch fails on the
scenarios whose rho is large (Sec. V names the choice of eps and D as open).
This module estimates rho for every Jacobian of a batch with a few power
iterations on a slightly perturbed factorisation, picks
    eps_0 = 10^-(ceil(log10 rho) + 2),   eps_k = eps_0 ratio^k,
so that eps_0 rho <= 0.01, and solves each group of Jacobians that share an
eps_0 with one batched call.  The power iteration and every factorisation
and solve run in the library's kernels; this module draws the start vectors
and groups the Jacobians by eps_0 on the host.
"""
from __future__ import annotations

import math

import numpy as np

from . import psp


def estimate_rho(plan: psp.Plan, values, d=None, probe: float = 1e-8, iters: int = 24, seed: int = 0):
    """rho(A_s^{-1} D) for every Jacobian s of `values` (batch, nnz), as a float64 numpy array.

    Power iteration with M = (A + probe D)^{-1} D on the library's factors
    (psp_estimate_rho); the estimate is the mean growth factor over the second
    half of the iterations, which is robust when the dominant eigenvalues are a
    complex pair.  The start vectors are standard normal draws from `seed`."""
    import torch
    batch, n = values.shape[0], plan.n
    gen = torch.Generator(device="cpu").manual_seed(seed)
    v0 = torch.randn((batch, n), generator=gen, dtype=torch.float64).to(values.device)
    return psp.estimate_rho(plan, values, v0, d=d, probe=probe, iters=iters).cpu().numpy()


def choose_eps0(rho, offset: int = 2):
    """eps_0 = 10^-(ceil(log10 rho) + offset) per Jacobian (rho <= 0 or non-finite: 1e-3 * 10^-offset)."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.empty_like(rho)
    for i, r in enumerate(rho):
        e = math.ceil(math.log10(r)) if (np.isfinite(r) and r > 0) else 3
        out[i] = 10.0 ** (-(e + offset))
    return out


def solve_adaptive(plan: psp.Plan, values, b, K: int = 5, ratio: float = 0.5, d=None, offset: int = 2,
                   rho=None, path: str = "auto"):
    """Alg. 1 with eps chosen per Jacobian: returns (x, info, eps0) with x shaped like b,
    info (batch, K) and eps0 (batch,) the first node used for each Jacobian."""
    import torch
    if rho is None:
        rho = estimate_rho(plan, values, d=d)
    eps0 = choose_eps0(rho, offset)
    x = torch.empty_like(b)
    info = torch.empty((values.shape[0], K), dtype=torch.int32, device=values.device)
    for e0 in np.unique(eps0):
        idx_np = np.nonzero(eps0 == e0)[0]
        idx = torch.from_numpy(idx_np).to(values.device)
        eps = e0 * ratio ** np.arange(K)
        xs, inf = psp.solve_batched(plan, values.index_select(0, idx).contiguous(), eps,
                                    b.index_select(0, idx).contiguous(), path=path, d=d)
        x.index_copy_(0, idx, xs)
        info.index_copy_(0, idx, inf)
    return x, info, eps0
