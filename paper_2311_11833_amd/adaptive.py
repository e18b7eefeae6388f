"""Per-Jacobian perturbation size on top of the C ABI.

The expansion behind the method converges only while every node satisfies
|eps_k| rho(A^{-1} D) < 1 (Sec. II-B), and its truncation error grows with
the nodes while the rounding of the pivot-free solves grows as they shrink,
so one node set for a whole batch fails on the Jacobians whose rho is large
(Sec. V names the choice of eps and D as open).  Two tools, both in the
library's kernels:

* solve_adaptive: psp_solve_adaptive, the error test of Alg. 1 step 5 taken
  from the perturbed solutions themselves, with a second, rescaled solve of the
  Jacobians that fail it (the rule lives behind the C ABI);
* estimate_rho: psp_estimate_rho, power iteration for rho(A^{-1} D) on a
  slightly perturbed pivot-free factorisation (diagnostics); this module only
  draws its start vectors.
"""
from __future__ import annotations

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


def solve_adaptive(plan: psp.Plan, values, b, eps, tol: float = 1e-10, d=None):
    """Alg. 1 with the error test choosing the node size per Jacobian; returns (x, info, est, scale)."""
    return psp.solve_adaptive(plan, values, eps, b, tol=tol, d=d)
