"""Newton-Raphson AC power flow around the perturbed solve (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
module; it shares no code with the GPU library.  The paper applies its method
to the linear solve of every Newton step of a distributed-slack AC power flow
(Sec. IV); this module is the plain reference for that loop:

* injections from the polar power-flow equations,
      P_i = sum_j V_i V_j (G_ij cos t_ij + B_ij sin t_ij),
      Q_i = sum_j V_i V_j (G_ij sin t_ij - B_ij cos t_ij),   t_ij = theta_i - theta_j,
  summed over row i of the bus admittance matrix in CSR order;
* the mismatch F(x) for x = [theta | |V| | lambda] and spec = [P0 | Q0 or
  V_set | theta_ref]:  F = [P - P0 - part*lambda | Q - Q0 (PQ bus) or
  |V| - V_set (PV bus) | theta_0 - theta_ref];
* its Jacobian from the closed-form derivatives of P and Q (off-diagonal and
  diagonal formulas below), with a unit row for every PV bus and for the
  angle reference, in the CSR order of the given pattern;
* the Newton loop: evaluate F; stop when max|F| <= tol (converged), when it
  is not finite (diverged) or after max_iter updates; otherwise solve J dx = F
  with Alg. 1 (the C oracle's perturbed sparse solve; any nonzero info stops
  the scenario as a breakdown) and set x <- x - dx.

Status codes: 0 converged, 1 iteration limit, 2 breakdown, 3 not finite.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

CONVERGED, MAXITER, BREAKDOWN, DIVERGED = 0, 1, 2, 3


def _rows(indptr):
    return np.repeat(np.arange(len(indptr) - 1), np.diff(indptr))


def injections(y_indptr, y_indices, g, b, x):
    """(P, Q) at the state x = [theta | |V| | lambda] (one scenario)."""
    N = len(y_indptr) - 1
    th, vm = x[:N], x[N:2 * N]
    i = _rows(y_indptr)
    j = np.asarray(y_indices)
    t = th[i] - th[j]
    c, s = np.cos(t), np.sin(t)
    w = vm[i] * vm[j]
    P = np.zeros(N)
    Q = np.zeros(N)
    np.add.at(P, i, w * (g * c + b * s))
    np.add.at(Q, i, w * (g * s - b * c))
    return P, Q


def mismatch(y_indptr, y_indices, g, b, pv, x, spec, part):
    N = len(y_indptr) - 1
    P, Q = injections(y_indptr, y_indices, g, b, x)
    vm, lam = x[N:2 * N], x[2 * N]
    fq = np.where(np.asarray(pv) != 0, vm - spec[N:2 * N], Q - spec[N:2 * N])
    return np.concatenate([P - spec[:N] - part * lam, fq, [x[0] - spec[2 * N]]])


def jacobian_values(y_indptr, y_indices, g, b, pv, x, part, indptr, indices):
    """dF/dx on the pattern (indptr, indices), as the nnz values in its CSR order.
    Raises if the pattern lacks an entry the derivatives need or holds one they do not."""
    N = len(y_indptr) - 1
    n = 2 * N + 1
    th, vm = x[:N], x[N:2 * N]
    P, Q = injections(y_indptr, y_indices, g, b, x)
    pos = {}
    for r in range(n):
        for e in range(indptr[r], indptr[r + 1]):
            pos[(r, int(indices[e]))] = e
    vals = np.full(int(indptr[-1]), np.nan)

    def put(r, c, v):
        vals[pos[(r, c)]] = v

    for i in range(N):
        for e in range(y_indptr[i], y_indptr[i + 1]):
            j = int(y_indices[e])
            G, B = g[e], b[e]
            if j != i:
                t = th[i] - th[j]
                c, s = np.cos(t), np.sin(t)
                put(i, j, vm[i] * vm[j] * (G * s - B * c))            # dP_i/dtheta_j
                put(i, N + j, vm[i] * (G * c + B * s))                # dP_i/d|V_j|
                dq_th = -vm[i] * vm[j] * (G * c + B * s)              # dQ_i/dtheta_j
                dq_v = vm[i] * (G * s - B * c)                        # dQ_i/d|V_j|
            else:
                put(i, i, -Q[i] - B * vm[i] ** 2)
                put(i, N + i, P[i] / vm[i] + G * vm[i])
                dq_th = P[i] - G * vm[i] ** 2
                dq_v = Q[i] / vm[i] - B * vm[i]
            if pv[i]:
                put(N + i, j, 0.0)
                put(N + i, N + j, 1.0 if j == i else 0.0)
            else:
                put(N + i, j, dq_th)
                put(N + i, N + j, dq_v)
        put(i, 2 * N, -part[i])
    put(2 * N, 0, 1.0)
    if np.isnan(vals).any():
        raise ValueError("pattern holds entries outside the power-flow Jacobian")
    return vals


def newton(y_indptr, y_indices, g, b, pv, indptr, indices, x0, spec, part, eps, tol=1e-9, max_iter=10,
           d=None, sym=None):
    """Batched Newton loop, one scenario at a time.  x0, spec: (batch, n); part (batch, N).
    Returns (x, iters, status, fnorm, history) with history[s] the max|F| of every evaluation."""
    x0 = np.atleast_2d(np.asarray(x0, dtype=np.float64))
    batch, n = x0.shape
    if sym is None:
        sym = O.symbolic(n, indptr, indices)
    x = x0.copy()
    iters = np.zeros(batch, dtype=np.int32)
    status = np.full(batch, MAXITER, dtype=np.int32)
    fnorm = np.zeros(batch)
    hist = []
    for s in range(batch):
        h = []
        for it in range(max_iter + 1):
            F = mismatch(y_indptr, y_indices, g, b, pv, x[s], spec[s], part[s])
            fn = np.abs(F).max()
            fnorm[s] = fn
            h.append(fn)
            if fn <= tol:
                status[s] = CONVERGED
                break
            if not np.isfinite(fn):
                status[s] = DIVERGED
                break
            if it == max_iter:
                status[s] = MAXITER
                break
            J = jacobian_values(y_indptr, y_indices, g, b, pv, x[s], part[s], indptr, indices)
            dx, info, _, _ = O.sparse_batch(n, indptr, indices, J[None], sym, eps, F[None], d=d)
            if np.any(info != 0):
                status[s] = BREAKDOWN
                break
            x[s] -= dx[0]
            iters[s] += 1
        hist.append(h)
    return x, iters, status, fnorm, hist
