"""Seeded synthetic inputs: power-flow Jacobians, right-hand sides, perturbation sets.

This module is shared by the oracle tests and the GPU path.  It holds none of
the method's arithmetic (no factorisation, substitution, weights or combine);
it only draws the systems that the method is applied to.

The paper evaluates the distributed-slack AC power-flow Jacobian of the PGLib
300-bus case at many voltage initialisations (Sec. IV).  That dataset is not
available here, so every workload is a seeded stand-in with the same
structure:

* network: a random spanning tree plus random extra branches, series
  impedance ``r ~ U[0.01, 0.1]``, ``x ~ U[0.05, 0.3]`` p.u., no shunts;
* state: ``|V| ~ U[0.95, 1.05]``, ``theta ~ U[-0.2, 0.2]``, slack
  participation ``p ~ Dirichlet(1)``;
* Jacobian of ``[P(theta, V) - P0 - p*lambda ; Q(theta, V) - Q0 ; theta_ref]``
  with respect to ``[theta, |V|, lambda]``: ``n = 2N + 1``.  All buses are
  treated as PQ buses and bus 0 is the angle reference.

Because P and Q depend on angles only through differences, the leading
2N x 2N block is singular, which is what makes the unperturbed pivot-free
factorisation break down (Sec. IV, first observation).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Network", "Jacobian", "branch_count", "make_network", "make_state",
    "jacobian", "rhs", "geometric_eps", "config_eps", "seed_net",
    "seed_state", "seed_rhs", "scenario_batch", "to_dense",
    "PowerFlowCase", "PowerFlowScenarios", "pf_case", "pf_scenarios",
]


def seed_net(N: int, inst: int = 0) -> int:
    return 1000 * inst + N


def seed_state(N: int, scenario: int) -> int:
    return 7_000_000 + 1000 * scenario + N


def seed_rhs(N: int, scenario: int) -> int:
    return seed_state(N, scenario) + 1


def branch_count(N: int) -> int:
    """Branch count used for an N-bus synthetic network."""
    fixed = {14: 20, 300: 411, 10000: 13000}
    return fixed.get(N, int(round(1.37 * N)))


@dataclass
class Network:
    N: int
    fbus: np.ndarray  # int64 [L]
    tbus: np.ndarray  # int64 [L]
    r: np.ndarray     # float64 [L]
    x: np.ndarray     # float64 [L]


@dataclass
class Jacobian:
    """A square sparse matrix in CSR form (sorted columns, no duplicates)."""
    n: int
    indptr: np.ndarray   # int32 [n+1]
    indices: np.ndarray  # int32 [nnz]
    data: np.ndarray     # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])


def make_network(N: int, L: int | None = None, seed: int | None = None) -> Network:
    """Random connected network: spanning tree, then distinct extra branches."""
    if L is None:
        L = branch_count(N)
    if L < N - 1 or L > N * (N - 1) // 2:
        raise ValueError("branch count out of range")
    rng = np.random.default_rng(seed_net(N) if seed is None else seed)
    order = rng.permutation(N)
    edges: list[tuple[int, int]] = []
    seen: set[tuple[int, int]] = set()
    for i in range(1, N):
        j = int(rng.integers(0, i))
        a, b = int(order[i]), int(order[j])
        e = (min(a, b), max(a, b))
        seen.add(e)
        edges.append(e)
    while len(edges) < L:
        a, b = (int(v) for v in rng.integers(0, N, 2))
        if a == b:
            continue
        e = (min(a, b), max(a, b))
        if e in seen:
            continue
        seen.add(e)
        edges.append(e)
    r = rng.uniform(0.01, 0.1, L)
    x = rng.uniform(0.05, 0.3, L)
    ed = np.array(edges, dtype=np.int64)
    return Network(N, ed[:, 0].copy(), ed[:, 1].copy(), r, x)


def make_state(N: int, seed: int):
    rng = np.random.default_rng(seed)
    vm = rng.uniform(0.95, 1.05, N)
    va = rng.uniform(-0.2, 0.2, N)
    part = rng.dirichlet(np.ones(N))
    return vm, va, part


def _ybus_entries(net: Network):
    """Bus admittance matrix as (row, col, G, B) over its structural pattern."""
    N = net.N
    y = 1.0 / (net.r + 1j * net.x)
    diag = np.zeros(N, dtype=np.complex128)
    np.add.at(diag, net.fbus, y)
    np.add.at(diag, net.tbus, y)
    rows = np.concatenate([np.arange(N), net.fbus, net.tbus])
    cols = np.concatenate([np.arange(N), net.tbus, net.fbus])
    vals = np.concatenate([diag, -y, -y])
    return rows, cols, vals


def jacobian(net: Network, vm: np.ndarray, va: np.ndarray, part: np.ndarray) -> Jacobian:
    """Distributed-slack polar power-flow Jacobian, n = 2N+1, CSR."""
    N = net.N
    yr, yc, yv = _ybus_entries(net)
    G, B = yv.real, yv.imag
    dth = va[yr] - va[yc]
    c, s = np.cos(dth), np.sin(dth)
    # injections P_i, Q_i
    tp = vm[yr] * vm[yc] * (G * c + B * s)
    tq = vm[yr] * vm[yc] * (G * s - B * c)
    P = np.zeros(N)
    Q = np.zeros(N)
    np.add.at(P, yr, tp)
    np.add.at(Q, yr, tq)
    off = yr != yc
    dP_dth = np.where(off, vm[yr] * vm[yc] * (G * s - B * c), 0.0)
    dP_dv = np.where(off, vm[yr] * (G * c + B * s), 0.0)
    dQ_dth = np.where(off, -vm[yr] * vm[yc] * (G * c + B * s), 0.0)
    dQ_dv = np.where(off, vm[yr] * (G * s - B * c), 0.0)
    d = ~off
    i = yr[d]
    Gd, Bd = G[d], B[d]
    dP_dth[d] = -Q[i] - Bd * vm[i] ** 2
    dP_dv[d] = P[i] / vm[i] + Gd * vm[i]
    dQ_dth[d] = P[i] - Gd * vm[i] ** 2
    dQ_dv[d] = Q[i] / vm[i] - Bd * vm[i]

    n = 2 * N + 1
    rows = np.concatenate([yr, yr, N + yr, N + yr, np.arange(N), [2 * N]])
    cols = np.concatenate([yc, N + yc, yc, N + yc, np.full(N, 2 * N), [0]])
    vals = np.concatenate([dP_dth, dP_dv, dQ_dth, dQ_dv, -part, [1.0]])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if np.any((rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])):
        raise RuntimeError("duplicate Jacobian entry")
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr).astype(np.int32)
    return Jacobian(n, indptr, cols.astype(np.int32), vals.astype(np.float64))


def rhs(n: int, seed: int, nrhs: int = 1, scale_range: tuple[float, float] | None = None) -> np.ndarray:
    """b ~ N(0,1), shape (n,) or (n, nrhs); optional per-scenario load scale."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    if scale_range is not None:
        b = b * rng.uniform(*scale_range)
    return b


def geometric_eps(eps0: float, K: int, ratio: float = 0.5) -> np.ndarray:
    """Positive geometric perturbation set eps0 * ratio**k, k = 0..K-1."""
    return np.array([eps0 * ratio ** k for k in range(K)], dtype=np.float64)


def config_eps(name: str) -> np.ndarray:
    """Perturbation sets of the named workloads (small: K=3; n=601 family: K=5)."""
    if name == "small":
        return np.array([1e-2, 5e-3, 2.5e-3])
    if name in ("n601", "uneven", "adjoint"):
        return geometric_eps(1e-3, 5)
    raise KeyError(name)


def large_eps(K: int = 4) -> np.ndarray:
    """Nodes for the 20,001-unknown workload: the symmetric scheme +-eps0, +-2 eps0 (Sec. III's
    +-alpha eps nodes), eps0 = 1e-5.

    The Neumann series of (A + eps D)^{-1} converges for |eps| rho(A^{-1} D) < 1
    (Sec. II-B).  For the seeded 10,000-bus states rho(A^{-1}) is 2e2 to 1e3
    (measured offline by power iteration), so eps0 = 10^-(ceil(log10 rho) + 2)
    keeps eps0 * rho near 1e-2.  At this size the error of the recovered solution
    is dominated by the rounding of the pivot-free solves (a pivot the perturbation
    controls is of order eps), which the combination amplifies by
    sum_k |c_k| / |eps_k|: 36 / eps0 for the geometric nodes eps0 * 2^-k, 1.5 / eps0
    for these.  K other than 4 takes the geometric nodes eps0 * 2^-k.
    """
    if K != 4:
        return geometric_eps(1e-5, K)
    return np.array([1e-5, -1e-5, 2e-5, -2e-5], dtype=np.float64)


def scenario_batch(N: int, count: int, inst: int = 0, first: int = 0,
                   scale_range: tuple[float, float] | None = None):
    """`count` Jacobians of one network at seeded states, plus their RHS.

    Returns (indptr, indices, values[count, nnz], b[count, n]).  Every
    Jacobian shares the network's sparsity pattern.
    """
    net = make_network(N, seed=seed_net(N, inst))
    vals = []
    bs = []
    pat = None
    for s in range(first, first + count):
        vm, va, part = make_state(N, seed_state(N, s))
        J = jacobian(net, vm, va, part)
        if pat is None:
            pat = (J.indptr, J.indices)
        elif not (np.array_equal(pat[0], J.indptr) and np.array_equal(pat[1], J.indices)):
            raise RuntimeError("pattern changed between scenarios")
        vals.append(J.data)
        bs.append(rhs(J.n, seed_rhs(N, s), scale_range=scale_range))
    return pat[0], pat[1], np.stack(vals), np.stack(bs)


UNEVEN_NETWORKS = (30, 118, 300, 500, 1354)


def uneven_batch(total: int = 512, networks=UNEVEN_NETWORKS, seed: int = 2311):
    """Jacobians of several networks in one batch: each of `total` Jacobians picks its
    network uniformly (seeded), then gets its own seeded state and RHS.  Returns a list
    of (N, indptr, indices, values[count, nnz], b[count, n]) per network that was drawn."""
    pick = np.random.default_rng(seed).integers(0, len(networks), size=total)
    out = []
    for i, N in enumerate(networks):
        count = int(np.sum(pick == i))
        if count:
            out.append((N,) + scenario_batch(N, count))
    return out


# ---------------------------------------------------------------------------
# Newton-Raphson power flows (the setting of Sec. IV: a Jacobian solve per
# Newton step of a distributed-slack AC power flow).
#
# Unknowns x = [theta (N) | |V| (N) | lambda] and equations
#   F = [P(x) - P0 - part*lambda (N) | Q(x) - Q0 on PQ buses, |V| - V_set on
#        PV buses (N) | theta_0 - theta_ref],
# with the injection specification spec = [P0 | Q0 or V_set | theta_ref] laid
# out like x.  A PV (generator) bus holds its voltage magnitude and lets its
# reactive output float, as in the paper's reduced 531-unknown system of the
# 300-bus case (69 generator buses: 2*300 - 69 = 531); here the reduction is
# replaced by a unit row, so the Jacobian keeps the pattern of `jacobian`.
# Generator buses carry the distributed slack (part > 0 only there).

PV_FRACTION = 69 / 300


@dataclass
class PowerFlowCase:
    net: Network
    pv: np.ndarray          # int32 [N]: 1 = voltage-controlled bus (bus 0 always)
    y_indptr: np.ndarray    # int32 [N+1]: bus admittance matrix, CSR, sorted, diagonal present
    y_indices: np.ndarray   # int32 [ny]
    g: np.ndarray           # float64 [ny]: conductance G_ij
    b: np.ndarray           # float64 [ny]: susceptance B_ij
    indptr: np.ndarray      # int32 [n+1]: Jacobian pattern (n = 2N+1), that of `jacobian`
    indices: np.ndarray     # int32 [nnz]

    @property
    def N(self) -> int:
        return self.net.N

    @property
    def n(self) -> int:
        return 2 * self.net.N + 1


@dataclass
class PowerFlowScenarios:
    x_target: np.ndarray    # [batch, n]: the state the specification was drawn from (a solution)
    spec: np.ndarray        # [batch, n]
    part: np.ndarray        # [batch, N]: slack participation, sums to 1, zero on PQ buses
    x0: np.ndarray          # [batch, n]: flat start (theta = 0, |V| = 1 or V_set, lambda = 0)


def pf_case(N: int, pv_fraction: float = PV_FRACTION, seed: int | None = None) -> PowerFlowCase:
    net = make_network(N, seed=seed)
    rng = np.random.default_rng(seed_net(N) + 17 if seed is None else seed + 17)
    ng = max(1, int(round(pv_fraction * N)))
    pv = np.zeros(N, dtype=np.int32)
    pv[0] = 1
    if ng > 1:
        pv[rng.choice(np.arange(1, N), ng - 1, replace=False)] = 1
    yr, yc, yv = _ybus_entries(net)
    order = np.lexsort((yc, yr))
    yr, yc, yv = yr[order], yc[order], yv[order]
    if np.any((yr[1:] == yr[:-1]) & (yc[1:] == yc[:-1])):
        raise RuntimeError("duplicate admittance entry")
    y_indptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(y_indptr, yr + 1, 1)
    y_indptr = np.cumsum(y_indptr).astype(np.int32)
    J = jacobian(net, np.ones(N), np.zeros(N), np.full(N, 1.0 / N))
    return PowerFlowCase(net, pv, y_indptr, yc.astype(np.int32), yv.real.copy(), yv.imag.copy(),
                         J.indptr, J.indices)


def pf_scenarios(case: PowerFlowCase, batch: int, seed: int = 3110, p_sigma: float = 0.5,
                 v_spread: float = 0.02) -> PowerFlowScenarios:
    """Seeded solvable scenarios: scenario s draws balanced active injections
    p ~ N(0, p_sigma), takes the DC power-flow angles for them as its target
    angles (bus 0 the reference), |V| ~ U[1 - v_spread, 1 + v_spread],
    part ~ Dirichlet(1) over the generator buses and lambda ~ U[-1, 1], and
    specifies the injections that this target implies (so the target is a
    root of F).  Draws depend only on (seed, s)."""
    import scipy.sparse as sps
    import scipy.sparse.linalg as spl
    net, N, n = case.net, case.N, case.n
    bl = 1.0 / net.x
    Bdc = sps.coo_matrix((np.concatenate([bl, bl, -bl, -bl]),
                          (np.concatenate([net.fbus, net.tbus, net.fbus, net.tbus]),
                           np.concatenate([net.fbus, net.tbus, net.tbus, net.fbus]))), shape=(N, N)).tocsc()
    lu = spl.splu(Bdc[1:, 1:].tocsc())
    Y = sps.csr_matrix((case.g + 1j * case.b, case.y_indices, case.y_indptr), shape=(N, N))
    pvb = case.pv.astype(bool)
    xt = np.zeros((batch, n))
    spec = np.zeros((batch, n))
    part = np.zeros((batch, N))
    x0 = np.zeros((batch, n))
    for s in range(batch):
        rng = np.random.default_rng((seed, N, s))
        p = rng.normal(0.0, p_sigma, N)
        p -= p.mean()
        th = np.zeros(N)
        th[1:] = lu.solve(p[1:])
        vm = rng.uniform(1.0 - v_spread, 1.0 + v_spread, N)
        part[s, pvb] = rng.dirichlet(np.ones(int(pvb.sum())))
        lam = rng.uniform(-1.0, 1.0)
        V = vm * np.exp(1j * th)
        S = V * np.conj(Y @ V)
        xt[s] = np.concatenate([th, vm, [lam]])
        spec[s] = np.concatenate([S.real - part[s] * lam, np.where(pvb, vm, S.imag), [0.0]])
        x0[s] = np.concatenate([np.zeros(N), np.where(pvb, vm, 1.0), [0.0]])
    return PowerFlowScenarios(xt, spec, part, x0)


def to_dense(n: int, indptr: np.ndarray, indices: np.ndarray, data: np.ndarray) -> np.ndarray:
    A = np.zeros((n, n))
    for i in range(n):
        A[i, indices[indptr[i]:indptr[i + 1]]] = data[indptr[i]:indptr[i + 1]]
    return A

