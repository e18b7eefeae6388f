"""Oracle pins for the symbolic analysis (static pivot sequence, Sec. II-C): minimum-degree
order, fill, elimination tree and level sets, each checked against a brute-force
construction from its definition, plus a sanity bound against SuperLU's MMD ordering."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _sym_adj(n, ip, ix):
    adj = [set() for _ in range(n)]
    for i in range(n):
        for j in ix[ip[i]:ip[i + 1]]:
            if j != i:
                adj[i].add(int(j))
                adj[int(j)].add(i)
    return adj


def _brute_md(n, ip, ix):
    """Minimum degree by explicit elimination with Python sets (definition in the oracle header)."""
    adj0 = _sym_adj(n, ip, ix)
    dense = [i for i in range(n) if len(adj0[i]) > 16 and len(adj0[i]) ** 2 > 100 * n]
    ds = set(dense)
    g = {i: {j for j in adj0[i] if j not in ds} for i in range(n) if i not in ds}
    order = []
    while g:
        p = min(g, key=lambda i: (len(g[i]), i))
        nb = g.pop(p)
        for u in nb:
            g[u] |= nb
            g[u].discard(u)
            g[u].discard(p)
        order.append(p)
    return np.array(order + sorted(dense), dtype=np.int32)


def _brute_fill(n, ip, ix, perm):
    """Boolean Gaussian elimination on P S P^T (S = pat(A) | pat(A^T) | I)."""
    S = np.zeros((n, n), dtype=bool)
    for i in range(n):
        S[i, ix[ip[i]:ip[i + 1]]] = True
    S = S | S.T | np.eye(n, dtype=bool)
    B = S[np.ix_(perm, perm)].copy()
    for k in range(n):
        rows = np.nonzero(B[k + 1:, k])[0] + k + 1
        cols = np.nonzero(B[k, k + 1:])[0] + k + 1
        if len(rows) and len(cols):
            B[np.ix_(rows, cols)] = True
    return B


def _liu_etree(n, ip, ix, iperm):
    """Liu's elimination-tree algorithm (path-compressed ancestors) on P S P^T."""
    adj = _sym_adj(n, ip, ix)
    rows = [sorted(iperm[j] for j in adj[i]) for i in range(n)]
    byperm = [None] * n
    for i in range(n):
        byperm[iperm[i]] = rows[i]
    parent = [-1] * n
    anc = [-1] * n
    for i in range(n):
        for k in byperm[i]:
            if k >= i:
                continue
            r = k
            while anc[r] != -1 and anc[r] != i:
                nxt = anc[r]
                anc[r] = i
                r = nxt
            if anc[r] == -1:
                anc[r] = i
                parent[r] = i
    return np.array(parent, dtype=np.int32)


def _patterns(W):
    out = []
    for N in (14, 30, 118):
        ip, ix, _, _ = W.scenario_batch(N, 1)
        out.append((f"jac{N}", len(ip) - 1, ip, ix))
    rng = np.random.default_rng(9)
    for t, (n, p) in enumerate([(12, 0.25), (40, 0.08), (70, 0.05), (90, 0.3)]):
        M = sp.random(n, n, density=p, random_state=np.random.RandomState(t), format="csr")
        M = (M + sp.eye(n)).tocsr()
        M.sort_indices()
        if t == 3:   # add a few dense rows/columns to exercise the dense rule
            M = M.tolil()
            for r in rng.choice(n, 3, replace=False):
                M[r, :] = 1.0
            M = M.tocsr()
            M.sort_indices()
        out.append((f"rand{n}", n, M.indptr.astype(np.int32), M.indices.astype(np.int32)))
    return out


def test_md_order_matches_brute_force(O, W):
    for name, n, ip, ix in _patterns(W):
        s = O.symbolic(n, ip, ix)
        assert np.array_equal(s.perm, _brute_md(n, ip, ix)), name
        assert np.array_equal(np.sort(s.perm), np.arange(n))
        assert np.array_equal(s.iperm[s.perm], np.arange(n))


def test_dense_rule_catches_slack_column_at_601(O, W):
    ip, ix, _, _ = W.scenario_batch(300, 1)
    n = len(ip) - 1
    s = O.symbolic(n, ip, ix)
    assert s.ndense == 1 and s.perm[-1] == n - 1      # the slack (lambda) column is ordered last


@pytest.mark.parametrize("natural", [False, True])
def test_fill_etree_levels_vs_definitions(O, W, natural):
    cases = _patterns(W)
    ip, ix, _, _ = W.scenario_batch(300, 1)
    cases.append(("jac300", len(ip) - 1, ip, ix))
    for name, n, ip, ix in cases:
        s = O.symbolic(n, ip, ix, natural=natural)
        if natural:
            assert np.array_equal(s.perm, np.arange(n))
        B = _brute_fill(n, ip, ix, s.perm)
        for j in range(n):
            want = np.nonzero(B[j + 1:, j])[0] + j + 1
            assert np.array_equal(s.li[s.lp[j]:s.lp[j + 1]], want), (name, j)
        # U pattern is the transpose: the boolean elimination fills symmetrically
        assert np.array_equal(np.triu(B, 1), np.tril(B, -1).T)
        par = _liu_etree(n, ip, ix, s.iperm)
        assert np.array_equal(s.parent, par), name
        # levels from their definitions
        height = np.zeros(n, int)
        for j in range(n):
            if par[j] >= 0:
                height[par[j]] = max(height[par[j]], height[j] + 1)
        L = np.tril(B, -1)
        lev_l = np.zeros(n, int)
        for i in range(n):
            deps = np.nonzero(L[i, :i])[0]
            lev_l[i] = 1 + lev_l[deps].max() if len(deps) else 0
        lev_u = np.zeros(n, int)
        for i in range(n - 1, -1, -1):
            deps = np.nonzero(L[i + 1:, i])[0] + i + 1      # U_ij != 0, j > i
            lev_u[i] = 1 + lev_u[deps].max() if len(deps) else 0
        for t, lev in enumerate((height, lev_l, lev_u)):
            ptr, idx = s.levels[t]
            assert len(ptr) - 1 == lev.max() + 1
            for l in range(len(ptr) - 1):
                assert np.array_equal(idx[ptr[l]:ptr[l + 1]], np.nonzero(lev == l)[0]), (name, t, l)


def test_md_fill_sanity_vs_superlu(O, W):
    """Sanity (not a parity pin): MD fill within 1.5x of SuperLU's MMD on A^T + A."""
    for N in (118, 300):
        ip, ix, vals, _ = W.scenario_batch(N, 1)
        n = len(ip) - 1
        s = O.symbolic(n, ip, ix)
        A = sp.csc_matrix(sp.csr_matrix((vals[0], ix, ip), shape=(n, n)) + 1e-3 * sp.eye(n))
        lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        ours = 2 * s.nnzL + n
        assert ours <= 1.5 * (lu.L.nnz + lu.U.nnz)
        nat = O.symbolic(n, ip, ix, natural=True)
        assert s.nnzL < nat.nnzL


@pytest.mark.parametrize("bad", ["unsorted", "dup", "range", "ptr"])
def test_malformed_csr_rejected(O, bad):
    ip = np.array([0, 2, 3, 5], np.int32)
    ix = np.array([0, 2, 1, 0, 2], np.int32)
    if bad == "unsorted":
        ix = np.array([2, 0, 1, 0, 2], np.int32)
    elif bad == "dup":
        ix = np.array([0, 0, 1, 0, 2], np.int32)
    elif bad == "range":
        ix = np.array([0, 3, 1, 0, 2], np.int32)
    else:
        ip = np.array([0, 3, 2, 5], np.int32)
    with pytest.raises(ValueError):
        O.symbolic(3, ip, ix)
