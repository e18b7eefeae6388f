/*
 * psp_oracle_sparse.c -- symbolic analysis, sparse pivot-free LU, sparse
 * substitutions and the adjoint gradient for the oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see psp_oracle.c).  Shares no code with the GPU
 * path.
 *
 * The static pivot sequence of Sec. II-C is computed once per sparsity
 * pattern and reused for every perturbed system.  The sparse batched
 * factorisation is the direction the paper names in Sec. IV and Sec. V.
 * Definitions used here (the paper fixes none of them):
 *
 *   S        symmetric pattern: pat(A) union pat(A^T) union the diagonal.
 *   order    minimum degree on the elimination graph of S.  A vertex whose
 *            degree in S exceeds 16 and 10*sqrt(n) (tested as d*d > 100 n)
 *            is set aside and ordered last, in ascending index.  At every
 *            step the remaining vertex with the smallest degree in the
 *            current elimination graph is eliminated, ties to the smallest
 *            original index; eliminating v joins all its neighbours
 *            pairwise.  The degree is exact (not approximated), so the
 *            order is a function of the pattern alone.
 *   fill     struct(L(:,j)) = neighbours of j with larger position in the
 *            elimination graph of P S P^T at the moment j is eliminated.
 *            U has the transposed pattern plus the diagonal.
 *   etree    parent(j) = min struct(L(:,j)), -1 for a root.
 *   levels   factor: height in the etree (0 for a leaf).
 *            L-solve: lev(i) = 1 + max{lev(j) : L_ij != 0}, 0 if none.
 *            U-solve: lev(i) = 1 + max{lev(j) : U_ij != 0, j > i}, 0 if none.
 *            Each level lists its indices in ascending order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* ---------------- small growable sorted int sets ---------------- */
typedef struct { int* v; int n, cap; } iset;

static void iset_reserve(iset* s, int cap) {
    if (cap <= s->cap) return;
    int c = s->cap ? s->cap : 4;
    while (c < cap) c *= 2;
    s->v = (int*)realloc(s->v, sizeof(int) * (size_t)c);
    s->cap = c;
}

/* s <- (s union add) minus {x, y}; both sorted ascending. */
static void iset_merge_minus(iset* s, const int* add, int na, int x, int y, int* tmp) {
    int i = 0, j = 0, m = 0;
    while (i < s->n || j < na) {
        int v;
        if (j >= na || (i < s->n && s->v[i] < add[j])) v = s->v[i++];
        else if (i >= s->n || add[j] < s->v[i]) v = add[j++];
        else { v = s->v[i]; ++i; ++j; }
        if (v != x && v != y) tmp[m++] = v;
    }
    iset_reserve(s, m);
    memcpy(s->v, tmp, sizeof(int) * (size_t)m);
    s->n = m;
}

static int cmp_int(const void* a, const void* b) {
    const int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

typedef struct {
    int n, ndense;
    int *perm, *iperm, *parent;
    int *lp, *li;             /* L pattern, CSC, strictly lower, rows ascending (permuted indices) */
    int nlev[3];              /* factor, L-solve, U-solve */
    int *levp[3], *levi[3];
    int64_t nnzL;
} osym;

/* Validate CSR and build the symmetric adjacency (no self loops). */
static int build_sym(int n, const int* rp, const int* ci, iset* adj) {
    if (n < 1 || rp[0] != 0) return -1;
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return -1;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return -1;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return -1;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = ci[e];
            if (j == i) continue;
            iset_reserve(&adj[i], adj[i].n + 1); adj[i].v[adj[i].n++] = j;
            iset_reserve(&adj[j], adj[j].n + 1); adj[j].v[adj[j].n++] = i;
        }
    for (int i = 0; i < n; ++i) {
        qsort(adj[i].v, (size_t)adj[i].n, sizeof(int), cmp_int);
        int m = 0;
        for (int t = 0; t < adj[i].n; ++t)
            if (m == 0 || adj[i].v[t] != adj[i].v[m - 1]) adj[i].v[m++] = adj[i].v[t];
        adj[i].n = m;
    }
    return 0;
}

static void free_adj(iset* adj, int n) {
    for (int i = 0; i < n; ++i) free(adj[i].v);
    free(adj);
}

/* Minimum degree on the explicit elimination graph (see header). */
static void md_order(int n, const iset* adj0, int* perm, int* ndense_out) {
    char* dense = (char*)calloc((size_t)n, 1);
    int ndense = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t d = adj0[i].n;
        if (d > 16 && d * d > 100 * (int64_t)n) { dense[i] = 1; ++ndense; }
    }
    iset* g = (iset*)calloc((size_t)n, sizeof(iset));
    for (int i = 0; i < n; ++i) {
        if (dense[i]) continue;
        for (int t = 0; t < adj0[i].n; ++t) {
            const int j = adj0[i].v[t];
            if (dense[j]) continue;
            iset_reserve(&g[i], g[i].n + 1); g[i].v[g[i].n++] = j;
        }
    }
    char* done = (char*)calloc((size_t)n, 1);
    int* tmp = (int*)malloc(sizeof(int) * (size_t)(2 * n + 2));
    int* nb = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    int pos = 0;
    for (int step = 0; step < n - ndense; ++step) {
        int p = -1, best = 0;
        for (int i = 0; i < n; ++i) {
            if (dense[i] || done[i]) continue;
            if (p < 0 || g[i].n < best) { p = i; best = g[i].n; }
        }
        perm[pos++] = p;
        done[p] = 1;
        const int m = g[p].n;
        memcpy(nb, g[p].v, sizeof(int) * (size_t)m);
        for (int t = 0; t < m; ++t) iset_merge_minus(&g[nb[t]], nb, m, nb[t], p, tmp);
        g[p].n = 0;
    }
    for (int i = 0; i < n; ++i)
        if (dense[i]) perm[pos++] = i;
    for (int i = 0; i < n; ++i) free(g[i].v);
    free(g); free(done); free(tmp); free(nb); free(dense);
    *ndense_out = ndense;
}

/* Fill by elimination of P S P^T in position order. */
static void fill_pattern(int n, const iset* adj0, const int* iperm, osym* s) {
    iset* g = (iset*)calloc((size_t)n, sizeof(iset));
    for (int i = 0; i < n; ++i) {
        const int pi = iperm[i];
        iset_reserve(&g[pi], adj0[i].n);
        for (int t = 0; t < adj0[i].n; ++t) g[pi].v[t] = iperm[adj0[i].v[t]];
        g[pi].n = adj0[i].n;
        qsort(g[pi].v, (size_t)g[pi].n, sizeof(int), cmp_int);
    }
    int* tmp = (int*)malloc(sizeof(int) * (size_t)(2 * n + 2));
    int* nb = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    int64_t cap = 1024, used = 0;
    int* li = (int*)malloc(sizeof(int) * (size_t)cap);
    int* lp = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    lp[0] = 0;
    for (int j = 0; j < n; ++j) {
        const int m = g[j].n;  /* all neighbours left are > j */
        memcpy(nb, g[j].v, sizeof(int) * (size_t)m);
        if (used + m > cap) { while (used + m > cap) cap *= 2; li = (int*)realloc(li, sizeof(int) * (size_t)cap); }
        memcpy(li + used, nb, sizeof(int) * (size_t)m);
        used += m;
        if (used > INT32_MAX) abort();
        lp[j + 1] = (int)used;
        for (int t = 0; t < m; ++t) iset_merge_minus(&g[nb[t]], nb, m, nb[t], j, tmp);
        free(g[j].v); g[j].v = NULL; g[j].n = g[j].cap = 0;
    }
    for (int i = 0; i < n; ++i) free(g[i].v);
    free(g); free(tmp); free(nb);
    s->lp = lp; s->li = li; s->nnzL = used;
}

static void make_levels(int n, const int* lev, int* nlev, int** lp, int** li) {
    int L = 0;
    for (int i = 0; i < n; ++i) if (lev[i] + 1 > L) L = lev[i] + 1;
    int* p = (int*)calloc((size_t)L + 1, sizeof(int));
    for (int i = 0; i < n; ++i) p[lev[i] + 1]++;
    for (int l = 0; l < L; ++l) p[l + 1] += p[l];
    int* fillp = (int*)malloc(sizeof(int) * (size_t)(L + 1));
    memcpy(fillp, p, sizeof(int) * (size_t)(L + 1));
    int* idx = (int*)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) idx[fillp[lev[i]]++] = i;   /* ascending i within a level */
    free(fillp);
    *nlev = L; *lp = p; *li = idx;
}

EXPORT int oracle_symbolic(int n, const int* rowptr, const int* colidx, int natural, osym** out) {
    *out = NULL;
    iset* adj = (iset*)calloc((size_t)n, sizeof(iset));
    if (build_sym(n, rowptr, colidx, adj) != 0) { free_adj(adj, n); return -1; }
    osym* s = (osym*)calloc(1, sizeof(osym));
    s->n = n;
    s->perm = (int*)malloc(sizeof(int) * (size_t)n);
    s->iperm = (int*)malloc(sizeof(int) * (size_t)n);
    s->parent = (int*)malloc(sizeof(int) * (size_t)n);
    if (natural) { for (int i = 0; i < n; ++i) s->perm[i] = i; s->ndense = 0; }
    else md_order(n, adj, s->perm, &s->ndense);
    for (int q = 0; q < n; ++q) s->iperm[s->perm[q]] = q;
    fill_pattern(n, adj, s->iperm, s);
    free_adj(adj, n);
    for (int j = 0; j < n; ++j) s->parent[j] = (s->lp[j + 1] > s->lp[j]) ? s->li[s->lp[j]] : -1;

    int* lev = (int*)malloc(sizeof(int) * (size_t)n);
    /* factor levels: etree height */
    for (int j = 0; j < n; ++j) lev[j] = 0;
    for (int j = 0; j < n; ++j)
        if (s->parent[j] >= 0 && lev[s->parent[j]] < lev[j] + 1) lev[s->parent[j]] = lev[j] + 1;
    make_levels(n, lev, &s->nlev[0], &s->levp[0], &s->levi[0]);
    /* L-solve levels: row i depends on every j with L_ij != 0 */
    for (int i = 0; i < n; ++i) lev[i] = 0;
    for (int j = 0; j < n; ++j)
        for (int t = s->lp[j]; t < s->lp[j + 1]; ++t)
            if (lev[s->li[t]] < lev[j] + 1) lev[s->li[t]] = lev[j] + 1;
    make_levels(n, lev, &s->nlev[1], &s->levp[1], &s->levi[1]);
    /* U-solve levels: row i depends on every j > i with U_ij != 0, i.e. j in struct(L(:,i)) */
    for (int i = n - 1; i >= 0; --i) {
        int m = 0;
        for (int t = s->lp[i]; t < s->lp[i + 1]; ++t)
            if (lev[s->li[t]] + 1 > m) m = lev[s->li[t]] + 1;
        lev[i] = m;
    }
    make_levels(n, lev, &s->nlev[2], &s->levp[2], &s->levi[2]);
    free(lev);
    *out = s;
    return 0;
}

/* sizes: n, nnzL, ndense, nlev_factor, nlev_lsolve, nlev_usolve */
EXPORT void oracle_symbolic_sizes(const osym* s, int64_t* sz) {
    sz[0] = s->n; sz[1] = s->nnzL; sz[2] = s->ndense;
    sz[3] = s->nlev[0]; sz[4] = s->nlev[1]; sz[5] = s->nlev[2];
}

EXPORT void oracle_symbolic_get(const osym* s, int* perm, int* iperm, int* parent, int* lp, int* li,
                                int* l0p, int* l0i, int* l1p, int* l1i, int* l2p, int* l2i) {
    const int n = s->n;
    memcpy(perm, s->perm, sizeof(int) * (size_t)n);
    memcpy(iperm, s->iperm, sizeof(int) * (size_t)n);
    memcpy(parent, s->parent, sizeof(int) * (size_t)n);
    memcpy(lp, s->lp, sizeof(int) * (size_t)(n + 1));
    memcpy(li, s->li, sizeof(int) * (size_t)s->nnzL);
    int* P[3] = {l0p, l1p, l2p};
    int* I[3] = {l0i, l1i, l2i};
    for (int t = 0; t < 3; ++t) {
        memcpy(P[t], s->levp[t], sizeof(int) * (size_t)(s->nlev[t] + 1));
        memcpy(I[t], s->levi[t], sizeof(int) * (size_t)n);
    }
}

EXPORT void oracle_symbolic_free(osym* s) {
    if (!s) return;
    free(s->perm); free(s->iperm); free(s->parent); free(s->lp); free(s->li);
    for (int t = 0; t < 3; ++t) { free(s->levp[t]); free(s->levi[t]); }
    free(s);
}

/* ------------------------------------------------------------------ */
/* Sparse pivot-free LU of P (A + eps D) P^T on the fill pattern,         */
/* left-looking.  Storage: udiag[n]; lval[nnzL] on the L pattern (CSC);   */
/* uval[nnzL]: U's strictly upper part stored by rows, where row k of U   */
/* has the column pattern struct(L(:,k)) (S is symmetric).                */
/* For column j: w = column j of the perturbed matrix; for each k < j     */
/* with U_kj != 0, ascending: u_kj = w_k, then w_i <- fma(-l_ik, w_k, w_i) */
/* for i in struct(L(:,k)); finally u_jj = w_j and l_ij = w_i / w_j.      */
/* Every entry sees the same update sequence as the dense factorisation.  */
/* Returns 0 or j+1 at the first zero / non-finite pivot.                 */
/* ------------------------------------------------------------------ */
static int find_pos(const int* a, int lo, int hi, int key) {
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Row structure of L (columns k < i with L_ik != 0), ascending. */
static void l_rows(int n, const int* lp, const int* li, int** rp_out, int** ri_out) {
    int* rp = (int*)calloc((size_t)n + 1, sizeof(int));
    for (int t = 0; t < lp[n]; ++t) rp[li[t] + 1]++;
    for (int i = 0; i < n; ++i) rp[i + 1] += rp[i];
    int* fill = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    memcpy(fill, rp, sizeof(int) * (size_t)(n + 1));
    int* ri = (int*)malloc(sizeof(int) * (size_t)(lp[n] > 0 ? lp[n] : 1));
    for (int k = 0; k < n; ++k)
        for (int t = lp[k]; t < lp[k + 1]; ++t) ri[fill[li[t]]++] = k;
    free(fill);
    *rp_out = rp; *ri_out = ri;
}

EXPORT int oracle_sparse_lu(int n, const int* rowptr, const int* colidx, const double* val,
                            const int* perm, const int* lp, const int* li, double eps, const double* d,
                            double* udiag, double* lval, double* uval) {
    int* ip = (int*)malloc(sizeof(int) * (size_t)n);
    for (int q = 0; q < n; ++q) ip[perm[q]] = q;
    /* permuted matrix by columns: (row, value) lists */
    int* cp = (int*)calloc((size_t)n + 1, sizeof(int));
    for (int i = 0; i < n; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) cp[ip[colidx[e]] + 1]++;
    for (int j = 0; j < n; ++j) cp[j + 1] += cp[j];
    int* fill = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    memcpy(fill, cp, sizeof(int) * (size_t)(n + 1));
    int* cr = (int*)malloc(sizeof(int) * (size_t)(rowptr[n] > 0 ? rowptr[n] : 1));
    double* cv = (double*)malloc(sizeof(double) * (size_t)(rowptr[n] > 0 ? rowptr[n] : 1));
    for (int i = 0; i < n; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int c = ip[colidx[e]];
            cr[fill[c]] = ip[i]; cv[fill[c]] = val[e]; fill[c]++;
        }
    free(fill);
    int *rp, *ri;
    l_rows(n, lp, li, &rp, &ri);
    double* w = (double*)calloc((size_t)n, sizeof(double));
    int info = 0;
    for (int j = 0; j < n && !info; ++j) {
        for (int t = cp[j]; t < cp[j + 1]; ++t) w[cr[t]] = cv[t];
        w[j] += eps * (d ? d[perm[j]] : 1.0);
        for (int t = rp[j]; t < rp[j + 1]; ++t) {       /* k ascending, U_kj != 0 */
            const int k = ri[t];
            const double wk = w[k];
            for (int s = lp[k]; s < lp[k + 1]; ++s) w[li[s]] = fma(-lval[s], wk, w[li[s]]);
        }
        const double piv = w[j];
        if (piv == 0.0 || !isfinite(piv)) { info = j + 1; break; }
        udiag[j] = piv;
        for (int t = rp[j]; t < rp[j + 1]; ++t) {
            const int k = ri[t];
            uval[find_pos(li, lp[k], lp[k + 1], j)] = w[k];
        }
        for (int s = lp[j]; s < lp[j + 1]; ++s) lval[s] = w[li[s]] / piv;
        /* clear the work vector on the column's pattern */
        for (int t = rp[j]; t < rp[j + 1]; ++t) w[ri[t]] = 0.0;
        for (int s = lp[j]; s < lp[j + 1]; ++s) w[li[s]] = 0.0;
        w[j] = 0.0;
    }
    free(w); free(rp); free(ri); free(cp); free(cr); free(cv); free(ip);
    return info;
}

/* Sparse substitutions, same operation order as the dense ones.
 * trans = 0: x = U^{-1} L^{-1} y;  trans = 1: x = L^{-T} U^{-T} y.
 * y (length n, permuted order) is overwritten. */
EXPORT void oracle_sparse_solve(int n, const int* lp, const int* li, const double* udiag,
                                const double* lval, const double* uval, int trans, double* y) {
    int *rp, *ri;
    l_rows(n, lp, li, &rp, &ri);
    if (!trans) {
        for (int k = 0; k < n; ++k)
            for (int s = lp[k]; s < lp[k + 1]; ++s) y[li[s]] = fma(-lval[s], y[k], y[li[s]]);
        for (int j = n - 1; j >= 0; --j) {
            const double xj = y[j] / udiag[j];
            y[j] = xj;
            for (int t = rp[j]; t < rp[j + 1]; ++t) {      /* U column j: rows i < j */
                const int i = ri[t];
                y[i] = fma(-uval[find_pos(li, lp[i], lp[i + 1], j)], xj, y[i]);
            }
        }
    } else {
        for (int k = 0; k < n; ++k) {
            const double zk = y[k] / udiag[k];
            y[k] = zk;
            for (int s = lp[k]; s < lp[k + 1]; ++s) y[li[s]] = fma(-uval[s], zk, y[li[s]]);
        }
        for (int k = n - 1; k >= 0; --k) {
            const double vk = y[k];
            for (int t = rp[k]; t < rp[k + 1]; ++t) {      /* L row k: columns i < k */
                const int i = ri[t];
                y[i] = fma(-lval[find_pos(li, lp[i], lp[i + 1], k)], vk, y[i]);
            }
        }
    }
    free(rp); free(ri);
}

/* One perturbed sparse system end to end for nrhs right-hand sides
 * (b, x: n x nrhs row-major, original order).  Factors go to the caller's
 * arrays when non-NULL.  Returns the LU info. */
EXPORT int oracle_sparse_system(int n, const int* rowptr, const int* colidx, const double* val,
                                const int* perm, const int* lp, const int* li, double eps,
                                const double* d, int nrhs, int trans, const double* b, double* x,
                                double* udiag_o, double* lval_o, double* uval_o) {
    const int64_t nl = lp[n] > 0 ? lp[n] : 1;
    double* ud = udiag_o ? udiag_o : (double*)malloc(sizeof(double) * (size_t)n);
    double* lv = lval_o ? lval_o : (double*)malloc(sizeof(double) * (size_t)nl);
    double* uv = uval_o ? uval_o : (double*)malloc(sizeof(double) * (size_t)nl);
    const int info = oracle_sparse_lu(n, rowptr, colidx, val, perm, lp, li, eps, d, ud, lv, uv);
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    for (int r = 0; r < nrhs; ++r) {
        for (int q = 0; q < n; ++q) t[q] = b[(size_t)perm[q] * nrhs + r];
        if (info == 0) oracle_sparse_solve(n, lp, li, ud, lv, uv, trans, t);
        else for (int q = 0; q < n; ++q) t[q] = NAN;
        for (int q = 0; q < n; ++q) x[(size_t)perm[q] * nrhs + r] = t[q];
    }
    free(t);
    if (!udiag_o) free(ud);
    if (!lval_o) free(lv);
    if (!uval_o) free(uv);
    return info;
}

/* ------------------------------------------------------------------ */
/* Adjoint of x = sum_k c_k (A + eps_k D)^{-1} b for L = sum_r w_r . x_r: */
/*   lambda_k = (A + eps_k D)^{-T} W,  dL/db = sum_k c_k lambda_k,         */
/*   dL/dA_ij = - sum_k c_k sum_r lambda_k[i,r] x_k[j,r]  on pat(A).       */
/* xk, lamk: K x n x nrhs row-major; gA in the CSR entry order of A.       */
/* ------------------------------------------------------------------ */
EXPORT void oracle_grad_values(int n, const int* rowptr, const int* colidx, int K, const double* c,
                               int nrhs, const double* xk, const double* lamk, double* gA) {
    const size_t blk = (size_t)n * nrhs;
    for (int i = 0; i < n; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int j = colidx[e];
            double acc = 0.0;
            for (int k = 0; k < K; ++k) {
                double s = 0.0;
                for (int r = 0; r < nrhs; ++r)
                    s = fma(lamk[k * blk + (size_t)i * nrhs + r], xk[k * blk + (size_t)j * nrhs + r], s);
                acc = fma(c[k], s, acc);
            }
            gA[e] = -acc;
        }
}

/* Sparse batch: each (s, k) system in parallel, then the combine per s. */
EXPORT int oracle_sparse_batch(int n, const int* rowptr, const int* colidx, int batch,
                               const double* vals, const int* perm, const int* lp, const int* li,
                               int K, const double* eps, const double* c, const double* d, int nrhs,
                               int trans, const double* b, double* x, double* xk_out, int* info) {
    const size_t nn = (size_t)n * nrhs;
    const int64_t nnz = rowptr[n];
    double* xk = xk_out ? xk_out : (double*)malloc(sizeof(double) * (size_t)batch * K * nn);
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            used = omp_get_num_threads();
#endif
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < (int64_t)batch * K; ++t) {
            const int s = (int)(t / K), k = (int)(t % K);
            info[t] = oracle_sparse_system(n, rowptr, colidx, vals + (size_t)s * nnz, perm, lp, li,
                                           eps[k], d, nrhs, trans, b + (size_t)s * nn,
                                           xk + (size_t)t * nn, NULL, NULL, NULL);
        }
    }
    for (int s = 0; s < batch; ++s) {
        for (size_t i = 0; i < nn; ++i) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc = fma(c[k], xk[((size_t)s * K + k) * nn + i], acc);
            x[(size_t)s * nn + i] = acc;
        }
    }
    if (!xk_out) free(xk);
    return used;
}
