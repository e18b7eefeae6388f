// plan.cpp -- symbolic analysis on the host: validation, minimum-degree order
// on the quotient graph, elimination tree (Liu), fill by row subtrees, and
// the three level schedules.  Definitions are the ones stated in psp.h.
#include "plan.h"

#include <algorithm>
#include <cstdint>
#include <set>
#include <utility>

namespace psp {

std::string validate_csr(int32_t n, const int32_t* rp, const int32_t* ci) {
    if (n < 1) return "n must be >= 1";
    if (!rp || !ci) return "row_ptr / col_idx must not be NULL";
    if (rp[0] != 0) return "row_ptr[0] must be 0";
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return "row_ptr must be non-decreasing";
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return "column index out of range";
            if (e > rp[i] && ci[e] <= ci[e - 1]) return "column indices must be strictly ascending in each row";
        }
    }
    return {};
}

namespace {

// Symmetric adjacency of pat(A) | pat(A^T) without the diagonal, CSR, sorted.
void symmetric_adjacency(int32_t n, const int32_t* rp, const int32_t* ci,
                         std::vector<int32_t>& ap, std::vector<int32_t>& ai) {
    std::vector<int32_t> cnt(n + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] != i) { cnt[i + 1]++; cnt[ci[e] + 1]++; }
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> tmp(cnt[n]);
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] != i) { tmp[pos[i]++] = ci[e]; tmp[pos[ci[e]]++] = i; }
    ap.assign(n + 1, 0);
    ai.clear();
    ai.reserve(tmp.size());
    for (int32_t i = 0; i < n; ++i) {
        auto b = tmp.begin() + cnt[i], en = tmp.begin() + cnt[i + 1];
        std::sort(b, en);
        en = std::unique(b, en);
        ai.insert(ai.end(), b, en);
        ap[i + 1] = (int32_t)ai.size();
    }
}

// Minimum degree with exact external degrees on the quotient graph.
// Variables keep a list of adjacent variables (A_i) and adjacent elements
// (E_i); element p (created when p is eliminated) keeps its variable list
// L_p.  The neighbourhood of i in the elimination graph is
// A_i | union_{e in E_i} L_e minus {i}, so its size is the exact degree.
void minimum_degree(int32_t n, const std::vector<int32_t>& ap, const std::vector<int32_t>& ai,
                    std::vector<int32_t>& perm, int32_t& ndense) {
    std::vector<char> dense(n, 0), gone(n, 0), elem_alive(n, 0);
    ndense = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t d = ap[i + 1] - ap[i];
        if (d > 16 && d * d > 100 * (int64_t)n) { dense[i] = 1; ++ndense; }
    }
    std::vector<std::vector<int32_t>> A(n), E(n), Le(n);
    std::vector<int32_t> deg(n, 0);
    std::set<std::pair<int32_t, int32_t>> queue;
    for (int32_t i = 0; i < n; ++i) {
        if (dense[i]) continue;
        for (int32_t t = ap[i]; t < ap[i + 1]; ++t)
            if (!dense[ai[t]]) A[i].push_back(ai[t]);
        deg[i] = (int32_t)A[i].size();
        queue.insert({deg[i], i});
    }
    std::vector<int32_t> in_lp(n, -1), seen(n, -1);
    int32_t stamp = 0;
    perm.clear();
    perm.reserve(n);
    while (!queue.empty()) {
        const int32_t p = queue.begin()->second;
        queue.erase(queue.begin());
        perm.push_back(p);
        gone[p] = 1;
        // new element: every live variable reachable from p
        std::vector<int32_t> lp;
        for (int32_t j : A[p])
            if (!gone[j] && in_lp[j] != p) { in_lp[j] = p; lp.push_back(j); }
        for (int32_t e : E[p]) {
            if (!elem_alive[e]) continue;
            for (int32_t j : Le[e])
                if (!gone[j] && in_lp[j] != p) { in_lp[j] = p; lp.push_back(j); }
            elem_alive[e] = 0;                     // absorbed into element p
            std::vector<int32_t>().swap(Le[e]);
        }
        std::vector<int32_t>().swap(A[p]);
        std::vector<int32_t>().swap(E[p]);
        Le[p] = lp;
        elem_alive[p] = 1;
        for (int32_t i : lp) {
            auto& Ai = A[i];
            Ai.erase(std::remove_if(Ai.begin(), Ai.end(), [&](int32_t j) { return j == p || in_lp[j] == p; }),
                     Ai.end());
            auto& Ei = E[i];
            Ei.erase(std::remove_if(Ei.begin(), Ei.end(), [&](int32_t e) { return !elem_alive[e]; }), Ei.end());
            Ei.push_back(p);
            ++stamp;
            seen[i] = stamp;
            int32_t d = 0;
            for (int32_t j : Ai)
                if (seen[j] != stamp) { seen[j] = stamp; ++d; }
            for (int32_t e : Ei)
                for (int32_t j : Le[e])
                    if (seen[j] != stamp) { seen[j] = stamp; ++d; }
            if (d != deg[i]) {
                queue.erase({deg[i], i});
                deg[i] = d;
                queue.insert({d, i});
            }
        }
    }
    for (int32_t i = 0; i < n; ++i)
        if (dense[i]) perm.push_back(i);
}

void levels_from(const std::vector<int32_t>& lev, int32_t n, std::vector<int32_t>& lp, std::vector<int32_t>& li) {
    int32_t L = 0;
    for (int32_t i = 0; i < n; ++i) L = std::max(L, lev[i] + 1);
    lp.assign(L + 1, 0);
    for (int32_t i = 0; i < n; ++i) lp[lev[i] + 1]++;
    for (int32_t l = 0; l < L; ++l) lp[l + 1] += lp[l];
    std::vector<int32_t> pos(lp.begin(), lp.end() - 1);
    li.assign(n, 0);
    for (int32_t i = 0; i < n; ++i) li[pos[lev[i]]++] = i;
}

}  // namespace

void analyse(int32_t n, const int32_t* rp, const int32_t* ci, bool natural, Symbolic& s) {
    s.n = n;
    s.nnz = rp[n];
    s.row_ptr.assign(rp, rp + n + 1);
    s.col_idx.assign(ci, ci + rp[n]);
    std::vector<int32_t> ap, ai;
    symmetric_adjacency(n, rp, ci, ap, ai);
    if (natural) {
        s.perm.resize(n);
        for (int32_t i = 0; i < n; ++i) s.perm[i] = i;
        s.ndense = 0;
    } else {
        minimum_degree(n, ap, ai, s.perm, s.ndense);
    }
    s.iperm.assign(n, 0);
    for (int32_t q = 0; q < n; ++q) s.iperm[s.perm[q]] = q;

    // permuted adjacency, lower part only (k < i), per row i
    std::vector<int32_t> pp(n + 1, 0), pi;
    for (int32_t q = 0; q < n; ++q) {
        const int32_t i = s.perm[q];
        for (int32_t t = ap[i]; t < ap[i + 1]; ++t)
            if (s.iperm[ai[t]] < q) pp[q + 1]++;
    }
    for (int32_t q = 0; q < n; ++q) pp[q + 1] += pp[q];
    pi.assign(pp[n], 0);
    for (int32_t q = 0; q < n; ++q) {
        int32_t w = pp[q];
        const int32_t i = s.perm[q];
        for (int32_t t = ap[i]; t < ap[i + 1]; ++t)
            if (s.iperm[ai[t]] < q) pi[w++] = s.iperm[ai[t]];
    }

    // elimination tree, Liu's algorithm with path-compressed ancestors
    s.parent.assign(n, -1);
    std::vector<int32_t> anc(n, -1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t t = pp[i]; t < pp[i + 1]; ++t) {
            int32_t r = pi[t];
            while (anc[r] != -1 && anc[r] != i) {
                const int32_t nx = anc[r];
                anc[r] = i;
                r = nx;
            }
            if (anc[r] == -1) { anc[r] = i; s.parent[r] = i; }
        }

    // row subtrees: L(i, j) != 0 for every j on the etree path from k (S_ik != 0, k < i) up to i
    std::vector<int32_t> mark(n, -1), colcnt(n + 1, 0), rowcnt(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        mark[i] = i;
        for (int32_t t = pp[i]; t < pp[i + 1]; ++t)
            for (int32_t j = pi[t]; mark[j] != i; j = s.parent[j]) { mark[j] = i; colcnt[j + 1]++; rowcnt[i + 1]++; }
    }
    for (int32_t j = 0; j < n; ++j) { colcnt[j + 1] += colcnt[j]; rowcnt[j + 1] += rowcnt[j]; }
    s.l_ptr = colcnt;
    s.lrow_ptr = rowcnt;
    s.l_idx.assign(colcnt[n], 0);
    s.lrow_idx.assign(rowcnt[n], 0);
    std::vector<int32_t> cpos(colcnt.begin(), colcnt.end() - 1);
    std::fill(mark.begin(), mark.end(), -1);
    for (int32_t i = 0; i < n; ++i) {
        mark[i] = i;
        int32_t w = s.lrow_ptr[i];
        for (int32_t t = pp[i]; t < pp[i + 1]; ++t)
            for (int32_t j = pi[t]; mark[j] != i; j = s.parent[j]) {
                mark[j] = i;
                s.l_idx[cpos[j]++] = i;      // rows appended in ascending i
                s.lrow_idx[w++] = j;
            }
        std::sort(s.lrow_idx.begin() + s.lrow_ptr[i], s.lrow_idx.begin() + s.lrow_ptr[i + 1]);
    }

    // levels
    std::vector<int32_t> lev(n, 0);
    for (int32_t j = 0; j < n; ++j)
        if (s.parent[j] >= 0) lev[s.parent[j]] = std::max(lev[s.parent[j]], lev[j] + 1);
    levels_from(lev, n, s.lev_ptr[0], s.lev_idx[0]);
    std::fill(lev.begin(), lev.end(), 0);
    for (int32_t j = 0; j < n; ++j)
        for (int32_t t = s.l_ptr[j]; t < s.l_ptr[j + 1]; ++t) lev[s.l_idx[t]] = std::max(lev[s.l_idx[t]], lev[j] + 1);
    levels_from(lev, n, s.lev_ptr[1], s.lev_idx[1]);
    for (int32_t i = n - 1; i >= 0; --i) {
        int32_t m = 0;
        for (int32_t t = s.l_ptr[i]; t < s.l_ptr[i + 1]; ++t) m = std::max(m, lev[s.l_idx[t]] + 1);
        lev[i] = m;
    }
    levels_from(lev, n, s.lev_ptr[2], s.lev_idx[2]);

    // dense trailing block (see plan.h)
    int32_t t = 0;
    while (t < n && s.l_ptr[n - t] - s.l_ptr[n - t - 1] == t) ++t;
    s.tail_n = 0;
    if (t >= kTailMin && n - t <= kTailAsmMaxB0) {
        std::vector<int32_t> flev(n);
        for (size_t l = 0; l + 1 < s.lev_ptr[0].size(); ++l)
            for (int32_t q = s.lev_ptr[0][l]; q < s.lev_ptr[0][l + 1]; ++q) flev[s.lev_idx[0][q]] = (int32_t)l;
        const int32_t b0 = n - t;
        int32_t max_sp = -1, min_tail = INT32_MAX;
        for (int32_t j = 0; j < b0; ++j) max_sp = std::max(max_sp, flev[j]);
        for (int32_t j = b0; j < n; ++j) min_tail = std::min(min_tail, flev[j]);
        if (max_sp < min_tail) {
            s.tail_n = t;
            s.tail_b0 = b0;
            s.fac_lev_sp = max_sp + 1;
            // solve levels of the rows < b0 among themselves (the block's rows are solved densely
            // in between: after every L-solve dependency of theirs, before every U-solve one)
            std::vector<int32_t> lv(b0, 0);
            for (int32_t j = 0; j < b0; ++j)
                for (int32_t q = s.l_ptr[j]; q < s.l_ptr[j + 1]; ++q)
                    if (s.l_idx[q] < b0) lv[s.l_idx[q]] = std::max(lv[s.l_idx[q]], lv[j] + 1);
            levels_from(lv, b0, s.lev_sp_ptr[0], s.lev_sp_idx[0]);
            for (int32_t i = b0 - 1; i >= 0; --i) {
                int32_t m = 0;
                for (int32_t q = s.l_ptr[i]; q < s.l_ptr[i + 1]; ++q)
                    if (s.l_idx[q] < b0) m = std::max(m, lv[s.l_idx[q]] + 1);
                lv[i] = m;
            }
            levels_from(lv, b0, s.lev_sp_ptr[1], s.lev_sp_idx[1]);
            // tiles of 16 block rows for the assembly on the MFMA unit (see plan.h): rows placed
            // greedily so that a tile's rows share their columns below b0
            const int32_t tiles = (t + 15) / 16;
            std::vector<int32_t> rp(t + 1, 0), inv_ptr(b0 + 1, 0), inv;
            for (int32_t r = 0; r < t; ++r) {
                int32_t q = s.lrow_ptr[b0 + r];
                while (q < s.lrow_ptr[b0 + r + 1] && s.lrow_idx[q] < b0) ++inv_ptr[s.lrow_idx[q++] + 1];
                rp[r + 1] = q - s.lrow_ptr[b0 + r];
            }
            for (int32_t r = 0; r < t; ++r) rp[r + 1] += rp[r];
            for (int32_t k = 0; k < b0; ++k) inv_ptr[k + 1] += inv_ptr[k];
            inv.resize(inv_ptr[b0]);
            {
                std::vector<int32_t> fill(inv_ptr.begin(), inv_ptr.end() - 1);
                for (int32_t r = 0; r < t; ++r)
                    for (int32_t q = 0; q < rp[r + 1] - rp[r]; ++q) inv[fill[s.lrow_idx[s.lrow_ptr[b0 + r] + q]]++] = r;
            }
            auto row_k = [&](int32_t r, int32_t q) { return s.lrow_idx[s.lrow_ptr[b0 + r] + q]; };
            s.tail_rord.assign((size_t)16 * tiles, -1);
            std::vector<char> placed(t, 0), in_u(b0, 0);
            std::vector<int32_t> newc(t), touched;
            int32_t slot = 0;
            for (int32_t tt = 0; tt < tiles; ++tt) {
                for (int32_t r = 0; r < t; ++r) newc[r] = rp[r + 1] - rp[r];
                touched.clear();
                for (int32_t m = 0; m < 16 && slot < t; ++m, ++slot) {
                    // seed: smallest first column; then fewest new columns; longer rows, then lower index, first
                    int32_t best = -1;
                    int64_t bkey = INT64_MAX;
                    for (int32_t r = 0; r < t; ++r) {
                        if (placed[r]) continue;
                        const int64_t len = rp[r + 1] - rp[r];
                        const int64_t lead = m == 0 ? (len ? row_k(r, 0) : b0) : newc[r];
                        const int64_t key = lead * ((int64_t)1 << 32) - len;
                        if (key < bkey) { bkey = key; best = r; }
                    }
                    placed[best] = 1;
                    s.tail_rord[slot] = best;
                    for (int32_t q = 0; q < rp[best + 1] - rp[best]; ++q) {
                        const int32_t k = row_k(best, q);
                        if (in_u[k]) continue;
                        in_u[k] = 1;
                        touched.push_back(k);
                        for (int32_t z = inv_ptr[k]; z < inv_ptr[k + 1]; ++z) --newc[inv[z]];
                    }
                }
                for (int32_t k : touched) in_u[k] = 0;
            }
            s.tail_kt_ptr.assign(1, 0);
            s.tail_kt.clear();
            bool ok = true;
            std::vector<int32_t> uni;
            for (int32_t tt = 0; tt < tiles && ok; ++tt) {
                uni.clear();
                for (int32_t m = 16 * tt; m < 16 * tt + 16; ++m) {
                    const int32_t r = s.tail_rord[m];
                    if (r < 0) continue;
                    for (int32_t q = 0; q < rp[r + 1] - rp[r]; ++q) uni.push_back(row_k(r, q));
                }
                std::sort(uni.begin(), uni.end());
                uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
                if (uni.size() >= 65535) ok = false;
                s.tail_kt.insert(s.tail_kt.end(), uni.begin(), uni.end());
                s.tail_kt_ptr.push_back((int32_t)s.tail_kt.size());
            }
            // the common columns of every tile pair, ascending, padded to a multiple of four with
            // the two zero columns
            s.tail_pp_ptr.assign(ok ? (size_t)tiles * tiles + 1 : 1, 0);
            s.tail_pairs.clear();
            for (int32_t a = 0; a < tiles && ok; ++a)
                for (int32_t b = 0; b < tiles && ok; ++b) {
                    s.tail_pp_ptr[(size_t)a * tiles + b] = (int32_t)s.tail_pairs.size();
                    const int32_t *A = s.tail_kt.data() + s.tail_kt_ptr[a], *B = s.tail_kt.data() + s.tail_kt_ptr[b];
                    const uint32_t na = s.tail_kt_ptr[a + 1] - s.tail_kt_ptr[a], nb = s.tail_kt_ptr[b + 1] - s.tail_kt_ptr[b];
                    uint32_t x = 0, y = 0;
                    while (x < na && y < nb) {
                        if (A[x] == B[y]) s.tail_pairs.push_back((int32_t)(x++ | (y++ << 16)));
                        else if (A[x] < B[y]) ++x;
                        else ++y;
                    }
                    while (s.tail_pairs.size() % 4) s.tail_pairs.push_back((int32_t)(na | (nb << 16)));
                    if (s.tail_pairs.size() > kTailMaxPairs) ok = false;
                }
            if (ok) s.tail_pp_ptr[(size_t)tiles * tiles] = (int32_t)s.tail_pairs.size();
            else {
                s.tail_kt_ptr.clear();
                s.tail_kt.clear();
                s.tail_rord.clear();
                s.tail_pp_ptr.clear();
                s.tail_pairs.clear();
            }
            s.tail_tiles = ok ? tiles : 0;
        }
    }

    const int64_t N = n;
    s.flops_dense = N * (N - 1) / 2 + (N - 1) * N * (2 * N - 1) / 3;
    s.flops_sparse = 0;
    for (int32_t j = 0; j < n; ++j) {
        const int64_t c = s.l_ptr[j + 1] - s.l_ptr[j];
        s.flops_sparse += c + 2 * c * c;
    }
}

}  // namespace psp
