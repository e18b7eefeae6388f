// sparse.hip -- pivot-free LU and substitutions on the plan's fill pattern,
// level-scheduled, for gfx950.
//
// Factorisation in dot-product (Crout) form.  With R_i the columns k < i of
// row i of L (ascending) and S symmetric, every factor entry is one sparse dot
// product over the intersection of two rows of L:
//   u_jj = a_jj - sum_{k in R_j}        l_jk u_kj
//   u_jm = a_jm - sum_{k in R_j ^ R_m}  l_jk u_km     (m in struct L(:,j))
//   l_ij = (a_ij - sum_{k in R_i ^ R_j} l_ik u_kj) / u_jj
// each summed as an fma chain in ascending k -- the same operations, in the
// same order, that left-looking elimination applies to that entry -- so the
// factors equal the reference factors bit for bit.  Column j and row j depend
// only on the columns in R_j, which are etree descendants of j, so the etree
// height gives the schedule: per level, the diagonals first, then every other
// entry of the level's columns and rows in parallel.
//
// Substitutions are row-oriented and level-scheduled, one lane per
// right-hand side (RHS vectors are row-major, so a row's RHS values are
// contiguous):
//   L y = b     y_i -= l_ik y_k    k in R_i ascending
//   U x = y     x_i = (y_i - sum u_im x_m) / u_ii, m in struct L(:,i) descending
//   U^T z = w   z_i = (w_i - sum u_ki z_k) / u_ii, k in R_i ascending
//   L^T v = z   v_i -= l_mi v_m   m in struct L(:,i) descending
// which again reproduces the reference order per entry.
//
// Two executions of the same device code:
//   * in-LDS: one workgroup per perturbed system keeps that system's factors
//     and RHS in LDS and runs every level with workgroup barriers (used when
//     (n + 2 nnz(L) + n nrhs) doubles fit);
//   * global: factors in the workspace, one launch per level and phase, all
//     systems of the batch in each launch.
#include <algorithm>
#include <climits>
#include <vector>

#include "dense.h"
#include "sparse.h"
#include "dense_ops.h"

namespace psp {

bool sparse_fits_lds(const Symbolic& s, int32_t nrhs);

namespace {
constexpr int kLdsLimit = 152 * 1024;    // bytes of LDS the in-LDS kernel may use
constexpr int kLdsThreads = 512;
constexpr int kThreads = 256;
// Update lists (precomputed pairs of every factor entry's dot product) are kept
// for at most this many pairs (256 MB of the plan image); beyond, the dot
// products merge the two rows on the fly.
constexpr int64_t kMaxPairs = 32LL << 20;

// acc - sum_{k in R_a ^ R_b, k < bound} lv[pos(a,k)] * uv[pos(b,k)], ascending k.  Rows of
// similar length are merged; when one row is much longer (the dense slack row has an entry in
// every column) the shorter one is walked and each of its k is found in the longer one by
// galloping search, so the cost follows the shorter row.  Either way the matches are taken in
// ascending k.
__device__ __forceinline__ double merge_dot_below(const SpIdx& ix, int a, int b, int bound, const double* lv,
                                                  const double* uv, double acc) {
    int p = ix.r_ptr[a], pe = ix.r_ptr[a + 1];
    int q = ix.r_ptr[b], qe = ix.r_ptr[b + 1];
    const int la = pe - p, lb = qe - q;
    if (la > 8 * lb || lb > 8 * la) {
        const bool a_short = la <= lb;
        int s = a_short ? p : q;
        const int se = a_short ? pe : qe;
        int l = a_short ? q : p;
        const int le = a_short ? qe : pe;
        for (; s < se && l < le; ++s) {
            const int k = ix.r_idx[s];
            if (k >= bound) break;
            // first index in [l, le) with r_idx >= k
            int lo = l, hi = l, step = 1;
            while (hi < le && ix.r_idx[hi] < k) {
                lo = hi + 1;
                hi += step;
                step <<= 1;
            }
            if (hi > le) hi = le;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ix.r_idx[mid] < k) lo = mid + 1;
                else hi = mid;
            }
            l = lo;
            if (l < le && ix.r_idx[l] == k) {
                const int pa = a_short ? s : l, pb = a_short ? l : s;
                acc = fmad(-lv[ix.r_pos[pa]], uv[ix.r_pos[pb]], acc);
                ++l;
            }
        }
        return acc;
    }
    while (p < pe && q < qe) {
        const int ka = ix.r_idx[p], kb = ix.r_idx[q];
        if (ka >= bound || kb >= bound) break;
        if (ka == kb) {
            acc = fmad(-lv[ix.r_pos[p]], uv[ix.r_pos[q]], acc);
            ++p;
            ++q;
        } else if (ka < kb) {
            ++p;
        } else {
            ++q;
        }
    }
    return acc;
}

__device__ __forceinline__ double merge_dot(const SpIdx& ix, int a, int b, const double* lv, const double* uv,
                                            double acc) {
    return merge_dot_below(ix, a, b, INT_MAX, lv, uv, acc);
}

// acc - sum lv[pl] * uv[pu] over the precomputed pairs of item id, in order
// The loads of a block of U iterations are issued before its fma chain so
// that U index/value fetches are in flight at once; the chain itself keeps
// the ascending order.
constexpr int U8 = 8;
constexpr int U16 = 16;   // the block rows' updates from the sparse part: more loads in flight per step
constexpr int U32 = 32;

__device__ __forceinline__ double pair_dot(const SpIdx& ix, int id, const double* lv, const double* uv, double acc) {
    const int p1 = ix.pair_ptr[id + 1];
    int p = ix.pair_ptr[id];
    if (p + U8 <= p1) {
        // the next block's pairs are fetched while this block's values are in flight
        int2 pq[U8];
#pragma unroll
        for (int u = 0; u < U8; ++u) pq[u] = ix.pairs[p + u];
        for (; p + U8 <= p1; p += U8) {
            double a[U8], b[U8];
#pragma unroll
            for (int u = 0; u < U8; ++u) { a[u] = lv[pq[u].x]; b[u] = uv[pq[u].y]; }
            if (p + 2 * U8 <= p1) {
#pragma unroll
                for (int u = 0; u < U8; ++u) pq[u] = ix.pairs[p + U8 + u];
            }
#pragma unroll
            for (int u = 0; u < U8; ++u) acc = fmad(-a[u], b[u], acc);
        }
    }
    for (; p < p1; ++p) {
        const int2 pq = ix.pairs[p];
        acc = fmad(-lv[pq.x], uv[pq.y], acc);
    }
    return acc;
}

__device__ __forceinline__ double diag_dot(const SpIdx& ix, int j, const double* lv, const double* uv, double acc) {
    if (ix.use_pairs && j < ix.pairs_below) return pair_dot(ix, j, lv, uv, acc);
    for (int p = ix.r_ptr[j]; p < ix.r_ptr[j + 1]; ++p) {
        const int t = ix.r_pos[p];
        acc = fmad(-lv[t], uv[t], acc);
    }
    return acc;
}

// Values of P (A + eps D) P^T on the fill pattern.
__device__ __forceinline__ void gather_item(const SpIdx& ix, int t, const double* v, double* lv, double* uv) {
    const int sl = ix.src_l[t], su = ix.src_u[t];
    lv[t] = sl >= 0 ? v[sl] : 0.0;
    uv[t] = su >= 0 ? v[su] : 0.0;
}

__device__ __forceinline__ double gather_diag(const SpIdx& ix, int j, const double* v, double eps, const double* dvec) {
    const int sd = ix.src_d[j];
    const double a = sd >= 0 ? v[sd] : 0.0;
    const double dq = dvec ? dvec[ix.perm[j]] : 1.0;
    return __dadd_rn(a, __dmul_rn(eps, dq));
}

// phase B item: it < npos -> U entry at position t, else L entry at position t
__device__ __forceinline__ void factor_item(const SpIdx& ix, int t, bool is_l, double* ud, double* lv, double* uv) {
    const int j = ix.col_of[t], m = ix.l_idx[t];
    if (ix.use_pairs && j < ix.pairs_below) {
        if (!is_l) uv[t] = pair_dot(ix, ix.n + t, lv, uv, uv[t]);
        else lv[t] = pair_dot(ix, ix.n + ix.nnzl + t, lv, uv, lv[t]) / ud[j];
        return;
    }
    if (!is_l) {
        uv[t] = merge_dot(ix, j, m, lv, uv, uv[t]);
    } else {
        lv[t] = merge_dot(ix, m, j, lv, uv, lv[t]) / ud[j];
    }
}

template <int TRANS>
__device__ __forceinline__ double fwd_row(const SpIdx& ix, int i, int r, int nrhs, const double* ud, const double* lv,
                                          const double* uv, const double* y) {
    double acc = y[(int64_t)i * nrhs + r];
    const double* m = TRANS ? uv : lv;
    const int p1 = ix.r_ptr[i + 1];
    int p = ix.r_ptr[i];
    for (; p + U8 <= p1; p += U8) {
        double a[U8], b[U8];
#pragma unroll
        for (int u = 0; u < U8; ++u) { a[u] = m[ix.r_pos[p + u]]; b[u] = y[(int64_t)ix.r_idx[p + u] * nrhs + r]; }
#pragma unroll
        for (int u = 0; u < U8; ++u) acc = fmad(-a[u], b[u], acc);
    }
    for (; p < p1; ++p) acc = fmad(-m[ix.r_pos[p]], y[(int64_t)ix.r_idx[p] * nrhs + r], acc);
    return TRANS ? acc / ud[i] : acc;
}

// t_end: positions of column i from t_end on were applied beforehand (the dense trailing block's
// rows, tail_bwd_ext_kernel); -1: none.
template <int TRANS>
__device__ __forceinline__ double bwd_row(const SpIdx& ix, int i, int r, int nrhs, const double* ud, const double* lv,
                                          const double* uv, const double* y, int t_end = -1) {
    double acc = y[(int64_t)i * nrhs + r];
    const double* m = TRANS ? lv : uv;
    const int t0 = ix.l_ptr[i];
    int t = (t_end < 0 ? ix.l_ptr[i + 1] : t_end) - 1;
    for (; t - U8 + 1 >= t0; t -= U8) {
        double a[U8], b[U8];
#pragma unroll
        for (int u = 0; u < U8; ++u) { a[u] = m[t - u]; b[u] = y[(int64_t)ix.l_idx[t - u] * nrhs + r]; }
#pragma unroll
        for (int u = 0; u < U8; ++u) acc = fmad(-a[u], b[u], acc);
    }
    for (; t >= t0; --t) acc = fmad(-m[t], y[(int64_t)ix.l_idx[t] * nrhs + r], acc);
    return TRANS ? acc : acc / ud[i];
}

struct SpArgs {
    SpIdx ix;
    int32_t nnz, nrhs, ntasks, K, trans;
    const double* values;   // batch x nnz
    const double* dvec;
    const double* B;        // batch x n x nrhs
    double* Xk;             // batch x K x n x nrhs
    int32_t* info;          // batch x K
    double* fac;            // global factors: ntasks x fstride (ud | lv | uv)
    int64_t fstride;
    double* y;              // global RHS scratch: ntasks x n x nrhs
    double* X;              // batch x n x nrhs, combined in-kernel when per_jacobian
    int32_t per_jacobian, batch;
    // Dense trailing block kernels (tail_*): value t of system s of the [u_jj | L | U] arrays at
    // fac[s * ts + t * vs], its block, right-hand-side scratch and panels at dense + s * dstride,
    // entry (i, r) of its substitution vector at y[s * yt + (i * nrhs + r) * yv].  Task-major
    // factors (vs = 1, ts = fstride, block inside each system's factors) or systems interleaved
    // (vs = TP, ts = 1, blocks in a region of their own).
    int64_t vs, ts, dstride, yv, yt;
    double* dense;
    const double* scale;    // or NULL: Jacobian s at the nodes scale[s] eps_k (a power of two)
};

// ---------------------------------------------------------------- in-LDS kernel
__global__ __launch_bounds__(kLdsThreads) void sparse_lds_kernel(SpArgs a, EpsSet es, int store_factors) {
    extern __shared__ double lds[];
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, nrhs = a.nrhs, tid = threadIdx.x;
    double* ud = lds;
    double* lv = ud + n;
    double* uv = lv + nl;
    double* y = uv + nl;
    __shared__ int s_bad;
    const int ntask = a.per_jacobian ? a.batch : a.ntasks;
    for (int tk = blockIdx.x; tk < ntask; tk += gridDim.x) {
      const int s = a.per_jacobian ? tk : tk / es.K;
      const int k0 = a.per_jacobian ? 0 : tk % es.K, k1 = a.per_jacobian ? es.K : k0 + 1;
      for (int kk = k0; kk < k1; ++kk) {
        const int task = s * es.K + kk;
        const double* v = a.values + (int64_t)s * a.nnz;
        if (tid == 0) s_bad = INT_MAX;
        for (int t = tid; t < nl; t += kLdsThreads) gather_item(ix, t, v, lv, uv);
        for (int j = tid; j < n; j += kLdsThreads) ud[j] = gather_diag(ix, j, v, eps_at(es, kk), a.dvec);
        if (nrhs > 0) {
            const double* b = a.B + (int64_t)s * n * nrhs;
            for (int t = tid; t < n * nrhs; t += kLdsThreads) {
                const int q = t / nrhs, r = t % nrhs;
                y[t] = b[(int64_t)ix.perm[q] * nrhs + r];
            }
        }
        __syncthreads();
        for (int l = 0; l < ix.nlev[0]; ++l) {
            const int c0 = ix.lev_ptr[0][l], c1 = ix.lev_ptr[0][l + 1];
            for (int t = c0 + tid; t < c1; t += kLdsThreads) {
                const int j = ix.lev_idx[0][t];
                const double u = diag_dot(ix, j, lv, uv, ud[j]);
                ud[j] = u;
                if (bad_pivot(u)) atomicMin(&s_bad, j + 1);
            }
            __syncthreads();
            const int p0 = ix.lpos_ptr[l], np = ix.lpos_ptr[l + 1] - p0;
            for (int it = tid; it < 2 * np; it += kLdsThreads) {
                const bool is_l = it >= np;
                factor_item(ix, ix.lpos[p0 + (is_l ? it - np : it)], is_l, ud, lv, uv);
            }
            __syncthreads();
        }
        const int bad = s_bad == INT_MAX ? 0 : s_bad;
        if (store_factors) {
            double* f = a.fac + (int64_t)task * a.fstride;
            for (int t = tid; t < n + 2 * nl; t += kLdsThreads) f[t] = lds[t];
        }
        if (nrhs > 0) {
            if (!bad) {
                for (int l = 0; l < ix.nlev[1]; ++l) {
                    const int c0 = ix.lev_ptr[1][l], c1 = ix.lev_ptr[1][l + 1];
                    for (int t = c0 * nrhs + tid; t < c1 * nrhs; t += kLdsThreads) {
                        const int i = ix.lev_idx[1][t / nrhs], r = t % nrhs;
                        y[(int64_t)i * nrhs + r] = fwd_row<0>(ix, i, r, nrhs, ud, lv, uv, y);
                    }
                    __syncthreads();
                }
                for (int l = 0; l < ix.nlev[2]; ++l) {
                    const int c0 = ix.lev_ptr[2][l], c1 = ix.lev_ptr[2][l + 1];
                    for (int t = c0 * nrhs + tid; t < c1 * nrhs; t += kLdsThreads) {
                        const int i = ix.lev_idx[2][t / nrhs], r = t % nrhs;
                        y[(int64_t)i * nrhs + r] = bwd_row<0>(ix, i, r, nrhs, ud, lv, uv, y);
                    }
                    __syncthreads();
                }
            }
            double* x = a.per_jacobian ? a.X + (int64_t)s * n * nrhs : a.Xk + (int64_t)task * n * nrhs;
            for (int t = tid; t < n * nrhs; t += kLdsThreads) {
                const int q = t / nrhs, r = t % nrhs;
                const double val = bad ? __builtin_nan("") : y[t];
                double* dst = x + (int64_t)ix.perm[q] * nrhs + r;
                *dst = a.per_jacobian ? fmad(c_at(es, kk), val, kk == 0 ? 0.0 : *dst) : val;
            }
        }
        if (tid == 0) a.info[task] = bad;
        __syncthreads();
      }
    }
}

// ---------------------------------------------------------------- global, per-level kernels
__global__ void sp_gather_kernel(SpArgs a, EpsSet es) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl;
    const int64_t per = n + nl;
    const int64_t total = per * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / per), t = (int)(g % per);
        const int s = task / es.K, kk = task % es.K;
        const double* v = a.values + (int64_t)s * a.nnz;
        double* ud = a.fac + (int64_t)task * a.fstride;
        if (t < nl) gather_item(ix, t, v, ud + n, ud + n + nl);
        else ud[t - nl] = gather_diag(ix, t - nl, v, eps_at(es, kk), a.dvec);
        if (t == 0) a.info[task] = INT_MAX;
    }
}

__global__ void sp_diag_kernel(SpArgs a, int c0, int cnt) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl;
    const int64_t total = (int64_t)cnt * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / cnt), j = ix.lev_idx[0][c0 + (int)(g % cnt)];
        double* ud = a.fac + (int64_t)task * a.fstride;
        const double u = diag_dot(ix, j, ud + n, ud + n + nl, ud[j]);
        ud[j] = u;
        if (bad_pivot(u)) atomicMin(&a.info[task], j + 1);
    }
}

__global__ void sp_offdiag_kernel(SpArgs a, int p0, int np) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl;
    const int64_t total = (int64_t)2 * np * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / (2 * np)), it = (int)(g % (2 * np));
        const bool is_l = it >= np;
        double* ud = a.fac + (int64_t)task * a.fstride;
        factor_item(ix, ix.lpos[p0 + (is_l ? it - np : it)], is_l, ud, ud + n, ud + n + nl);
    }
}

__global__ void sp_info_kernel(int32_t* info, int ntasks) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntasks && info[t] == INT_MAX) info[t] = 0;
}

__global__ void sp_rhs_in_kernel(SpArgs a) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nrhs = a.nrhs;
    const int64_t per = (int64_t)n * nrhs, total = per * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / per), t = (int)(g % per);
        const int s = task / a.K, q = t / nrhs, r = t % nrhs;
        a.y[g] = a.B[(int64_t)s * per + (int64_t)ix.perm[q] * nrhs + r];
    }
}

// sparse_only (U pass below a dense trailing block): the block rows' terms were applied beforehand.
template <int UPPER_PASS>
__global__ void sp_solve_level_kernel(SpArgs a, const int32_t* lev_idx, int c0, int cnt, int sparse_only) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, nrhs = a.nrhs;
    const int64_t per = (int64_t)cnt * nrhs, total = per * a.ntasks;
    // pass 0: L (or U^T when transposed), ascending schedule; pass 1: U (or L^T), descending schedule
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / per), t = (int)(g % per);
        if (a.info[task]) continue;
        const int i = lev_idx[c0 + t / nrhs], r = t % nrhs;
        const double* ud = a.fac + (int64_t)task * a.fstride;
        double* y = a.y + (int64_t)task * n * nrhs;
        double v;
        if (!UPPER_PASS) v = a.trans ? fwd_row<1>(ix, i, r, nrhs, ud, ud + n, ud + n + nl, y)
                                     : fwd_row<0>(ix, i, r, nrhs, ud, ud + n, ud + n + nl, y);
        else {
            const int te = sparse_only ? ix.l_ptr[i] + ix.tail_ccnt[i] : -1;
            v = a.trans ? bwd_row<1>(ix, i, r, nrhs, ud, ud + n, ud + n + nl, y, te)
                        : bwd_row<0>(ix, i, r, nrhs, ud, ud + n, ud + n + nl, y, te);
        }
        y[(int64_t)i * nrhs + r] = v;
    }
}

__global__ void sp_rhs_out_kernel(SpArgs a) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nrhs = a.nrhs;
    const int64_t per = (int64_t)n * nrhs, total = per * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / per), t = (int)(g % per);
        const int q = t / nrhs, r = t % nrhs;
        a.Xk[(int64_t)task * per + (int64_t)ix.perm[q] * nrhs + r] = a.info[task] ? __builtin_nan("") : a.y[g];
    }
}

// ---------------------------------------------------------------- dense trailing block
// The last tail_n columns of the factors are full, and their factor levels lie above every other
// column's (plan.h), so the sparse part (columns < b0) is factored first on its own levels.  Each
// entry (i, j) of the trailing block then starts from a_ij (+ eps d on the diagonal), takes the
// updates of the sparse part, l_ik u_kj for k < b0 in ascending k (one thread per entry, the two
// rows merged), and the block is factored densely in panels of NB columns on the MFMA unit, which
// continues every entry's chain over k >= b0 in ascending order: the reference sequence.

// Each entry (i, j) of the block takes l_ik u_kj for k < b0 in ascending k.  One workgroup per
// (system, tile of kAsmCols block columns): the U values of the tile's columns below b0 (row j of the
// factor pattern, at most kAsmUnion distinct k over the tile) are staged in LDS with a map
// k -> slot over the b0 sparse columns and a mask of the columns present at each slot; each thread
// then walks one block row i below b0 in ascending k (indices prefetched kAsmUnroll at a time) and
// applies every match to the tile's columns that have it.  The last unknown (the slack column,
// ordered last) has a full row and column below b0 whose factor entries sit last in every column:
// they are read directly.  A tile that holds the slack column, or whose staged values would not
// fit, is assembled one column at a time (staged, or by merging the two rows per entry).
constexpr int kAsmThreads = 256;
constexpr int kAsmCols = 4;
constexpr int kAsmUnion = 1024;
constexpr int kAsmUnroll = 8;

struct AsmLds {
    double* u4;        // kAsmUnion x kAsmCols (one column: kAsmUnion values)
    int32_t* kidx;     // kAsmUnion
    uint8_t* mask;     // kAsmUnion
    int16_t* kmap;     // b0
};

__device__ __forceinline__ AsmLds asm_lds(double* smem) {
    AsmLds L;
    L.u4 = smem;
    L.kidx = reinterpret_cast<int32_t*>(smem + kAsmUnion * kAsmCols);
    L.mask = reinterpret_cast<uint8_t*>(L.kidx + kAsmUnion);
    L.kmap = reinterpret_cast<int16_t*>(L.mask + kAsmUnion);
    return L;
}

// Initial value of block entry (gi, gj): a_ij (+ eps d on the diagonal) as gathered (values vs apart).
__device__ __forceinline__ double block_a(const SpIdx& ix, const double* ud, const double* lv, const double* uv,
                                          int gi, int gj, int64_t vs = 1) {
    return gi == gj ? ud[gj * vs]
                    : (gi > gj ? lv[(ix.l_ptr[gj] + (gi - gj - 1)) * vs] : uv[(ix.l_ptr[gi] + (gj - gi - 1)) * vs]);
}

// Column j of the block, alone.
__device__ void assemble_column(const SpIdx& ix, double* ud, int j, const AsmLds& L) {
    const int n = ix.n, nl = ix.nnzl, b0 = ix.tail_b0, nt = ix.tail_n, ld = ix.tail_ld, tid = threadIdx.x;
    const int last = n - 1;
    double* T = ud + ix.tail_off + (int64_t)j * ld;
    if (j >= nt) {                                       // identity padding column
        for (int i = tid; i < ld; i += kAsmThreads) T[i] = i == j ? 1.0 : 0.0;
        return;
    }
    const double* lv = ud + n;
    const double* uv = ud + n + nl;
    double* uval = L.u4;
    const int gj = b0 + j, lenj = ix.tail_rcnt[j], pj = ix.r_ptr[gj];
    const int32_t* lpos = ix.tail_lastpos;
    const bool owner_last = gj == last;
    const bool staged = !owner_last && lenj <= kAsmUnion;
    if (staged) {
        for (int k = tid; k < b0; k += kAsmThreads) L.kmap[k] = -1;
        __syncthreads();
        for (int q = tid; q < lenj; q += kAsmThreads) {
            const int k = ix.r_idx[pj + q];
            L.kmap[k] = (int16_t)q;
            L.kidx[q] = k;
            uval[q] = uv[ix.r_pos[pj + q]];
        }
        __syncthreads();
    }
    constexpr int UN = kAsmUnroll;
    for (int i = tid; i < ld; i += kAsmThreads) {
        if (i >= nt) {
            T[i] = 0.0;
            continue;
        }
        const int gi = b0 + i;
        double v = block_a(ix, ud, lv, uv, gi, gj);
        const bool row_last = gi == last;
        if (staged && row_last) {
            // l_{last,k} at lastpos[k] (no entry: -1)
            int q = 0;
            for (; q + UN <= lenj; q += UN) {
                int tt[UN];
                double l[UN];
#pragma unroll
                for (int w = 0; w < UN; ++w) tt[w] = lpos[L.kidx[q + w]];
#pragma unroll
                for (int w = 0; w < UN; ++w) l[w] = tt[w] >= 0 ? lv[tt[w]] : 0.0;
#pragma unroll
                for (int w = 0; w < UN; ++w)
                    if (tt[w] >= 0) v = fmad(-l[w], uval[q + w], v);
            }
            for (; q < lenj; ++q) {
                const int t = lpos[L.kidx[q]];
                if (t >= 0) v = fmad(-lv[t], uval[q], v);
            }
        } else if (staged) {
            const int p0 = ix.r_ptr[gi], pe = p0 + ix.tail_rcnt[i];
            int p = p0;
            for (; p + UN <= pe; p += UN) {
                int qq[UN], tt[UN];
                double l[UN];
#pragma unroll
                for (int w = 0; w < UN; ++w) {
                    qq[w] = ix.r_idx[p + w];
                    tt[w] = ix.r_pos[p + w];
                }
#pragma unroll
                for (int w = 0; w < UN; ++w) {
                    qq[w] = L.kmap[qq[w]];
                    l[w] = qq[w] >= 0 ? lv[tt[w]] : 0.0;
                }
#pragma unroll
                for (int w = 0; w < UN; ++w)
                    if (qq[w] >= 0) v = fmad(-l[w], uval[qq[w]], v);
            }
            for (; p < pe; ++p) {
                const int q = L.kmap[ix.r_idx[p]];
                if (q >= 0) v = fmad(-lv[ix.r_pos[p]], uval[q], v);
            }
        } else if (owner_last && row_last) {
            // (last, last): every k below b0 with both factors at lastpos[k]
            int k = 0;
            for (; k + UN <= b0; k += UN) {
                int tt[UN];
                double l[UN], u[UN];
#pragma unroll
                for (int w = 0; w < UN; ++w) tt[w] = lpos[k + w];
#pragma unroll
                for (int w = 0; w < UN; ++w) {
                    l[w] = tt[w] >= 0 ? lv[tt[w]] : 0.0;
                    u[w] = tt[w] >= 0 ? uv[tt[w]] : 0.0;
                }
#pragma unroll
                for (int w = 0; w < UN; ++w)
                    if (tt[w] >= 0) v = fmad(-l[w], u[w], v);
            }
            for (; k < b0; ++k) {
                const int t = lpos[k];
                if (t >= 0) v = fmad(-lv[t], uv[t], v);
            }
        } else if (owner_last) {
            // u_{k,last} at lastpos[k]
            const int p0 = ix.r_ptr[gi], pe = p0 + ix.tail_rcnt[i];
            int p = p0;
            for (; p + UN <= pe; p += UN) {
                int tt[UN], pp[UN];
                double l[UN], u[UN];
#pragma unroll
                for (int w = 0; w < UN; ++w) {
                    tt[w] = ix.r_idx[p + w];
                    pp[w] = ix.r_pos[p + w];
                }
#pragma unroll
                for (int w = 0; w < UN; ++w) tt[w] = lpos[tt[w]];
#pragma unroll
                for (int w = 0; w < UN; ++w) {
                    l[w] = tt[w] >= 0 ? lv[pp[w]] : 0.0;
                    u[w] = tt[w] >= 0 ? uv[tt[w]] : 0.0;
                }
#pragma unroll
                for (int w = 0; w < UN; ++w)
                    if (tt[w] >= 0) v = fmad(-l[w], u[w], v);
            }
            for (; p < pe; ++p) {
                const int t = lpos[ix.r_idx[p]];
                if (t >= 0) v = fmad(-lv[ix.r_pos[p]], uv[t], v);
            }
        } else {
            v = merge_dot_below(ix, gi, gj, b0, lv, uv, v);
        }
        T[i] = v;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kAsmThreads) void tail_assemble_kernel(SpArgs a, int cols) {
    extern __shared__ __align__(16) double smem[];
    __shared__ int s_cnt;
    const AsmLds L = asm_lds(smem);
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, b0 = ix.tail_b0, nt = ix.tail_n, ld = ix.tail_ld, tid = threadIdx.x;
    const int last = n - 1;
    const int32_t* lpos = ix.tail_lastpos;
    const int ntile = ld / cols;
    const int64_t total = (int64_t)ntile * a.ntasks;
    constexpr int UN = kAsmUnroll;
    for (int64_t wg = blockIdx.x; wg < total; wg += gridDim.x) {
        const int task = (int)(wg / ntile), j0 = (int)(wg % ntile) * cols;
        double* ud = a.fac + (int64_t)task * a.fstride;
        int lens = 0;
        bool has_last = false;
        for (int c = 0; c < cols; ++c)
            if (j0 + c < nt) {
                lens += ix.tail_rcnt[j0 + c];
                has_last |= b0 + j0 + c == last;
            }
        if (cols != kAsmCols || has_last || lens > kAsmUnion) {
            for (int c = 0; c < cols; ++c) assemble_column(ix, ud, j0 + c, L);
            continue;
        }
        const double* lv = ud + n;
        const double* uv = ud + n + nl;
        // stage: slots for the distinct k of the tile's columns, their U values and presence mask
        if (tid == 0) s_cnt = 0;
        for (int k = tid; k < b0; k += kAsmThreads) L.kmap[k] = -1;
        __syncthreads();
        for (int c = 0; c < kAsmCols; ++c) {
            if (j0 + c < nt) {
                const int gj = b0 + j0 + c, pj = ix.r_ptr[gj], len = ix.tail_rcnt[j0 + c];
                for (int q = tid; q < len; q += kAsmThreads) {
                    const int k = ix.r_idx[pj + q];
                    int sl = L.kmap[k];
                    if (sl < 0) {
                        sl = atomicAdd(&s_cnt, 1);
                        L.kmap[k] = (int16_t)sl;
                        L.mask[sl] = 0;
#pragma unroll
                        for (int w = 0; w < kAsmCols; ++w) L.u4[sl * kAsmCols + w] = 0.0;
                    }
                    L.u4[sl * kAsmCols + c] = uv[ix.r_pos[pj + q]];
                    L.mask[sl] |= (uint8_t)(1u << c);
                }
            }
            __syncthreads();
        }
        for (int i = tid; i < ld; i += kAsmThreads) {
            double acc[kAsmCols];
            const int gi = b0 + i;
#pragma unroll
            for (int c = 0; c < kAsmCols; ++c)
                acc[c] = (i < nt && j0 + c < nt) ? block_a(ix, ud, lv, uv, gi, b0 + j0 + c) : 0.0;
            if (i < nt && gi == last) {
                // the slack row: each column's own list, l_{last,k} at lastpos[k]
                for (int c = 0; c < kAsmCols; ++c) {
                    if (j0 + c >= nt) continue;
                    const int gj = b0 + j0 + c, pj = ix.r_ptr[gj], len = ix.tail_rcnt[j0 + c];
                    double v = acc[c];
                    int q = 0;
                    for (; q + UN <= len; q += UN) {
                        // indices, then the column ends, then the values: three round trips per UN entries
                        int kk[UN], tt[UN];
                        double l[UN], u[UN];
#pragma unroll
                        for (int w = 0; w < UN; ++w) {
                            kk[w] = ix.r_idx[pj + q + w];
                            tt[w] = ix.r_pos[pj + q + w];
                        }
#pragma unroll
                        for (int w = 0; w < UN; ++w) kk[w] = lpos[kk[w]];
#pragma unroll
                        for (int w = 0; w < UN; ++w) {
                            l[w] = kk[w] >= 0 ? lv[kk[w]] : 0.0;
                            u[w] = kk[w] >= 0 ? uv[tt[w]] : 0.0;
                        }
#pragma unroll
                        for (int w = 0; w < UN; ++w)
                            if (kk[w] >= 0) v = fmad(-l[w], u[w], v);
                    }
                    for (; q < len; ++q) {
                        const int t = lpos[ix.r_idx[pj + q]];
                        if (t >= 0) v = fmad(-lv[t], uv[ix.r_pos[pj + q]], v);
                    }
                    acc[c] = v;
                }
            } else if (i < nt) {
                const int p0 = ix.r_ptr[gi], pe = p0 + ix.tail_rcnt[i];
                int p = p0;
                for (; p + UN <= pe; p += UN) {
                    int qq[UN], tt[UN];
                    double l[UN];
#pragma unroll
                    for (int w = 0; w < UN; ++w) {
                        qq[w] = ix.r_idx[p + w];
                        tt[w] = ix.r_pos[p + w];
                    }
#pragma unroll
                    for (int w = 0; w < UN; ++w) {
                        qq[w] = L.kmap[qq[w]];
                        l[w] = qq[w] >= 0 ? lv[tt[w]] : 0.0;
                    }
#pragma unroll
                    for (int w = 0; w < UN; ++w) {
                        if (qq[w] < 0) continue;
                        const int m = L.mask[qq[w]];
#pragma unroll
                        for (int c = 0; c < kAsmCols; ++c)
                            if ((m >> c) & 1) acc[c] = fmad(-l[w], L.u4[qq[w] * kAsmCols + c], acc[c]);
                    }
                }
                for (; p < pe; ++p) {
                    const int q = L.kmap[ix.r_idx[p]];
                    if (q < 0) continue;
                    const double l = lv[ix.r_pos[p]];
                    const int m = L.mask[q];
#pragma unroll
                    for (int c = 0; c < kAsmCols; ++c)
                        if ((m >> c) & 1) acc[c] = fmad(-l, L.u4[q * kAsmCols + c], acc[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < kAsmCols; ++c) {
                const int j = j0 + c;
                ud[ix.tail_off + (int64_t)j * ld + i] = j < nt ? (i < nt ? acc[c] : 0.0) : (i == j ? 1.0 : 0.0);
            }
        }
        __syncthreads();
    }
}

int64_t tail_asm_lds(int32_t b0) {
    return (int64_t)kAsmUnion * (kAsmCols * 8 + 4 + 1) + ((int64_t)b0 * 2 + 15) / 16 * 16;
}

// ---- assembly by tile pairs on the MFMA unit
// Block tile (t, u) (16 x 16) receives sum_k l_ik u_kj over the columns k < tail_b0 common to
// K_t and K_u, ascending; a column in the union of a tile's rows contributes exact zeros to the
// rows without it (a product with a zero factor leaves a nonzero accumulator unchanged), so the
// chain of every entry equals the reference's.  Each system's panels are gathered once, then one
// wave per tile pair runs the chain four columns per v_mfma_f64_16x16x4f64 (which accumulates in
// ascending k), computed transposed like gemm_mfma: A = -U panel of u, B = L panel of t, so lane
// l, register q holds the entry of slots (16t + l%16, 16u + 4q + l/16); the chains start from the
// block's initial values, written beforehand.
constexpr int kTpWaves = 8;
constexpr int kTpUnroll = 8;
constexpr int kTileLongSteps = 512;   // tile pairs with this many steps take the staged path
// Staged path of the long tile pairs: chunks of kLcSteps MFMA steps, kLcDepth chunks in flight,
// a ring of kLcDepth + 1 chunk slots in LDS (A columns then B columns, 16 doubles each), and per
// wave two blocks of 8 chunks' pair words (68 KB in all: the two workgroups per CU that the
// registers allow still fit).
constexpr int kLcSteps = 16, kLcDepth = 3, kLcSlots = kLcDepth + 1;
constexpr int kLcSlot = 2 * 4 * kLcSteps * 16;

__device__ __forceinline__ double* tail_panels(const SpIdx& ix, double* T) {
    return T + (int64_t)ix.tail_ld * ix.tail_ld + (int64_t)ix.tail_ld * 64;
}

// Every block entry's initial value a_ij (+ eps d on the diagonal) straight from the Jacobian's
// values, the identity on the padding rows and columns: a workgroup per (column, system), one
// thread per row, so that the per-system values and the column's L positions are uniform and no
// index needs a division.
__global__ __launch_bounds__(256) void tail_block_init_kernel(SpArgs a, EpsSet es) {
    const SpIdx& ix = a.ix;
    const int ld = ix.tail_ld, nt = ix.tail_n, b0 = ix.tail_b0;
    for (int task = blockIdx.y; task < a.ntasks; task += gridDim.y) {
        const double* vals = a.values + (int64_t)(task / es.K) * a.nnz;
        const double e = a.scale ? __dmul_rn(eps_at(es, task % es.K), a.scale[task / es.K]) : eps_at(es, task % es.K);
        double* out = a.dense + (int64_t)task * a.dstride;
        for (int j = blockIdx.x; j < ld; j += gridDim.x) {
            const int gj = b0 + j;
            for (int i = threadIdx.x; i < ld; i += 256) {
                double v;
                if (i >= nt || j >= nt) v = i == j ? 1.0 : 0.0;
                else {
                    const int gi = b0 + i;
                    if (i == j) v = gather_diag(ix, gj, vals, e, a.dvec);
                    else {
                        const int src = i > j ? ix.src_l[ix.l_ptr[gj] + (gi - gj - 1)] : ix.src_u[ix.l_ptr[gi] + (gj - gi - 1)];
                        v = src >= 0 ? vals[src] : 0.0;
                    }
                }
                out[(int64_t)j * ld + i] = v;
            }
        }
    }
}

// Panels, task-major factors: one thread per panel entry.
__global__ void tail_panel_gather_kernel(SpArgs a) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl;
    const int64_t P = ix.tail_panel, total = P * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / P);
        const int64_t q = g % P;
        const int pos = ix.tail_mpos[q];
        const double* ud = a.fac + (int64_t)task * a.ts;
        double* PL = tail_panels(ix, a.dense + (int64_t)task * a.dstride);
        PL[q] = pos >= 0 ? ud[n + pos] : 0.0;
        PL[P + q] = pos >= 0 ? ud[n + nl + pos] : 0.0;
    }
}

// Panels, interleaved factors: 64 entries x 64 systems per workgroup, read along the systems and
// written along the entries through LDS.
__global__ __launch_bounds__(256) void tail_panel_gather_il_kernel(SpArgs a, int echunks) {
    __shared__ double sv[64][65];
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl;
    const int64_t P = ix.tail_panel, TP = a.vs;
    const int64_t e0 = (int64_t)(blockIdx.x % echunks) * 64;
    const int t0 = (int)(blockIdx.x / echunks) * 64;
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    int pos[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) pos[k] = e0 + y + 4 * k < P ? ix.tail_mpos[e0 + y + 4 * k] : -1;
    for (int side = 0; side < 2; ++side) {          // L values, then U values
        const double* src = a.fac + (int64_t)(side ? n + nl : n) * TP + t0 + x;
        const bool tok = t0 + x < a.ntasks;
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = (pos[k] >= 0 && tok) ? src[(int64_t)pos[k] * TP] : 0.0;
        if (side) __syncthreads();                  // the L values have been written out
#pragma unroll
        for (int k = 0; k < 16; ++k) sv[y + 4 * k][x] = v[k];
        __syncthreads();
        if (e0 + x < P)
            for (int tt = y; tt < 64 && t0 + tt < a.ntasks; tt += 4)
                tail_panels(ix, a.dense + (int64_t)(t0 + tt) * a.dstride)[side * P + e0 + x] = sv[x][tt];
    }
}

// LDS byte address of a pointer into a __shared__ array.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// The staged path's LDS reads are written out with their wait in the same block: they follow
// the wait and barrier that complete the copies they read, and left to the compiler each read
// would also wait for every copy still in flight (it cannot tell the ring slots apart).
// Eight steps of a chunk's operands at LDS address s (A: steps 64 doubles apart, B 8 KB on),
// and the pair word at LDS address w, under one wait.
__device__ __forceinline__ void read_half(uint32_t s, uint32_t w, double* av, double* bv, int& wd) {
    static_assert(kLcSlot == 2048, "offsets below assume chunks of 16 steps of 4 x 16 doubles");
    asm volatile(
        "ds_read_b32 %16, %18\n\t"
        "ds_read_b64 %0, %17\n\t"
        "ds_read_b64 %1, %17 offset:512\n\t"
        "ds_read_b64 %2, %17 offset:1024\n\t"
        "ds_read_b64 %3, %17 offset:1536\n\t"
        "ds_read_b64 %4, %17 offset:2048\n\t"
        "ds_read_b64 %5, %17 offset:2560\n\t"
        "ds_read_b64 %6, %17 offset:3072\n\t"
        "ds_read_b64 %7, %17 offset:3584\n\t"
        "ds_read_b64 %8, %17 offset:8192\n\t"
        "ds_read_b64 %9, %17 offset:8704\n\t"
        "ds_read_b64 %10, %17 offset:9216\n\t"
        "ds_read_b64 %11, %17 offset:9728\n\t"
        "ds_read_b64 %12, %17 offset:10240\n\t"
        "ds_read_b64 %13, %17 offset:10752\n\t"
        "ds_read_b64 %14, %17 offset:11264\n\t"
        "ds_read_b64 %15, %17 offset:11776\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(av[0]), "=&v"(av[1]), "=&v"(av[2]), "=&v"(av[3]), "=&v"(av[4]), "=&v"(av[5]), "=&v"(av[6]),
          "=&v"(av[7]), "=&v"(bv[0]), "=&v"(bv[1]), "=&v"(bv[2]), "=&v"(bv[3]), "=&v"(bv[4]), "=&v"(bv[5]),
          "=&v"(bv[6]), "=&v"(bv[7]), "=&v"(wd)
        : "v"(s), "v"(w)
        : "memory");
}

// The pair word at LDS address w alone.
__device__ __forceinline__ int read_word(uint32_t w) {
    int wd;
    asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(wd) : "v"(w) : "memory");
    return wd;
}

// One long tile pair per workgroup at a time (see tail_tile_kernel): the eight waves copy the
// panel columns of chunk c + kLcDepth while wave 0 runs the MFMAs of chunk c.
__device__ __forceinline__ void tail_tile_long(const SpArgs& a, int lwgs, double* ring, int32_t* words) {
    const SpIdx& ix = a.ix;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    constexpr int CW = 4 * kLcSteps;   // pair words (columns of A, and of B) per chunk
    // this lane's share of a chunk's copies: column q of A and of B, rows r0 and r0 + 1
    const int q = 8 * wave + (lane >> 3), r0 = 2 * (lane & 7);
    static_assert(kTpWaves == 8 && CW == 64, "eight waves copy a chunk's 64 + 64 columns, 8 + 8 each");
    int32_t* Wd = words + wave * 128;   // this wave's words: two blocks of 8 chunks x its 8 columns
    const int64_t items = (int64_t)ix.tail_nlpairs * a.ntasks;
    for (int64_t it = blockIdx.x; it < items; it += lwgs) {
        const int task = (int)(it / ix.tail_nlpairs), pi = ix.tail_lpairs[it % ix.tail_nlpairs];
        const int TT = ix.tail_tiles, t = pi / TT, u = pi % TT;
        double* T = a.dense + (int64_t)task * a.dstride;
        const double* PL = tail_panels(ix, T);
        const double* Lt = PL + 16 * (int64_t)ix.tail_kt_ptr[t] + r0;
        const double* Uu = PL + ix.tail_panel + 16 * (int64_t)ix.tail_kt_ptr[u] + r0;
        // past the end: the zero column of each panel (the pair lists' own padding), so that the
        // last chunk's extra steps leave the sums unchanged
        const int zw = (ix.tail_kt_ptr[t + 1] - ix.tail_kt_ptr[t] - 1) | (ix.tail_kt_ptr[u + 1] - ix.tail_kt_ptr[u] - 1) << 16;
        const int p0 = ix.tail_pp_ptr[pi], p1 = ix.tail_pp_ptr[pi + 1];
        const int len = p1 - p0, nch = (len + CW - 1) / CW;
        // Word block m (chunks 8m .. 8m + 7) into block slot m % 2: lane l takes the word of chunk
        // 8m + l / 8, column 8 wave + l % 8 (clamped in bounds).
        const int wcol = 8 * wave + (lane & 7), wch = lane >> 3;
        auto load_words = [&](int m) {
            __builtin_amdgcn_global_load_lds(ix.tail_pairs + p0 + min(CW * (8 * m + wch) + wcol, len - 1),
                                             Wd + (m % 2) * 64, 4, 0, 0);
        };
        auto word_addr = [&](int j) { return lds_addr(Wd + ((j >> 3) % 2) * 64 + (j & 7) * 8 + (lane >> 3)); };
        // Columns of chunk j into ring slot j % kLcSlots.
        auto copy = [&](int j, int wd) {
            wd = CW * j + q < len ? wd : zw;
            double* S = ring + (j % kLcSlots) * kLcSlot + 128 * wave;
            __builtin_amdgcn_global_load_lds(Uu + 16 * (int)((uint32_t)wd >> 16), S, 16, 0, 0);
            __builtin_amdgcn_global_load_lds(Lt + 16 * (wd & 0xFFFF), S + kLcSlot / 2, 16, 0, 0);
        };
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        int gi = -1, gj[4] = {-1, -1, -1, -1};
        if (wave == 0) {
            gi = ix.tail_rord[16 * t + li];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                gj[x] = ix.tail_rord[16 * u + 4 * x + lk];
                acc[x] = (gi >= 0 && gj[x] >= 0) ? T[(int64_t)gj[x] * ix.tail_ld + gi] : 0.0;
            }
        }
        static_assert(kLcDepth < 8, "the first kLcDepth copies take their words from block 0");
        load_words(0);
        load_words(1);
        __builtin_amdgcn_s_waitcnt(0);
        for (int j = 0; j < kLcDepth; ++j) copy(j, read_word(word_addr(j)));
        __builtin_amdgcn_s_waitcnt(0);
        for (int c = 0; c < nch; ++c) {
            // Each iteration issues two copies per wave (and every eighth one word load as well).
            // Waiting until 2 (kLcDepth - 1) loads remain completes the copies of chunk c, issued
            // kLcDepth iterations back, and the word block that chunk c + kLcDepth reads, issued
            // eight iterations before its first use; the barrier then makes chunk c visible and
            // tells that wave 0 is done with chunk c - 1, whose slot is refilled next.
            static_assert(2 * (kLcDepth - 1) < 16, "the wait below encodes vmcnt in its low four bits");
            __builtin_amdgcn_s_waitcnt(0x0070 | (2 * (kLcDepth - 1)));   // vmcnt(2 (kLcDepth - 1)) lgkmcnt(0)
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            const uint32_t S = lds_addr(ring + (c % kLcSlots) * kLcSlot + 16 * lk + li);
            double av[8], bv[8];
            int wd;
            if (wave == 0)
                read_half(S, word_addr(c + kLcDepth), av, bv, wd);
            else
                wd = read_word(word_addr(c + kLcDepth));
            copy(c + kLcDepth, wd);
            // block m is first read by the copy of chunk 8 m, at iteration 8 m - kLcDepth; it
            // is loaded eight iterations before, after the last read of block m - 2
            if (((c + 8 + kLcDepth) & 7) == 0) load_words((c + 8 + kLcDepth) >> 3);
            if (wave == 0) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (h == 1) read_half(S + 4096, word_addr(c + kLcDepth), av, bv, wd);
#pragma unroll
                    for (int x = 0; x < 8; ++x)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[x], bv[x], acc, 0, 0, 0);
                }
            }
        }
        if (wave == 0) {
#pragma unroll
            for (int x = 0; x < 4; ++x)
                if (gi >= 0 && gj[x] >= 0) T[(int64_t)gj[x] * ix.tail_ld + gi] = acc[x];
        }
        // the loads past the end land before the ring is used again
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// Logical workgroup l of a launch of G = 8 m workgroups runs as hardware workgroup
// (l % m) * 8 + l / m, so consecutive logical workgroups (the tile pairs of one system, which
// share its panels) are dispatched to the same XCD and its L2.  Wave w of logical workgroup l
// takes tile pair l * kTpWaves + w (item = system * tiles^2 + t * tiles + u).  The panel loads
// of the next kTpUnroll steps are issued before the MFMAs of the current ones (the chain of a
// long pair, the slack row's tile with itself, is otherwise one memory latency per step).
//
// The long pairs (the slack row's tile with itself: 4,620 steps at n = 20,001) are not left to
// one wave's register prefetch: the first lwgs workgroups of the launch (a multiple of 8, so the
// XCD mapping of the others is unchanged) take one long pair each, and all eight waves stage its
// panel columns through an LDS ring (global_load_lds, kLcDepth chunks of kLcSteps steps in
// flight) while wave 0 runs the chain from LDS in the same step order.  They run beside the
// regular pairs instead of after them.
__global__ __launch_bounds__(64 * kTpWaves) void tail_tile_kernel(SpArgs a, int64_t items, int lwgs) {
    __shared__ __align__(16) double ring[kLcSlots * kLcSlot];
    __shared__ __align__(16) int32_t words[kTpWaves * 128];
    if ((int)blockIdx.x < lwgs) {   // uniform per workgroup
        tail_tile_long(a, lwgs, ring, words);
        return;
    }
    const SpIdx& ix = a.ix;
    const int64_t bid = blockIdx.x - lwgs;
    const int64_t m = (gridDim.x - lwgs) / 8;
    const int64_t lw = (bid % 8) * m + bid / 8;
    const int64_t it = lw * kTpWaves + (threadIdx.x >> 6);
    if (it >= items) return;                     // uniform per wave; the kernel has no barrier
    const int TT = ix.tail_tiles;
    const int64_t pairs_per = (int64_t)TT * TT;
    const int task = (int)(it / pairs_per), pi = (int)(it % pairs_per);
    const int t = pi / TT, u = pi % TT;
    const int p0 = ix.tail_pp_ptr[pi], p1 = ix.tail_pp_ptr[pi + 1];
    if (lwgs > 0 && (p1 - p0) / 4 >= kTileLongSteps) return;   // a long pair: the staged path's
    const int ld = ix.tail_ld;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    double* T = a.dense + (int64_t)task * a.dstride;
    const double* PL = tail_panels(ix, T);
    const double* Lt = PL + 16 * (int64_t)ix.tail_kt_ptr[t] + li;
    const double* Uu = PL + ix.tail_panel + 16 * (int64_t)ix.tail_kt_ptr[u] + li;
    const int gi = ix.tail_rord[16 * t + li];
    int gj[4];
    v4d acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        gj[q] = ix.tail_rord[16 * u + 4 * q + lk];
        acc[q] = (gi >= 0 && gj[q] >= 0) ? T[(int64_t)gj[q] * ld + gi] : 0.0;
    }
    const int32_t* pr = ix.tail_pairs + lk;
    constexpr int UN = kTpUnroll;
    // pair words: a | b << 16 (past the end: column 0 of both panels, never used)
    auto word = [&](int p) { return p < p1 ? pr[p] : 0; };
    int w[UN];
    double av[UN], bv[UN];
#pragma unroll
    for (int x = 0; x < UN; ++x) w[x] = word(p0 + 4 * x);
#pragma unroll
    for (int x = 0; x < UN; ++x) {
        av[x] = -Uu[16 * (int)((uint32_t)w[x] >> 16)];
        bv[x] = Lt[16 * (w[x] & 0xFFFF)];
    }
#pragma unroll
    for (int x = 0; x < UN; ++x) w[x] = word(p0 + 4 * UN + 4 * x);
    for (int p = p0; p < p1; p += 4 * UN) {
        double an[UN], bn[UN];
#pragma unroll
        for (int x = 0; x < UN; ++x) {
            an[x] = -Uu[16 * (int)((uint32_t)w[x] >> 16)];
            bn[x] = Lt[16 * (w[x] & 0xFFFF)];
        }
#pragma unroll
        for (int x = 0; x < UN; ++x) w[x] = word(p + 8 * UN + 4 * x);
#pragma unroll
        for (int x = 0; x < UN; ++x)
            if (p + 4 * x < p1) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[x], acc, 0, 0, 0);
#pragma unroll
        for (int x = 0; x < UN; ++x) {
            av[x] = an[x];
            bv[x] = bn[x];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (gi >= 0 && gj[q] >= 0) T[(int64_t)gj[q] * ld + gi] = acc[q];
}


// Panel p0 of every system's block: the diagonal block's GETRF (one wave per system), then the
// multipliers below it and the rows of U to its right in chunks of kTrsmThreads items (rows
// below, then columns to the right) over many workgroups, each reloading the factored diagonal
// block.
__global__ __launch_bounds__(64) void tail_getrf_kernel(SpArgs a, int p0) {
    __shared__ double D[NB * NB];
    const int ld = a.ix.tail_ld;
    for (int task = blockIdx.x; task < a.ntasks; task += gridDim.x) {
        const int bad = panel_getrf(a.dense + (int64_t)task * a.dstride, ld, p0, D);
        if (threadIdx.x == 0 && bad) atomicMin(&a.info[task], a.ix.tail_b0 + bad);
    }
}

constexpr int kTrsmThreads = 256;

__global__ __launch_bounds__(kTrsmThreads) void tail_trsm_kernel(SpArgs a, int p0, int chunks) {
    __shared__ double D[NB * NB];
    const int ld = a.ix.tail_ld, rest = ld - p0 - NB;
    const int64_t total = (int64_t)chunks * a.ntasks;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int task = (int)(b / chunks), c = (int)(b % chunks);
        double* T = a.dense + (int64_t)task * a.dstride;
        load_diag(T, ld, p0, D);
        __syncthreads();
        const int i0 = c * kTrsmThreads, i1 = min(i0 + kTrsmThreads, 2 * rest);
        const int r_lo = p0 + NB + min(i0, rest), r_hi = p0 + NB + min(i1, rest);
        const int c_lo = p0 + NB + max(i0 - rest, 0), c_hi = p0 + NB + max(i1 - rest, 0);
        panel_trsm(T, ld, p0, D, r_lo, r_hi, c_lo, c_hi);
        __syncthreads();
    }
}

// Rank-NB update of the trailing matrix after panel p0: one workgroup per 128 x 64 tile.
__global__ __launch_bounds__(WG) void tail_update_kernel(SpArgs a, int p0, int tiles_r, int tiles_c) {
    __shared__ double Us[NB * 64];
    const int ld = a.ix.tail_ld;
    const int64_t per = (int64_t)tiles_r * tiles_c, total = per * a.ntasks;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int task = (int)(b / per), tt = (int)(b % per);
        double* T = a.dense + (int64_t)task * a.dstride;
        const int r0 = p0 + NB + 128 * (tt / tiles_c), c0 = p0 + NB + 64 * (tt % tiles_c);
        gemm_mfma<NB>(T, ld, r0, min(r0 + 128, ld), c0, min(c0 + 64, ld), p0, NB, Us);
    }
}

// Rows of the block, updates from the sparse part (k < b0, ascending): L (or U^T) without the
// division, which the dense solve applies after the block's own updates.
constexpr int kExtThreads = 128;   // the block-row update kernel: room for 32 loads in flight per lane

// A block row with this many terms from the sparse part (the slack row: 18,480 at n = 20,001)
// is one long fma chain per system and right-hand side; one lane per chain keeps only ~32 terms'
// loads in flight, so such rows get a wave per chain instead (tail_fwd_long_kernel).
constexpr int kTailLongRow = 2048;

// One wave per (long row, system, right-hand side), grid-stride: lane l fetches term 64 b + l of
// batch b, its index three batches and its values (the L (U^T) entry and the solution entry) two
// batches before the batch is applied; the index of batch b + 3 is waited for only once batch b's
// values are due anyway (loads complete in order).  A batch's 64 pairs go through LDS and every
// lane applies them in ascending order to the same accumulator with broadcast reads: the chain
// and its rounding are those of one lane walking the row.  Terms past the row's end read a valid
// entry and count as 0 x 0.
template <int TRANS>
__global__ __launch_bounds__(64) void tail_fwd_long_kernel(SpArgs a) {
    constexpr int DV = 2, DI = 4;            // batches of values / of indices in flight
    __shared__ __align__(16) double sp[64][2];
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, nrhs = a.nrhs, b0 = ix.tail_b0, lane = threadIdx.x;
    const int64_t per_row = (int64_t)nrhs * a.ntasks, chains = (int64_t)ix.tail_nlong * per_row;
    const bool il = a.vs != 1;
    for (int64_t c = blockIdx.x; c < chains; c += gridDim.x) {
        const int lr = (int)(c / per_row);
        const int q = (int)(c % per_row);
        const int task = il ? q % a.ntasks : q / nrhs;
        const int r = il ? q / a.ntasks : q % nrhs;
        if (a.info[task]) continue;                       // uniform per wave
        const int i = b0 + ix.tail_long[lr];
        const int64_t vs = a.vs, ys = a.yv;
        const double* m = a.fac + (int64_t)task * a.ts + (int64_t)(TRANS ? n + nl : n) * vs;
        double* y = a.y + (int64_t)task * a.yt + (int64_t)r * ys;
        const int p0 = ix.r_ptr[i], len = ix.tail_rcnt[i - b0], pl = p0 + len - 1;
        const int nb = (len + 63) / 64;
        double acc = y[(int64_t)i * nrhs * ys];
        int ip[DI], iy[DI];
        double mv[DV], yw[DV];
        auto load_idx = [&](int b, int& ipo, int& iyo) {
            const int p = min(p0 + 64 * b + lane, pl);
            ipo = ix.r_pos[p];
            iyo = ix.r_idx[p];
        };
        auto load_val = [&](int b, int ipi, int iyi, double& mo, double& yo) {
            const bool ok = 64 * b + lane < len;
            const double mm = m[(int64_t)ipi * vs], yy = y[(int64_t)iyi * nrhs * ys];
            mo = ok ? mm : 0.0;
            yo = ok ? yy : 0.0;
        };
#pragma unroll
        for (int d = 0; d < DI; ++d) load_idx(d, ip[d], iy[d]);
#pragma unroll
        for (int d = 0; d < DV; ++d) load_val(d, ip[d], iy[d], mv[d], yw[d]);
        for (int bb = 0; bb < nb; bb += DI) {
#pragma unroll
            for (int d = 0; d < DI; ++d) {
                const int b = bb + d;
                if (b >= nb) break;
                const int dv = d % DV;
                sp[lane][0] = mv[dv];
                sp[lane][1] = yw[dv];
                // batch b + DV's values from the indices fetched DI - DV batches ago, then the
                // indices of batch b + DI into the slot batch b's indices used
                load_val(b + DV, ip[(d + DV) % DI], iy[(d + DV) % DI], mv[dv], yw[dv]);
                load_idx(b + DI, ip[d], iy[d]);
                __builtin_amdgcn_wave_barrier();
                // all 64 slots (past the row's end they hold 0 x 0, which leaves acc as it is), a
                // fixed count so that the reads run ahead of the chain
#pragma unroll 16
                for (int j = 0; j < 64; ++j) acc = fmad(-sp[j][0], sp[j][1], acc);
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (lane == 0) y[(int64_t)i * nrhs * ys] = acc;
    }
}

template <int TRANS>
__global__ __launch_bounds__(kExtThreads) void tail_fwd_ext_kernel(SpArgs a) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, nrhs = a.nrhs, b0 = ix.tail_b0;
    const int64_t per = (int64_t)ix.tail_n * nrhs, total = per * a.ntasks;
    const bool il = a.vs != 1;      // interleaved: consecutive threads serve consecutive systems
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = il ? (int)(g % a.ntasks) : (int)(g / per);
        const int t = il ? (int)(g / a.ntasks) : (int)(g % per);
        if (a.info[task]) continue;
        const int i = b0 + t / nrhs, r = t % nrhs;
        if (ix.tail_rcnt[i - b0] >= kTailLongRow) continue;   // tail_fwd_long_kernel's
        const int64_t vs = a.vs, ys = a.yv;
        const double* m = a.fac + (int64_t)task * a.ts + (int64_t)(TRANS ? n + nl : n) * vs;
        double* y = a.y + (int64_t)task * a.yt + (int64_t)r * ys;
        double acc = y[(int64_t)i * nrhs * ys];
        const int p0 = ix.r_ptr[i], pe = p0 + ix.tail_rcnt[i - b0];
        int p = p0;
        if (p + U32 <= pe) {
            // the indices of the next block are fetched while this block's values are in flight
            int ip[U32], iy[U32];
#pragma unroll
            for (int w = 0; w < U32; ++w) {
                ip[w] = ix.r_pos[p + w];
                iy[w] = ix.r_idx[p + w];
            }
            for (; p + U32 <= pe; p += U32) {
                double mv[U32], yw[U32];
#pragma unroll
                for (int w = 0; w < U32; ++w) {
                    mv[w] = m[ip[w] * vs];
                    yw[w] = y[(int64_t)iy[w] * nrhs * ys];
                }
                if (p + 2 * U32 <= pe) {
#pragma unroll
                    for (int w = 0; w < U32; ++w) {
                        ip[w] = ix.r_pos[p + U32 + w];
                        iy[w] = ix.r_idx[p + U32 + w];
                    }
                }
#pragma unroll
                for (int w = 0; w < U32; ++w) acc = fmad(-mv[w], yw[w], acc);
            }
        }
        for (; p < pe; ++p) acc = fmad(-m[ix.r_pos[p] * vs], y[(int64_t)ix.r_idx[p] * nrhs * ys], acc);
        y[(int64_t)i * nrhs * ys] = acc;
    }
}

// Rows before the block, backward pass (U, or L^T when transposed): each row's chain starts with
// the terms of the block's columns (its highest positions, descending); they are applied to every
// row at once once the block is solved, and the levels run the rest of the chains.
template <int TRANS>
__global__ void tail_bwd_ext_kernel(SpArgs a) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, nrhs = a.nrhs, b0 = ix.tail_b0;
    const int64_t per = (int64_t)b0 * nrhs, total = per * a.ntasks;
    const bool il = a.vs != 1;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = il ? (int)(g % a.ntasks) : (int)(g / per);
        const int q = il ? (int)(g / a.ntasks) : (int)(g % per);
        if (a.info[task]) continue;
        const int i = q / nrhs, r = q % nrhs;
        const int t0 = ix.l_ptr[i] + ix.tail_ccnt[i];
        int t = ix.l_ptr[i + 1] - 1;
        if (t < t0) continue;
        const int64_t vs = a.vs, ys = a.yv;
        const double* m = a.fac + (int64_t)task * a.ts + (int64_t)(TRANS ? n : n + nl) * vs;
        double* y = a.y + (int64_t)task * a.yt + (int64_t)r * ys;
        double acc = y[(int64_t)i * nrhs * ys];
        if (t - U16 + 1 >= t0) {
            int iy[U16];
#pragma unroll
            for (int w = 0; w < U16; ++w) iy[w] = ix.l_idx[t - w];
            for (; t - U16 + 1 >= t0; t -= U16) {
                double mv[U16], yw[U16];
#pragma unroll
                for (int w = 0; w < U16; ++w) {
                    mv[w] = m[(int64_t)(t - w) * vs];
                    yw[w] = y[(int64_t)iy[w] * nrhs * ys];
                }
                if (t - 2 * U16 + 1 >= t0) {
#pragma unroll
                    for (int w = 0; w < U16; ++w) iy[w] = ix.l_idx[t - U16 - w];
                }
#pragma unroll
                for (int w = 0; w < U16; ++w) acc = fmad(-mv[w], yw[w], acc);
            }
        }
        for (; t >= t0; --t) acc = fmad(-m[(int64_t)t * vs], y[(int64_t)ix.l_idx[t] * nrhs * ys], acc);
        y[(int64_t)i * nrhs * ys] = acc;
    }
}

// The block's own triangular solves (forward then backward, or the transposed pair) on a
// column-major copy R of its right-hand sides (nrhs columns of stride tail_ld), by blocks of SB
// rows: the diagonal block of every system in one workgroup (one wave per right-hand side, the
// pivot values passed by readlane), then the rows outside it on the whole device.  The updates of
// an entry arrive block by block in the order of the reference substitution (ascending for the
// forward pass, descending for the backward one).
__global__ void tail_rhs_in_kernel(SpArgs a) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nrhs = a.nrhs, ld = ix.tail_ld;
    const int64_t per = (int64_t)ld * nrhs, total = per * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / per), t = (int)(g % per);
        const int q = t % ld, r = t / ld;
        double* R = a.dense + (int64_t)task * a.dstride + (int64_t)ld * ld;
        R[(int64_t)r * ld + q] = q < ix.tail_n ? a.y[task * a.yt + ((int64_t)(ix.tail_b0 + q) * nrhs + r) * a.yv] : 0.0;
    }
}

__global__ void tail_rhs_out_kernel(SpArgs a) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nrhs = a.nrhs, ld = ix.tail_ld, nt = ix.tail_n;
    const int64_t per = (int64_t)nt * nrhs, total = per * a.ntasks;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int task = (int)(g / per), t = (int)(g % per);
        const int q = t % nt, r = t / nt;
        const double* R = a.dense + (int64_t)task * a.dstride + (int64_t)ld * ld;
        a.y[task * a.yt + ((int64_t)(ix.tail_b0 + q) * nrhs + r) * a.yv] = R[(int64_t)r * ld + q];
    }
}

template <int LOWER, int TRANS>
__global__ __launch_bounds__(WG) void tail_tri_diag_kernel(SpArgs a, int c0) {
    constexpr bool UNIT = (LOWER && !TRANS) || (!LOWER && TRANS);
    constexpr int NW = WG / 64;                  // right-hand sides per workgroup, one per wave
    constexpr int TP = SB + 1;                  // padded rows: the solve's column reads hit distinct banks
    __shared__ double Tri[SB * TP];
    const int ld = a.ix.tail_ld, nrhs = a.nrhs, bs = min(SB, ld - c0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int groups = (nrhs + NW - 1) / NW;     // workgroup b: system b / groups, waves' RHS from (b % groups) * NW
    for (int64_t b = blockIdx.x; b < (int64_t)a.ntasks * groups; b += gridDim.x) {
        const int task = (int)(b / groups), r0 = (int)(b % groups) * NW;
        if (a.info[task]) continue;
        const double* M = a.dense + (int64_t)task * a.dstride;
        double* R = const_cast<double*>(M) + (int64_t)ld * ld;
        constexpr int QT = SB * SB / WG;          // all of the block's loads in flight first
        double vt[QT];
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            const int t = tid + WG * q, i = t % SB, j = t / SB;
            vt[q] = (i < bs && j < bs) ? (TRANS ? M[(int64_t)(c0 + i) * ld + c0 + j] : M[(int64_t)(c0 + j) * ld + c0 + i])
                                       : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            const int t = tid + WG * q;
            Tri[(t % SB) * TP + t / SB] = vt[q];
        }
        __syncthreads();
        for (int r = r0 + wave; r < min(nrhs, r0 + NW); r += NW) {
            double* tc = R + (int64_t)r * ld + c0;
            double t = lane < bs ? tc[lane] : 0.0;
            if (LOWER) {
                for (int k = 0; k < bs; ++k) {
                    double xk = readlane_d(t, k);
                    if (!UNIT) xk = xk / Tri[k * TP + k];
                    if (lane == k) t = xk;
                    if (lane > k) t = fmad(-Tri[lane * TP + k], xk, t);
                }
            } else {
                for (int k = bs - 1; k >= 0; --k) {
                    double xk = readlane_d(t, k);
                    if (!UNIT) xk = xk / Tri[k * TP + k];
                    if (lane == k) t = xk;
                    if (lane < k) t = fmad(-Tri[lane * TP + k], xk, t);
                }
            }
            if (lane < bs) tc[lane] = t;
        }
        __syncthreads();
    }
}

// The rows outside the solved 64-row block, each (row, right-hand side) updated by the block's
// bs terms in the order of the solve.  A workgroup takes one system, 64 rows and up to 32
// right-hand sides: it stages the 64 x bs multipliers (transposed when TRANS, so that both
// orientations are read along a row index) and the bs x 32 solved values in LDS, and wave w
// runs eight right-hand sides' chains, lane = row.  Each chain is the same sequence of fmas as
// one thread per (row, right-hand side) would run.
constexpr int kRestRows = 64, kRestRhs = 32, kRestMP = SB + 1, kRestXP = kRestRhs + 2;
template <int LOWER, int TRANS>
__global__ __launch_bounds__(256) void tail_tri_rest_kernel(SpArgs a, int c0) {
    __shared__ double Ms[SB * kRestMP];       // Ms[k * kRestMP + row]
    __shared__ double Xs[SB * kRestXP];       // Xs[k * kRestXP + rhs]
    const int ld = a.ix.tail_ld, nrhs = a.nrhs, bs = min(SB, ld - c0);
    const int lo = LOWER ? c0 + bs : 0, hi = LOWER ? ld : c0;
    if (hi <= lo) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row_tiles = (hi - lo + kRestRows - 1) / kRestRows, rhs_chunks = (nrhs + kRestRhs - 1) / kRestRhs;
    const int64_t per = (int64_t)row_tiles * rhs_chunks;
    for (int64_t b = blockIdx.x; b < per * a.ntasks; b += gridDim.x) {   // uniform per workgroup
        const int task = (int)(b / per), rt = (int)(b % per) / rhs_chunks, rc = (int)(b % per) % rhs_chunks;
        if (a.info[task]) continue;
        const int i0 = lo + rt * kRestRows, rows = min(kRestRows, hi - i0);
        const int r0 = rc * kRestRhs, nr = min(kRestRhs, nrhs - r0);
        const double* M = a.dense + (int64_t)task * a.dstride;
        double* R = const_cast<double*>(M) + (int64_t)ld * ld;
        // all of the tile's loads in flight before the first LDS store
        constexpr int QM = SB * kRestRows / 256, QX = SB * kRestRhs / 256;
        double vm[QM], vx[QX];
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            // coalesced along the row index (not TRANS) or along k (TRANS)
            const int t = tid + 256 * q;
            const int k = TRANS ? t % SB : t / kRestRows, ii = TRANS ? t / SB : t % kRestRows;
            vm[q] = (k < bs && ii < rows) ? (TRANS ? M[(int64_t)(i0 + ii) * ld + c0 + k] : M[(int64_t)(c0 + k) * ld + i0 + ii])
                                          : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int t = tid + 256 * q, k = t % SB, rr = t / SB;
            vx[q] = (k < bs && rr < nr) ? R[(int64_t)(r0 + rr) * ld + c0 + k] : 0.0;
        }
        __syncthreads();                          // the previous item's reads are done
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int t = tid + 256 * q;
            const int k = TRANS ? t % SB : t / kRestRows, ii = TRANS ? t / SB : t % kRestRows;
            Ms[k * kRestMP + ii] = vm[q];
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int t = tid + 256 * q;
            Xs[(t % SB) * kRestXP + t / SB] = vx[q];
        }
        __syncthreads();
        const int rw = 8 * wave;                  // this wave's right-hand sides: r0 + rw .. + 7
        if (rw < nr && lane < rows) {              // uniform in the first, per lane in the second
            double acc[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = rw + j < nr ? R[(int64_t)(r0 + rw + j) * ld + i0 + lane] : 0.0;
            for (int kk = 0; kk < bs; ++kk) {
                const int k = LOWER ? kk : bs - 1 - kk;
                const double m = Ms[k * kRestMP + lane];
                const double* x = Xs + k * kRestXP + rw;
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[j] = fmad(-m, x[j], acc[j]);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (rw + j < nr) R[(int64_t)(r0 + rw + j) * ld + i0 + lane] = acc[j];
        }
    }
}

// One workgroup per system (large batches): the block's whole LU with super-panels and MFMA
// updates, or one triangular solve; the same operations in the same order as the per-panel and
// per-block kernels above, so the same bits.
// The LU takes the dense path's configuration: 256-lane workgroups, two per CU.
__global__ __launch_bounds__(WGD, 2) void tail_lu_slot_kernel(SpArgs a) {
    extern __shared__ double lds[];
    const int ld = a.ix.tail_ld;
    for (int task = blockIdx.x; task < a.ntasks; task += gridDim.x) {
        double* T = a.dense + (int64_t)task * a.dstride;
        const int bad = factor_slot<WGD, kFusedBuf, kFusedCT>(T, ld, ld, ld, lds);
        if (threadIdx.x == 0 && bad) atomicMin(&a.info[task], a.ix.tail_b0 + bad);
        __syncthreads();
    }
}

template <int LOWER, int TRANS>
__global__ __launch_bounds__(WG) void tail_tri_slot_kernel(SpArgs a) {
    extern __shared__ double lds[];
    const int ld = a.ix.tail_ld;
    for (int task = blockIdx.x; task < a.ntasks; task += gridDim.x) {
        if (a.info[task]) continue;                  // uniform per workgroup
        double* T = a.dense + (int64_t)task * a.dstride;
        tri_solve<LOWER, TRANS>(T, ld, ld, T + (int64_t)ld * ld, a.nrhs, lds);
    }
}

int grid_for(int64_t items, int threads);

template <int LOWER, int TRANS>
hipError_t tail_tri(SpArgs a, hipStream_t st) {
    const int ld = a.ix.tail_ld, nblk = (ld + SB - 1) / SB;
    const int tgrid = (int)std::min<int64_t>((int64_t)a.ntasks * ((a.nrhs + WG / 64 - 1) / (WG / 64)), 65535);
    for (int bb = 0; bb < nblk; ++bb) {
        const int blk = LOWER ? bb : nblk - 1 - bb, c0 = blk * SB, bs = std::min(SB, ld - c0);
        hipLaunchKernelGGL((tail_tri_diag_kernel<LOWER, TRANS>), dim3(tgrid), dim3(WG), 0, st, a, c0);
        const int rows = LOWER ? ld - c0 - bs : c0;
        if (rows > 0) {
            const int64_t wgs = (int64_t)a.ntasks * ((rows + kRestRows - 1) / kRestRows) * ((a.nrhs + kRestRhs - 1) / kRestRhs);
            hipLaunchKernelGGL((tail_tri_rest_kernel<LOWER, TRANS>), dim3((unsigned)std::min<int64_t>(wgs, 1 << 20)),
                               dim3(256), 0, st, a, c0);
        }
    }
    return hipGetLastError();
}


// ---------------------------------------------------------------- batched, systems interleaved
// Many systems share one pattern, so the index data of an item is the same for
// all of them.  Values are stored system-innermost, value v of task q at
// v * TP + q (TP = ntasks rounded up to 64), and a wave handles one item for 64
// consecutive systems: the index loads are uniform and the value loads are
// contiguous.  One launch per level and phase covers every system.
struct IlArgs {
    SpIdx ix;
    int32_t nnz, nrhs, ntasks, TP, K, batch;
    const double* values;
    const double* dvec;
    const double* B;
    double* X;
    int32_t* info;
    double* fac;     // (n + 2 nnzl) x TP
    double* y;       // (n * nrhs) x TP
    double* Xk;              // or NULL: the per-system solutions too, batch x K x n x nrhs (NaN if broken)
    const double* scale;     // or NULL: Jacobian s at the nodes scale[s] eps_k (a power of two)
};

// UNIFORM: every lane of the wave works on the same item (the per-level
// kernels, where a wave covers 64 consecutive tasks of one item), so the pair
// range is made wave-uniform; the grouped kernel mixes items within a wave.
template <bool UNIFORM>
__device__ __forceinline__ double il_pair_dot(const SpIdx& ix, int id, const double* lv, const double* uv, int TP,
                                              int q, double acc) {
    const int p0 = UNIFORM ? __builtin_amdgcn_readfirstlane(ix.pair_ptr[id]) : ix.pair_ptr[id];
    const int p1 = UNIFORM ? __builtin_amdgcn_readfirstlane(ix.pair_ptr[id + 1]) : ix.pair_ptr[id + 1];
    int p = p0;
    if (p + U8 <= p1) {
        // the next block's pair indices are fetched while this block's values are in flight
        int2 pq[U8];
#pragma unroll
        for (int u = 0; u < U8; ++u) pq[u] = ix.pairs[p + u];
        for (; p + U8 <= p1; p += U8) {
            double a[U8], b[U8];
#pragma unroll
            for (int u = 0; u < U8; ++u) {
                a[u] = lv[(int64_t)pq[u].x * TP + q];
                b[u] = uv[(int64_t)pq[u].y * TP + q];
            }
            if (p + 2 * U8 <= p1) {
#pragma unroll
                for (int u = 0; u < U8; ++u) pq[u] = ix.pairs[p + U8 + u];
            }
#pragma unroll
            for (int u = 0; u < U8; ++u) acc = fmad(-a[u], b[u], acc);
        }
    }
    for (; p < p1; ++p) {
        const int2 pq = ix.pairs[p];
        acc = fmad(-lv[(int64_t)pq.x * TP + q], uv[(int64_t)pq.y * TP + q], acc);
    }
    return acc;
}

// ---- per-item work of the batched execution, shared by the per-level
// kernels and the grouped kernel (q = task index)
__device__ __forceinline__ void il_gather_item(const IlArgs& a, const EpsSet& es, int v, int q) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl;
    double* ud = a.fac;
    double* lv = a.fac + (int64_t)n * a.TP;
    double* uv = lv + (int64_t)nl * a.TP;
    const int s = q / es.K, kk = q % es.K;
    const double* vals = a.values + (int64_t)s * a.nnz;
    if (v < nl) {
        const int sl = ix.src_l[v], su = ix.src_u[v];
        lv[(int64_t)v * a.TP + q] = sl >= 0 ? vals[sl] : 0.0;
        uv[(int64_t)v * a.TP + q] = su >= 0 ? vals[su] : 0.0;
    } else {
        const int j = v - nl;
        const double e = a.scale ? __dmul_rn(eps_at(es, kk), a.scale[s]) : eps_at(es, kk);
        ud[(int64_t)j * a.TP + q] = gather_diag(ix, j, vals, e, a.dvec);
        if (j == 0) a.info[q] = INT_MAX;
    }
}

template <bool UNIFORM>
__device__ __forceinline__ void il_diag_item(const IlArgs& a, int j, int q) {
    const SpIdx& ix = a.ix;
    double* ud = a.fac;
    const double* lv = a.fac + (int64_t)ix.n * a.TP;
    const double* uv = lv + (int64_t)ix.nnzl * a.TP;
    const double u = il_pair_dot<UNIFORM>(ix, j, lv, uv, a.TP, q, ud[(int64_t)j * a.TP + q]);
    ud[(int64_t)j * a.TP + q] = u;
    if (bad_pivot(u)) atomicMin(&a.info[q], j + 1);
}

template <bool UNIFORM>
__device__ __forceinline__ void il_offdiag_item(const IlArgs& a, int p0, int np, int it, int q) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl;
    const double* ud = a.fac;
    double* lv = a.fac + (int64_t)n * a.TP;
    double* uv = lv + (int64_t)nl * a.TP;
    const bool is_l = it >= np;
    const int t = ix.lpos[p0 + (is_l ? it - np : it)];
    const int64_t o = (int64_t)t * a.TP + q;
    if (!is_l) {
        uv[o] = il_pair_dot<UNIFORM>(ix, n + t, lv, uv, a.TP, q, uv[o]);
    } else {
        const int j = ix.col_of[t];
        lv[o] = il_pair_dot<UNIFORM>(ix, n + nl + t, lv, uv, a.TP, q, lv[o]) / ud[(int64_t)j * a.TP + q];
    }
}

__device__ __forceinline__ void il_rhs_item(const IlArgs& a, int v, int q) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nrhs = a.nrhs;
    const int s = q / a.K, i = v / nrhs, r = v % nrhs;
    a.y[(int64_t)v * a.TP + q] = a.B[((int64_t)s * n + ix.perm[i]) * nrhs + r];
}

template <int UPPER>
__device__ __forceinline__ void il_solve_item(const IlArgs& a, int i, int r, int q, int sparse_only = 0) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, nrhs = a.nrhs, TP = a.TP;
    const double* ud = a.fac;
    const double* lv = a.fac + (int64_t)n * TP;
    const double* uv = lv + (int64_t)nl * TP;
    double* y = a.y;
    double acc = y[((int64_t)i * nrhs + r) * TP + q];
    if (!UPPER) {
        const int p1 = ix.r_ptr[i + 1];
        int p = ix.r_ptr[i];
        if (p + U8 <= p1) {
            int ip[U8], iy[U8];
#pragma unroll
            for (int u = 0; u < U8; ++u) {
                ip[u] = ix.r_pos[p + u];
                iy[u] = ix.r_idx[p + u];
            }
            for (; p + U8 <= p1; p += U8) {
                double x[U8], z[U8];
#pragma unroll
                for (int u = 0; u < U8; ++u) {
                    x[u] = lv[(int64_t)ip[u] * TP + q];
                    z[u] = y[((int64_t)iy[u] * nrhs + r) * TP + q];
                }
                if (p + 2 * U8 <= p1) {
#pragma unroll
                    for (int u = 0; u < U8; ++u) {
                        ip[u] = ix.r_pos[p + U8 + u];
                        iy[u] = ix.r_idx[p + U8 + u];
                    }
                }
#pragma unroll
                for (int u = 0; u < U8; ++u) acc = fmad(-x[u], z[u], acc);
            }
        }
        for (; p < p1; ++p)
            acc = fmad(-lv[(int64_t)ix.r_pos[p] * TP + q], y[((int64_t)ix.r_idx[p] * nrhs + r) * TP + q], acc);
    } else {
        const int t0 = ix.l_ptr[i];
        int t = (sparse_only ? t0 + ix.tail_ccnt[i] : ix.l_ptr[i + 1]) - 1;
        if (t - U8 + 1 >= t0) {
            int iy[U8];
#pragma unroll
            for (int u = 0; u < U8; ++u) iy[u] = ix.l_idx[t - u];
            for (; t - U8 + 1 >= t0; t -= U8) {
                double x[U8], z[U8];
#pragma unroll
                for (int u = 0; u < U8; ++u) {
                    x[u] = uv[(int64_t)(t - u) * TP + q];
                    z[u] = y[((int64_t)iy[u] * nrhs + r) * TP + q];
                }
                if (t - 2 * U8 + 1 >= t0) {
#pragma unroll
                    for (int u = 0; u < U8; ++u) iy[u] = ix.l_idx[t - U8 - u];
                }
#pragma unroll
                for (int u = 0; u < U8; ++u) acc = fmad(-x[u], z[u], acc);
            }
        }
        for (; t >= t0; --t)
            acc = fmad(-uv[(int64_t)t * TP + q], y[((int64_t)ix.l_idx[t] * nrhs + r) * TP + q], acc);
        acc = acc / ud[(int64_t)i * TP + q];
    }
    y[((int64_t)i * nrhs + r) * TP + q] = acc;
}

// Positions [0, npos) of L and U and diagonal entries [0, ndiag) (all of them: nnzl and n; below
// a dense trailing block only its columns' positions and diagonal, the block being gathered on
// its own).
__global__ void il_gather_kernel(IlArgs a, EpsSet es, int npos, int ndiag) {
    const int64_t total = (int64_t)(npos + ndiag) * a.TP;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(g % a.TP), v = (int)(g / a.TP);
        if (q < a.ntasks) il_gather_item(a, es, v < npos ? v : a.ix.nnzl + (v - npos), q);
    }
}

__global__ void il_diag_kernel(IlArgs a, int c0, int cnt) {
    const int64_t total = (int64_t)cnt * a.TP;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(g % a.TP);
        if (q < a.ntasks) il_diag_item<true>(a, a.ix.lev_idx[0][c0 + (int)(g / a.TP)], q);
    }
}

__global__ void il_offdiag_kernel(IlArgs a, int p0, int np) {
    const int64_t total = (int64_t)2 * np * a.TP;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(g % a.TP);
        if (q < a.ntasks) il_offdiag_item<true>(a, p0, np, (int)(g / a.TP), q);
    }
}

__global__ void il_rhs_in_kernel(IlArgs a) {
    const int64_t total = (int64_t)a.ix.n * a.nrhs * a.TP;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(g % a.TP), v = (int)(g / a.TP);
        if (q >= a.ntasks) continue;
        if (v == 0 && a.info[q] == INT_MAX) a.info[q] = 0;
        il_rhs_item(a, v, q);
    }
}

template <int UPPER>
__global__ void il_solve_level_kernel(IlArgs a, const int32_t* lev_idx, int c0, int cnt, int sparse_only) {
    const int nrhs = a.nrhs;
    const int64_t total = (int64_t)cnt * nrhs * a.TP;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(g % a.TP), v = (int)(g / a.TP);
        if (q < a.ntasks) il_solve_item<UPPER>(a, lev_idx[c0 + v / nrhs], v % nrhs, q, sparse_only);
    }
}

// Grouped execution: workgroup g owns tasks [g*GS, g*GS + GS) and walks every
// level of the factorisation and both substitutions itself, with workgroup
// barriers between phases instead of kernel boundaries.  Lane l serves task
// g*GS + l%GS; the 64/GS lane groups of a wave and the waves of the
// workgroup share out the items of a phase.
template <int GS>
__global__ __launch_bounds__(512) void il_group_kernel(IlArgs a, EpsSet es) {
    const SpIdx& ix = a.ix;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = wave * (64 / GS) + lane / GS;
    const int nslot = (blockDim.x >> 6) * (64 / GS);
    const int q = blockIdx.x * GS + lane % GS;
    const bool act = q < a.ntasks;
    const int n = ix.n, nl = ix.nnzl, nrhs = a.nrhs;
    for (int v = slot; v < n + nl; v += nslot)
        if (act) il_gather_item(a, es, v, q);
    __syncthreads();
    for (int l = 0; l < ix.nlev[0]; ++l) {
        const int c0 = ix.lev_ptr[0][l], cnt = ix.lev_ptr[0][l + 1] - c0;
        for (int ci = slot; ci < cnt; ci += nslot)
            if (act) il_diag_item<GS == 64>(a, ix.lev_idx[0][c0 + ci], q);
        __syncthreads();
        const int p0 = ix.lpos_ptr[l], np = ix.lpos_ptr[l + 1] - p0;
        for (int it = slot; it < 2 * np; it += nslot)
            if (act) il_offdiag_item<GS == 64>(a, p0, np, it, q);
        __syncthreads();
    }
    if (act && slot == 0 && a.info[q] == INT_MAX) a.info[q] = 0;
    for (int v = slot; v < n * nrhs; v += nslot)
        if (act) il_rhs_item(a, v, q);
    __syncthreads();
    for (int l = 0; l < ix.nlev[1]; ++l) {
        const int c0 = ix.lev_ptr[1][l], cnt = ix.lev_ptr[1][l + 1] - c0;
        for (int t = slot; t < cnt * nrhs; t += nslot)
            if (act) il_solve_item<0>(a, ix.lev_idx[1][c0 + t / nrhs], t % nrhs, q);
        __syncthreads();
    }
    for (int l = 0; l < ix.nlev[2]; ++l) {
        const int c0 = ix.lev_ptr[2][l], cnt = ix.lev_ptr[2][l + 1] - c0;
        for (int t = slot; t < cnt * nrhs; t += nslot)
            if (act) il_solve_item<1>(a, ix.lev_idx[2][c0 + t / nrhs], t % nrhs, q);
        __syncthreads();
    }
}

// X[s][perm[i]][r] = sum_k c_k x_(s,k)[i][r], ascending k; NaN for a broken-down system
__global__ void il_combine_kernel(IlArgs a, EpsSet es) {
    const SpIdx& ix = a.ix;
    const int n = ix.n, nrhs = a.nrhs;
    const int64_t total = (int64_t)a.batch * n * nrhs;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(g / ((int64_t)n * nrhs)), v = (int)(g % ((int64_t)n * nrhs));
        const int i = v / nrhs, r = v % nrhs;
        double acc = 0.0;
        for (int k = 0; k < es.K; ++k) {
            const int q = s * es.K + k;
            const double x = a.info[q] ? __builtin_nan("") : a.y[(int64_t)v * a.TP + q];
            if (a.Xk) a.Xk[((int64_t)q * n + ix.perm[i]) * nrhs + r] = x;
            acc = fmad(c_at(es, k), x, acc);
        }
        a.X[((int64_t)s * n + ix.perm[i]) * nrhs + r] = acc;
    }
}

int grid_for(int64_t items, int threads) {
    int64_t g = (items + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

int64_t lds_bytes(const Symbolic& s, int nrhs) {
    return ((int64_t)s.n + 2 * (int64_t)s.l_ptr[s.n] + (int64_t)s.n * nrhs) * 8;
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

int64_t tail_ld_of(const Symbolic& s) { return s.tail_n ? (s.tail_n + NB - 1) / NB * NB : 0; }

// doubles of one system's factors: [u_jj | L | U] rounded to 32, then (dense trailing block) the
// block, its right-hand-side scratch (tail_ld x 64) and the L and U panels of the tile-pair
// assembly
int64_t fbase_of(const Symbolic& s) { return (s.n + 2 * (int64_t)s.l_ptr[s.n] + 31) / 32 * 32; }
// doubles of one panel set of the tile-pair assembly (0: none)
int64_t tail_panel_of(const Symbolic& s) {
    return s.tail_tiles ? (16 * ((int64_t)s.tail_kt.size() + s.tail_tiles) + 31) / 32 * 32 : 0;
}
int64_t dstride_of(const Symbolic& s) {
    const int64_t ld = tail_ld_of(s);
    return ld * ld + ld * 64 + 2 * tail_panel_of(s);
}
int64_t fstride_of(const Symbolic& s) { return fbase_of(s) + dstride_of(s); }

int64_t tp_of(int64_t ntasks) { return (ntasks + 63) / 64 * 64; }

bool pairs_ok(const Symbolic& s) { return (s.flops_sparse - s.l_ptr[s.n]) / 2 <= kMaxPairs; }

// Fused-call variant: many systems -> interleaved batched kernels; a small
// fill -> one workgroup per system in LDS; otherwise per-level kernels over
// task-major factors.  `forced` (a kVar value, or -1) selects one explicitly;
// an impossible choice returns -1.
int variant_of(const Symbolic& s, int64_t ntasks, int32_t nrhs, int forced) {
    if (forced == kVarLds) return sparse_fits_lds(s, nrhs) ? kVarLds : -1;
    if (forced == kVarBatched) return pairs_ok(s) ? kVarBatched : -1;
    if (forced == kVarGrouped) return pairs_ok(s) ? kVarGrouped : -1;
    if (forced == kVarGlobal) return kVarGlobal;
    if (forced == kVarSteps) return steps_fit(s, nrhs) ? kVarSteps : -1;
    if (forced == kVarTail) return s.tail_n > 0 ? kVarTail : -1;
    if (ntasks >= 256 && pairs_ok(s) && s.tail_n == 0) return kVarBatched;
    if (sparse_fits_lds(s, nrhs)) return kVarLds;
    return s.tail_n > 0 ? kVarTail : kVarGlobal;
}

// workspace, keep = 0:
//   LDS      [ Xk (ntasks x n x nrhs) ]
//   global   [ factors (ntasks x fstride) | y (ntasks x n x nrhs) | Xk ]
//   batched  [ factors ((n + 2 nnzl) x TP) | y ((n nrhs) x TP) ]
// keep = 1:  [ factors (ntasks x fstride) | y (ntasks x n x nrhs) ]
struct SpLayout {
    int64_t off_fac, off_y, off_xk, total;
};

SpLayout sp_layout(const Symbolic& s, int32_t batch, int32_t K, int32_t nrhs, int32_t keep, int forced = -1) {
    const int64_t ntasks = (int64_t)batch * K;
    SpLayout L{};
    L.off_fac = 0;
    int var = keep ? kVarGlobal : variant_of(s, ntasks, nrhs, forced);
    if (var < 0) var = kVarGlobal;
    if (var == kVarBatched || var == kVarGrouped) {
        const int64_t TP = tp_of(ntasks);
        L.off_y = align256(((int64_t)s.n + 2 * (int64_t)s.l_ptr[s.n]) * TP * 8);
        L.off_xk = align256(L.off_y + (int64_t)s.n * nrhs * TP * 8);
        L.total = L.off_xk;
        return L;
    }
    const bool lds = var == kVarLds || var == kVarSteps;
    int64_t off = lds ? 0 : align256(ntasks * fstride_of(s) * 8);
    if (var == kVarTail && !keep) {
        // the interleaved form of the fused call: [ factors ((n + 2 nnzl) x TP) | blocks | y ((n nrhs) x TP) ]
        const int64_t TP = tp_of(ntasks);
        const int64_t il = align256(align256(align256(((int64_t)s.n + 2 * (int64_t)s.l_ptr[s.n]) * TP * 8) +
                                             ntasks * dstride_of(s) * 8) + (int64_t)s.n * nrhs * TP * 8);
        L.total = std::max<int64_t>(il, align256(off + 2 * ntasks * (int64_t)s.n * nrhs * 8));
    }
    L.off_y = off;
    if (!lds) off = align256(off + ntasks * (int64_t)s.n * nrhs * 8);
    L.off_xk = off;
    if (!keep) off = align256(off + ntasks * (int64_t)s.n * nrhs * 8);
    L.total = std::max<int64_t>(std::max<int64_t>(off, 256), L.total);
    return L;
}

hipError_t batched_run(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values, const EpsSet& es,
                       const double* dvec, int32_t nrhs, const double* B, double* X, int32_t* info, char* w,
                       const SpLayout& L, hipStream_t st, bool grouped) {
    IlArgs a{};
    a.ix = d.idx;
    a.nnz = s.nnz; a.nrhs = nrhs; a.ntasks = batch * es.K; a.TP = (int32_t)tp_of(a.ntasks); a.K = es.K;
    a.batch = batch; a.values = values; a.dvec = dvec; a.B = B; a.X = X; a.info = info;
    a.fac = (double*)(w + L.off_fac);
    a.y = (double*)(w + L.off_y);
    const int n = s.n, nl = s.l_ptr[n];
    if (grouped) {
        constexpr int GS = 32;
        hipLaunchKernelGGL(il_group_kernel<GS>, dim3((a.ntasks + GS - 1) / GS), dim3(512), 0, st, a, es);
        hipLaunchKernelGGL(il_combine_kernel, dim3(grid_for((int64_t)batch * n * nrhs, kThreads)), dim3(kThreads), 0, st,
                           a, es);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(il_gather_kernel, dim3(grid_for((int64_t)(n + nl) * a.TP, kThreads)), dim3(kThreads), 0, st, a, es,
                       nl, n);
    for (int l = 0; l < a.ix.nlev[0]; ++l) {
        const int c0 = d.h_lev_ptr[0][l], cnt = d.h_lev_ptr[0][l + 1] - c0;
        hipLaunchKernelGGL(il_diag_kernel, dim3(grid_for((int64_t)cnt * a.TP, kThreads)), dim3(kThreads), 0, st, a, c0, cnt);
        const int p0 = d.h_lpos_ptr[l], np = d.h_lpos_ptr[l + 1] - p0;
        if (np > 0)
            hipLaunchKernelGGL(il_offdiag_kernel, dim3(grid_for((int64_t)2 * np * a.TP, kThreads)), dim3(kThreads), 0, st,
                               a, p0, np);
    }
    hipLaunchKernelGGL(il_rhs_in_kernel, dim3(grid_for((int64_t)n * nrhs * a.TP, kThreads)), dim3(kThreads), 0, st, a);
    for (int l = 0; l < a.ix.nlev[1]; ++l) {
        const int c0 = d.h_lev_ptr[1][l], cnt = d.h_lev_ptr[1][l + 1] - c0;
        hipLaunchKernelGGL(il_solve_level_kernel<0>, dim3(grid_for((int64_t)cnt * nrhs * a.TP, kThreads)),
                           dim3(kThreads), 0, st, a, a.ix.lev_idx[1], c0, cnt, 0);
    }
    for (int l = 0; l < a.ix.nlev[2]; ++l) {
        const int c0 = d.h_lev_ptr[2][l], cnt = d.h_lev_ptr[2][l + 1] - c0;
        hipLaunchKernelGGL(il_solve_level_kernel<1>, dim3(grid_for((int64_t)cnt * nrhs * a.TP, kThreads)),
                           dim3(kThreads), 0, st, a, a.ix.lev_idx[2], c0, cnt, 0);
    }
    hipLaunchKernelGGL(il_combine_kernel, dim3(grid_for((int64_t)batch * n * nrhs, kThreads)), dim3(kThreads), 0, st, a,
                       es);
    return hipGetLastError();
}

SpArgs make_args(const SparseDevice& d, const Symbolic& s, int32_t ntasks, int32_t K, int32_t nrhs) {
    SpArgs a{};
    a.ix = d.idx;
    a.nnz = s.nnz;
    a.nrhs = nrhs;
    a.ntasks = ntasks;
    a.K = K;
    a.fstride = fstride_of(s);
    return a;
}

hipError_t factor_global(const SparseDevice& d, SpArgs a, const EpsSet& es, hipStream_t st) {
    hipLaunchKernelGGL(sp_gather_kernel, dim3(grid_for((int64_t)(a.ix.n + a.ix.nnzl) * a.ntasks, kThreads)),
                       dim3(kThreads), 0, st, a, es);
    for (int l = 0; l < a.ix.nlev[0]; ++l) {
        const int c0 = d.h_lev_ptr[0][l], cnt = d.h_lev_ptr[0][l + 1] - c0;
        hipLaunchKernelGGL(sp_diag_kernel, dim3(grid_for((int64_t)cnt * a.ntasks, kThreads)), dim3(kThreads), 0, st,
                           a, c0, cnt);
        const int p0 = d.h_lpos_ptr[l], np = d.h_lpos_ptr[l + 1] - p0;
        if (np > 0)
            hipLaunchKernelGGL(sp_offdiag_kernel, dim3(grid_for((int64_t)2 * np * a.ntasks, kThreads)), dim3(kThreads),
                               0, st, a, p0, np);
    }
    hipLaunchKernelGGL(sp_info_kernel, dim3((a.ntasks + 255) / 256), dim3(256), 0, st, a.info, a.ntasks);
    return hipGetLastError();
}

// Task-major addressing of the dense-block kernels: each system's block inside its factors.
void tail_task_major(SpArgs& a) {
    a.vs = 1;
    a.ts = a.fstride;
    a.dense = a.fac + a.ix.tail_off;
    a.dstride = a.fstride;
    a.yv = 1;
    a.yt = (int64_t)a.ix.n * a.nrhs;
}

// One workgroup per system for the block's LU and solves (a tuning choice: at n = 2709 and 550
// systems the per-panel launches across the device are faster).
bool tail_slot(const Knobs& kn, int64_t) { return kn.tail_lu == 1; }

// Assembly and LU of every system's dense block, the factors below it done (any addressing; the
// column-wise assembly only task-major).
hipError_t tail_dense_factor(SpArgs a, const EpsSet& es, hipStream_t st, int cols, bool slot) {
    const int ld = a.ix.tail_ld;
    if (cols == 16 && a.ix.tail_tiles > 0) {
        if (!a.values) return hipErrorInvalidValue;   // the block's initial values come from the Jacobians
        hipLaunchKernelGGL(tail_block_init_kernel, dim3((unsigned)std::min(ld, 65535), (unsigned)std::min(a.ntasks, 65535)), dim3(256),
                           0, st, a, es);
        if (a.vs == 1) {
            hipLaunchKernelGGL(tail_panel_gather_kernel, dim3(grid_for(a.ix.tail_panel * a.ntasks, kThreads)),
                               dim3(kThreads), 0, st, a);
        } else {
            const int64_t ech = (a.ix.tail_panel + 63) / 64, tch = (a.ntasks + 63) / 64;
            if (ech * tch > INT32_MAX) return hipErrorInvalidValue;
            hipLaunchKernelGGL(tail_panel_gather_il_kernel, dim3((unsigned)(ech * tch)), dim3(256), 0, st, a, (int)ech);
        }
        const int64_t items = (int64_t)a.ix.tail_tiles * a.ix.tail_tiles * a.ntasks;
        const int64_t wgs = (items + kTpWaves - 1) / kTpWaves;
        if ((wgs + 7) / 8 * 8 > INT32_MAX) return hipErrorInvalidValue;
        const int64_t litems = (int64_t)a.ix.tail_nlpairs * a.ntasks;
        const int lwgs = (int)((std::min<int64_t>(litems, 1 << 16) + 7) / 8 * 8);
        hipLaunchKernelGGL(tail_tile_kernel, dim3((unsigned)((wgs + 7) / 8 * 8 + lwgs)), dim3(64 * kTpWaves), 0, st, a,
                           items, lwgs);
    } else {
        if (a.vs != 1) return hipErrorInvalidValue;
        cols = cols == 1 ? 1 : kAsmCols;
        hipLaunchKernelGGL(tail_assemble_kernel, dim3((int)std::min<int64_t>((int64_t)(ld / cols) * a.ntasks, 1 << 20)),
                           dim3(kAsmThreads), (int)tail_asm_lds(a.ix.tail_b0), st, a, cols);
    }
    if (slot) {
        hipLaunchKernelGGL(tail_lu_slot_kernel, dim3(std::min(a.ntasks, 65535)), dim3(WGD), kLdsFused, st, a);
        return hipGetLastError();
    }
    for (int p0 = 0; p0 < ld; p0 += NB) {
        const int rest = ld - p0 - NB;
        hipLaunchKernelGGL(tail_getrf_kernel, dim3(std::min(a.ntasks, 65535)), dim3(64), 0, st, a, p0);
        if (rest > 0) {
            const int chunks = (2 * rest + kTrsmThreads - 1) / kTrsmThreads;
            hipLaunchKernelGGL(tail_trsm_kernel, dim3((int)std::min<int64_t>((int64_t)chunks * a.ntasks, 65535)),
                               dim3(kTrsmThreads), 0, st, a, p0, chunks);
        }
        const int rem = rest;
        if (rem > 0) {
            const int tr = (rem + 127) / 128, tc = (rem + 63) / 64;
            const int64_t blocks = (int64_t)tr * tc * a.ntasks;
            hipLaunchKernelGGL(tail_update_kernel, dim3((int)std::min<int64_t>(blocks, 65535)), dim3(WG), 0, st, a, p0,
                               tr, tc);
        }
    }
    return hipGetLastError();
}

hipError_t factor_tail(const SparseDevice& d, SpArgs a, const EpsSet& es, hipStream_t st, const Knobs& kn = Knobs()) {
    tail_task_major(a);
    hipLaunchKernelGGL(sp_gather_kernel, dim3(grid_for((int64_t)(a.ix.n + a.ix.nnzl) * a.ntasks, kThreads)),
                       dim3(kThreads), 0, st, a, es);
    for (int l = 0; l < a.ix.fac_lev_sp; ++l) {
        const int c0 = d.h_lev_ptr[0][l], cnt = d.h_lev_ptr[0][l + 1] - c0;
        hipLaunchKernelGGL(sp_diag_kernel, dim3(grid_for((int64_t)cnt * a.ntasks, kThreads)), dim3(kThreads), 0, st,
                           a, c0, cnt);
        const int p0 = d.h_lpos_ptr[l], np = d.h_lpos_ptr[l + 1] - p0;
        if (np > 0)
            hipLaunchKernelGGL(sp_offdiag_kernel, dim3(grid_for((int64_t)2 * np * a.ntasks, kThreads)), dim3(kThreads),
                               0, st, a, p0, np);
    }
    hipError_t e = tail_dense_factor(a, es, st, kn.tail_cols, tail_slot(kn, a.ntasks));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sp_info_kernel, dim3((a.ntasks + 255) / 256), dim3(256), 0, st, a.info, a.ntasks);
    return hipGetLastError();
}

// The block rows of the substitutions: their updates from the sparse part, the block's own
// triangular solves, then the block's terms of the backward chains of the rows before it (any
// addressing).
hipError_t tail_dense_solve(SpArgs a, hipStream_t st, bool slot) {
    const int64_t trows = (int64_t)a.ix.tail_n * a.nrhs * a.ntasks;
    const int64_t tpad = (int64_t)a.ix.tail_ld * a.nrhs * a.ntasks;
    if (a.trans)
        hipLaunchKernelGGL(tail_fwd_ext_kernel<1>, dim3(grid_for(trows, kExtThreads)), dim3(kExtThreads), 0, st, a);
    else
        hipLaunchKernelGGL(tail_fwd_ext_kernel<0>, dim3(grid_for(trows, kExtThreads)), dim3(kExtThreads), 0, st, a);
    const int64_t lchains = (int64_t)a.ix.tail_nlong * a.nrhs * a.ntasks;
    if (lchains > 0) {
        const dim3 lg((unsigned)std::min<int64_t>(lchains, 1 << 20));
        if (a.trans)
            hipLaunchKernelGGL(tail_fwd_long_kernel<1>, lg, dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL(tail_fwd_long_kernel<0>, lg, dim3(64), 0, st, a);
    }
    hipLaunchKernelGGL(tail_rhs_in_kernel, dim3(grid_for(tpad, kThreads)), dim3(kThreads), 0, st, a);
    if (slot) {
        const dim3 g(std::min(a.ntasks, 65535));
        if (a.trans) {
            hipLaunchKernelGGL((tail_tri_slot_kernel<1, 1>), g, dim3(WG), kLdsSolve, st, a);
            hipLaunchKernelGGL((tail_tri_slot_kernel<0, 1>), g, dim3(WG), kLdsSolve, st, a);
        } else {
            hipLaunchKernelGGL((tail_tri_slot_kernel<1, 0>), g, dim3(WG), kLdsSolve, st, a);
            hipLaunchKernelGGL((tail_tri_slot_kernel<0, 0>), g, dim3(WG), kLdsSolve, st, a);
        }
    } else {
        hipError_t e = a.trans ? tail_tri<1, 1>(a, st) : tail_tri<1, 0>(a, st);
        if (e != hipSuccess) return e;
        e = a.trans ? tail_tri<0, 1>(a, st) : tail_tri<0, 0>(a, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(tail_rhs_out_kernel, dim3(grid_for(trows, kThreads)), dim3(kThreads), 0, st, a);
    const int64_t srows = (int64_t)a.ix.tail_b0 * a.nrhs * a.ntasks;
    if (a.trans)
        hipLaunchKernelGGL(tail_bwd_ext_kernel<1>, dim3(grid_for(srows, kThreads)), dim3(kThreads), 0, st, a);
    else
        hipLaunchKernelGGL(tail_bwd_ext_kernel<0>, dim3(grid_for(srows, kThreads)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t solve_tail(const SparseDevice& d, SpArgs a, hipStream_t st, const Knobs& kn = Knobs()) {
    tail_task_major(a);
    const int64_t items = (int64_t)a.ix.n * a.nrhs * a.ntasks;
    hipLaunchKernelGGL(sp_rhs_in_kernel, dim3(grid_for(items, kThreads)), dim3(kThreads), 0, st, a);
    for (int l = 0; l < a.ix.nlev_sp[0]; ++l) {
        const int c0 = d.h_lev_sp_ptr[0][l], cnt = d.h_lev_sp_ptr[0][l + 1] - c0;
        hipLaunchKernelGGL(sp_solve_level_kernel<0>, dim3(grid_for((int64_t)cnt * a.nrhs * a.ntasks, kThreads)),
                           dim3(kThreads), 0, st, a, a.ix.lev_sp_idx[0], c0, cnt, 0);
    }
    hipError_t e = tail_dense_solve(a, st, tail_slot(kn, a.ntasks));
    if (e != hipSuccess) return e;
    for (int l = 0; l < a.ix.nlev_sp[1]; ++l) {
        const int c0 = d.h_lev_sp_ptr[1][l], cnt = d.h_lev_sp_ptr[1][l + 1] - c0;
        hipLaunchKernelGGL(sp_solve_level_kernel<1>, dim3(grid_for((int64_t)cnt * a.nrhs * a.ntasks, kThreads)),
                           dim3(kThreads), 0, st, a, a.ix.lev_sp_idx[1], c0, cnt, 1);
    }
    hipLaunchKernelGGL(sp_rhs_out_kernel, dim3(grid_for(items, kThreads)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

// The fused call on the dense-block path with the systems interleaved below the block (the
// batched kernels' layout: a wave serves one item of 64 systems, index loads uniform, value
// loads contiguous), each system's block task-major in a region of its own.
// The interleaved form needs the pair lists below the block and the tile-pair assembly; by
// default it is taken for 64 systems or more.
bool tail_il_ok(const Symbolic& s, const SparseDevice& d, int64_t ntasks, const Knobs& kn) {
    if (!d.idx.use_pairs || d.idx.pairs_below < s.tail_b0 || d.idx.tail_tiles == 0 || kn.tail_cols != 16) return false;
    return kn.tail_il < 0 ? ntasks >= 64 : kn.tail_il == 1;
}

hipError_t tail_il_run(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                       const EpsSet& es, const double* dvec, int32_t nrhs, const double* B, double* X, int32_t* info,
                       char* w, hipStream_t st, const Knobs& kn, double* Xk = nullptr, const double* scale = nullptr) {
    if (!d.idx.use_pairs || d.idx.pairs_below < s.tail_b0 || d.idx.tail_tiles == 0) return hipErrorInvalidValue;
    IlArgs ia{};
    ia.ix = d.idx;
    ia.nnz = s.nnz; ia.nrhs = nrhs; ia.ntasks = batch * es.K; ia.TP = (int32_t)tp_of(ia.ntasks); ia.K = es.K;
    ia.batch = batch; ia.values = values; ia.dvec = dvec; ia.B = B; ia.X = X; ia.info = info;
    ia.Xk = Xk;
    ia.scale = scale;
    const int n = s.n, nl = s.l_ptr[n];
    const int64_t off_dense = align256(((int64_t)n + 2 * (int64_t)nl) * ia.TP * 8);
    const int64_t off_y = align256(off_dense + (int64_t)ia.ntasks * dstride_of(s) * 8);
    ia.fac = (double*)w;
    ia.y = (double*)(w + off_y);
    const int npos = s.l_ptr[s.tail_b0];
    hipLaunchKernelGGL(il_gather_kernel, dim3(grid_for((int64_t)(npos + s.tail_b0) * ia.TP, kThreads)), dim3(kThreads), 0,
                       st, ia, es, npos, s.tail_b0);
    for (int l = 0; l < ia.ix.fac_lev_sp; ++l) {
        const int c0 = d.h_lev_ptr[0][l], cnt = d.h_lev_ptr[0][l + 1] - c0;
        hipLaunchKernelGGL(il_diag_kernel, dim3(grid_for((int64_t)cnt * ia.TP, kThreads)), dim3(kThreads), 0, st, ia, c0,
                           cnt);
        const int p0 = d.h_lpos_ptr[l], np = d.h_lpos_ptr[l + 1] - p0;
        if (np > 0)
            hipLaunchKernelGGL(il_offdiag_kernel, dim3(grid_for((int64_t)2 * np * ia.TP, kThreads)), dim3(kThreads), 0, st,
                               ia, p0, np);
    }
    SpArgs a = make_args(d, s, ia.ntasks, es.K, nrhs);
    a.values = values;
    a.dvec = dvec;
    a.B = B;
    a.info = info;
    a.scale = scale;
    a.fac = ia.fac;
    a.vs = ia.TP;
    a.ts = 1;
    a.dense = (double*)(w + off_dense);
    a.dstride = dstride_of(s);
    a.y = ia.y;
    a.yv = ia.TP;
    a.yt = 1;
    const bool slot = tail_slot(kn, a.ntasks);
    hipError_t e = tail_dense_factor(a, es, st, 16, slot);
    if (e != hipSuccess) return e;
    // clears the unbroken systems' info (the gather's INT_MAX) before anything reads it
    hipLaunchKernelGGL(il_rhs_in_kernel, dim3(grid_for((int64_t)n * nrhs * ia.TP, kThreads)), dim3(kThreads), 0, st, ia);
    for (int l = 0; l < ia.ix.nlev_sp[0]; ++l) {
        const int c0 = d.h_lev_sp_ptr[0][l], cnt = d.h_lev_sp_ptr[0][l + 1] - c0;
        hipLaunchKernelGGL(il_solve_level_kernel<0>, dim3(grid_for((int64_t)cnt * nrhs * ia.TP, kThreads)),
                           dim3(kThreads), 0, st, ia, ia.ix.lev_sp_idx[0], c0, cnt, 0);
    }
    e = tail_dense_solve(a, st, slot);
    if (e != hipSuccess) return e;
    for (int l = 0; l < ia.ix.nlev_sp[1]; ++l) {
        const int c0 = d.h_lev_sp_ptr[1][l], cnt = d.h_lev_sp_ptr[1][l + 1] - c0;
        hipLaunchKernelGGL(il_solve_level_kernel<1>, dim3(grid_for((int64_t)cnt * nrhs * ia.TP, kThreads)),
                           dim3(kThreads), 0, st, ia, ia.ix.lev_sp_idx[1], c0, cnt, 1);
    }
    hipLaunchKernelGGL(il_combine_kernel, dim3(grid_for((int64_t)batch * n * nrhs, kThreads)), dim3(kThreads), 0, st, ia,
                       es);
    return hipGetLastError();
}

hipError_t solve_global(const SparseDevice& d, SpArgs a, hipStream_t st) {
    const int64_t items = (int64_t)a.ix.n * a.nrhs * a.ntasks;
    hipLaunchKernelGGL(sp_rhs_in_kernel, dim3(grid_for(items, kThreads)), dim3(kThreads), 0, st, a);
    // forward pass uses the L-solve levels, backward pass the U-solve levels (both for the transposed solve)
    for (int l = 0; l < a.ix.nlev[1]; ++l) {
        const int c0 = d.h_lev_ptr[1][l], cnt = d.h_lev_ptr[1][l + 1] - c0;
        hipLaunchKernelGGL(sp_solve_level_kernel<0>, dim3(grid_for((int64_t)cnt * a.nrhs * a.ntasks, kThreads)),
                           dim3(kThreads), 0, st, a, a.ix.lev_idx[1], c0, cnt, 0);
    }
    for (int l = 0; l < a.ix.nlev[2]; ++l) {
        const int c0 = d.h_lev_ptr[2][l], cnt = d.h_lev_ptr[2][l + 1] - c0;
        hipLaunchKernelGGL(sp_solve_level_kernel<1>, dim3(grid_for((int64_t)cnt * a.nrhs * a.ntasks, kThreads)),
                           dim3(kThreads), 0, st, a, a.ix.lev_idx[2], c0, cnt, 0);
    }
    hipLaunchKernelGGL(sp_rhs_out_kernel, dim3(grid_for(items, kThreads)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

bool sparse_fits_lds(const Symbolic& s, int32_t nrhs) { return lds_bytes(s, nrhs) <= kLdsLimit; }

int sparse_variant(const Symbolic& s, int64_t ntasks, int32_t nrhs, int forced) {
    return variant_of(s, ntasks, nrhs, forced);
}

void sparse_image(const Symbolic& s, PlanImage& img, SparseDevice& d) {
    if (d.imaged) return;
    const int n = s.n, nl = s.l_ptr[n];
    std::vector<int32_t> col_of(nl), r_pos(nl), src_l(nl, -1), src_u(nl, -1), src_d(n, -1);
    for (int j = 0; j < n; ++j)
        for (int t = s.l_ptr[j]; t < s.l_ptr[j + 1]; ++t) col_of[t] = j;
    auto pos_in_col = [&](int col, int row) {
        const int* b = s.l_idx.data() + s.l_ptr[col];
        const int* e = s.l_idx.data() + s.l_ptr[col + 1];
        const int* p = std::lower_bound(b, e, row);
        return (p != e && *p == row) ? (int)(p - s.l_idx.data()) : -1;
    };
    for (int i = 0; i < n; ++i)
        for (int p = s.lrow_ptr[i]; p < s.lrow_ptr[i + 1]; ++p) r_pos[p] = pos_in_col(s.lrow_idx[p], i);
    for (int r = 0; r < n; ++r)
        for (int e = s.row_ptr[r]; e < s.row_ptr[r + 1]; ++e) {
            const int pr = s.iperm[r], pc = s.iperm[s.col_idx[e]];
            if (pr == pc) src_d[pr] = e;
            else if (pr > pc) src_l[pos_in_col(pc, pr)] = e;
            else src_u[pos_in_col(pr, pc)] = e;
        }
    // positions of the columns of each factor level
    const int L0 = (int)s.lev_ptr[0].size() - 1;
    std::vector<int32_t> lpos_ptr(L0 + 1, 0), lpos;
    lpos.reserve(nl);
    for (int l = 0; l < L0; ++l) {
        for (int t = s.lev_ptr[0][l]; t < s.lev_ptr[0][l + 1]; ++t) {
            const int j = s.lev_idx[0][t];
            for (int q = s.l_ptr[j]; q < s.l_ptr[j + 1]; ++q) lpos.push_back(q);
        }
        lpos_ptr[l + 1] = (int32_t)lpos.size();
    }
    // update lists, when the total stays modest: for every item, or (a plan with a dense
    // trailing block whose full lists are too long) for the items of the columns before the block,
    // the only ones its per-level kernels evaluate
    const int64_t npairs_est = (s.flops_sparse - nl) / 2;
    std::vector<int32_t> pair_ptr, pairs;
    int32_t below = npairs_est <= kMaxPairs ? n : (s.tail_n > 0 ? s.tail_b0 : 0);
    if (below > 0) {
        pair_ptr.assign((size_t)n + 2 * (size_t)nl + 1, 0);
        pairs.reserve(2 * (size_t)std::min<int64_t>(std::max<int64_t>(npairs_est, 1), kMaxPairs));
        auto push_merge = [&](int a, int b) {   // pairs (pos(a,k), pos(b,k)) for k in R_a ^ R_b
            int p = s.lrow_ptr[a], pe = s.lrow_ptr[a + 1], q = s.lrow_ptr[b], qe = s.lrow_ptr[b + 1];
            if (pe - p > 8 * (qe - q) || qe - q > 8 * (pe - p)) {
                // very different lengths: look the shorter row's columns up in the longer one
                const bool a_short = pe - p <= qe - q;
                const int* lb = s.lrow_idx.data() + (a_short ? q : p);
                const int* le = s.lrow_idx.data() + (a_short ? qe : pe);
                for (int x = a_short ? p : q; x < (a_short ? pe : qe); ++x) {
                    const int* f = std::lower_bound(lb, le, s.lrow_idx[x]);
                    if (f == le) break;
                    if (*f == s.lrow_idx[x]) {
                        const int y = (int)(f - s.lrow_idx.data());
                        pairs.push_back(r_pos[a_short ? x : y]);
                        pairs.push_back(r_pos[a_short ? y : x]);
                    }
                    lb = f;
                }
                return;
            }
            while (p < pe && q < qe) {
                const int ka = s.lrow_idx[p], kb = s.lrow_idx[q];
                if (ka == kb) { pairs.push_back(r_pos[p]); pairs.push_back(r_pos[q]); ++p; ++q; }
                else if (ka < kb) ++p;
                else ++q;
            }
        };
        int64_t id = 0;
        for (int j = 0; j < n; ++j, ++id) {
            pair_ptr[id] = (int32_t)(pairs.size() / 2);
            if (j < below)
                for (int p = s.lrow_ptr[j]; p < s.lrow_ptr[j + 1]; ++p) { pairs.push_back(r_pos[p]); pairs.push_back(r_pos[p]); }
        }
        for (int t = 0; t < nl; ++t, ++id) {
            pair_ptr[id] = (int32_t)(pairs.size() / 2);
            if (col_of[t] < below) push_merge(col_of[t], s.l_idx[t]);
        }
        for (int t = 0; t < nl; ++t, ++id) {
            pair_ptr[id] = (int32_t)(pairs.size() / 2);
            if (col_of[t] < below) push_merge(s.l_idx[t], col_of[t]);
        }
        pair_ptr[id] = (int32_t)(pairs.size() / 2);
        if ((int64_t)pairs.size() / 2 > kMaxPairs) {
            below = 0;
            pair_ptr.clear();
            pairs.clear();
        }
    }
    const bool use_pairs = below > 0;
    SpIdx& ix = d.idx;
    ix.n = n;
    ix.nnzl = nl;
    img.bind(&ix.perm, img.put(s.perm));
    img.bind(&ix.l_ptr, img.put(s.l_ptr));
    img.bind(&ix.l_idx, img.put(s.l_idx));
    img.bind(&ix.col_of, img.put(col_of));
    img.bind(&ix.r_ptr, img.put(s.lrow_ptr));
    img.bind(&ix.r_idx, img.put(s.lrow_idx));
    img.bind(&ix.r_pos, img.put(r_pos));
    img.bind(&ix.src_l, img.put(src_l));
    img.bind(&ix.src_u, img.put(src_u));
    img.bind(&ix.src_d, img.put(src_d));
    for (int t = 0; t < 3; ++t) {
        img.bind(&ix.lev_ptr[t], img.put(s.lev_ptr[t]));
        img.bind(&ix.lev_idx[t], img.put(s.lev_idx[t]));
        ix.nlev[t] = (int32_t)s.lev_ptr[t].size() - 1;
        d.h_lev_ptr[t] = s.lev_ptr[t];
    }
    img.bind(&ix.lpos_ptr, img.put(lpos_ptr));
    img.bind(&ix.lpos, img.put(lpos));
    ix.use_pairs = use_pairs ? 1 : 0;
    ix.pairs_below = below;
    img.bind(&ix.pair_ptr, img.put(pair_ptr));
    img.bind(&ix.pairs, img.put(pairs));
    d.h_lpos_ptr = lpos_ptr;
    ix.tail_n = s.tail_n;
    ix.tail_b0 = s.tail_b0;
    ix.tail_ld = (int32_t)tail_ld_of(s);
    ix.fac_lev_sp = s.fac_lev_sp;
    ix.tail_off = fbase_of(s);
    {
        std::vector<int32_t> rc(std::max(s.tail_n, 1), 0);
        for (int i = 0; i < s.tail_n; ++i) {
            const int r = s.tail_b0 + i;
            rc[i] = (int32_t)(std::lower_bound(s.lrow_idx.begin() + s.lrow_ptr[r], s.lrow_idx.begin() + s.lrow_ptr[r + 1],
                                               s.tail_b0) - (s.lrow_idx.begin() + s.lrow_ptr[r]));
        }
        img.bind(&ix.tail_rcnt, img.put(rc));
        std::vector<int32_t> lr;
        for (int i = 0; i < s.tail_n; ++i)
            if (rc[i] >= kTailLongRow) lr.push_back(i);
        ix.tail_nlong = (int32_t)lr.size();
        if (lr.empty()) lr.push_back(0);
        img.bind(&ix.tail_long, img.put(lr));
        std::vector<int32_t> lp(std::max(s.tail_b0, 1), -1);
        for (int k = 0; k < s.tail_b0; ++k)
            if (s.l_ptr[k + 1] > s.l_ptr[k] && s.l_idx[s.l_ptr[k + 1] - 1] == n - 1) lp[k] = s.l_ptr[k + 1] - 1;
        img.bind(&ix.tail_lastpos, img.put(lp));
        std::vector<int32_t> cc(std::max(s.tail_b0, 1), 0);
        for (int k = 0; k < s.tail_b0; ++k)
            cc[k] = (int32_t)(std::lower_bound(s.l_idx.begin() + s.l_ptr[k], s.l_idx.begin() + s.l_ptr[k + 1], s.tail_b0) -
                              (s.l_idx.begin() + s.l_ptr[k]));
        img.bind(&ix.tail_ccnt, img.put(cc));
        // tile-pair assembly: panel positions and the pair lists
        const int TT = s.tail_tiles;
        ix.tail_tiles = TT;
        ix.tail_panel = tail_panel_of(s);
        std::vector<int32_t> ktp(TT + 1, 0), mpos(std::max<int64_t>(ix.tail_panel, 1), -1), ppp(1, 0), prs;
        if (TT > 0) {
            for (int t = 0; t <= TT; ++t) ktp[t] = s.tail_kt_ptr[t] + t;
            for (int slot = 0; slot < 16 * TT; ++slot) {
                if (s.tail_rord[slot] < 0) continue;
                const int t = slot / 16, r = slot % 16, row = s.tail_b0 + s.tail_rord[slot];
                const int32_t* K = s.tail_kt.data() + s.tail_kt_ptr[t];
                int c = 0;
                for (int q = s.lrow_ptr[row]; q < s.lrow_ptr[row + 1] && s.lrow_idx[q] < s.tail_b0; ++q) {
                    while (K[c] < s.lrow_idx[q]) ++c;
                    mpos[16 * ((int64_t)ktp[t] + c) + r] = r_pos[q];
                }
            }
            ppp = s.tail_pp_ptr;
            prs = s.tail_pairs;
            d.h_tail_pairs = (int64_t)prs.size();
        }
        if (prs.empty()) prs.push_back(0);
        std::vector<int32_t> rord = TT ? s.tail_rord : std::vector<int32_t>(1, -1);
        img.bind(&ix.tail_rord, img.put(rord));
        img.bind(&ix.tail_kt_ptr, img.put(ktp));
        img.bind(&ix.tail_mpos, img.put(mpos));
        img.bind(&ix.tail_pp_ptr, img.put(ppp));
        img.bind(&ix.tail_pairs, img.put(prs));
        std::vector<int32_t> lpr;
        for (int64_t pi = 0; pi + 1 < (int64_t)ppp.size(); ++pi)
            if ((ppp[pi + 1] - ppp[pi]) / 4 >= kTileLongSteps) lpr.push_back((int32_t)pi);
        ix.tail_nlpairs = TT ? (int32_t)lpr.size() : 0;
        if (lpr.empty()) lpr.push_back(0);
        img.bind(&ix.tail_lpairs, img.put(lpr));
    }
    for (int w = 0; w < 2; ++w) {
        ix.nlev_sp[w] = s.tail_n ? (int32_t)s.lev_sp_ptr[w].size() - 1 : 0;
        img.bind(&ix.lev_sp_ptr[w], img.put(s.lev_sp_ptr[w]));
        img.bind(&ix.lev_sp_idx[w], img.put(s.lev_sp_idx[w]));
        d.h_lev_sp_ptr[w] = s.lev_sp_ptr[w];
    }
    steps_image(s, r_pos, img, d);
    d.imaged = true;
}

hipError_t sparse_kernel_attrs() {
    static hipError_t e = [] {
        hipError_t r = hipFuncSetAttribute((const void*)sparse_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kLdsLimit);
        if (r == hipSuccess)
            r = hipFuncSetAttribute((const void*)tail_assemble_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)tail_asm_lds(kTailAsmMaxB0));
        if (r == hipSuccess)
            r = hipFuncSetAttribute((const void*)tail_lu_slot_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    kLdsFused);
        return r;
    }();
    return e;
}

size_t sparse_workspace_bytes(const Symbolic& s, int32_t batch, int32_t K, int32_t nrhs, int32_t keep, int forced) {
    return (size_t)sp_layout(s, batch, K, nrhs, keep, forced).total;
}

int32_t sparse_nrhs_capacity(const Symbolic& s, int32_t batch, int32_t K, size_t ws_bytes) {
    const SpLayout L = sp_layout(s, batch, K, 0, 1);
    const int64_t per = (int64_t)batch * K * s.n * 8;
    return (int32_t)std::min<int64_t>(64, std::max<int64_t>(0, ((int64_t)ws_bytes - L.off_y) / per));
}

hipError_t sparse_solve_batched(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                                const EpsSet& es, const double* dvec, int32_t nrhs, const double* B, double* X,
                                int32_t* info, void* ws, hipStream_t st, int forced, const Knobs& kn) {
    const int32_t ntasks = batch * es.K;
    const SpLayout L = sp_layout(s, batch, es.K, nrhs, 0, forced);
    char* w = (char*)ws;
    SpArgs a = make_args(d, s, ntasks, es.K, nrhs);
    a.values = values; a.dvec = dvec; a.B = B; a.info = info;
    a.Xk = (double*)(w + L.off_xk);
    int var = variant_of(s, ntasks, nrhs, forced);
    if (var < 0) return hipErrorInvalidValue;
    if (forced < 0 && var != kVarGrouped && nrhs == 1 && steps_ready(d)) {
        // the step schedule beats the per-level launches and the level-scheduled LDS
        // kernel whenever it exists; its Xk (when not fused) fits in the interleaved
        // layout or the LDS variant's Xk reserved above
        var = kVarSteps;
        a.Xk = (double*)w;
    }
    if (var == kVarBatched || var == kVarGrouped)
        return batched_run(s, d, batch, values, es, dvec, nrhs, B, X, info, w, L, st, var == kVarGrouped);
    if (var == kVarSteps) {
        return steps_solve(d, s.n, s.nnz, batch, values, es, dvec, B, X, info, a.Xk, st, kn);
    }
    if (var == kVarLds) {
        const int lds = (int)lds_bytes(s, nrhs);
        hipError_t e = sparse_kernel_attrs();
        if (e != hipSuccess) return e;
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int resident = cus * std::max(1, (160 * 1024) / std::max(lds, 1));
        // Enough Jacobians to fill the GPU: one task per Jacobian, combine fused.
        a.per_jacobian = batch >= resident ? 1 : 0;
        a.batch = batch;
        a.X = X;
        const int grid = std::min(a.per_jacobian ? batch : ntasks, resident);
        hipLaunchKernelGGL(sparse_lds_kernel, dim3(grid), dim3(kLdsThreads), lds, st, a, es, 0);
        e = hipGetLastError();
        if (e != hipSuccess || a.per_jacobian) return e;
    } else {
        const bool tail = var == kVarTail;
        if (tail && tail_il_ok(s, d, ntasks, kn))
            return tail_il_run(s, d, batch, values, es, dvec, nrhs, B, X, info, w, st, kn);
        a.fac = (double*)(w + L.off_fac);
        a.y = (double*)(w + L.off_y);
        hipError_t e = tail ? factor_tail(d, a, es, st, kn) : factor_global(d, a, es, st);
        if (e != hipSuccess) return e;
        e = tail ? solve_tail(d, a, st, kn) : solve_global(d, a, st);
        if (e != hipSuccess) return e;
    }
    return launch_combine((int64_t)s.n * nrhs, batch, es, a.Xk, X, st);
}

bool sparse_tail_adaptive_ok(const Symbolic& s, const SparseDevice& d) {
    return s.tail_n > 0 && d.idx.use_pairs && d.idx.pairs_below >= s.tail_b0 && d.idx.tail_tiles > 0;
}

size_t sparse_tail_run_bytes(const Symbolic& s, int32_t batch, int32_t K) {
    return (size_t)sp_layout(s, batch, K, 1, 0, kVarTail).total;
}

hipError_t sparse_tail_run(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                           const EpsSet& es, const double* dvec, const double* B, double* X, int32_t* info, double* Xk,
                           const double* scale, void* ws, hipStream_t st, const Knobs& kn) {
    if (!sparse_tail_adaptive_ok(s, d)) return hipErrorInvalidValue;
    return tail_il_run(s, d, batch, values, es, dvec, 1, B, X, info, (char*)ws, st, kn, Xk, scale);
}

hipError_t sparse_factor(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                         const EpsSet& es, const double* dvec, int32_t* info, void* ws, hipStream_t st) {
    const int32_t ntasks = batch * es.K;
    const SpLayout L = sp_layout(s, batch, es.K, 0, 1);
    SpArgs a = make_args(d, s, ntasks, es.K, 0);
    a.values = values; a.dvec = dvec; a.info = info;
    a.fac = (double*)((char*)ws + L.off_fac);
    if (s.tail_n > 0) return factor_tail(d, a, es, st);
    if (sparse_fits_lds(s, 0)) {
        const int lds = (int)lds_bytes(s, 0);
        hipError_t e = sparse_kernel_attrs();
        if (e != hipSuccess) return e;
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int grid = std::min(ntasks, cus * std::max(1, (160 * 1024) / std::max(lds, 1)));
        hipLaunchKernelGGL(sparse_lds_kernel, dim3(grid), dim3(kLdsThreads), lds, st, a, es, 1);
        return hipGetLastError();
    }
    return factor_global(d, a, es, st);
}

hipError_t sparse_solve(const Symbolic& s, const SparseDevice& d, int32_t batch, const EpsSet& es, int32_t nrhs,
                        const double* B, double* Xk, int32_t transpose, const int32_t* info, void* ws,
                        hipStream_t st) {
    const int32_t ntasks = batch * es.K;
    const SpLayout L = sp_layout(s, batch, es.K, 0, 1);
    SpArgs a = make_args(d, s, ntasks, es.K, nrhs);
    a.B = B; a.Xk = Xk; a.info = const_cast<int32_t*>(info); a.trans = transpose ? 1 : 0;
    a.fac = (double*)((char*)ws + L.off_fac);
    a.y = (double*)((char*)ws + L.off_y);
    return s.tail_n > 0 ? solve_tail(d, a, st) : solve_global(d, a, st);
}

}  // namespace psp
