// dense.hip -- dense batched pivot-free LU, substitutions and combine for
// gfx950, one workgroup (4 waves) per perturbed system.
//
// Each perturbed system P (A_s + eps_k D) P^T is assembled from the CSR
// values straight into a column-major n_pad x (n_pad + nrhs) slot of the
// workspace (n_pad = n rounded up to the panel width; the padding rows and
// columns form an identity block, which leaves the leading n x n block's
// arithmetic untouched).  The right-hand sides ride along as extra columns,
// so the forward substitution L y = P b is performed by the factorisation
// itself, exactly as elimination on [A | b] does.
//
// Factorisation: right-looking, panels of NB = 32 columns:
//   1. GETRF of the NB x NB diagonal block by one wave (lane = row,
//      pivot row broadcast with readlane);
//   2. TRSM of the block column below (one thread per row) and of the block
//      row to the right, RHS columns included (one thread per column);
//   3. rank-NB update of the trailing matrix in 64 x 64 tiles staged in LDS.
// Every entry receives its updates a <- fma(-l, u, a) in ascending pivot
// order and every multiplier is an IEEE division, which is the operation
// sequence of the reference factorisation; the results are therefore
// identical bit for bit.
//
// Back substitution U x = y: blocks of 64 columns from the right; the
// diagonal triangle is staged in LDS and solved by one wave per RHS column,
// then the rows above are updated in descending column order.
#include "dense.h"

namespace psp {

constexpr int NB = 32;        // panel width
constexpr int TB = 64;        // trailing-update tile (TB x TB)
constexpr int SB = 64;        // triangular-solve block
constexpr int WG = 512;       // threads per workgroup (8 waves)

// ---------------------------------------------------------------- assembly
__device__ __forceinline__ void assemble(const DenseArgs& a, double* M, int s, double eps, int ncols) {
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)a.ld * ncols;
    for (int64_t i = tid; i < total; i += WG) M[i] = 0.0;
    __syncthreads();
    const double* v = a.values + (int64_t)s * a.nnz;
    for (int e = tid; e < a.nnz; e += WG) M[a.dst[e]] = v[e];
    __syncthreads();
    for (int q = tid; q < a.n_pad; q += WG) {
        const int64_t o = (int64_t)q * a.ld + q;
        if (q < a.n) {
            const double dq = a.dvec ? a.dvec[a.perm[q]] : 1.0;
            M[o] = __dadd_rn(M[o], __dmul_rn(eps, dq));
        } else {
            M[o] = 1.0;
        }
    }
    if (a.nrhs > 0) {
        const double* b = a.B + (int64_t)s * a.n * a.nrhs;
        for (int t = tid; t < a.n * a.nrhs; t += WG) {
            const int q = t / a.nrhs, r = t % a.nrhs;
            M[(int64_t)(a.n_pad + r) * a.ld + q] = b[(int64_t)a.perm[q] * a.nrhs + r];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- factorisation
// GETRF of the NB x NB diagonal block at (c0, c0) by wave 0 (lane = row); the
// factored block is left in M and in D (row-major, LDS).  Returns the 1-based
// position of the first bad pivot or 0 (valid in wave 0 only).
__device__ __forceinline__ int panel_getrf(double* M, int ld, int c0, double* D) {
    const int lane = threadIdx.x & 63;
    double r[NB];
    const bool act = lane < NB;
#pragma unroll
    for (int j = 0; j < NB; ++j) r[j] = act ? M[(int64_t)(c0 + j) * ld + c0 + lane] : 0.0;
    int bad = 0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const double ukk = readlane_d(r[k], k);
        if (!bad && bad_pivot(ukk)) bad = c0 + k + 1;
        const bool below = lane > k;
        const double l = r[k] / ukk;
        r[k] = below ? l : r[k];
#pragma unroll
        for (int j = k + 1; j < NB; ++j) {
            const double ukj = readlane_d(r[j], k);
            r[j] = below ? fmad(-l, ukj, r[j]) : r[j];
        }
    }
    if (act) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            M[(int64_t)(c0 + j) * ld + c0 + lane] = r[j];
            D[lane * NB + j] = r[j];
        }
    }
    return bad;
}

// Load the factored diagonal block at (c0, c0) into D.
__device__ __forceinline__ void load_diag(const double* M, int ld, int c0, double* D) {
    for (int t = threadIdx.x; t < NB * NB; t += WG) {
        const int i = t % NB, j = t / NB;
        D[i * NB + j] = M[(int64_t)(c0 + j) * ld + c0 + i];
    }
}

// One thread per item: rows [r_lo, r_hi) get l = a U^{-1} on the panel columns
// (TRSM from the right with the upper triangle of D, IEEE divisions), columns
// [c_lo, c_hi) get u = L^{-1} a on the panel rows (unit lower triangle of D).
__device__ __forceinline__ void panel_trsm(double* M, int ld, int c0, const double* D, int r_lo, int r_hi, int c_lo, int c_hi) {
    const int nrows = max(0, r_hi - r_lo), ncolr = max(0, c_hi - c_lo);
    for (int t = threadIdx.x; t < nrows + ncolr; t += WG) {
        double r[NB];
        // keep the LDS reads of D inside the loop (hoisting them all would exhaust registers)
        int z;
        asm volatile("v_mov_b32 %0, 0" : "=v"(z));   // opaque zero offset
        const double* Dv = D + z;
        if (t < nrows) {
            const int i = r_lo + t;
#pragma unroll
            for (int j = 0; j < NB; ++j) r[j] = M[(int64_t)(c0 + j) * ld + i];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const double l = r[k] / Dv[k * NB + k];
                r[k] = l;
#pragma unroll
                for (int j = k + 1; j < NB; ++j) r[j] = fmad(-l, Dv[k * NB + j], r[j]);
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) M[(int64_t)(c0 + j) * ld + i] = r[j];
        } else {
            const int j = c_lo + (t - nrows);
            double* col = M + (int64_t)j * ld + c0;
#pragma unroll
            for (int i = 0; i < NB; ++i) r[i] = col[i];
#pragma unroll
            for (int k = 0; k < NB; ++k)
#pragma unroll
                for (int i = k + 1; i < NB; ++i) r[i] = fmad(-Dv[i * NB + k], r[k], r[i]);
#pragma unroll
            for (int i = 0; i < NB; ++i) col[i] = r[i];
        }
    }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// C[r_lo:r_hi, c_lo:c_hi] -= L[:, k_lo:k_lo+KD] * U[k_lo:k_lo+KD, :] on the
// MFMA unit.  v_mfma_f64_16x16x4f64 accumulates each output as a chain of
// fmas in ascending k (checked on gfx950), so feeding k in ascending order
// keeps the reference operation sequence.  Each 16 x 16 block is computed
// transposed (D = (-U)^T L^T + C^T) so that a lane's accumulators run down a
// column of the column-major matrix: lane l, register q holds
// C[row0 + l%16][col0 + 4q + l/16].  Each wave keeps its 16 rows of L
// (the b operand) in registers for the whole sweep; the U tile (KD x 64) is
// staged in LDS and shared by the 8 waves; the workgroup covers 128 rows x 64
// columns per step.
constexpr int KDMAX = 128;

__device__ __forceinline__ void gemm_mfma(double* M, int ld, int r_lo, int r_hi, int c_lo, int c_hi, int k_lo, int kd,
                                          double* Us) {
    constexpr int KS = KDMAX / 4;
    constexpr int NW = WG / 64;                 // waves; each owns 16 rows of the 16*NW-row group
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int ks = kd / 4;
    for (int rg = r_lo; rg < r_hi; rg += 16 * NW) {
        const int wr = rg + 16 * wave;
        const bool wact = wr < r_hi;
        const bool rok = wact && wr + li < r_hi;
        double bop[KS];
        {
            const double* lb = M + (int64_t)(k_lo + lk) * ld + wr + li;
#pragma unroll
            for (int s = 0; s < KS; ++s) bop[s] = (rok && s < ks) ? lb[(int64_t)(4 * s) * ld] : 0.0;
        }
        for (int ct = c_lo; ct < c_hi; ct += 64) {
            __syncthreads();
            for (int t = tid; t < kd * 64; t += WG) {
                const int k = t % kd, c = t / kd;
                Us[k * 64 + c] = (ct + c < c_hi) ? -M[(int64_t)(ct + c) * ld + k_lo + k] : 0.0;
            }
            __syncthreads();
            if (!wact) continue;
            double* cb0 = M + (int64_t)(ct + lk) * ld + wr + li;
            v4d acc[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool ok = rok && (ct + 16 * cb + 4 * q + lk < c_hi);
                    acc[cb][q] = ok ? cb0[(int64_t)(16 * cb + 4 * q) * ld] : 0.0;
                }
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s < ks) {
                    double aop[4];
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) aop[cb] = Us[(4 * s + lk) * 64 + 16 * cb + li];
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[cb], bop[s], acc[cb], 0, 0, 0);
                }
            }
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool ok = rok && (ct + 16 * cb + 4 * q + lk < c_hi);
                    if (ok) cb0[(int64_t)(16 * cb + 4 * q) * ld] = acc[cb][q];
                }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void gemm_kd(int kd, double* M, int ld, int r_lo, int r_hi, int c_lo, int c_hi, int k_lo,
                                        double* Us) {
    if (r_lo >= r_hi || c_lo >= c_hi) return;
    gemm_mfma(M, ld, r_lo, r_hi, c_lo, c_hi, k_lo, kd, Us);
}

// Right-looking factorisation with super-panels of SP = 4 NB columns:
//   inside a super-panel, NB-wide panels are factored left to right and the
//   rest of the super-panel is updated after each (GETRF, TRSM, rank-NB);
//   the block row to the right is then solved panel by panel (TRSM, rank-NB
//   update of the lower panel rows), and the trailing matrix receives one
//   rank-SP update.  Every entry still sees its updates in ascending pivot
//   order.  Returns 0 or the 1-based position of the first bad pivot.
constexpr int SP = 4 * NB;
__device__ __forceinline__ int factor_slot(double* M, int n_pad, int ld, int ncols, double* lds) {
    double* D = lds;                // NB x NB
    double* Us = lds + NB * NB;     // SP x 64
    __shared__ int s_info;
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int c0 = 0; c0 < n_pad; c0 += SP) {
        const int ce = min(c0 + SP, n_pad);
        for (int p = c0; p < ce; p += NB) {
            if (wave == 0) {
                const int bad = panel_getrf(M, ld, p, D);
                if ((tid & 63) == 0) s_info = bad;
            }
            __syncthreads();
            if (s_info) return s_info;
            panel_trsm(M, ld, p, D, p + NB, n_pad, p + NB, ce);
            __syncthreads();
            gemm_kd(NB, M, ld, p + NB, n_pad, p + NB, ce, p, Us);
        }
        if (ce < ncols) {
            for (int p = c0; p < ce; p += NB) {
                load_diag(M, ld, p, D);
                __syncthreads();
                panel_trsm(M, ld, p, D, 0, 0, ce, ncols);
                __syncthreads();
                gemm_kd(NB, M, ld, p + NB, ce, ce, ncols, p, Us);
            }
            gemm_kd(ce - c0, M, ld, ce, n_pad, ce, ncols, c0, Us);
        }
    }
    return 0;
}

// ---------------------------------------------------------------- triangular solves
// T holds nrhs columns of length n_pad with stride ld.  Variants (reference order):
//   LOWER=1, TRANS=0: L y = b  (unit, a_ik = M[i + k ld]), ascending
//   LOWER=0, TRANS=0: U x = y  (a_ij = M[i + j ld], diag u_jj), descending
//   LOWER=1, TRANS=1: U^T z = w (a_ik = M[k + i ld], diag u_kk), ascending
//   LOWER=0, TRANS=1: L^T v = z (unit, a_ij = M[j + i ld]), descending
template <int LOWER, int TRANS>
__device__ __forceinline__ void tri_solve(const double* M, int n_pad, int ld, double* T, int nrhs, double* lds) {
    constexpr bool UNIT = (LOWER && !TRANS) || (!LOWER && TRANS);
    double* Tri = lds;                 // SB x SB, Tri[i*SB + j] = a(b0+i, b0+j)
    double* Xs = lds + SB * SB;        // SB x nrhs (nrhs <= 64)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n_pad + SB - 1) / SB;
    for (int bb = 0; bb < nblk; ++bb) {
        const int blk = LOWER ? bb : nblk - 1 - bb;
        const int b0 = blk * SB, bs = min(SB, n_pad - b0);
        for (int t = tid; t < SB * SB; t += WG) {
            const int i = t % SB, j = t / SB;
            double v = 0.0;
            if (i < bs && j < bs) v = TRANS ? M[(int64_t)(b0 + i) * ld + b0 + j] : M[(int64_t)(b0 + j) * ld + b0 + i];
            Tri[i * SB + j] = v;
        }
        __syncthreads();
        for (int r = wave; r < nrhs; r += WG / 64) {
            double* tc = T + (int64_t)r * ld + b0;
            double t = lane < bs ? tc[lane] : 0.0;
            if (LOWER) {
                for (int k = 0; k < bs; ++k) {
                    double xk = readlane_d(t, k);
                    if (!UNIT) xk = xk / Tri[k * SB + k];
                    if (lane == k) t = xk;
                    if (lane > k) t = fmad(-Tri[lane * SB + k], xk, t);
                    if (lane == 0) Xs[k * 64 + r] = xk;
                }
            } else {
                for (int k = bs - 1; k >= 0; --k) {
                    double xk = readlane_d(t, k);
                    if (!UNIT) xk = xk / Tri[k * SB + k];
                    if (lane == k) t = xk;
                    if (lane < k) t = fmad(-Tri[lane * SB + k], xk, t);
                    if (lane == 0) Xs[k * 64 + r] = xk;
                }
            }
            if (lane < bs) tc[lane] = t;
        }
        __syncthreads();
        // rows outside the block
        const int lo = LOWER ? b0 + bs : 0, hi = LOWER ? n_pad : b0;
        for (int t = tid; t < (hi - lo) * nrhs; t += WG) {
            const int i = lo + t % (hi - lo), r = t / (hi - lo);
            double v = T[(int64_t)r * ld + i];
            if (LOWER) {
                for (int k = 0; k < bs; ++k) {
                    const double a = TRANS ? M[(int64_t)i * ld + b0 + k] : M[(int64_t)(b0 + k) * ld + i];
                    v = fmad(-a, Xs[k * 64 + r], v);
                }
            } else {
                for (int k = bs - 1; k >= 0; --k) {
                    const double a = TRANS ? M[(int64_t)i * ld + b0 + k] : M[(int64_t)(b0 + k) * ld + i];
                    v = fmad(-a, Xs[k * 64 + r], v);
                }
            }
            T[(int64_t)r * ld + i] = v;
        }
        __syncthreads();
    }
}

constexpr int kLdsFactor = (NB * NB + SP * 64) * 8;
constexpr int kLdsSolve = (SB * SB + SB * 64) * 8;
constexpr int kLdsDense = kLdsFactor > kLdsSolve ? kLdsFactor : kLdsSolve;

// ---------------------------------------------------------------- kernels
// Fused: assemble, factor, forward (augmented), back substitution, write x_k.
// Tasks are either single systems (s, k), writing x_sk to Xk, or whole
// Jacobians s (per_jacobian), which run their K systems one after the other
// and accumulate x_s = sum_k c_k x_sk in ascending k straight into X, each
// thread owning the same entries for every k.
__global__ __launch_bounds__(WG) void dense_factor_solve_kernel(DenseArgs a, EpsSet es) {
    extern __shared__ double lds[];
    const int K = es.K;
    const int ntask = a.per_jacobian ? a.batch : a.ntasks;
    for (int task = blockIdx.x; task < ntask; task += gridDim.x) {
        const int s = a.per_jacobian ? task : task / K;
        const int k0 = a.per_jacobian ? 0 : task % K, k1 = a.per_jacobian ? K : k0 + 1;
        for (int k = k0; k < k1; ++k) {
            const int sys = s * K + k;
            double* M = a.slots + (a.keep ? (int64_t)sys : (int64_t)blockIdx.x) * a.slot_stride;
            const int ncols = a.n_pad + a.nrhs;
            assemble(a, M, s, eps_at(es, k), ncols);
            const int info = factor_slot(M, a.n_pad, a.ld, ncols, lds);
            if (info == 0 && a.nrhs > 0) tri_solve<0, 0>(M, a.n_pad, a.ld, M + (int64_t)a.n_pad * a.ld, a.nrhs, lds);
            if (threadIdx.x == 0) a.info[sys] = info;
            if (a.nrhs > 0) {
                double* x = a.per_jacobian ? a.X + (int64_t)s * a.n * a.nrhs : a.Xk + (int64_t)sys * a.n * a.nrhs;
                for (int t = threadIdx.x; t < a.n * a.nrhs; t += WG) {
                    const int q = t / a.nrhs, r = t % a.nrhs;
                    const double v = info ? __builtin_nan("") : M[(int64_t)(a.n_pad + r) * a.ld + q];
                    double* dst = x + (int64_t)a.perm[q] * a.nrhs + r;
                    *dst = a.per_jacobian ? fmad(c_at(es, k), v, k == 0 ? 0.0 : *dst) : v;
                }
            }
            __syncthreads();
        }
    }
}

// Split solve with stored factors, one WG per (s, k).
__global__ __launch_bounds__(WG) void dense_solve_kernel(DenseSolveArgs a) {
    extern __shared__ double lds[];
    for (int task = blockIdx.x; task < a.ntasks; task += gridDim.x) {
        const int s = task / a.K;
        const double* M = a.slots + (int64_t)task * a.slot_stride;
        double* T = a.tmp + (int64_t)task * a.ld * a.nrhs;
        const double* b = a.B + (int64_t)s * a.n * a.nrhs;
        for (int t = threadIdx.x; t < a.n_pad * a.nrhs; t += WG) {
            const int q = t % a.n_pad, r = t / a.n_pad;
            T[(int64_t)r * a.ld + q] = q < a.n ? b[(int64_t)a.perm[q] * a.nrhs + r] : 0.0;
        }
        __syncthreads();
        const int info = a.info[task];
        if (!info) {
            if (!a.trans) {
                tri_solve<1, 0>(M, a.n_pad, a.ld, T, a.nrhs, lds);
                tri_solve<0, 0>(M, a.n_pad, a.ld, T, a.nrhs, lds);
            } else {
                tri_solve<1, 1>(M, a.n_pad, a.ld, T, a.nrhs, lds);
                tri_solve<0, 1>(M, a.n_pad, a.ld, T, a.nrhs, lds);
            }
        }
        double* x = a.Xk + (int64_t)task * a.n * a.nrhs;
        for (int t = threadIdx.x; t < a.n * a.nrhs; t += WG) {
            const int q = t / a.nrhs, r = t % a.nrhs;
            x[(int64_t)a.perm[q] * a.nrhs + r] = info ? __builtin_nan("") : T[(int64_t)r * a.ld + q];
        }
        __syncthreads();
    }
}

// X[s] = sum_k c_k Xk[s][k], ascending k, fma chain from zero.
__global__ void combine_kernel(int64_t len, int32_t batch, EpsSet es, const double* Xk, double* X) {
    const int64_t total = len * batch;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = t / len, i = t % len;
        const double* p = Xk + s * es.K * len + i;
        double acc = 0.0;
        for (int k = 0; k < es.K; ++k) acc = fmad(c_at(es, k), p[k * len], acc);
        X[t] = acc;
    }
}

// gA[s][e] = - sum_k c_k sum_r Lam[s][k][i][r] X[s][k][j][r] on the CSR entries of A.
__global__ void grad_values_kernel(int32_t n, int32_t nnz, int32_t batch, int32_t nrhs, EpsSet es,
                                   const int32_t* rows, const int32_t* cols,
                                   const double* Lamk, const double* Xk, double* gA) {
    const int64_t total = (int64_t)nnz * batch;
    const int64_t blk = (int64_t)n * nrhs;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = t / nnz;
        const int e = (int)(t % nnz);
        const int i = rows[e], j = cols[e];
        double acc = 0.0;
        for (int k = 0; k < es.K; ++k) {
            const double* lam = Lamk + (s * es.K + k) * blk + (int64_t)i * nrhs;
            const double* x = Xk + (s * es.K + k) * blk + (int64_t)j * nrhs;
            double sum = 0.0;
            for (int r = 0; r < nrhs; ++r) sum = fmad(lam[r], x[r], sum);
            acc = fmad(c_at(es, k), sum, acc);
        }
        gA[t] = -acc;
    }
}

// ---------------------------------------------------------------- host launchers
int dense_lds_bytes() { return kLdsDense; }
int dense_panel() { return NB; }

hipError_t launch_dense_factor_solve(const DenseArgs& a, const EpsSet& es, int grid, hipStream_t st) {
    hipLaunchKernelGGL(dense_factor_solve_kernel, dim3(grid), dim3(WG), kLdsDense, st, a, es);
    return hipGetLastError();
}

hipError_t launch_dense_solve(const DenseSolveArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(dense_solve_kernel, dim3(grid), dim3(WG), kLdsDense, st, a);
    return hipGetLastError();
}

hipError_t launch_combine(int64_t len, int32_t batch, const EpsSet& es, const double* Xk, double* X, hipStream_t st) {
    const int64_t total = len * batch;
    int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(combine_kernel, dim3(grid), dim3(256), 0, st, len, batch, es, Xk, X);
    return hipGetLastError();
}

hipError_t launch_grad_values(int32_t n, int32_t nnz, int32_t batch, int32_t nrhs, const EpsSet& es,
                              const int32_t* rows, const int32_t* cols, const double* Lamk, const double* Xk,
                              double* gA, hipStream_t st) {
    const int64_t total = (int64_t)nnz * batch;
    int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(grad_values_kernel, dim3(grid), dim3(256), 0, st, n, nnz, batch, nrhs, es, rows, cols, Lamk,
                       Xk, gA);
    return hipGetLastError();
}

hipError_t dense_occupancy(int* blocks_per_cu) {
    // queried once per process (a launch-independent property of the compiled kernel)
    static int occ = 0;
    static const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, dense_factor_solve_kernel, WG, kLdsDense);
    *blocks_per_cu = occ;
    return e;
}

}  // namespace psp
