// dense_ops.h -- the dense pivot-free LU building blocks for gfx950 (internal),
// shared by the dense path (one workgroup per system) and the dense trailing
// block of the sparse path (one large block per system, many workgroups).
// Every routine runs in one workgroup, of W threads where it takes a width
// (WG otherwise).
//
// Every entry receives its updates a <- fma(-l, u, a) in ascending pivot
// order and every multiplier is an IEEE division, which is the operation
// sequence of the reference factorisation; results are identical bit for bit.
#pragma once

#include "common.h"

namespace psp {

constexpr int NB = 32;        // panel width
constexpr int SB = 64;        // triangular-solve block
constexpr int WG = 512;       // threads per workgroup (8 waves)

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
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t % NB, j = t / NB;
        D[i * NB + j] = M[(int64_t)(c0 + j) * ld + c0 + i];
    }
}

// One thread per item (any workgroup width): rows [r_lo, r_hi) get l = a U^{-1} on the panel columns
// (TRSM from the right with the upper triangle of D, IEEE divisions), columns
// [c_lo, c_hi) get u = L^{-1} a on the panel rows (unit lower triangle of D).
__device__ __forceinline__ void panel_trsm(double* M, int ld, int c0, const double* D, int r_lo, int r_hi, int c_lo, int c_hi) {
    const int nrows = max(0, r_hi - r_lo), ncolr = max(0, c_hi - c_lo);
    for (int t = threadIdx.x; t < nrows + ncolr; t += blockDim.x) {
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
// staged in LDS and shared by the workgroup's W/64 waves, which cover 16 W/64
// rows x 64 columns per step.
constexpr int KDMAX = 128;

template <int KDM = KDMAX, int W = WG>
__device__ __forceinline__ void gemm_mfma(double* M, int ld, int r_lo, int r_hi, int c_lo, int c_hi, int k_lo, int kd,
                                          double* Us) {
    constexpr int KS = KDM / 4;
    constexpr int NW = W / 64;                  // waves; each owns 16 rows of the 16*NW-row group
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
            for (int t = tid; t < kd * 64; t += W) {
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

// The same update, software-pipelined for one workgroup sweeping a whole
// block: the (row group, column tile) iterations run as one sequence, and
// while iteration i runs its MFMAs the U tile of iteration i+1 is copied from
// global memory straight into the other half of a double buffer in LDS
// (global_load_lds: one instruction moves one column of the tile, 64 lanes x
// KDM/8 bytes, to consecutive LDS addresses) and its C tile is fetched into
// registers; each iteration ends with one barrier.  The staged tile is
// column-major with a padded column stride (UP = KDM + 2 doubles), so the
// MFMA operand reads (16 columns x 4 k per read) hit distinct LDS banks.  The
// L rows are kept negated in registers (B = -L): the products -l u enter each
// chain exactly as in the plain update.
// With a single buffer (NBUF = 1) the next tile is copied between two
// barriers after the MFMAs instead.  A tile is 16 rows per wave (16 W/64
// rows per row group) by CT columns; the U tile is fetched again for every
// row group, which is the largest share of this update's HBM traffic.
// Us: NBUF x CT x (KDM + 2) doubles.  Rows [r_lo, r_hi) must not overlap the
// U rows [k_lo, k_lo + kd), nor columns [c_lo, c_hi) the L columns; r_lo and
// ld are multiples of 16 and r_hi <= ld.  W: workgroup width.
template <int KDM, int NBUF, int CT = 64>
constexpr int gemm_pipe_lds_doubles() { return NBUF * CT * (KDM + 2); }

// kd == KDM (a full panel or super-panel).
template <int KDM, int W, int NBUF, int CT = 64>
__device__ __forceinline__ void gemm_mfma_pipe(double* M, int ld, int r_lo, int r_hi, int c_lo, int c_hi, int k_lo,
                                               double* Us) {
    constexpr int KS = KDM / 4;
    constexpr int UP = KDM + 2;
    constexpr int USZ = CT * UP;
    constexpr int NCB = CT / 16;                // 16-column blocks per tile
    constexpr int NW = W / 64;
    static_assert(NBUF == 1 || NBUF == 2, "one or two staged U tiles");
    constexpr int BPL = KDM * 8 / 64;           // bytes per lane of one column copy (16 or 4)
    constexpr int CPW = CT / NW;                // tile columns copied per wave
    static_assert(BPL == 16 || BPL == 4, "column copy must be a dword or dwordx4 per lane");
    static_assert(KS % 2 == 0, "operand double buffering takes the k steps in pairs");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int nct = (c_hi - c_lo + CT - 1) / CT;
    const int nrg = (r_hi - r_lo + 16 * NW - 1) / (16 * NW);
    const int total = nct * nrg;
    if (total <= 0) return;

    auto stage_u = [&](double* U, int ct) {
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int c = wave * CPW + j;
            if (ct + c < c_hi) {
                const char* src = reinterpret_cast<const char*>(M + (int64_t)(ct + c) * ld + k_lo) + lane * BPL;
                if constexpr (BPL == 16)
                    __builtin_amdgcn_global_load_lds(src, U + c * UP, 16, 0, 0);
                else
                    __builtin_amdgcn_global_load_lds(src, U + c * UP, 4, 0, 0);
            }
        }
    };
    const uint32_t loff = (uint32_t)(lk * ld + li) * 8u;   // this lane's byte offset in a 4-column block
    v4d cpre[NCB];
    auto load_c = [&](int rg, int ct) {
        const int wr = r_lo + rg * 16 * NW + 16 * wave;
        if (wr >= r_hi) return;
        const bool rok = wr + li < r_hi;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = ct + 16 * cb + 4 * q;
                const char* base = reinterpret_cast<const char*>(M + (int64_t)col * ld + wr);
                double v = 0.0;
                if (rok && col + lk < c_hi) v = *reinterpret_cast<const double*>(base + loff);
                cpre[cb][q] = v;
            }
    };
    double bop[KS];
    auto load_l = [&](int rg) {
        const int wr = r_lo + rg * 16 * NW + 16 * wave;
        if (wr >= r_hi) return;
        const bool rok = wr + li < r_hi;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const char* base = reinterpret_cast<const char*>(M + (int64_t)(k_lo + 4 * s) * ld + wr);
            double v = 0.0;
            if (rok) v = -*reinterpret_cast<const double*>(base + loff);
            bop[s] = v;
        }
    };

    stage_u(Us, c_lo);
    load_l(0);
    load_c(0, c_lo);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const int rg = it / nct, ct = c_lo + CT * (it % nct);
        const int it1 = it + 1;
        const bool more = it1 < total;
        const int rg1 = it1 / nct, ct1 = c_lo + CT * (it1 % nct);
        const double* U = Us + (NBUF == 2 ? (it & 1) * USZ : 0) + li * UP + lk;
        const int wr = r_lo + rg * 16 * NW + 16 * wave;
        v4d acc[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = cpre[cb];
        if (more) {
            if constexpr (NBUF == 2) stage_u(Us + (it1 & 1) * USZ, ct1);
            load_c(rg1, ct1);
        }
        if (wr < r_hi) {
            // A operands one k step ahead of the MFMAs that use them
            double a0[NCB], a1[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) a0[cb] = U[16 * cb * UP];
#pragma unroll
            for (int s = 0; s < KS; s += 2) {
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) a1[cb] = U[16 * cb * UP + 4 * (s + 1)];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[cb], bop[s], acc[cb], 0, 0, 0);
                if (s + 2 < KS) {
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) a0[cb] = U[16 * cb * UP + 4 * (s + 2)];
                }
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[cb], bop[s + 1], acc[cb], 0, 0, 0);
            }
            const bool rok = wr + li < r_hi;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = ct + 16 * cb + 4 * q;
                    char* base = reinterpret_cast<char*>(M + (int64_t)col * ld + wr);
                    if (rok && col + lk < c_hi) *reinterpret_cast<double*>(base + loff) = acc[cb][q];
                }
        }
        if constexpr (NBUF == 1) {
            if (!more) break;
            __syncthreads();          // every wave is done with the tile
            stage_u(Us, ct1);
        }
        if (more && rg1 != rg) load_l(rg1);
        // this wave's copies into the next buffer have landed before anyone reads them
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if constexpr (NBUF == 1) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// A partial super-panel (kd other than NB or KDMAX; none occurs with rows to update): the
// plain update, kept out of line so that it does not weigh on the callers' registers.
template <int W>
__device__ __attribute__((noinline)) void gemm_mfma_cold(double* M, int ld, int r_lo, int r_hi, int c_lo, int c_hi,
                                                         int k_lo, int kd, double* Us) {
    gemm_mfma<KDMAX, W>(M, ld, r_lo, r_hi, c_lo, c_hi, k_lo, kd, Us);
}

template <int W, int NBUF, int CT = 64>
__device__ __forceinline__ void gemm_kd(int kd, double* M, int ld, int r_lo, int r_hi, int c_lo, int c_hi, int k_lo,
                                        double* Us) {
    if (r_lo >= r_hi || c_lo >= c_hi) return;
    if (kd == NB)
        gemm_mfma_pipe<NB, W, NBUF, CT>(M, ld, r_lo, r_hi, c_lo, c_hi, k_lo, Us);
    else if (kd == KDMAX)
        gemm_mfma_pipe<KDMAX, W, NBUF, CT>(M, ld, r_lo, r_hi, c_lo, c_hi, k_lo, Us);
    else
        gemm_mfma_cold<W>(M, ld, r_lo, r_hi, c_lo, c_hi, k_lo, kd, Us);
}

// Right-looking factorisation with super-panels of SP = 4 NB columns:
//   inside a super-panel, NB-wide panels are factored left to right and the
//   rest of the super-panel is updated after each (GETRF, TRSM, rank-NB);
//   the block row to the right is then solved panel by panel (TRSM, rank-NB
//   update of the lower panel rows), and the trailing matrix receives one
//   rank-SP update.  Every entry still sees its updates in ascending pivot
//   order.  Returns 0 or the 1-based position of the first bad pivot.
// W: workgroup width; NBUF: staged U tiles of the updates (2: double buffered).
constexpr int SP = 4 * NB;
template <int W = WG, int NBUF = 2, int CT = 64>
__device__ __forceinline__ int factor_slot(double* M, int n_pad, int ld, int ncols, double* lds) {
    double* D = lds;                // NB x NB
    double* Us = lds + NB * NB;     // the staged U tiles of gemm_mfma_pipe
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
            gemm_kd<W, NBUF, CT>(NB, M, ld, p + NB, n_pad, p + NB, ce, p, Us);
        }
        if (ce < ncols) {
            for (int p = c0; p < ce; p += NB) {
                load_diag(M, ld, p, D);
                __syncthreads();
                panel_trsm(M, ld, p, D, 0, 0, ce, ncols);
                __syncthreads();
                gemm_kd<W, NBUF, CT>(NB, M, ld, p + NB, ce, ce, ncols, p, Us);
            }
            gemm_kd<W, NBUF, CT>(ce - c0, M, ld, ce, n_pad, ce, ncols, c0, Us);
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
template <int LOWER, int TRANS, int W = WG>
__device__ __forceinline__ void tri_solve(const double* M, int n_pad, int ld, double* T, int nrhs, double* lds) {
    constexpr bool UNIT = (LOWER && !TRANS) || (!LOWER && TRANS);
    // SB x SB, Tri[i*(SB+1) + j] = a(b0+i, b0+j): the padded row stride puts the column reads of
    // the diagonal solve (one row per lane) on distinct banks
    constexpr int TP = SB + 1;
    double* Tri = lds;
    double* Xs = lds + SB * TP;        // SB x nrhs (nrhs <= 64)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n_pad + SB - 1) / SB;
    for (int bb = 0; bb < nblk; ++bb) {
        const int blk = LOWER ? bb : nblk - 1 - bb;
        const int b0 = blk * SB, bs = min(SB, n_pad - b0);
        for (int t = tid; t < SB * SB; t += W) {
            const int i = t % SB, j = t / SB;
            double v = 0.0;
            if (i < bs && j < bs) v = TRANS ? M[(int64_t)(b0 + i) * ld + b0 + j] : M[(int64_t)(b0 + j) * ld + b0 + i];
            Tri[i * TP + j] = v;
        }
        __syncthreads();
        for (int r = wave; r < nrhs; r += W / 64) {
            double* tc = T + (int64_t)r * ld + b0;
            double t = lane < bs ? tc[lane] : 0.0;
            if (LOWER) {
                for (int k = 0; k < bs; ++k) {
                    double xk = readlane_d(t, k);
                    if (!UNIT) xk = xk / Tri[k * TP + k];
                    if (lane == k) t = xk;
                    if (lane > k) t = fmad(-Tri[lane * TP + k], xk, t);
                    if (lane == 0) Xs[k * 64 + r] = xk;
                }
            } else {
                for (int k = bs - 1; k >= 0; --k) {
                    double xk = readlane_d(t, k);
                    if (!UNIT) xk = xk / Tri[k * TP + k];
                    if (lane == k) t = xk;
                    if (lane < k) t = fmad(-Tri[lane * TP + k], xk, t);
                    if (lane == 0) Xs[k * 64 + r] = xk;
                }
            }
            if (lane < bs) tc[lane] = t;
        }
        __syncthreads();
        // rows outside the block
        const int lo = LOWER ? b0 + bs : 0, hi = LOWER ? n_pad : b0;
        for (int t = tid; t < (hi - lo) * nrhs; t += W) {
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

// U x = y for one right-hand side T (length n_pad, overwritten by x), in the
// order of tri_solve<0, 0> (x_i: the terms u_ij x_j for j descending, then the
// division by u_ii), in blocks of BS1 = 32 rows from the bottom: wave 0 holds
// row `lane` of the diagonal block in registers (no LDS staging of the
// triangle) and solves it, then every thread takes one row above the block
// and applies the block's terms, with all loads issued before the chain.
// xs: BS1 doubles of LDS.
constexpr int BS1 = 32;
template <int W = WG>
__device__ __forceinline__ void upper_solve_1rhs(const double* M, int n_pad, int ld, double* T, double* xs) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n_pad + BS1 - 1) / BS1;
    for (int blk = nblk - 1; blk >= 0; --blk) {
        const int b0 = blk * BS1, bs = min(BS1, n_pad - b0);
        if (wave == 0) {
            const bool act = lane < bs;
            double r[BS1];
#pragma unroll
            for (int k = 0; k < BS1; ++k) r[k] = (act && k < bs) ? M[(int64_t)(b0 + k) * ld + b0 + lane] : 0.0;
            double t = act ? T[b0 + lane] : 0.0;
#pragma unroll
            for (int k = BS1 - 1; k >= 0; --k) {
                if (k < bs) {
                    const double xk = readlane_d(t, k) / readlane_d(r[k], k);
                    if (lane == k) t = xk;
                    if (lane < k) t = fmad(-r[k], xk, t);
                }
            }
            if (act) {
                T[b0 + lane] = t;
                xs[lane] = t;
            }
        }
        __syncthreads();
        for (int i = tid; i < b0; i += W) {
            double a[BS1];
#pragma unroll
            for (int k = 0; k < BS1; ++k) a[k] = k < bs ? M[(int64_t)(b0 + k) * ld + i] : 0.0;
            double v = T[i];
#pragma unroll
            for (int k = BS1 - 1; k >= 0; --k)
                if (k < bs) v = fmad(-a[k], xs[k], v);
            T[i] = v;
        }
        __syncthreads();
    }
}

template <int NBUF, int CT = 64>
constexpr int lds_factor_bytes() { return (NB * NB + gemm_pipe_lds_doubles<SP, NBUF, CT>()) * 8; }
constexpr int kLdsFactor = lds_factor_bytes<2>();
constexpr int kLdsSolve = (SB * (SB + 1) + SB * 64) * 8;
constexpr int kLdsDense = kLdsFactor > kLdsSolve ? kLdsFactor : kLdsSolve;
// the fused dense kernel: two 256-lane workgroups per CU, whose updates double-buffer
// U tiles of 32 columns (74.75 KB of LDS with the diagonal block)
constexpr int WGD = 256;
constexpr int kFusedBuf = 2, kFusedCT = 32;
constexpr int kLdsFused = lds_factor_bytes<kFusedBuf, kFusedCT>() > kLdsSolve ? lds_factor_bytes<kFusedBuf, kFusedCT>()
                                                                               : kLdsSolve;

}  // namespace psp
