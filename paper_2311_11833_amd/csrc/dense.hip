// dense.hip -- dense batched pivot-free LU, substitutions and combine for
// gfx950, one workgroup per perturbed system (or per Jacobian and its K systems).
//
// Each perturbed system P (A_s + eps_k D) P^T is assembled from the CSR
// values straight into a column-major n_pad x (n_pad + nrhs) slot of the
// workspace (n_pad = n rounded up to the panel width; the padding rows and
// columns form an identity block, which leaves the leading n x n block's
// arithmetic untouched).  The right-hand sides ride along as extra columns,
// so the forward substitution L y = P b is performed by the factorisation
// itself, exactly as elimination on [A | b] does.
//
// Factorisation (factor_slot): right-looking, super-panels of 128 columns
// made of panels of NB = 32:
//   1. GETRF of the NB x NB diagonal block by one wave (lane = row,
//      pivot row broadcast with readlane);
//   2. TRSM of the block column below (one thread per row) and of the block
//      row to the right, RHS columns included (one thread per column);
//   3. rank-NB updates inside the super-panel and of its block row, then one
//      rank-128 update of the trailing matrix, all on the MFMA unit with the
//      U tiles double-buffered in LDS (gemm_mfma_pipe).
// Every entry receives its updates a <- fma(-l, u, a) in ascending pivot
// order and every multiplier is an IEEE division, which is the operation
// sequence of the reference factorisation; the results are therefore
// identical bit for bit.
//
// Back substitution U x = y (one RHS: upper_solve_1rhs): blocks of 32 rows
// from the bottom; wave 0 solves the diagonal triangle from registers, then
// the rows above are updated in descending column order.
//
// Two 256-lane workgroups share a CU, so that one system's in-order panel
// steps overlap the other's updates.  At n = 608 the kernel streams each
// system's 3 MB slot from HBM several times (about 24 MB read and 13 MB
// written per system), half the HBM bandwidth at the measured speed.
#include "dense.h"
#include "dense_ops.h"

namespace psp {

// ---------------------------------------------------------------- assembly
__device__ __forceinline__ void assemble(const DenseArgs& a, double* M, int s, double eps, int ncols) {
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)a.ld * ncols;
    for (int64_t i = tid; i < total; i += WGD) M[i] = 0.0;
    __syncthreads();
    const double* v = a.values + (int64_t)s * a.nnz;
    for (int e = tid; e < a.nnz; e += WGD) M[a.dst[e]] = v[e];
    __syncthreads();
    for (int q = tid; q < a.n_pad; q += WGD) {
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
        for (int t = tid; t < a.n * a.nrhs; t += WGD) {
            const int q = t / a.nrhs, r = t % a.nrhs;
            M[(int64_t)(a.n_pad + r) * a.ld + q] = b[(int64_t)a.perm[q] * a.nrhs + r];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- kernels
// Fused: assemble, factor, forward (augmented), back substitution, write x_k.
// Tasks are either single systems (s, k), writing x_sk to Xk, or whole
// Jacobians s (per_jacobian), which run their K systems one after the other
// and accumulate x_s = sum_k c_k x_sk in ascending k straight into X, each
// thread owning the same entries for every k.
// 256-lane workgroups, two per CU (two waves per SIMD, at most 256 registers per wave, at
// most 80 KB of LDS each), so that one system's in-order panel steps overlap the other's
// MFMA updates.
__global__ __launch_bounds__(WGD, 2) void dense_factor_solve_kernel(DenseArgs a, EpsSet es) {
    extern __shared__ double lds[];
    // the nodes and weights in LDS: held in scalar registers for the whole kernel they
    // crowd out the update's addresses
    __shared__ double s_eps[kMaxK], s_c[kMaxK];
    if (threadIdx.x < kMaxK) {
        s_eps[threadIdx.x] = eps_at(es, threadIdx.x);
        s_c[threadIdx.x] = c_at(es, threadIdx.x);
    }
    __syncthreads();
    const int K = es.K;
    const int ntask = a.per_jacobian ? a.batch : a.ntasks;
    for (int task = blockIdx.x; task < ntask; task += gridDim.x) {
        const int s = a.per_jacobian ? task : task / K;
        const int k0 = a.per_jacobian ? 0 : task % K, k1 = a.per_jacobian ? K : k0 + 1;
        for (int k = k0; k < k1; ++k) {
            const int sys = s * K + k;
            double* M = a.slots + (a.keep ? (int64_t)sys : (int64_t)blockIdx.x) * a.slot_stride;
            const int ncols = a.n_pad + a.nrhs;
            assemble(a, M, s, s_eps[k], ncols);
            const int info = factor_slot<WGD, kFusedBuf, kFusedCT>(M, a.n_pad, a.ld, ncols, lds);
            if (info == 0 && a.nrhs == 1) upper_solve_1rhs<WGD>(M, a.n_pad, a.ld, M + (int64_t)a.n_pad * a.ld, lds);
            else if (info == 0 && a.nrhs > 0)
                tri_solve<0, 0, WGD>(M, a.n_pad, a.ld, M + (int64_t)a.n_pad * a.ld, a.nrhs, lds);
            if (threadIdx.x == 0) a.info[sys] = info;
            if (a.nrhs > 0) {
                double* x = a.per_jacobian ? a.X + (int64_t)s * a.n * a.nrhs : a.Xk + (int64_t)sys * a.n * a.nrhs;
                for (int t = threadIdx.x; t < a.n * a.nrhs; t += WGD) {
                    const int q = t / a.nrhs, r = t % a.nrhs;
                    const double v = info ? __builtin_nan("") : M[(int64_t)(a.n_pad + r) * a.ld + q];
                    double* dst = x + (int64_t)a.perm[q] * a.nrhs + r;
                    *dst = a.per_jacobian ? fmad(s_c[k], v, k == 0 ? 0.0 : *dst) : v;
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
int dense_lds_bytes() { return kLdsFused; }
int dense_panel() { return NB; }

hipError_t launch_dense_factor_solve(const DenseArgs& a, const EpsSet& es, int grid, hipStream_t st) {
    hipLaunchKernelGGL(dense_factor_solve_kernel, dim3(grid), dim3(WGD), kLdsFused, st, a, es);
    return hipGetLastError();
}

hipError_t launch_dense_solve(const DenseSolveArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(dense_solve_kernel, dim3(grid), dim3(WG), kLdsSolve, st, a);
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

hipError_t dense_kernel_attrs() {
    static const hipError_t e = [] {
        hipError_t r = hipFuncSetAttribute((const void*)dense_factor_solve_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kLdsFused);
        if (r == hipSuccess)
            r = hipFuncSetAttribute((const void*)dense_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    kLdsSolve);
        return r;
    }();
    return e;
}

hipError_t dense_occupancy(int* blocks_per_cu) {
    // queried once per process (a launch-independent property of the compiled kernel)
    static int occ = 0;
    static const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, dense_factor_solve_kernel, WGD, kLdsFused);
    *blocks_per_cu = occ;
    return e;
}

}  // namespace psp
