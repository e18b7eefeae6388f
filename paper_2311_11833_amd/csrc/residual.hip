// residual.hip -- the optional error test of Alg. 1 (step 5), for gfx950:
// r = b - A x and the 2-norms of r and b per Jacobian and RHS column (the
// residual norm the paper's Fig. 1 reports).
//
// One workgroup per (Jacobian, RHS column).  Each r_i is b_i followed by
// fma(-a_ie, x_j, .) over row i in CSR order; the sums of squares are fma
// chains in ascending row order, taken by one lane (n dependent fmas, a few
// microseconds at n ~ 600) so that they match a sequential evaluation bit for
// bit.  r is staged in LDS (n <= kResLds) or read back from R.
#include "dense.h"

namespace psp {

namespace {
constexpr int kResThreads = 256;

__global__ __launch_bounds__(kResThreads) void residual_kernel(ResArgs a) {
    extern __shared__ __align__(16) double rs[];
    const int job = blockIdx.x, s = job / a.nrhs, q = job % a.nrhs;
    const int64_t nn = (int64_t)a.n * a.nrhs;
    const double* v = a.values + (int64_t)s * a.nnz;
    const double* b = a.B + s * nn;
    const double* x = a.X + s * nn;
    double* r = a.R ? a.R + s * nn : nullptr;
    for (int i = threadIdx.x; i < a.n; i += kResThreads) {
        double acc = b[(int64_t)i * a.nrhs + q];
        for (int e = a.rowptr[i]; e < a.rowptr[i + 1]; ++e) acc = fmad(-v[e], x[(int64_t)a.cols[e] * a.nrhs + q], acc);
        if (a.stage) rs[i] = acc;
        if (r) r[(int64_t)i * a.nrhs + q] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sq = 0.0;
        for (int i = 0; i < a.n; ++i) {
            const double ri = a.stage ? rs[i] : r[(int64_t)i * a.nrhs + q];
            sq = fmad(ri, ri, sq);
        }
        a.rnorm[job] = __dsqrt_rn(sq);
    } else if (threadIdx.x == 64 && a.bnorm) {   // another wave
        double sq = 0.0;
        for (int i = 0; i < a.n; ++i) {
            const double bi = b[(int64_t)i * a.nrhs + q];
            sq = fmad(bi, bi, sq);
        }
        a.bnorm[job] = __dsqrt_rn(sq);
    }
}
}  // namespace

hipError_t launch_residual(ResArgs a, hipStream_t st) {
    a.stage = a.n <= kResLds ? 1 : 0;
    const int lds = a.stage ? a.n * 8 : 0;
    if (lds > 48 * 1024) {
        // once per process, for the largest staged size
        static const hipError_t e = hipFuncSetAttribute((const void*)residual_kernel,
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, kResLds * 8);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(residual_kernel, dim3(a.batch * a.nrhs), dim3(kResThreads), lds, st, a);
    return hipGetLastError();
}

}  // namespace psp
