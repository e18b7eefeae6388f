// estimate.hip -- power iteration for rho(A^{-1} D), the quantity that decides
// whether the expansion behind the method converges (|eps_k| rho < 1, Sec. II-B)
// and how large its truncation error is (about prod_k |eps_k| rho^K); the
// perturbation size per Jacobian is chosen from it.
//
// The iteration runs M = (A + p D)^{-1} D with a perturbed, pivot-free
// factorisation (small p, so M is A^{-1} D to within p rho): each step solves
// (a fused factor-and-solve on the step kernel, or kept factors for patterns
// too large for it) and then this kernel, one workgroup per
// Jacobian, takes g = ||x||_2 (one lane's ascending fma chain of squares, then
// a correctly rounded sqrt), sets v = x / g, writes the next right-hand side
// D v, and adds log g to a sum over the second half of the steps; the
// estimate is exp(mean log g), which also settles when the dominant
// eigenvalues are a complex pair of equal modulus.
#include "estimate.h"

namespace psp {

namespace {
constexpr int kRhoThreads = 256;
constexpr int kRhoStage = 4096;   // vectors up to this length are staged in LDS (32 KB) for the chain

__global__ __launch_bounds__(kRhoThreads) void rho_step_kernel(RhoArgs a) {
    __shared__ double gs;
    __shared__ double xl[kRhoStage];
    const int s = blockIdx.x;
    const int64_t off = (int64_t)s * a.n;
    const double* x = a.src + off;
    const bool stage = a.n <= kRhoStage;
    if (stage)
        for (int i = threadIdx.x; i < a.n; i += kRhoThreads) xl[i] = x[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        // one ascending fma chain, so the norm (and with it every iterate) is reproducible bit for bit
        const double* xs = stage ? xl : x;
        double ss = 0.0;
        for (int i = 0; i < a.n; ++i) ss = fma(xs[i], xs[i], ss);
        gs = __dsqrt_rn(ss);
    }
    __syncthreads();
    const double g = gs;
    for (int i = threadIdx.x; i < a.n; i += kRhoThreads) {
        const double vi = x[i] / g;
        a.v[off + i] = vi;
        a.B[off + i] = a.d ? a.d[i] * vi : vi;
    }
    if (threadIdx.x == 0) {
        if (a.mode == 0) a.acc[s] = 0.0;
        else if (a.mode >= 2) a.acc[s] += log(g);
        if (a.mode == 3) a.rho[s] = exp(a.acc[s] * a.inv_count);
    }
}
}  // namespace

hipError_t launch_rho_step(const RhoArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(rho_step_kernel, dim3(a.batch), dim3(kRhoThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace psp
