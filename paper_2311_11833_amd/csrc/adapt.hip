// adapt.hip -- the error test of Alg. 1 step 5 computed from the perturbed
// solutions alone, and the choice of a smaller node set for the Jacobians that
// fail it (the perturbation strategy that Sec. V leaves open).
//
// By the expansion of Sec. II-B, x(eps) = sum_j (-eps)^j M^j x* with
// M = A^{-1} D, so the divided difference of the perturbed solutions over the
// first j+1 nodes is (-1)^j M^j x* up to terms of order eps, and the
// combination's leading error is -(prod_k eps_k) M^K x* (Theorem 1 for general
// nodes).  Per Jacobian, with m_j = max_i |f[eps_0..eps_j]_i|:
//     rho_hat = m_{K-1} / m_{K-2},  est = |prod eps_k| m_{K-1} rho_hat / ||x_hat||_inf.
// A Jacobian whose est exceeds the caller's tolerance (or is NaN) is solved
// again at the nodes s eps_k, s = 2^-j: the error at scale s is modelled as
// a s^K (truncation; a = est, or |prod eps| rho_hat^K when est >= 1e-2 and the
// series may diverge) plus b / s (rounding, b = 50 u / max|eps_k|, the pivot
// the perturbation controls growing like 1/eps), whose minimiser is
// s* = (b / (K a))^{1/(K+1)}; s is the largest power of two at most
// min(s*, 1/2), found exactly from the binary exponent of b / (K a).  Scaling
// by a power of two leaves the combination weights unchanged and scales the
// divided-difference weights exactly, so the second estimate needs no new
// weights.
//
// Every divided difference and combination entry is an fma chain over
// ascending k from zero; maxima are exact; so est and the choice of s are the
// same bits as the reference's.
#include "adapt.h"

namespace psp {

namespace {
constexpr int kAdThreads = 256;

struct MaxNaN {
    double m;
    int nan;
};

__device__ __forceinline__ void take(MaxNaN& r, double v) {
    const double a = __builtin_fabs(v);
    if (a != a) r.nan = 1;
    else if (a > r.m) r.m = a;
}

// Block-wide exact maximum with a NaN flag (NaN wins, as in the reference's maximum).
__device__ double block_max(MaxNaN r, double* sm, int* sn) {
    const int t = threadIdx.x;
    sm[t] = r.m;
    sn[t] = r.nan;
    __syncthreads();
    for (int h = kAdThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            sm[t] = sm[t] > sm[t + h] ? sm[t] : sm[t + h];
            sn[t] |= sn[t + h];
        }
        __syncthreads();
    }
    const double out = sn[0] ? __builtin_nan("") : sm[0];
    __syncthreads();
    return out;
}

// j of the node scale 2^-j (see the file comment).
__device__ int scale_exponent(int K, const AdaptConst& c, double est, double rho) {
    if (est != est) return 10;
    double a = est;
    if (!(est < 1e-2)) {
        a = c.P;
        for (int k = 0; k < K; ++k) a = __dmul_rn(a, rho);
    }
    const double q = __ddiv_rn(c.b, __dmul_rn((double)K, a));
    if (!(q > 0.0) || !__builtin_isfinite(q)) return 10;
    const uint64_t bits = __builtin_bit_cast(uint64_t, q);
    const int E = (int)((bits >> 52) & 0x7FF);
    if (E == 0) return 60;                       // below 2^-1022: the cap
    const int e = E - 1023;                      // 2^e <= q < 2^{e+1}
    int j = e >= 0 ? 1 : (-e + K) / (K + 1);
    return j < 1 ? 1 : (j > 60 ? 60 : j);
}

// One workgroup per Jacobian (pass 1: Jacobian blockIdx.x; pass 2: entry blockIdx.x of the list).
__global__ __launch_bounds__(kAdThreads) void adapt_kernel(AdaptArgs a, AdaptConst c) {
    __shared__ double sm[kAdThreads];
    __shared__ int sn[kAdThreads];
    const int K = a.K, n = a.n;
    int s = blockIdx.x;
    double f1 = 1.0, f2 = 1.0, fP = 1.0, sc = 1.0;
    if (a.pass == 2) {
        if (blockIdx.x >= *a.count) return;      // uniform per workgroup
        s = a.list[blockIdx.x];
        // nodes s eps_k with s = 2^-j: the weights of f[..K-1] scale by 2^{j(K-1)}, those of f[..K-2] by
        // 2^{j(K-2)}, the node product by 2^{-jK}, all exactly
        sc = a.scale[s];
        const int j = 1023 - (int)((__builtin_bit_cast(uint64_t, sc) >> 52) & 0x7FF);   // sc = 2^-j
        f1 = __builtin_ldexp(1.0, j * (K - 1));
        f2 = __builtin_ldexp(1.0, j * (K - 2));
        fP = __builtin_ldexp(1.0, -j * K);
    }
    const double* xk = a.Xk + (int64_t)s * K * n;
    double* x = a.X + (int64_t)s * n;
    MaxNaN r1{0.0, 0}, r2{0.0, 0}, rx{0.0, 0};
    for (int i = threadIdx.x; i < n; i += kAdThreads) {
        double d1 = 0.0, d2 = 0.0, xc = 0.0;
        for (int k = 0; k < K; ++k) {
            const double v = xk[(int64_t)k * n + i];
            d1 = fmad(__dmul_rn(c.w1[k], f1), v, d1);
            if (k < K - 1) d2 = fmad(__dmul_rn(c.w2[k], f2), v, d2);
            if (a.combine) xc = fmad(c.c[k], v, xc);
        }
        if (a.combine) x[i] = xc;
        else xc = x[i];
        take(r1, d1);
        take(r2, d2);
        take(rx, xc);
    }
    const double m1 = block_max(r1, sm, sn);
    const double m2 = block_max(r2, sm, sn);
    const double mx = block_max(rx, sm, sn);
    if (threadIdx.x != 0) return;
    double est, rho;
    if (m1 != m1 || m2 != m2 || mx != mx) {
        est = rho = __builtin_nan("");
    } else if (m1 == 0.0) {
        est = rho = 0.0;
    } else {
        rho = __ddiv_rn(m1, m2);
        est = __ddiv_rn(__dmul_rn(__dmul_rn(__dmul_rn(c.P, fP), m1), rho), mx);
    }
    a.est[s] = est;
    if (a.pass == 1) {
        double out = 1.0;
        if (!(est <= a.tol)) {
            out = __builtin_ldexp(1.0, -scale_exponent(K, c, est, rho));
            a.list[atomicAdd(a.count, 1)] = s;
        }
        a.scale[s] = out;
    }
}

__global__ void adapt_reset_kernel(int32_t* count) {
    if (threadIdx.x == 0) *count = 0;
}
}  // namespace

hipError_t launch_adapt_reset(int32_t* count, hipStream_t st) {
    hipLaunchKernelGGL(adapt_reset_kernel, dim3(1), dim3(64), 0, st, count);
    return hipGetLastError();
}

hipError_t launch_adapt(const AdaptArgs& a, const AdaptConst& c, hipStream_t st) {
    hipLaunchKernelGGL(adapt_kernel, dim3(a.batch), dim3(kAdThreads), 0, st, a, c);
    return hipGetLastError();
}

}  // namespace psp
