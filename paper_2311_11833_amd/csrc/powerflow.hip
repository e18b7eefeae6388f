// powerflow.hip -- the Newton-Raphson power flow that the paper's solve sits
// in (Sec. IV: one Jacobian solve per Newton step of a distributed-slack AC
// power flow), for gfx950, FP64.
//
// pf_eval: one workgroup per scenario, one lane per bus (strided).  The lane
// for bus i walks row i of the bus admittance matrix once: for each entry it
// forms cos/sin of theta_i - theta_j, accumulates
//     P_i += V_i V_j (G cos + B sin),   Q_i += V_i V_j (G sin - B cos)
// (plain multiply-adds in CSR order, no contraction), and writes the four
// off-diagonal Jacobian entries of (i, j) straight into the caller's CSR
// values; the diagonal entries need P_i and Q_i and follow the row.  A PV
// bus writes the unit row |V_i| - V_set instead of its Q row.  The mismatch
// F and its max-norm (a workgroup reduction) come out of the same pass.  The
// work is a few kB per scenario, latency-bound, and one pass replaces the
// mismatch and Jacobian-assembly kernels a host loop would launch.
//
// pf_update: x <- x - dx for scenarios still running whose K perturbed
// factorisations all succeeded; a nonzero info marks a breakdown instead.
//
// Inside the Newton loop both kernels take a list of the scenarios still
// running (block r works on scenario idx[r] and on row r of F, J, dx and
// info), so evaluations and solves shrink with the set of running scenarios.
#include "powerflow.h"

namespace psp {

namespace {
constexpr int kPfThreads = 256;

// max that keeps a NaN once one is seen
__device__ __forceinline__ double nanmax(double m, double a) { return (a != a || a > m) ? a : m; }

__global__ __launch_bounds__(kPfThreads) void pf_eval_kernel(PfArgs a) {
    __shared__ double red[kPfThreads];
    const int r = blockIdx.x;
    const int s = a.idx ? a.idx[r] : r;
    const int N = a.N;
    const double* xs = a.x + (int64_t)s * a.n;
    const double* sp = a.spec + (int64_t)s * a.n;
    const double* pt = a.part + (int64_t)s * N;
    double* F = a.F + (int64_t)r * a.n;
    double* J = a.J ? a.J + (int64_t)r * a.nnz : nullptr;
    double m = 0.0;
    for (int i = threadIdx.x; i < N; i += kPfThreads) {
        const double ti = xs[i], vi = xs[N + i];
        const bool isPV = a.pv[i] != 0;
        double P = 0.0, Q = 0.0, Gd = 0.0, Bd = 0.0;
        int ed = -1;
        for (int e = a.yptr[i]; e < a.yptr[i + 1]; ++e) {
            const int j = a.ycol[e];
            const double G = a.g[e], B = a.b[e];
            double c = 1.0, sn = 0.0;
            if (j != i) sincos(ti - xs[j], &sn, &c);
            const double w = vi * xs[N + j];
            const double pa = G * c + B * sn;
            const double qa = G * sn - B * c;
            P = P + w * pa;
            Q = Q + w * qa;
            if (j == i) {
                ed = e;
                Gd = G;
                Bd = B;
            } else if (J) {
                const int4 p = a.pos[e];
                J[p.x] = w * qa;
                J[p.y] = vi * pa;
                J[p.z] = isPV ? 0.0 : -(w * pa);
                J[p.w] = isPV ? 0.0 : vi * qa;
            }
        }
        const double v2 = vi * vi;
        if (J && ed >= 0) {
            const int4 p = a.pos[ed];
            J[p.x] = -Q - Bd * v2;
            J[p.y] = P / vi + Gd * vi;
            J[p.z] = isPV ? 0.0 : P - Gd * v2;
            J[p.w] = isPV ? 1.0 : Q / vi - Bd * vi;
        }
        if (J) J[a.pos_lam[i]] = -pt[i];
        const double fp = (P - sp[i]) - pt[i] * xs[2 * N];
        const double fq = isPV ? vi - sp[N + i] : Q - sp[N + i];
        F[i] = fp;
        F[N + i] = fq;
        m = nanmax(nanmax(m, fabs(fp)), fabs(fq));
        if (i == 0) {
            const double fr = xs[0] - sp[2 * N];
            F[2 * N] = fr;
            if (J) J[a.pos_ref] = 1.0;
            m = nanmax(m, fabs(fr));
        }
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kPfThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double fn = red[0];
        if (a.fnorm) a.fnorm[s] = fn;
        if (a.status && a.status[s] == kPfRunning) {
            if (fn <= a.tol) a.status[s] = kPfConverged;
            else if (!isfinite(fn)) a.status[s] = kPfDiverged;
        }
    }
}

__global__ void pf_status_kernel(int32_t batch, int32_t* status, int32_t* iters, int32_t finish) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    if (finish) {
        if (status[s] == kPfRunning) status[s] = kPfMaxIter;
    } else {
        status[s] = kPfRunning;
        iters[s] = 0;
    }
}

__global__ __launch_bounds__(kPfThreads) void pf_update_kernel(int32_t n, int32_t K, const int32_t* idx, double* x,
                                                              const double* dx, const int32_t* info, int32_t* status,
                                                              int32_t* iters) {
    const int r = blockIdx.x;
    const int s = idx ? idx[r] : r;
    __shared__ int go;
    if (threadIdx.x == 0) {
        int g = status[s] == kPfRunning ? 1 : 0;
        if (g)
            for (int k = 0; k < K; ++k)
                if (info[(int64_t)r * K + k] != 0) g = 2;
        if (g == 2) status[s] = kPfBreakdown;
        if (g == 1) iters[s] += 1;
        go = g;
    }
    __syncthreads();
    if (go != 1) return;
    double* xs = x + (int64_t)s * n;
    const double* d = dx + (int64_t)r * n;
    for (int i = threadIdx.x; i < n; i += kPfThreads) xs[i] = xs[i] - d[i];
}
}  // namespace

hipError_t launch_pf_eval(const PfArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(pf_eval_kernel, dim3(a.batch), dim3(kPfThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pf_status(int32_t batch, int32_t* status, int32_t* iters, int32_t finish, hipStream_t st) {
    hipLaunchKernelGGL(pf_status_kernel, dim3((batch + 255) / 256), dim3(256), 0, st, batch, status, iters, finish);
    return hipGetLastError();
}

hipError_t launch_pf_update(int32_t batch, int32_t n, int32_t K, const int32_t* idx, double* x, const double* dx,
                            const int32_t* info, int32_t* status, int32_t* iters, hipStream_t st) {
    hipLaunchKernelGGL(pf_update_kernel, dim3(batch), dim3(kPfThreads), 0, st, n, K, idx, x, dx, info, status, iters);
    return hipGetLastError();
}

}  // namespace psp
