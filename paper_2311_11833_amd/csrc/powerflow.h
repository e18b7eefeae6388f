// powerflow.h -- launch parameters of the Newton-Raphson power-flow kernels (internal).
#pragma once

#include "common.h"

namespace psp {

// Scenario status inside the Newton loop (the public codes are 0..3).
constexpr int32_t kPfRunning = -1;
constexpr int32_t kPfConverged = 0, kPfMaxIter = 1, kPfBreakdown = 2, kPfDiverged = 3;

struct PfArgs {
    int32_t N, n, nnz, batch;
    const int32_t* yptr;      // N+1: bus admittance CSR
    const int32_t* ycol;      // ny
    const double* g;          // ny
    const double* b;          // ny
    const int32_t* pv;        // N: nonzero = voltage-controlled bus
    const int4* pos;          // ny: Jacobian CSR positions of (dP/dtheta_j, dP/dV_j, dQ/dtheta_j, dQ/dV_j)
    const int32_t* pos_lam;   // N: position of dP_i/dlambda
    int32_t pos_ref;          // position of the angle-reference entry
    const int32_t* idx;       // batch: scenario of block r, or NULL (block r is scenario r)
    const double* x;          // scenarios x n: [theta | |V| | lambda]
    const double* spec;       // scenarios x n: [P0 | Q0 or V_set | theta_ref]
    const double* part;       // scenarios x N
    double* F;                // batch x n, row r for block r
    double* J;                // batch x nnz, row r for block r, or NULL
    double* fnorm;            // per scenario, or NULL: max |F| (NaN if any entry is NaN)
    int32_t* status;          // per scenario, or NULL: running -> converged / diverged
    double tol;
};

hipError_t launch_pf_eval(const PfArgs& a, hipStream_t st);
hipError_t launch_pf_status(int32_t batch, int32_t* status, int32_t* iters, int32_t finish, hipStream_t st);
// block r updates scenario idx[r] (idx NULL: scenario r) from dx row r and info row r
hipError_t launch_pf_update(int32_t batch, int32_t n, int32_t K, const int32_t* idx, double* x, const double* dx,
                            const int32_t* info, int32_t* status, int32_t* iters, hipStream_t st);

}  // namespace psp
