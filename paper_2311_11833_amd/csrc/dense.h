// dense.h -- launch parameters and launchers of the dense path (internal).
#pragma once

#include "common.h"

namespace psp {

struct DenseArgs {
    int32_t n, n_pad, ld, nrhs, nnz, batch;
    const int32_t* dst;       // nnz: slot offset (column-major) of each CSR entry, permuted
    const int32_t* perm;      // n: position -> original index
    const double* values;     // batch x nnz
    const double* dvec;       // n (original order) or NULL (D = I)
    const double* B;          // batch x n x nrhs, or NULL when nrhs == 0
    double* Xk;               // batch x K x n x nrhs, or NULL when nrhs == 0
    int32_t* info;            // batch x K
    double* slots;            // workspace slots
    int64_t slot_stride;      // doubles per slot
    int32_t ntasks;           // batch * K
    int32_t keep;             // slot = task (1) or slot = blockIdx.x (0)
    int32_t per_jacobian;     // 1: one task per Jacobian, combine into X in-kernel
    double* X;                // batch x n x nrhs (per_jacobian only)
};

struct DenseSolveArgs {
    int32_t n, n_pad, ld, nrhs, K, ntasks, trans;
    const int32_t* perm;
    const double* slots;      // factors, one slot per task
    int64_t slot_stride;
    const double* B;          // batch x n x nrhs
    double* Xk;               // batch x K x n x nrhs
    const int32_t* info;      // batch x K
    double* tmp;              // ntasks x (ld * nrhs) scratch
};

int dense_lds_bytes();
int dense_panel();
hipError_t launch_dense_factor_solve(const DenseArgs& a, const EpsSet& es, int grid, hipStream_t st);
hipError_t launch_dense_solve(const DenseSolveArgs& a, int grid, hipStream_t st);
hipError_t launch_combine(int64_t len, int32_t batch, const EpsSet& es, const double* Xk, double* X, hipStream_t st);

// error test (residual.hip)
constexpr int32_t kResLds = 16384;   // rows whose residual is staged in LDS; beyond, R is required
struct ResArgs {
    int32_t n, nnz, batch, nrhs, stage;
    const int32_t* rowptr;   // n+1, user CSR
    const int32_t* cols;     // nnz
    const double* values;    // batch x nnz
    const double* B;         // batch x n x nrhs
    const double* X;         // batch x n x nrhs
    double* R;               // batch x n x nrhs or NULL
    double* rnorm;           // batch x nrhs
    double* bnorm;           // batch x nrhs or NULL
};
hipError_t launch_residual(ResArgs a, hipStream_t st);
hipError_t launch_grad_values(int32_t n, int32_t nnz, int32_t batch, int32_t nrhs, const EpsSet& es,
                              const int32_t* rows, const int32_t* cols, const double* Lamk, const double* Xk,
                              double* gA, hipStream_t st);
hipError_t dense_occupancy(int* blocks_per_cu);
hipError_t dense_kernel_attrs();   // once per process: the dense kernels' dynamic LDS limit

}  // namespace psp
