// sparse.h -- the sparse (fill-pattern) path (internal).
#pragma once

#include "common.h"
#include "plan.h"

namespace psp {

// Device copies of the plan's sparse index arrays.
struct SparseDevice {
    bool ready = false;
    int32_t* buf = nullptr;   // one allocation holding every array below
    const int32_t *perm, *l_ptr, *l_idx, *lrow_ptr, *lrow_idx, *upos, *lev_ptr[3], *lev_idx[3];
    const int32_t *a_ptr, *a_row, *a_src;   // permuted matrix by columns: row and CSR entry index
    const int32_t *diag_src;                 // per position: CSR entry of the diagonal or -1
};

hipError_t sparse_upload(const Symbolic& s, SparseDevice& d);
void sparse_free(SparseDevice& d);
size_t sparse_workspace_bytes(const Symbolic& s, int32_t batch, int32_t K, int32_t nrhs, int32_t keep);
int32_t sparse_nrhs_capacity(const Symbolic& s, int32_t batch, int32_t K, size_t ws_bytes);
hipError_t sparse_solve_batched(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                                const EpsSet& es, const double* dvec, int32_t nrhs, const double* B, double* X,
                                int32_t* info, void* ws, hipStream_t st);
hipError_t sparse_factor(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                         const EpsSet& es, const double* dvec, int32_t* info, void* ws, hipStream_t st);
hipError_t sparse_solve(const Symbolic& s, const SparseDevice& d, int32_t batch, const EpsSet& es, int32_t nrhs,
                        const double* B, double* Xk, int32_t transpose, const int32_t* info, void* ws,
                        hipStream_t st);

}  // namespace psp
