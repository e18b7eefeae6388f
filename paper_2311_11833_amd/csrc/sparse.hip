// sparse.hip -- sparse (fill-pattern) path: placeholder until its kernels land.
#include "sparse.h"

namespace psp {

hipError_t sparse_upload(const Symbolic&, SparseDevice&) { return hipErrorNotSupported; }
void sparse_free(SparseDevice& d) { if (d.buf) (void)hipFree(d.buf); d.buf = nullptr; d.ready = false; }
size_t sparse_workspace_bytes(const Symbolic&, int32_t, int32_t, int32_t, int32_t) { return 0; }
int32_t sparse_nrhs_capacity(const Symbolic&, int32_t, int32_t, size_t) { return 0; }
hipError_t sparse_solve_batched(const Symbolic&, const SparseDevice&, int32_t, const double*, const EpsSet&,
                                const double*, int32_t, const double*, double*, int32_t*, void*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t sparse_factor(const Symbolic&, const SparseDevice&, int32_t, const double*, const EpsSet&, const double*,
                         int32_t*, void*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t sparse_solve(const Symbolic&, const SparseDevice&, int32_t, const EpsSet&, int32_t, const double*, double*,
                        int32_t, const int32_t*, void*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace psp
