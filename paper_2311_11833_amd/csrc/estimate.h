// estimate.h -- launch parameters of the rho(A^{-1} D) power iteration (internal).
#pragma once

#include "common.h"

namespace psp {

struct RhoArgs {
    int32_t n, batch;
    int32_t mode;          // 0: normalise the start vector, 1: step, 2: step and add log g, 3: as 2 and finish
    double inv_count;      // 1 / number of steps whose log g is summed
    const double* src;     // batch x n: start vectors (mode 0) or the last solve's output
    const double* d;       // n, diagonal of D, or NULL (D = I)
    double* v;             // batch x n: normalised iterate
    double* B;             // batch x n: next right-hand side D v
    double* acc;           // batch: sum of log g
    double* rho;           // batch: exp(acc * inv_count), written in mode 3
};

hipError_t launch_rho_step(const RhoArgs& a, hipStream_t st);

}  // namespace psp
