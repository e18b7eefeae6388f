// adapt.h -- launch parameters of the error test and node rescaling (internal).
#pragma once

#include "common.h"

namespace psp {

// Per-call constants, computed on the host from the first node set.
struct AdaptConst {
    double w1[kMaxK];   // weights of the divided difference over nodes 0..K-1
    double w2[kMaxK];   // ... over nodes 0..K-2 (entries K-1.. unused)
    double c[kMaxK];    // combination weights
    double P;           // prod_k |eps_k|, ascending k
    double b;           // (50 u) / max_k |eps_k|
};

struct AdaptArgs {
    int32_t n, K, batch;  // batch: Jacobians (pass 1) or list capacity (pass 2); the grid size
    int32_t pass;         // 1: estimate, decide, append to the list; 2: list entries, rescaled nodes
    int32_t combine;      // 1: X = sum_k c_k Xk (written); 0: X already holds the combination
    double tol;
    const double* Xk;     // batch x K x n perturbed solutions (original numbering)
    double* X;            // batch x n
    double* est;          // batch
    double* scale;        // batch: 1, or the node scale 2^-j of a rescaled Jacobian
    int32_t* list;        // Jacobians to solve again
    int32_t* count;       // their number (zeroed by launch_adapt_reset)
};

hipError_t launch_adapt_reset(int32_t* count, hipStream_t st);
hipError_t launch_adapt(const AdaptArgs& a, const AdaptConst& c, hipStream_t st);

}  // namespace psp
