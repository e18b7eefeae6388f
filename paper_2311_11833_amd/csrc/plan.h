// plan.h -- host-side symbolic analysis of one sparsity pattern (internal).
//
// The static pivot sequence (Sec. II-C) is computed once per pattern on the
// host and reused by every perturbed system.  The definitions (ordering
// rule, fill, etree, level sets) are the ones stated in psp.h.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace psp {

struct Symbolic {
    int32_t n = 0, nnz = 0, ndense = 0;
    std::vector<int32_t> row_ptr, col_idx;        // user pattern (CSR)
    std::vector<int32_t> perm, iperm, parent;     // perm[q] = original index at position q
    std::vector<int32_t> l_ptr, l_idx;            // L column pattern (strictly lower), permuted
    std::vector<int32_t> lrow_ptr, lrow_idx;      // L row pattern (k < i with L_ik != 0)
    std::vector<int32_t> lev_ptr[3], lev_idx[3];  // factor, L-solve, U-solve
    int64_t flops_dense = 0, flops_sparse = 0;
    // Dense trailing block: the last tail_n columns of L are full (|L(:,j)| = n-1-j) and every
    // column before tail_b0 = n - tail_n sits on a lower factor level than every tail column, so
    // factor levels [0, fac_lev_sp) hold exactly the columns < tail_b0.  lev_sp_* are the L-solve
    // and U-solve levels restricted to rows < tail_b0 (empty levels dropped).  tail_n = 0 when
    // the block is smaller than kTailMin or the levels do not separate.
    int32_t tail_n = 0, tail_b0 = 0, fac_lev_sp = 0;
    std::vector<int32_t> lev_sp_ptr[2], lev_sp_idx[2];
};

constexpr int32_t kTailMin = 64;
constexpr int32_t kTailAsmMaxB0 = 60000;   // columns before the block at most (an LDS map over them)

// Returns an empty string on success, else the reason the pattern was rejected.
std::string validate_csr(int32_t n, const int32_t* row_ptr, const int32_t* col_idx);

// Full analysis; natural = identity order.  Throws std::bad_alloc only.
void analyse(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, bool natural, Symbolic& s);

}  // namespace psp
