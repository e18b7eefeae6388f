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
    // Tiles of 16 block rows: slot 16 t + r of tile t holds block row tail_rord[16 t + r] (-1:
    // padding), rows grouped so that a tile's rows share their columns below tail_b0; tile t lists
    // K_t, the columns below tail_b0 in which any of its rows has an entry, ascending, at
    // tail_kt[tail_kt_ptr[t] ..); tail_tiles = 0 when a tile would list 65535 columns or more.
    // The columns common to K_t and K_u, ascending, as (index in K_t) | (index in K_u) << 16 at
    // tail_pairs[tail_pp_ptr[t * tail_tiles + u] ..), padded to a multiple of four with
    // |K_t| | |K_u| << 16; tail_tiles = 0 as well when the lists would exceed kTailMaxPairs.
    int32_t tail_tiles = 0;
    std::vector<int32_t> tail_rord, tail_kt_ptr, tail_kt, tail_pp_ptr, tail_pairs;
};

constexpr int32_t kTailMin = 64;
constexpr size_t kTailMaxPairs = (size_t)1 << 28;
constexpr int32_t kTailAsmMaxB0 = 60000;   // columns before the block at most (an LDS map over them)

// Returns an empty string on success, else the reason the pattern was rejected.
std::string validate_csr(int32_t n, const int32_t* row_ptr, const int32_t* col_idx);

// Full analysis; natural = identity order.  Throws std::bad_alloc only.
void analyse(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, bool natural, Symbolic& s);

}  // namespace psp
