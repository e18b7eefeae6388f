// sparse.h -- the sparse (fill-pattern) path (internal).
#pragma once

#include "common.h"
#include "image.h"
#include "plan.h"

namespace psp {

// Device copies of the plan's index arrays for the sparse path, in one
// allocation.  Positions t index the L column pattern (CSC); the strictly
// upper part of U is stored at the same positions (row k of U has the column
// pattern of column k of L).
struct SpIdx {
    int32_t n, nnzl, nlev[3];
    const int32_t* perm;        // n
    const int32_t* l_ptr;       // n+1   L columns
    const int32_t* l_idx;       // nnzl  rows of each L column, ascending
    const int32_t* col_of;      // nnzl  column of position t
    const int32_t* r_ptr;       // n+1   L rows
    const int32_t* r_idx;       // nnzl  columns k of row i, ascending
    const int32_t* r_pos;       // nnzl  position of (i, k) in the column pattern
    const int32_t* src_l;       // nnzl  CSR entry of A feeding L position t (or -1)
    const int32_t* src_u;       // nnzl  CSR entry of A feeding U position t (or -1)
    const int32_t* src_d;       // n     CSR entry of the diagonal (or -1)
    const int32_t* lev_ptr[3];  // factor, L-solve, U-solve
    const int32_t* lev_idx[3];
    const int32_t* lpos_ptr;    // factor level -> range in lpos
    const int32_t* lpos;        // positions t of the columns of each factor level
    // Update lists (present when use_pairs): for factor item id (diagonal j ->
    // j, U position t -> n + t, L position t -> n + nnzl + t), the (L position,
    // U position) pairs of its dot product in ascending k, items
    // [pair_ptr[id], pair_ptr[id+1]) of pairs (two int32 each).
    int32_t use_pairs;
    int32_t pairs_below;        // lists exist for the items of the columns before this one
    const int32_t* pair_ptr;    // n + 2 nnzl + 1
    const int2* pairs;
    // Dense trailing block (plan.h; tail_n = 0: none): columns >= tail_b0 are factored as one
    // column-major tail_ld x tail_ld block (identity padding) at offset tail_off (doubles) of each
    // system's factors, followed by tail_ld x 64 doubles of right-hand-side scratch.
    int32_t tail_n, tail_b0, tail_ld, fac_lev_sp, nlev_sp[2];
    int64_t tail_off;
    const int32_t* tail_rcnt;       // tail_n: entries below tail_b0 in each row of the block
    const int32_t* tail_long;       // tail_nlong: block rows with at least 2,048 such entries (long chains)
    int32_t tail_nlong;
    const int32_t* tail_lastpos;    // tail_b0: position of (n-1, k) in column k of L, or -1
    const int32_t* tail_ccnt;       // tail_b0: entries of column k of L in rows before tail_b0
    const int32_t* lev_sp_ptr[2];   // L-solve / U-solve levels of the rows < tail_b0
    const int32_t* lev_sp_idx[2];
    // Assembly of the block on the MFMA unit (tail_tiles > 0): tiles of 16 block rows, slot s
    // holding block row tail_rord[s] (-1: padding); tile t's panel holds, for each column k of K_t
    // (plan.h) and a final zero column, its 16 slots' entries l_ik (and, in the U panel, u_ki),
    // 16 doubles per column, from panel column tail_kt_ptr[t] + t.
    // tail_mpos gives each panel entry's position in the L pattern (or -1: zero).  The updates of
    // block tile (t, u) are the columns common to K_t and K_u, ascending, as pairs
    // (column in panel t) | (column in panel u) << 16 at tail_pairs[tail_pp_ptr[t * tiles + u] ..),
    // padded to a multiple of four with the two zero columns.
    int32_t tail_tiles;
    int64_t tail_panel;                 // doubles of one panel set (16 x columns, rounded to 32)
    const int32_t* tail_rord;           // 16 x tiles
    const int32_t* tail_kt_ptr;         // tiles + 1
    const int32_t* tail_mpos;           // 16 x panel columns
    const int32_t* tail_pp_ptr;         // tiles^2 + 1
    const int32_t* tail_lpairs;         // tail_nlpairs: tile pairs of 512 or more steps (long chains)
    int32_t tail_nlpairs;
    const int32_t* tail_pairs;
};

// Dataflow step schedule of one perturbed system (factor, forward and
// backward substitution), for the step kernel.  Each factor or RHS entry
// advances its own fma chain, in the reference order, as soon as the inputs
// of its next updates are final; a step is the set of such chain segments
// that can run between two workgroup barriers.  Descriptors are laid out
// per step as rows x active threads, row r of thread t at base + r*tact + t.
struct StepIdx {
    int32_t nsteps = 0, threads = 0, ndesc = 0;
    int32_t packed = 0;               // L and U values share LDS slots (see steps.hip)
    int32_t pool = 0;                 // LDS doubles holding the L and U values (2 nnzL when not packed)
    const int4* meta = nullptr;       // per step: slot base, active threads, rows, 0
    const int4* desc = nullptr;       // task descriptors, 16 bytes each (see steps.hip)
    const int32_t* slot_l = nullptr;  // nnzl: LDS index that L position t is gathered into, or -1
    const int32_t* slot_u = nullptr;  // nnzl: the same for U
};

// The sparse path's part of the plan: pointers into the uploaded plan image
// (set by relocation) and host copies of the level boundaries.
struct SparseDevice {
    bool imaged = false;
    SpIdx idx{};
    std::vector<int32_t> h_lev_ptr[3];   // host copies for per-level launches
    std::vector<int32_t> h_lpos_ptr;
    std::vector<int32_t> h_lev_sp_ptr[2];
    int64_t h_tail_pairs = 0;            // entries of the tile-pair lists (multiple of 4 per pair)
    StepIdx st{};                        // step schedule (nsteps = 0 when it does not fit in LDS)
};

enum { kVarLds = 0, kVarGlobal = 1, kVarBatched = 2, kVarGrouped = 3, kVarSteps = 4, kVarTail = 5 };

// Launch choices the autotuner searches (psp_tune); the defaults are the heuristics.
struct Knobs {
    int32_t steps_mode = -1;   // step kernel: -1 by batch size, 0 one workgroup per system, 1 per Jacobian
    int32_t steps_wgcu = 0;    // step kernel: 0 as many workgroups per CU as LDS allows, 1 one per CU
    int32_t ring = 7;          // step kernel: descriptors in flight (7 or 4)
    int32_t tail_cols = 16;    // dense-block assembly: 16 tile pairs on the MFMA unit, or 4 or 1
                               // block columns per workgroup
    int32_t tail_il = -1;      // dense-block path, fused call: systems interleaved below the block
                               // (1), task-major (0), or -1 by batch size
    int32_t tail_lu = 0;       // dense-block LU and solves: one workgroup per system (1), or each
                               // panel step across the device (0)
};
int sparse_variant(const Symbolic& s, int64_t ntasks, int32_t nrhs, int forced);

// Appends the sparse path's arrays (and the step schedule, when it fits) to the
// plan image and binds d's pointers to them.
void sparse_image(const Symbolic& s, PlanImage& img, SparseDevice& d);
// step schedule (steps.hip): built by sparse_image when the system fits
bool steps_fit(const Symbolic& s, int32_t nrhs);
bool steps_ready(const SparseDevice& d);   // schedule built (it may not fit even when steps_fit holds)
void steps_image(const Symbolic& s, const std::vector<int32_t>& r_pos, PlanImage& img, SparseDevice& d);
// Set the kernels' dynamic LDS limits once per process (idempotent).
hipError_t sparse_kernel_attrs();
hipError_t steps_kernel_attrs();
// one launch; X (batch x n) combined in-kernel when per_jacobian, else Xk (batch x K x n) is written
// (per_jacobian with xk_too: both)
int steps_per_cu(const SparseDevice& d);   // step-kernel workgroups resident per CU (1 or 2)
int64_t steps_lds_bytes(const SparseDevice& d);   // dynamic LDS of one step-kernel workgroup (0: no schedule)
hipError_t steps_run(const SparseDevice& d, int32_t nnz, int32_t batch, const double* values, const EpsSet& es,
                     const double* dvec, const double* B, double* X, double* Xk, int32_t* info, bool per_jacobian,
                     hipStream_t st, bool xk_too = false, const Knobs& kn = Knobs());
// Per-system launch over the Jacobians list[0 .. *count-1] (device count, at most batch) with the
// nodes scale[s] eps_k (scale: powers of two); writes Xk[s][k] and info[s*K + k] of those only.
hipError_t steps_run_list(const SparseDevice& d, int32_t nnz, int32_t batch, const double* values, const EpsSet& es,
                          const double* dvec, const double* B, double* Xk, int32_t* info, const int32_t* list,
                          const int32_t* count, const double* scale, hipStream_t st);
// One workgroup per Jacobian (combine fused, no workspace) once the batch fills every resident slot.
bool steps_per_jacobian(const SparseDevice& d, int32_t batch);
// steps_run in the mode steps_per_jacobian picks, plus the combine launch in per-system mode
// (Xk: batch x K x n doubles of device memory, unused in per-Jacobian mode).
hipError_t steps_solve(const SparseDevice& d, int32_t n, int32_t nnz, int32_t batch, const double* values,
                       const EpsSet& es, const double* dvec, const double* B, double* X, int32_t* info, double* Xk,
                       hipStream_t st, const Knobs& kn = Knobs());
// The library's static device scratch (noalloc.hip): its size, and the current device's address.
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch(void** out);
bool sparse_fits_lds(const Symbolic& s, int32_t nrhs);
size_t sparse_workspace_bytes(const Symbolic& s, int32_t batch, int32_t K, int32_t nrhs, int32_t keep, int forced = -1);
// The dense-trailing-block path's fused call with the factors below the block interleaved, one
// right-hand side, also writing the per-system solutions Xk (batch x K x n, NaN where broken) and,
// with scale, Jacobian s at the nodes scale[s] eps_k: the error test's first and second solves.
bool sparse_tail_adaptive_ok(const Symbolic& s, const SparseDevice& d);
size_t sparse_tail_run_bytes(const Symbolic& s, int32_t batch, int32_t K);
hipError_t sparse_tail_run(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                           const EpsSet& es, const double* dvec, const double* B, double* X, int32_t* info, double* Xk,
                           const double* scale, void* ws, hipStream_t st, const Knobs& kn);
int32_t sparse_nrhs_capacity(const Symbolic& s, int32_t batch, int32_t K, size_t ws_bytes);
hipError_t sparse_solve_batched(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                                const EpsSet& es, const double* dvec, int32_t nrhs, const double* B, double* X,
                                int32_t* info, void* ws, hipStream_t st, int forced = -1, const Knobs& kn = Knobs());
hipError_t sparse_factor(const Symbolic& s, const SparseDevice& d, int32_t batch, const double* values,
                         const EpsSet& es, const double* dvec, int32_t* info, void* ws, hipStream_t st);
hipError_t sparse_solve(const Symbolic& s, const SparseDevice& d, int32_t batch, const EpsSet& es, int32_t nrhs,
                        const double* B, double* Xk, int32_t transpose, const int32_t* info, void* ws,
                        hipStream_t st);

}  // namespace psp
