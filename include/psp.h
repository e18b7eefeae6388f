/*
 * psp.h -- C ABI of libpsp: perturbation-induced static pivoting on MI355X
 * (gfx950), FP64 throughout.
 *
 * Method (arXiv 2311.11833, Alg. 1): instead of pivoting, factor K perturbed
 * systems A + eps_k D without row exchanges, solve each, and combine the
 * perturbed solutions x_k with weights c_k so that the A^{-1} b term is kept
 * and the first K-1 powers of eps cancel (Sec. III-A, Theorem 1, Remark 2):
 *     x_hat = sum_k c_k x_k,    sum_k c_k eps_k^j = delta_{j0}, j < K.
 *
 * Conventions shared by every call:
 *   - Every call returns psp_status; no C++ exception crosses the ABI.  The
 *     text of the last failure on the calling thread is psp_last_error().
 *   - All reals are IEEE binary64, all indices int32.  Matrices arrive in
 *     CSR form for one sparsity pattern; "values" are the nnz entries in that
 *     CSR order.  Dense vectors with nrhs right-hand sides are row-major
 *     n x nrhs (entry (i, r) at i*nrhs + r).
 *   - Pointers documented "device" are device memory owned by the caller;
 *     the library never allocates or frees device memory.  That includes the
 *     plan's own index arrays: psp_plan_device_bytes sizes them and
 *     psp_plan_upload copies them into a caller buffer, once per plan, before
 *     any numeric call (which then allocates nothing and may be captured in a
 *     HIP graph).  Pointers documented "host" are read
 *     during the call only.  "stream" is a hipStream_t (NULL = the null
 *     stream); device work is enqueued on it and the call returns without
 *     waiting, so device outputs are valid after the caller synchronises
 *     the stream.
 *   - Numerical breakdown is not a call error: it is reported per system in
 *     the device array "info" (0 = ok, j+1 = pivot j was exactly zero or not
 *     finite; the LAPACK getrf convention), written by the kernels.  The
 *     outputs of a system with info != 0 are NaN.
 *   - Handles (psp_plan, psp_factors) are host objects owned by the library
 *     and freed by the matching destroy/release call.
 */
#ifndef PSP_H
#define PSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSP_API __attribute__((visibility("default")))

typedef enum {
    PSP_OK = 0,
    PSP_E_INVALID = 1,      /* bad size, NULL pointer or malformed CSR pattern          */
    PSP_E_EPS = 2,          /* perturbation nodes not distinct, zero or not finite      */
    PSP_E_NOMEM = 3,        /* caller workspace too small, or host allocation failed    */
    PSP_E_HIP = 4,          /* HIP runtime error (including one left by earlier work)   */
    PSP_E_STATE = 5,        /* handle used in the wrong order or with a mismatched plan */
    PSP_E_UNSUPPORTED = 6   /* device is not gfx950, or size beyond the chosen path     */
} psp_status;

/* Message describing the last non-OK status returned on this thread. */
PSP_API const char* psp_last_error(void);

/* ABI version (major*100 + minor). */
PSP_API int32_t psp_version(void);

/* ------------------------------------------------------------------------
 * Plan: symbolic analysis of one sparsity pattern, host CPU, once per
 * pattern.  This is the static pivot sequence of Sec. II-C, computed once and
 * reused by every perturbed system, every Newton step and every scenario.
 *   S      = pat(A) | pat(A^T) | diagonal (the diagonal is always present
 *            because D is diagonal).
 *   order  PSP_ORDER_MD: minimum degree on the elimination graph of S with
 *            exact degrees; ties go to the smallest index; a vertex whose
 *            degree d in S satisfies d > 16 and d*d > 100*n is set aside
 *            and ordered last (ascending index).
 *          PSP_ORDER_NATURAL: the identity.
 *   fill   L = strictly lower symbolic factor of P S P^T (column pattern),
 *          U = its transpose plus the diagonal.
 *   etree  parent[j] = smallest row index of L(:, j), -1 for a root.
 *   levels factor: etree height; L-solve: lev(i) = 1 + max lev(j) over
 *          L_ij != 0; U-solve: lev(i) = 1 + max lev(j) over U_ij != 0, j > i;
 *          each level lists its indices ascending.
 * row_ptr (host, n+1) and col_idx (host, nnz) must describe a square CSR
 * pattern with strictly ascending column indices in each row.
 * ---------------------------------------------------------------------- */
typedef struct psp_plan_s* psp_plan;

enum { PSP_ORDER_MD = 0, PSP_ORDER_NATURAL = 1 };

PSP_API psp_status psp_plan_create(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                           uint32_t flags, psp_plan* out);

typedef struct {
    int32_t n;
    int32_t nnz;               /* entries of A                                      */
    int64_t nnz_l;             /* strictly lower entries of L (= strictly upper of U) */
    int32_t ndense;            /* vertices set aside by the dense rule              */
    int32_t nlev[3];           /* levels: factor, L-solve, U-solve                  */
    int64_t flops_dense_factor;/* n(n-1)/2 divisions + 2 * sum_k (n-1-k)^2 fma flops */
    int64_t flops_sparse_factor;/* sum_j (|L(:,j)| + 2*|L(:,j)|^2) on the fill      */
    int32_t steps;             /* barrier steps of the LDS step schedule (0: none)  */
    int32_t steps_packed;      /* 1 if its L/U values share LDS slots               */
    int64_t steps_lds_bytes;   /* dynamic LDS of one step-kernel workgroup          */
    int32_t steps_per_cu;      /* step-kernel workgroups resident per CU (0, 1, 2)  */
    int64_t device_bytes;      /* psp_plan_device_bytes                              */
    int32_t tail_n;            /* columns of the dense trailing block (0: none)      */
    int32_t tail_fac_levels;   /* factor levels below it                             */
    int32_t tail_tiles;        /* 16-row tiles of its assembly on the MFMA unit (0: none) */
    int64_t tail_mfma;         /* 16x16x4 FP64 MFMA steps of one system's assembly  */
} psp_plan_info_t;

PSP_API psp_status psp_plan_info(psp_plan plan, psp_plan_info_t* out);

/* Copies the symbolic arrays (host buffers sized from psp_plan_info):
 * perm[n] (position -> original index), iperm[n], parent[n], l_ptr[n+1],
 * l_idx[nnz_l] (rows of each L column, ascending, permuted numbering), and
 * for t = 0, 1, 2 (factor, L-solve, U-solve) lev_ptr[t][nlev[t]+1] and
 * lev_idx[t][n].  Any output may be NULL to skip it. */
PSP_API psp_status psp_plan_export(psp_plan plan, int32_t* perm, int32_t* iperm, int32_t* parent,
                           int32_t* l_ptr, int32_t* l_idx, int32_t* lev_ptr[3], int32_t* lev_idx[3]);

PSP_API void psp_plan_destroy(psp_plan plan);

/* Device copy of the plan (the static pivot sequence of Sec. II-C and
 * everything derived from it: fill patterns, level lists, update lists, the
 * step schedule, dense slot offsets).  psp_plan_device_bytes returns the bytes
 * it needs (0 on host allocation failure); psp_plan_upload copies it into
 * `dev` (device, caller-owned, 256-byte aligned, at least that many bytes) on
 * `stream` and waits for the copy.  The plan then refers to that buffer, which
 * must stay alive and unmodified while the plan is used; a later upload
 * rebinds the plan to a new buffer (on the then current device).  Numeric calls
 * on a plan that is not uploaded to the current device return PSP_E_STATE.
 * PSP_E_UNSUPPORTED if the device is not gfx950. */
PSP_API size_t psp_plan_device_bytes(psp_plan plan);
PSP_API psp_status psp_plan_upload(psp_plan plan, void* dev, size_t dev_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Weights (host): c_k = prod_{l != k} eps_l / (eps_l - eps_k), the unique
 * solution of sum_k c_k eps_k^j = delta_{j0} for j < K.  For the paper's
 * nodes +-alpha*eps (alpha = 1..m) this is c = beta_alpha / 2 with
 * beta = (Gamma_m^T)^{-1} e1 (Remark 2).  eps (host, K), c (host, K).
 * PSP_E_EPS if the nodes are not distinct, zero or finite.
 * ---------------------------------------------------------------------- */
PSP_API psp_status psp_weights(int32_t K, const double* eps, double* c);

/* ------------------------------------------------------------------------
 * Numeric paths.
 *   PSP_PATH_DENSE    each perturbed system as a dense n x n matrix (the
 *                     batched dense factorisation of Sec. IV), n <= 4096.
 *   PSP_PATH_SPARSE   factors on the plan's fill pattern, level-scheduled
 *                     (the sparse batched factorisation named in Sec. IV/V);
 *                     the library picks one of the three executions below.
 *   PSP_PATH_SPARSE_BATCHED  systems interleaved across lanes, one launch per
 *                     level for the whole batch (needs the plan's update
 *                     lists: at most 32 Mi multiply-adds per factorisation).
 *   PSP_PATH_SPARSE_LDS      one workgroup per system, factors in LDS (needs
 *                     (n + 2 nnz_l + n nrhs) * 8 <= 152 KiB).
 *   PSP_PATH_SPARSE_LEVELS   one launch per level, factors in the workspace.
 *   PSP_PATH_SPARSE_GROUPED  systems interleaved as in _BATCHED, but each
 *                     workgroup walks all levels for 32 systems with
 *                     workgroup barriers (two launches per call).
 *   PSP_PATH_SPARSE_STEPS    one workgroup per Jacobian runs its K systems in
 *                     LDS on a dataflow step schedule: every factor and RHS
 *                     entry advances its own update chain as soon as its
 *                     inputs are final, forward substitution overlapping the
 *                     factorisation; one launch per call (needs nrhs = 1 and
 *                     (3 n + 2 nnz_l) * 8 <= 152 KiB).
 *   PSP_PATH_SPARSE_TAIL     per-level kernels for the columns before the
 *                     plan's dense trailing block (the last columns of the
 *                     factor when they are full and sit above every other
 *                     column in the elimination tree: the top separator and
 *                     the slack column), which is then factored and solved
 *                     densely in panels on the MFMA unit, several workgroups
 *                     per system (needs a trailing block of at least 64
 *                     columns).
 *   PSP_PATH_AUTO     the path psp_tune chose for this (batch, K, nrhs), else
 *                     a size heuristic.
 * A path that cannot run the plan returns PSP_E_UNSUPPORTED.  Every path
 * returns the same bits (each applies the same operation sequence).
 * ---------------------------------------------------------------------- */
enum {
    PSP_PATH_AUTO = 0,
    PSP_PATH_DENSE = 1,
    PSP_PATH_SPARSE = 2,
    PSP_PATH_SPARSE_BATCHED = 3,
    PSP_PATH_SPARSE_LDS = 4,
    PSP_PATH_SPARSE_LEVELS = 5,
    PSP_PATH_SPARSE_GROUPED = 6,
    PSP_PATH_SPARSE_STEPS = 7,
    PSP_PATH_SPARSE_TAIL = 8
};

/* Bytes of device workspace psp_factor / psp_solve_batched need for `batch`
 * Jacobians, K nodes and nrhs right-hand sides on `path` (the scratch of
 * Alg. 1 steps 2-4: factors of the perturbed systems and their solutions
 * before the combination).  With keep != 0 the factors of all batch*K systems
 * stay resident for psp_solve and the adjoint.  PSP_PATH_AUTO returns the
 * maximum over the paths.  0 for an invalid plan or size. */
PSP_API size_t psp_workspace_bytes(psp_plan plan, int32_t path, int32_t batch, int32_t K, int32_t nrhs,
                           int32_t keep);

/* ------------------------------------------------------------------------
 * psp_solve_batched -- Alg. 1 steps 1-4 for a batch of Jacobians that share
 * the plan's pattern, in one fused launch: for Jacobian s and node k it forms
 * P (A_s + eps_k D) P^T, factors it without pivoting, solves with the
 * nrhs right-hand sides, and accumulates x_hat_s = sum_k c_k x_sk (ascending
 * k) into X.
 *   values  device, batch x nnz           eps   host, K distinct nonzero
 *   d       device, n (NULL: D = I)       B     device, batch x n x nrhs
 *   X       device, batch x n x nrhs      info  device, batch x K (int32)
 *   ws      device workspace of at least psp_workspace_bytes(plan, path,
 *           batch, K, nrhs, 0) bytes.
 * ---------------------------------------------------------------------- */
PSP_API psp_status psp_solve_batched(psp_plan plan, int32_t path, int32_t batch, const double* values,
                             int32_t K, const double* eps, const double* d, int32_t nrhs,
                             const double* B, double* X, int32_t* info, void* ws, size_t ws_bytes,
                             void* stream);

/* ------------------------------------------------------------------------
 * psp_solve_adaptive -- Alg. 1 with its error test (step 5) deciding the
 * perturbation size per Jacobian (Sec. V leaves the perturbation strategy
 * open; the expansion of Sec. II-B converges only while |eps| rho(A^{-1}D) < 1
 * and its truncation grows with the nodes, its rounding with their inverse).
 * Step-schedule path (else, for a pattern without one, the dense-trailing-
 * block path, whose second solve runs every Jacobian again at its scale: 1
 * for those that passed, which reproduces their first solve bit for bit),
 * nrhs = 1, K >= 3 nodes eps (host, distinct, nonzero).
 *   1. Every Jacobian is solved at the nodes eps (as psp_solve_batched).
 *   2. Error test without A: with f_j the divided difference of the K
 *      perturbed solutions over nodes 0..j (= (-1)^j M^j x* up to O(eps),
 *      M = A^{-1} D) and m_j = max_i |f_j[i]|,
 *        rho_hat = m_{K-1} / m_{K-2},
 *        est     = |prod eps_k| m_{K-1} rho_hat / ||x_hat||_inf,
 *      the leading term -(prod eps_k) M^K x* of the combination's error
 *      (Theorem 1), relative.
 *   3. A Jacobian with est > tol (or NaN) is solved again at the nodes
 *      s eps_k, s = 2^-j (the weights do not change): j is the smallest
 *      j >= 1 with 2^{-j(K+1)} <= q = b / (K a), i.e. s is the largest power
 *      of two at most min(s*, 1/2) where s* minimises the error model
 *      a s^K + b / s; a = est (est < 1e-2) or |prod eps_k| rho_hat^K
 *      (series possibly divergent), b = 50 u / max|eps_k|, u = 2^-53 (the
 *      rounding of the pivot-free solves grows like 1/eps); at most j = 60,
 *      j = 10 for a NaN est.  Its est is then taken at the new nodes.
 *   values device batch x nnz;  d device n or NULL (D = I);  B, X device
 *   batch x n;  info device batch x K (of the nodes finally used);
 *   est device batch (final estimate);  scale device batch (1, or 2^-j);
 *   ws device, psp_solve_adaptive_workspace_bytes(plan, batch, K) bytes,
 *   256-byte aligned.  Asynchronous on `stream` (no host synchronisation:
 *   the list of rescaled Jacobians stays on the device).
 * PSP_E_INVALID for NULL pointers, batch < 1, K < 3 or a negative or
 * non-finite tol; PSP_E_UNSUPPORTED when the plan has neither path.
 * ---------------------------------------------------------------------- */
PSP_API size_t psp_solve_adaptive_workspace_bytes(psp_plan plan, int32_t batch, int32_t K);
PSP_API psp_status psp_solve_adaptive(psp_plan plan, int32_t batch, const double* values, int32_t K,
                                      const double* eps, const double* d, double tol, const double* B, double* X,
                                      int32_t* info, double* est, double* scale, void* ws, size_t ws_bytes,
                                      void* stream);

/* ------------------------------------------------------------------------
 * psp_solve_batched_noalloc -- psp_solve_batched on PSP_PATH_SPARSE_STEPS with
 * nrhs = 1 and no workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The call allocates nothing: when the batch is too
 * small for one workgroup per Jacobian, the per-system solutions (batch x K x n
 * doubles) go to a static scratch array that the library holds on every
 * device it runs on (16 MiB per device, kept until the process ends).
 * Arguments and results as for psp_solve_batched (the same bits).
 * PSP_E_UNSUPPORTED when the plan has no step schedule or the batch needs more
 * than the 16 MiB of scratch.  Every call on a device shares that device's
 * scratch: calls that overlap on one device (concurrent streams or threads)
 * race and must be serialised by the caller.
 * ---------------------------------------------------------------------- */
PSP_API psp_status psp_solve_batched_noalloc(psp_plan plan, int32_t batch, const double* values, int32_t K,
                                             const double* eps, const double* d, const double* B, double* X,
                                             int32_t* info, void* stream);

/* ------------------------------------------------------------------------
 * Groups: Alg. 1 steps 1-4 for an uneven batch, i.e. several items of
 * Jacobians of different patterns, enqueued together (Sec. IV: batched solves
 * whose time should not grow with the number of systems).  Item i holds
 * shapes[i].batch Jacobians sharing shapes[i].plan's pattern, solved on
 * shapes[i].path (PSP_PATH_AUTO: the plan's tuned choice, else the size
 * heuristic, resolved at creation).  psp_group_create (host) checks the
 * items (every plan must be uploaded to the current device), orders them
 * longest first by their symbolic flop count, deals them over up to four
 * stream lanes (the caller's stream and three the group owns, each at the
 * default priority) and lays out one workspace: psp_group_workspace_bytes.
 *   psp_group_run      enqueues every item: the lanes fork from `stream`
 *                      and join back into it, so the work is ordered after
 *                      earlier work on `stream` and later work waits for all
 *                      of it.  tasks[i] gives item i's device arrays:
 *                      values batch x nnz, d n or NULL (D = I), B and X
 *                      batch x n x nrhs, info batch x K.
 *   psp_group_capture  the same sequence captured from `stream` into one HIP
 *                      graph (thread-local capture mode); *graph_exec
 *                      receives the instantiated graph, which
 *                      psp_graph_launch replays on any stream and
 *                      psp_graph_destroy frees.  The graph keeps the task
 *                      pointers and the workspace it was captured with.
 *                      `stream` must be a created stream: the null stream
 *                      cannot be captured (PSP_E_INVALID).
 * Errors as for psp_solve_batched, plus PSP_E_STATE for a group used on
 * another device.  Calls on one group must not overlap (its lanes are shared).
 * ---------------------------------------------------------------------- */
typedef struct psp_group_s* psp_group;

typedef struct psp_group_shape {
    psp_plan plan;
    int32_t batch;
    int32_t path;
} psp_group_shape_t;

typedef struct psp_group_task {
    const double* values;
    const double* d;
    const double* B;
    double* X;
    int32_t* info;
} psp_group_task_t;

PSP_API psp_status psp_group_create(int32_t nitems, const psp_group_shape_t* shapes, int32_t K, const double* eps,
                                    int32_t nrhs, psp_group* out);
PSP_API size_t psp_group_workspace_bytes(psp_group g);
PSP_API psp_status psp_group_run(psp_group g, const psp_group_task_t* tasks, void* ws, size_t ws_bytes, void* stream);
PSP_API psp_status psp_group_capture(psp_group g, const psp_group_task_t* tasks, void* ws, size_t ws_bytes,
                                     void* stream, void** graph_exec);
/* Groups with the error test (psp_solve_adaptive for every item: the first
 * solve at eps, the estimate, the second solve at 2^-j eps for the Jacobians
 * above tol, on the step schedule or, for patterns without one, the dense
 * trailing block path).  nrhs = 1 and K >= 3 (else PSP_E_INVALID); an item
 * with neither path gives PSP_E_UNSUPPORTED.  outs[i] gives item i's device
 * arrays est and scale (batch each, as for psp_solve_adaptive); the workspace
 * is psp_group_adaptive_workspace_bytes.  Run and capture as above. */
typedef struct psp_group_adapt {
    double* est;
    double* scale;
} psp_group_adapt_t;

PSP_API size_t psp_group_adaptive_workspace_bytes(psp_group g);
PSP_API psp_status psp_group_run_adaptive(psp_group g, const psp_group_task_t* tasks, const psp_group_adapt_t* outs,
                                          double tol, void* ws, size_t ws_bytes, void* stream);
PSP_API psp_status psp_group_capture_adaptive(psp_group g, const psp_group_task_t* tasks, const psp_group_adapt_t* outs,
                                              double tol, void* ws, size_t ws_bytes, void* stream, void** graph_exec);
PSP_API psp_status psp_graph_launch(void* graph_exec, void* stream);
PSP_API void psp_graph_destroy(void* graph_exec);
PSP_API void psp_group_destroy(psp_group g);

/* ------------------------------------------------------------------------
 * psp_tune -- autotuner for Alg. 1 steps 2-4 in batch (Sec. IV: the batched
 * factorisation and solves are where the time goes): runs psp_solve_batched on the caller's data with
 * every path that can run this plan and fits ws_bytes (one warm-up, three
 * timed runs each, HIP events on `stream`; the call synchronises the stream),
 * and records the fastest as the PSP_PATH_AUTO choice for (batch, K, nrhs).
 * Arguments as for psp_solve_batched (X and info receive the last run's
 * results, which are the same on every path).  chosen (host, may be NULL)
 * receives the path id; ms (host, may be NULL, 9 entries indexed by path id)
 * receives the mean time per call, -1 for a path not run.  Size the
 * workspace with psp_workspace_bytes(plan, PSP_PATH_AUTO, ...), which covers
 * every candidate.
 * ---------------------------------------------------------------------- */
PSP_API psp_status psp_tune(psp_plan plan, int32_t batch, const double* values, int32_t K, const double* eps,
                            const double* d, int32_t nrhs, const double* B, double* X, int32_t* info, void* ws,
                            size_t ws_bytes, void* stream, int32_t* chosen, float* ms);

/* The tuner's choice for (batch, K, nrhs): the path and, for it, the launch
 * choices searched besides the path (Sec. IV: batched factorisation and
 * solves are where the time goes, so their launch shape is tuned per
 * workload):
 *   steps_mode  step schedule: -1 by batch size, 0 one workgroup per perturbed
 *               system, 1 one workgroup per Jacobian (combine fused);
 *   steps_wgcu  step schedule: 0 as many workgroups per CU as LDS allows,
 *               1 one per CU;
 *   ring        step schedule: descriptors in flight, 7 or 4;
 *   tail_cols   dense trailing block assembly: 16 by 16 x 16 tile pairs on
 *               the MFMA unit (where every tile's column union is below
 *               65535), else 4 or 1 block columns per workgroup;
 *   tail_il     dense trailing block, fused call: 1 the systems' factors
 *               below the block interleaved (a wave serves 64 systems),
 *               0 one system after another, -1 interleaved from 64
 *               systems on (needs tail_cols 16);
 *   tail_lu     dense trailing block LU and solves: 1 one workgroup per
 *               system, 0 each panel step across the device;
 *   ms          measured time per call (-1 when set by hand);
 *   source      0 none (the size heuristic applies), 1 tuned or set in this
 *               process, 2 read from the tuning cache file.
 * psp_tune records its choice in the plan and in the tuning cache file
 * ($PSP_TUNE_CACHE, else $HOME/.cache/psp/tune.txt; PSP_TUNE_CACHE set to ""
 * disables it), one line per (device, pattern hash, n, nnz, batch, K, nrhs),
 * so that PSP_PATH_AUTO in a later process uses it without tuning again.
 * psp_tune_choice reports the choice AUTO would use; psp_set_tune_choice
 * pins one by hand (PSP_E_INVALID for an unknown path or a launch choice
 * outside the values above).  All choices return the same bits. */
typedef struct {
    int32_t path;
    int32_t steps_mode;
    int32_t steps_wgcu;
    int32_t ring;
    int32_t tail_cols;
    int32_t tail_il;
    int32_t tail_lu;
    float ms;
    int32_t source;
} psp_tune_choice_t;

PSP_API psp_status psp_tune_choice(psp_plan plan, int32_t batch, int32_t K, int32_t nrhs, psp_tune_choice_t* out);
PSP_API psp_status psp_set_tune_choice(psp_plan plan, int32_t batch, int32_t K, int32_t nrhs,
                                       const psp_tune_choice_t* choice);

/* ------------------------------------------------------------------------
 * Split steps (plain, one call per step) -- the adjoint and the
 * one-system-at-a-time baseline use these.
 * psp_factor (Alg. 1 steps 1-2, the factorisation half; Sec. II-C: no row
 * exchange, the plan's static order): factors all batch*K perturbed systems
 * P (A_s + eps_k D) P^T into the workspace
 * (keep = 1 layout) and returns a host handle that refers to it.  The
 * handle is valid while the workspace memory is alive and unmodified.
 * ---------------------------------------------------------------------- */
typedef struct psp_factors_s* psp_factors;

PSP_API psp_status psp_factor(psp_plan plan, int32_t path, int32_t batch, const double* values, int32_t K,
                      const double* eps, const double* d, int32_t* info, void* ws, size_t ws_bytes,
                      void* stream, psp_factors* out);

/* Solves every perturbed system with its factors: Xk[s][k] = (A_s + eps_k D)^{-1} B[s]
 * (transpose = 0) or (A_s + eps_k D)^{-T} B[s] (transpose = 1).
 * B device batch x n x nrhs; Xk device batch x K x n x nrhs.  nrhs must not
 * exceed the nrhs the workspace was sized for. */
PSP_API psp_status psp_solve(psp_factors f, int32_t nrhs, const double* B, double* Xk, int32_t transpose,
                     void* stream);

/* X[s] = sum_k c_k Xk[s][k], ascending k (Alg. 1 steps 3-4).  Device arrays. */
PSP_API psp_status psp_combine(psp_factors f, int32_t nrhs, const double* Xk, double* X, void* stream);

/* Adjoint of L = sum_r w_r . x_hat_r with respect to the values of A:
 * gA[s][e] = - sum_k c_k sum_r Lamk[s][k][i][r] * Xk[s][k][j][r] for the CSR
 * entry e = (i, j).  Lamk = psp_solve(..., W, transpose=1) and Xk =
 * psp_solve(..., B, transpose=0); all device arrays. dL/dB is psp_combine of
 * Lamk. */
PSP_API psp_status psp_grad_values(psp_factors f, int32_t nrhs, const double* Lamk, const double* Xk,
                           double* gA, void* stream);

PSP_API psp_status psp_factors_release(psp_factors f);

/* ------------------------------------------------------------------------
 * Error test (Alg. 1 step 5, optional): for every Jacobian s and RHS column r,
 *   R[s][:, r] = B[s][:, r] - A_s X[s][:, r]
 *   rnorm[s*nrhs + r] = ||R[s][:, r]||_2,  bnorm[s*nrhs + r] = ||B[s][:, r]||_2
 * (the residual norm of the paper's Fig. 1; divide for the relative one).
 * Each R entry is b_i followed by fma(-a_ie, x_j, .) over row i in the
 * plan's CSR order; each norm is sqrt of the fma sum of squares in ascending
 * row order.  values device batch x nnz (CSR order); B, X device batch x n x
 * nrhs (row-major); R device batch x n x nrhs, or NULL when not wanted
 * (required for n > 16384); rnorm device batch x nrhs; bnorm device batch x
 * nrhs or NULL.  Asynchronous on `stream`.  PSP_E_INVALID for NULL required
 * pointers or batch/nrhs < 1, PSP_E_UNSUPPORTED for R = NULL with n > 16384.
 * ---------------------------------------------------------------------- */
PSP_API psp_status psp_residual(psp_plan plan, int32_t batch, const double* values, int32_t nrhs,
                                const double* B, const double* X, double* R, double* rnorm, double* bnorm,
                                void* stream);

/* ------------------------------------------------------------------------
 * psp_estimate_rho -- rho(A_s^{-1} D) for every Jacobian s of a batch, the
 * radius that decides convergence of the expansion behind the method
 * (|eps_k| rho < 1, Sec. II-B) and the size of its truncation error (about
 * prod_k |eps_k| rho^K); used to choose the perturbation size per Jacobian.
 * Power iteration with M = (A_s + probe D)^{-1} D, pivot-free (K = 1, sparse
 * path: a fused factor-and-solve per step when the step schedule fits, else one
 * kept factorisation and psp_solve per step; the same bits either way):
 *     v = v0 / ||v0||;  repeat iters times: x = M v, g = ||x||_2, v = x / g;
 *     rho = exp(mean of log g over the last iters - iters/2 steps).
 *   values  device batch x nnz;  d device n (NULL: D = I);  probe nonzero, small
 *   v0      device batch x n start vectors (the caller draws them)
 *   rho     device batch output (NaN if a factorisation broke down or x = 0)
 *   ws      device, psp_estimate_rho_workspace_bytes(plan, batch) bytes
 * Asynchronous on `stream`.  PSP_E_INVALID for NULL pointers, batch < 1 or
 * iters outside 1..100000; PSP_E_EPS for a zero or non-finite probe.
 * ---------------------------------------------------------------------- */
PSP_API size_t psp_estimate_rho_workspace_bytes(psp_plan plan, int32_t batch);
PSP_API psp_status psp_estimate_rho(psp_plan plan, int32_t batch, const double* values, const double* d, double probe,
                                    int32_t iters, const double* v0, double* rho, void* ws, size_t ws_bytes,
                                    void* stream);

/* ------------------------------------------------------------------------
 * Newton-Raphson power flow around Alg. 1 (Sec. IV: the method solves the
 * Jacobian system of every Newton step of a distributed-slack AC power flow).
 * Network: nbus buses, bus admittance matrix Y = G + jB in CSR form (sorted
 * columns, diagonal present in every row), and pv[i] != 0 for a
 * voltage-controlled bus.  Per scenario, with n = 2*nbus + 1:
 *   x    = [theta (nbus) | |V| (nbus) | lambda]
 *   spec = [P0 (nbus) | Q0 on PQ buses, V_set on PV buses (nbus) | theta_ref]
 *   part = slack participation (nbus)
 *   F(x) = [P_i - P0_i - part_i lambda | Q_i - Q0_i (PQ) or |V_i| - V_set_i (PV)
 *           | theta_0 - theta_ref],
 *   P_i = sum_j V_i V_j (G_ij cos t_ij + B_ij sin t_ij),
 *   Q_i = sum_j V_i V_j (G_ij sin t_ij - B_ij cos t_ij),  t_ij = theta_i - theta_j.
 * The plan's pattern must be exactly the pattern of dF/dx: for every Y entry
 * (i, j) the positions (i, j), (i, nbus+j), (nbus+i, j), (nbus+i, nbus+j),
 * plus (i, 2*nbus) for every bus and (2*nbus, 0); a PV bus's Q row keeps its
 * positions (values 0 except 1 on its |V| diagonal).
 * ---------------------------------------------------------------------- */
typedef struct psp_pf_s* psp_pf;

enum { PSP_PF_CONVERGED = 0, PSP_PF_MAXITER = 1, PSP_PF_BREAKDOWN = 2, PSP_PF_DIVERGED = 3 };

/* Checks the network against the plan's pattern (PSP_E_INVALID on any
 * mismatch, NULL pointer, malformed Y, missing diagonal or non-finite G/B),
 * then copies the network and the map from Y entries to Jacobian positions
 * into `dev` (device, caller-owned, 256-byte aligned, at least
 * psp_pf_device_bytes(nbus, y_row_ptr[nbus]) bytes) on `stream` and waits for
 * the copy.  The plan must be uploaded to the current device.  All other
 * arrays are host, read during the call.  The plan and `dev` must outlive the
 * handle; free it with psp_pf_destroy. */
PSP_API size_t psp_pf_device_bytes(int32_t nbus, int32_t nnz_y);
PSP_API psp_status psp_pf_create(psp_plan plan, int32_t nbus, const int32_t* y_row_ptr, const int32_t* y_col_idx,
                                 const double* g, const double* b, const int32_t* pv, void* dev, size_t dev_bytes,
                                 void* stream, psp_pf* out);
PSP_API void psp_pf_destroy(psp_pf pf);

/* One evaluation for `batch` scenarios (device arrays): F (batch x n), the
 * Jacobian values J (batch x nnz in the plan's CSR order, or NULL) and
 * fnorm[s] = max_i |F_s,i| (batch, or NULL; NaN if any entry is NaN).
 * x, spec device batch x n; part device batch x nbus.  Asynchronous. */
PSP_API psp_status psp_pf_eval(psp_pf pf, int32_t batch, const double* x, const double* spec, const double* part,
                               double* F, double* J, double* fnorm, void* stream);

/* Device workspace psp_pf_newton needs: psp_workspace_bytes(plan, path,
 * batch, K, 1, 0) for the solves plus F, J, dx and info. */
PSP_API size_t psp_pf_workspace_bytes(psp_pf pf, int32_t path, int32_t batch, int32_t K);

/* Newton loop for `batch` scenarios.  Each iteration evaluates F and J; a
 * scenario whose max|F| <= tol is converged and one whose max|F| is not
 * finite has diverged; if any scenario is still running and fewer than
 * max_iter updates were made, Alg. 1 (psp_solve_batched on `path` with the K
 * nodes eps and D = diag(d), d NULL for D = I) solves J dx = F for the batch
 * and every running scenario takes x <- x - dx, unless one of its K
 * factorisations broke down (info != 0), which stops it.
 *   x       device batch x n, in: start, out: last iterate
 *   iters   device batch (int32): updates applied
 *   status  device batch (int32): PSP_PF_* (MAXITER if still above tol)
 *   fnorm   device batch: max|F| at the last evaluation
 *   ws      device, psp_pf_workspace_bytes(pf, path, batch, K) bytes
 * Blocks the calling thread: after each evaluation it copies the status
 * array to the host and waits for `stream`.  Calls on one handle must not
 * overlap.  Errors as for psp_solve_batched; PSP_E_INVALID also for
 * max_iter < 0 or a negative / non-finite tol. */
PSP_API psp_status psp_pf_newton(psp_pf pf, int32_t path, int32_t batch, int32_t K, const double* eps,
                                 const double* d, double* x, const double* spec, const double* part, double tol,
                                 int32_t max_iter, int32_t* iters, int32_t* status, double* fnorm, void* ws,
                                 size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PSP_H */
