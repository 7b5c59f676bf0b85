/*
 * nolsm.h - C ABI of the MI355X (gfx950) NOLSM hot-path library, libnolsm.so.
 *
 * The library computes, for every column block J of two block-sparse matrices
 * K (the Hamiltonian H_0) and S (the overlap), the owned columns of the
 * non-orthogonal local submatrix purification of Schade et al., Sec. III-B.2
 * (Eq. purification_submatrix):
 *
 *   T_J(D) = 1/2 (I - sign(T_J(S)^-1 T_J(K) - mu I)) T_J(S)^-1,
 *
 * with sign() by the Newton-Schulz iteration (Eq. NS1-NS2), and writes those
 * columns back into a block-sparse D that keeps the merged pattern of K and S
 * (Sec. III-B.2, write-back step; Fig. 2 steps b-i).
 *
 * Conventions for every entry point:
 *   - All functions are extern "C", never throw, and return NOLSM_OK (0) or a
 *     negative nolsm_error code; nolsm_strerror() gives a message (the last
 *     HIP runtime message is appended for NOLSM_E_HIP).
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the current device, owned by the caller. The library
 *     never allocates or frees device memory; the plan owns host memory only.
 *     (The one device buffer of the library's own is the static workspace
 *     array of nolsm_sign_batch_noalloc, loaded with the library's code.)
 *   - `stream` is a hipStream_t passed as void*. All device work is enqueued
 *     asynchronously on it; NULL means the legacy default stream.
 *   - Blocks are bs x bs doubles stored row-major, bs*bs contiguous values per
 *     block, blocks in block-CSR order (row_ptr / col_idx, columns strictly
 *     increasing inside a row). This build supports bs = 6 (one molecule of
 *     the water-like systems) and bs = 1..6 in general.
 */
#ifndef NOLSM_H
#define NOLSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors -- */
typedef enum {
    NOLSM_OK = 0,
    NOLSM_E_ARG = -1,        /* null pointer, bad size or bad option            */
    NOLSM_E_PATTERN = -2,    /* row_ptr not monotone, column unsorted/duplicate/
                                out of range, pattern asymmetric, diagonal block
                                missing, or K and S disagree on nb/bs          */
    NOLSM_E_WORKSPACE = -3,  /* workspace or metadata buffer too small          */
    NOLSM_E_HIP = -4,        /* HIP runtime error                               */
    NOLSM_E_STATE = -5,      /* plan not configured/bound for these options     */
    NOLSM_E_NOT_SPD = -6,    /* some T_J(S) not positive definite (sync mode)   */
    NOLSM_E_NOCONV = -7,     /* some sign iteration hit max_iter (sync mode)    */
    NOLSM_E_NOMEM = -8       /* host allocation failed                          */
} nolsm_error;

/* Per-molecule status codes, in nolsm_mol_stats.status. */
enum {
    NOLSM_MOL_OK = 0,
    NOLSM_MOL_NOT_SPD = 1,   /* Cholesky pivot <= 0: Dcols left at zero         */
    NOLSM_MOL_NOCONV = 2     /* max_iter reached without meeting the stop rule  */
};

/* ------------------------------------------------------------- patterns -- */
/* A square block-sparse pattern: nb block rows, bs x bs blocks. The arrays
 * are host memory, read during nolsm_build_submatrices only. */
typedef struct {
    int32_t nb;
    int32_t bs;
    int64_t nnzb;
    const int32_t *row_ptr;  /* host, [nb+1], row_ptr[0] = 0, row_ptr[nb] = nnzb */
    const int32_t *col_idx;  /* host, [nnzb], strictly increasing within a row   */
} nolsm_pattern;

/* ------------------------------------------------------------- options -- */
typedef enum {
    NOLSM_FP64 = 0,          /* everything FP64 (the plain method)              */
    NOLSM_FP32 = 1,          /* FP64 setup, FP32 Newton-Schulz GEMMs            */
    NOLSM_FP16 = 2,          /* FP64 setup, FP16-in/FP32-accumulate MFMA GEMMs,
                                then n_final_fp32 FP32 finishing iterations     */
    NOLSM_BF16 = 3           /* as FP16 with bfloat16 inputs                    */
} nolsm_prec;

typedef enum {
    NOLSM_BOUNDS_GERSHGORIN = 0,   /* c_J = 1/min(||A||_inf, ||A||_1)           */
    NOLSM_BOUNDS_LEARNED = 1       /* c_J from the spectral-bound MLP, clamped
                                      at the Gershgorin scale                  */
} nolsm_bounds;

typedef enum {
    NOLSM_SCHED_GRAPH = 0,         /* whole batch captured once into a hipGraph
                                      and launched as one graph                */
    NOLSM_SCHED_STREAM = 1,        /* same kernels launched directly           */
    NOLSM_SCHED_PER_BUCKET = 2,    /* baseline: one launch per size bucket per
                                      phase (buckets of 64 rows)               */
    NOLSM_SCHED_PERSISTENT = 3,    /* as GRAPH, but each Newton-Schulz launch is a
                                      fixed grid (2 workgroups per CU) draining
                                      per-XCD device work queues of tiles      */
    NOLSM_SCHED_PIPELINE = 4       /* as GRAPH, with the workspace split into two
                                      chunk regions used in turn: the setup of
                                      chunk c + 1 (gather, factor, substitution,
                                      bounds) runs on a second stream of the
                                      library's, beside the sign iteration,
                                      finishing and extraction of chunk c, with
                                      events for the order; the stream of the
                                      call waits for all of it. Needs a stream
                                      other than the null stream (else runs as
                                      STREAM).                                 */
} nolsm_sched;

/* How T_J(S)^-1 is applied when forming A_J = T_J(S)^-1 T_J(K) - mu I and
 * Y_J = T_J(S)^-1 E_cJ. */
typedef enum {
    NOLSM_INV_CHOLESKY = 0,        /* FP64 Cholesky factor and substitution
                                      (default)                                 */
    NOLSM_INV_COUPLED_NS = 1,      /* FP16/BF16 only: the coupled Newton-Schulz
                                      iteration of Eq. inv1-inv3 on the matrix
                                      cores (FP32 accumulation): Y_0 = c S_J,
                                      Z_0 = I, R_k = I - Z_k Y_k,
                                      Y_{k+1} = Y_k + Y_k R_k / 2,
                                      Z_{k+1} = Z_k + R_k Z_k / 2 (the paper's
                                      update written with R_k, which keeps its
                                      relative precision in 16 bits), stopped
                                      like the sign iteration (stagnation of
                                      ||R_k||_F); then S^-1 = c Z^2 and A_J =
                                      S^-1 K_J - mu I by two more GEMMs, with
                                      c = 1 / max row sum of |S_J|. A diverging
                                      iteration, or one that does not stop
                                      within inv_max_iter, marks the molecule
                                      NOT_SPD (no inverse: its columns stay
                                      zero and its sign iteration is skipped). */
    NOLSM_INV_CHOLESKY_FP32 = 2,   /* FP16/BF16 only: the same
                                      Cholesky factor and substitution with FP32
                                      arithmetic on the matrix cores, FP64
                                      storage; its relative error, about
                                      kappa(S_J) 2^-24, stays far below the
                                      16-bit floor of the sign iteration.      */
    NOLSM_INV_CHOLESKY_APPLY_FP32 = 3  /* FP16/BF16 only: the FP64 Cholesky
                                      factor (FP64 pivots and NOT_SPD test), also
                                      stored in FP32 with its diagonal-tile
                                      inverses; the substitutions that form A_J
                                      (or L^-1 T_J(K) L^-T) and the E columns
                                      apply that FP32 copy with FP32 arithmetic
                                      on the matrix cores (twice the FP64 matrix
                                      rate), FP64 storage; the owned columns are
                                      taken back through the FP64 factor. Error
                                      of the application about kappa(S_J) 2^-24,
                                      far below the 16-bit floor.              */
} nolsm_inverse;

typedef struct {
    int32_t prec;            /* nolsm_prec                                       */
    int32_t n_final_fp32;    /* FP16/BF16: FP32 finishing iterations, 0..2
                                (default 2), applied column-restricted to Y_J   */
    double tol;              /* stop at ||X^2 - I||_F < tol (defaults FP64
                                1e-10, FP32 1e-5). FP16/BF16: the hand-over to
                                the FP32 finishing iterations; the default -1
                                derives it from the format and n_final_fp32
                                (FP16 0.104, BF16 0.174 with two finishing
                                iterations), 0 leaves only the stagnation test */
    int32_t max_iter;        /* iteration slots per solve, 2..128 (defaults:
                                FP64 48, FP32/FP16/BF16 40)                     */
    int32_t fixed_iters;     /* > 0: exactly this many low-precision updates, no
                                residual test (the paper's fixed step count)    */
    double switch_theta;     /* FP32/FP16/BF16: stop when r_k > theta r_{k-1}
                                and r_k < switch_rmax (defaults 0.7, 0.5)        */
    double switch_rmax;
    int32_t bounds;          /* nolsm_bounds                                     */
    const float *d_mlp;      /* device, packed MLP parameters (NOLSM_MLP_NPARAM) */
    const float *d_mlp_norm; /* device, 24 floats: feature mean[12], std[12]     */
    float mlp_safety;        /* c_J = 1/(safety * rho_hat); default 1.05         */
    int32_t sched;           /* nolsm_sched                                      */
    int32_t sync_errors;     /* != 0: synchronize and return E_NOT_SPD/E_NOCONV  */
    float *d_features;       /* optional device [nb][12] float: features of A_J
                                (of L^-1 T_J(K) L^-T - mu I with sym_sign)       */
    double debug_scale_mult; /* != 0: multiply c_J (tests of the restart guard)  */
    int32_t debug_poison_mol;/* >= 0: molecule whose S_J pivot is forced <= 0    */
    int32_t profile;         /* != 0: launch directly (no graph), time each phase
                                with HIP events on `stream`, synchronize, and keep
                                the times for nolsm_profile_last                 */
    uint64_t ns_small_tile_mask; /* FP16/BF16 GEMM tile per size bucket: bit b
                                set -> submatrices padded to 64(b+1) rows use
                                64x64 tiles, else 128x128 (default: bits 0, 2,
                                i.e. 64 and 192 rows). Used by configure.       */
    double *d_wcols;         /* optional device [sum_m*bs*bs], Dcols layout: the
                                owned columns of the energy-weighted density
                                matrix T_J(W) = T_J(D) T_J(K) T_J(D) (Sec. III-B.2).
                                Computed as (A_J + mu I) Dcols_J, which equals
                                the definition because T_J(D) = P T_J(S)^-1 with
                                P = (I - sign A_J)/2 a projector commuting with
                                A_J. Zero for NOT_SPD molecules. Null: skipped.
                                Assemble W with nolsm_assemble_D.                */
    int32_t inverse;         /* nolsm_inverse (default NOLSM_INV_CHOLESKY)       */
    int32_t inv_max_iter;    /* coupled Newton-Schulz iteration slots, 2..128
                                (default 40; used by configure)                  */
    int32_t sym_sign;        /* FP16/BF16 with a Cholesky route: != 0 runs the
                                sign iteration on the symmetric similar matrix
                                L^-1 T_J(K) L^-T - mu I (same spectrum;
                                sign(A_J) = L^-T sign(.) L^T), so each GEMM
                                computes its upper tiles only and mirrors
                                them; the owned columns are L^-T (y - sign(.) y)
                                / 2 with y = L^-1 E_cJ, the same D. The
                                features (d_features) and the learned bounds are
                                then those of that symmetric matrix (a network
                                trained on its features). Not with d_wcols.
                                Default 0; used by configure.                  */
    int32_t finish_rows;     /* FP16: != 0 runs the column-restricted finishing
                                products with the row-streaming vector kernel
                                (one launch per product) instead of the default
                                fused matrix-core kernel (both FP32-accurate:
                                the fused one splits each n x bs block into
                                FP16 high and low parts). BF16 always uses the
                                vector kernel. Default 0.                      */
    int32_t debug_force_stall;/* >= 0: molecule whose sign iteration is taken as
                                diverged after its residual at iteration 2, so
                                the guard restarts it from the Gershgorin scale
                                (fallback = 1, same result); -1: none        */
    int32_t subst_fp32;      /* sym_sign with FP32 substitutions (the FP32
                                factor, or the FP64 factor applied in FP32):
                                != 0 forms their tile products on the FP32
                                matrix cores. The default 0 forms them on the
                                FP16 matrix cores from operands split into
                                FP16 high and low parts, hi*hi + hi*lo + lo*hi
                                with FP32 accumulation (about 2^-22 relative
                                per operand, K scaled by a power of two into
                                FP16 range), far below the FP16 rounding of
                                the iterate that follows.                      */
} nolsm_solve_opts;

/* Fills *o with the defaults above for precision `prec`. */
void nolsm_default_opts(nolsm_solve_opts *o, int32_t prec);

/* The residual ||X^2 - I||_F at which a solve with these options stops the
 * sign iteration (Eq. NS1; the paper runs a fixed step count instead):
 * `tol` itself when tol >= 0; for tol < 0 the default of `prec`
 * (FP64 1e-10, FP32 1e-5) or, for FP16/BF16, the hand-over to the
 * n_final_fp32 exact FP32 steps: one step maps e = 1 - x^2 of an eigenvalue
 * to 3/4 e^2 + 1/4 e^3, so two leave 27/64 r^4 to leading order, held
 * below a tenth of the format's unit roundoff u (2^-11 FP16, 2^-8 BF16):
 * r = (64 u / 270)^(1/4); one step: r = (4 u / 30)^(1/2); none: 0 (the
 * stagnation test alone). Pure function of its arguments, host only. */
double nolsm_switch_tol(int32_t prec, int32_t n_final_fp32, double tol);

/* Per-molecule statistics, written to device memory by nolsm_sign_batch. */
typedef struct {
    int32_t iters;           /* Newton-Schulz updates taken in the main precision */
    int32_t iters_fp32;      /* finishing FP32 iterations (column-restricted)     */
    int32_t fallback;        /* 1 if the Gershgorin restart was used              */
    int32_t status;          /* NOLSM_MOL_*                                       */
    double scale;            /* c_J used for X_0 = c_J A_J                        */
    double resid;            /* ||X_k^2 - I||_F of the returned iterate           */
    double trace_SD;         /* N_J = sum_c (S_J Dcols_J)[cJ_c, c]                */
    double energy_KD;        /* E_J = sum_c (K_J Dcols_J)[cJ_c, c]                */
    int32_t iters_inv;       /* coupled Newton-Schulz inverse updates (0 with the
                                Cholesky route)                                   */
    int32_t reserved_;
} nolsm_mol_stats;

typedef struct nolsm_plan nolsm_plan;

typedef struct {
    int32_t nb, bs;
    int64_t sum_m;           /* sum_J m_J = nnzb(D) = number of Dcols blocks      */
    int32_t m_min, m_max;    /* blocks per submatrix                              */
    double sum_n3;           /* sum_J n_J^3 (true sizes)                          */
    int32_t nchunks;         /* after nolsm_plan_configure, else 0                */
    size_t meta_bytes;       /* device metadata bytes needed by nolsm_plan_bind   */
    size_t ws_min_bytes;     /* smallest workspace that holds the largest J       */
    size_t ws_full_bytes;    /* workspace holding the whole batch in one chunk    */
    int32_t ngroups;         /* submatrices after combination (= nb without it)   */
    int32_t g_m_max;         /* blocks of the largest submatrix                   */
    int64_t sum_gm;          /* sum over submatrices of their blocks              */
    double sum_gn3;          /* sum over submatrices of n^3 (n = bs blocks)       */
} nolsm_plan_sizes;

/* ------------------------------------------------------------- the path -- */

/* Flags of nolsm_build_submatrices. */
#define NOLSM_PLAN_COMBINE 1   /* combine submatrices (Sec. III-B, submatrix
                                  combination heuristic, Eq.
                                  combination_criterion): groups of molecules
                                  share one submatrix on the union R of their
                                  N(J) when (m_i + m_j - m_ij)^3 < m_i^3 + m_j^3
                                  (m in blocks, m_ij = common blocks); candidates
                                  of group i are the groups owning a block of
                                  R_i, merged one at a time in increasing order
                                  of the blocks one side adds to the other
                                  (ties: larger cubic drop, then lower group
                                  ids; the merged group keeps the lower id), at
                                  most floor(64 / bs) molecules per group. D
                                  keeps the merged pattern: only the rows N(J)
                                  of each owned molecule are written back.     */

/* Plan / index build (Sec. III-B.2 NOLSM generation step; Fig. 2 b-c).
 * Validates both patterns, merges them (block row I is in the submatrix of
 * column block J iff K_IJ or S_IJ is stored), and builds N(J) sorted
 * ascending, p_J = position of J in N(J), the pattern of D (= the merged
 * pattern) and the scatter positions; with NOLSM_PLAN_COMBINE also the
 * groups (otherwise every molecule is its own group). Host work only.
 * Errors: E_ARG (null, nb<1, bs outside 1..6, K/S disagree, unknown flag),
 * E_PATTERN, E_NOMEM.
 * On success *plan is owned by the caller (nolsm_plan_destroy). */
int nolsm_build_submatrices(const nolsm_pattern *K, const nolsm_pattern *S,
                            int32_t flags, nolsm_plan **plan);

/* Sizes of the plan; fields after sum_n3 are zero until configured. */
int nolsm_plan_info(const nolsm_plan *plan, nolsm_plan_sizes *out);

/* Copies the plan's integer arrays to host buffers (any may be NULL):
 * sub_ptr[nb+1], sub_blk[sum_m] (N(J) lists), self_pos[nb],
 * D_row_ptr[nb+1], D_col_idx[sum_m], scatter_pos[sum_m] (index in D's
 * block-CSR of block (N(J)_a, J), for entry sub_ptr[J]+a). */
int nolsm_plan_export(const nolsm_plan *plan, int32_t *sub_ptr, int32_t *sub_blk,
                      int32_t *self_pos, int32_t *D_row_ptr, int32_t *D_col_idx,
                      int32_t *scatter_pos);

/* Copies the submatrix groups to host buffers (any may be NULL):
 * grp_ptr[ngroups+1], grp_blk[sum_gm] (row blocks R_g, sorted),
 * own_ptr[ngroups+1], own_J[nb] (molecules owned by group g, sorted; groups
 * ordered by their smallest molecule). Sizes from nolsm_plan_info. */
int nolsm_plan_groups(const nolsm_plan *plan, int32_t *grp_ptr, int32_t *grp_blk,
                      int32_t *own_ptr, int32_t *own_J);

/* Chooses the schedule for `opts` and a workspace of ws_bytes: submatrices
 * grouped into chunks that fit the workspace, tile lists per chunk. Reports
 * the device metadata size in *meta_bytes. Host work only.
 * Submatrices have at most NOLSM_MAX_ROWS rows (the extraction keeps a
 * submatrix's whole FP64 column block in the 160 KB of LDS of one workgroup).
 * Errors: E_ARG (also: a submatrix above NOLSM_MAX_ROWS rows), E_WORKSPACE
 * (the largest submatrix does not fit). */
#define NOLSM_MAX_ROWS 3008
int nolsm_plan_configure(nolsm_plan *plan, const nolsm_solve_opts *opts,
                         size_t ws_bytes, size_t *meta_bytes);

/* Uploads the configured metadata to d_meta (device, >= meta_bytes, 256-byte
 * aligned) on `stream` and waits for the copy. d_meta must stay allocated and
 * unmodified while the plan is used. Errors: E_STATE (not configured),
 * E_WORKSPACE (too small), E_HIP. */
int nolsm_plan_bind(nolsm_plan *plan, void *d_meta, size_t meta_bytes, void *stream);

/* The batched sign solve (Eq. purification_submatrix for every J; Fig. 2 e-h
 * with the element generation replaced by a gather from K and S):
 *   dK_val, dS_val : device, [nnzb * bs * bs] doubles in K's / S's block-CSR;
 *   mu             : chemical potential;
 *   d_ws, ws_bytes : device workspace (>= the size given to configure);
 *   dDcols         : device, [sum_m * bs * bs] doubles; the rows of molecule J
 *                    start at element bs*bs*sub_ptr[J]: an n_J x bs row-major
 *                    block T_J(D)[:, cJ] (so each bs x bs block is contiguous);
 *   dD_val         : device or NULL; if given, also scattered into D's
 *                    block-CSR (the merged pattern), [sum_m * bs * bs];
 *   dstats         : device, [nb] nolsm_mol_stats.
 * Per-molecule numerical failures are reported in dstats[J].status, which
 * the caller reads after synchronizing; with opts->sync_errors the call
 * synchronizes and returns E_NOT_SPD / E_NOCONV if any molecule failed.
 * Errors: E_ARG, E_STATE (plan not configured/bound for opts->prec,
 * opts->sched or a larger workspace), E_WORKSPACE, E_HIP. */
int nolsm_sign_batch(nolsm_plan *plan, const double *dK_val, const double *dS_val,
                     double mu, const nolsm_solve_opts *opts, void *d_ws,
                     size_t ws_bytes, double *dDcols, double *dD_val,
                     nolsm_mol_stats *dstats, void *stream);

/* Allocation-free variant of nolsm_sign_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the workspace is a device array of the
 * library, NOLSM_NOALLOC_WS_BYTES per GPU, held by every GPU the library runs
 * on until the process ends. Same arguments and results as nolsm_sign_batch
 * without d_ws / ws_bytes; the plan must be configured with
 * ws_bytes <= NOLSM_NOALLOC_WS_BYTES (more chunks for a large batch) and bound
 * on the current device. The kernels are launched directly on `stream` (never
 * a graph of the library's), so the call may itself be captured by the
 * caller. It calls no hipMalloc / hipFree and no allocating routine; the
 * first call on a device looks up the array's address there.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on one
 * GPU (several streams or threads) race and must be serialised by the caller.
 * Errors: as nolsm_sign_batch; E_WORKSPACE when the plan's workspace exceeds
 * the array; E_ARG for the pipeline schedule, profile or sync_errors (each
 * would create library streams, events or host buffers); E_STATE when the
 * current device is not the plan's. */
#define NOLSM_NOALLOC_WS_BYTES ((size_t)64 << 20)
int nolsm_sign_batch_noalloc(nolsm_plan *plan, const double *dK_val, const double *dS_val,
                             double mu, const nolsm_solve_opts *opts, double *dDcols,
                             double *dD_val, nolsm_mol_stats *dstats, void *stream);

/* Write-back (Sec. III-B.2; Fig. 2 h-i): D block (N(J)_a, J) <- rows
 * bs*a .. bs*a+bs-1 of molecule J's Dcols. dDcols and dD_val are device
 * arrays of sum_m*bs*bs doubles. Requires a bound plan. */
int nolsm_assemble_D(const nolsm_plan *plan, const double *dDcols, double *dD_val,
                     void *stream);

/* FP64 trace sums over all molecules of the last solve whose stats are in
 * dstats (device): sums_out[0] = sum_J N_J = Tr(DS) share total,
 * sums_out[1] = sum_J E_J (band energy, Eq. e_elec), sums_out[2] = number of
 * molecules whose status is not OK. Uses the first 256 bytes of d_ws (the
 * workspace of the plan); synchronizes `stream`. */
int nolsm_trace_sums(const nolsm_plan *plan, const nolsm_mol_stats *dstats, void *d_ws,
                     double *sums_out, void *stream);

/* Chemical-potential bisection (Sec. IV-A: mu is fixed for charge neutrality
 * by a bisection-like outer loop around the method). Repeats
 * nolsm_sign_batch at mu = midpoint of [mu_lo, mu_hi] and halves the
 * interval until |sum_J N_J - n_target| <= tol_count or max_steps solves.
 * sum_J N_J must be increasing in mu (it counts occupied orbitals). On
 * return dDcols / dD_val / dstats hold the last solve; *mu_out, *count_out,
 * *steps_out (may be NULL) report it. Errors as nolsm_sign_batch, plus
 * E_ARG (mu_hi <= mu_lo, tol_count <= 0, max_steps < 1) and E_NOCONV when
 * the count is not reached, or when it is reached but some molecule of the
 * final solve is not NOLSM_MOL_OK (a mu inside a band converges slowly; its
 * NOCONV molecules still enter the count). With E_NOCONV the outputs, the
 * last solve and *mu_out / *count_out / *steps_out are still returned. */
int nolsm_mu_bisect(nolsm_plan *plan, const double *dK_val, const double *dS_val, double mu_lo,
                    double mu_hi, double n_target, double tol_count, int32_t max_steps,
                    const nolsm_solve_opts *opts, void *d_ws, size_t ws_bytes, double *dDcols,
                    double *dD_val, nolsm_mol_stats *dstats, void *stream, double *mu_out,
                    double *count_out, int32_t *steps_out);

void nolsm_plan_destroy(nolsm_plan *plan);
const char *nolsm_strerror(int code);

/* Phase times of the last nolsm_sign_batch call made with opts->profile,
 * in milliseconds, summed over chunks (HIP events on the call's stream). */
typedef struct {
    int32_t valid;
    int32_t nchunks;
    int32_t n_ns_launches;   /* Newton-Schulz GEMM launches (both halves)      */
    int32_t n_fin_launches;  /* finishing-product launches                     */
    double ms_gather;        /* control init + gather                          */
    double ms_chol;          /* Cholesky                                       */
    double ms_subst;         /* substitution (A_J and Y_J)                     */
    double ms_bounds;        /* bounds, scale and X_0                          */
    double ms_ns;            /* all Newton-Schulz GEMM launches                */
    double ms_finish;        /* finishing products                             */
    double ms_extract;       /* extraction, traces, write-back                 */
    double ms_total;         /* first to last event                            */
    double ms_wmat;          /* owned columns of T_J(W), when requested        */
    double ms_inverse;       /* coupled Newton-Schulz route: everything from
                                the scaled S_J to A_J (replaces chol + subst)  */
} nolsm_profile;
int nolsm_profile_last(const nolsm_plan *plan, nolsm_profile *out);

/* ---------------------------------------------- learned spectral bounds -- */
/* A 12 -> 64 -> 64 -> 2 perceptron (SiLU) mapping features of A_J to the
 * normalised extremes (lambda_min/G_lo, lambda_max/G_hi). Not in the paper:
 * it sets the pre-scaling that the paper only requires to exist
 * (Sec. III-B.2, after Eq. NS2). Parameters: float, packed W1[64][12], b1[64],
 * W2[64][64], b2[64], W3[2][64], b3[2]. All pointers are device memory. */
#define NOLSM_MLP_NFEAT 12
#define NOLSM_MLP_NPARAM 5122

/* out[B][2] = MLP((x[B][12] - mean) / std), norm = mean[12], std[12]. */
int nolsm_mlp_forward(const float *d_params, const float *d_norm, const float *d_x,
                      int32_t B, float *d_out, void *stream);

/* Loss = mean over B rows and 2 outputs of w (pred - y)^2, w = 4 where
 * pred < y, else 1. Writes *d_loss (1 float) and d_grad[NPARAM] (overwritten,
 * not accumulated). d_x are raw features (normalised inside with d_norm). */
int nolsm_mlp_loss_grad(const float *d_params, const float *d_norm, const float *d_x,
                        const float *d_y, int32_t B, float *d_grad, float *d_loss,
                        void *stream);

/* One Adam step with bias correction (t counts from 1) on all NPARAM values.
 * The hyper-parameters are taken in double: 1 - beta and the bias corrections
 * are formed on the host from the exact values and rounded once to FP32
 * (1 - (float)0.999 would differ from 0.001 by 1.3e-5 relative). */
int nolsm_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v,
                   int32_t t, double lr, double beta1, double beta2, double eps,
                   void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NOLSM_H */
