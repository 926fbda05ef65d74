/*
 * mgr.h -- C-ABI of the MI355X (gfx950) MGR + FGMRES library (libmgrhip.so).
 *
 * The library solves A x = b for a block system whose unknowns carry a
 * physical-field label (Bui et al., arXiv 2101.11649, Sec. 1, eq. (1)) with
 * flexible GMRES right-preconditioned by multigrid reduction (MGR, Sec. 2,
 * Algorithm 1).  Each MGR level splits the current unknowns into F-points (the
 * fields named by that level's bitmask) and C-points (the rest) (Sec. 2, the
 * partition under eq. (2)); the coarse system after the last level is solved by
 * a classical AMG V-cycle (Sec. 4.1).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers unless marked "(host)".
 *  - All device work is enqueued on the hipStream_t given to mgr_create.
 *    mgr_apply / mgr_apply_transpose / mgr_matvec are asynchronous;
 *    mgr_setup, mgr_solve*, mgr_export and mgr_hierarchy_info synchronise the
 *    stream before returning.
 *  - Inputs are only read during the call (setup copies what it keeps), so the
 *    caller may free them afterwards.  Outputs are caller-allocated.  The
 *    handle owns every internal buffer and frees it in mgr_destroy.
 *  - A handle is not thread-safe; separate handles are independent.
 *  - Return value: 0 = OK; > 0 = warning (1 = MGR_NOT_CONVERGED: X holds the
 *    last iterate); < 0 = error (see MGR_ERR_*).  No exception crosses the
 *    ABI; mgr_last_error(h) returns a host string describing the last error.
 *  - Indices are int32; values FP64 at the boundary, whatever the internal
 *    apply precision.
 */
#ifndef MGR_H
#define MGR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGR_OK 0
#define MGR_NOT_CONVERGED 1
#define MGR_ERR_ARG (-1)          /* invalid argument or call order            */
#define MGR_ERR_HIP (-2)          /* HIP runtime error                         */
#define MGR_ERR_ZERO_PIVOT (-3)   /* zero / non-finite F-pivot or singular block, singular coarse matrix */
#define MGR_ERR_OOM (-4)          /* device allocation failed                  */
#define MGR_ERR_BAD_LABELS (-5)   /* field label out of range, empty F or C set */
#define MGR_ERR_UNSUPPORTED (-6)  /* option combination or size not supported (e.g. a_ii <= 0 in AMG) */

/* F-relaxation M_FF^{-1} of Algorithm 1 (Sec. 2; choices discussed in Sec. 2 and Sec. 3). */
#define MGR_FRELAX_JACOBI 0        /* diag(A_FF)^{-1}                               */
#define MGR_FRELAX_BLOCK_JACOBI 1  /* inverse of the A_FF blocks formed by the F-points of one block row */
#define MGR_FRELAX_ILU0 2          /* ILU(0) of A_FF                                */
#define MGR_FRELAX_AMG 3           /* one AMG V-cycle on A_FF (Sec. 3.2, Sec. 3.3)   */

/* Restriction R~ (Sec. 2): injection, eq. (4), or Jacobi restriction, eq. (5). */
#define MGR_RESTRICT_INJECTION 0
#define MGR_RESTRICT_JACOBI 1

#define MGR_ORTHO_CGS2 0           /* classical Gram-Schmidt applied twice         */

/* AMG interpolation: direct (Stueben 2001; the reading of the BoomerAMG
 * settings of Sec. 4.1 both codes share) or extended+i (De Sterck, Falgout,
 * Nolting, Yang 2008: distance two, the long-range interpolation that
 * Sec. 4.1 pairs with HMIS coarsening).  Extended+i needs every interpolatory
 * set to stay within 256 points, else the setup fails with MGR_ERR_UNSUPPORTED. */
#define MGR_INTERP_DIRECT 0
#define MGR_INTERP_EXT_I 1

/* AMG smoother: L1-Jacobi (Baker, Falgout, Kolev, Yang 2011), or the paper's
 * hybrid L1 Gauss-Seidel (Sec. 4.1: one forward sweep on the way down, one
 * backward sweep on the way up) with chunks of gs_chunk consecutive rows in
 * place of the processors' row blocks: inside a chunk the rows are relaxed one
 * after another with this sweep's values of the chunk's earlier rows, the
 * previous values elsewhere, and a_ii plus the l1 norm of the row's entries
 * outside the chunk as the diagonal (gs_chunk = 1 is L1-Jacobi).  Levels are
 * then never applied in composed form. */
#define MGR_SMOOTH_L1_JACOBI 0
#define MGR_SMOOTH_HYBRID_GS 1

/* The AMG of an MGR_FRELAX_AMG level (mgr_level_opts.amg_unknown_based):
 * scalar; the unknown approach (strength and interpolation only between
 * unknowns of one field label); or the unknown approach built on the
 * separate-component approximation of A_FF, its couplings between unknowns of
 * different labels dropped (Sec. 4.4: the displacement block's AMG is built
 * on it, which sparsifies the block), the V-cycle then using that operator. */
#define MGR_AMG_SCALAR 0
#define MGR_AMG_UNKNOWN 1
#define MGR_AMG_SEPARATE 2

typedef struct mgr_ctx *mgr_handle;

/* Block-CSR matrix with b x b row-major dense blocks.  b = 1 is plain CSR.
 * Column indices ascending within a block row, no duplicates.  Scalar unknown
 * i = I*b + r for block row I, in-block row r. */
typedef struct {
    int32_t block_size;      /* b in {1,2,3,4}                                 */
    int32_t n_block_rows;    /* square: scalar n = b * n_block_rows            */
    const int32_t *row_ptr;  /* n_block_rows + 1                               */
    const int32_t *col_idx;  /* nnzb                                           */
    const double *values;    /* nnzb * b * b                                   */
} mgr_matrix;

/* One MGR reduction level. */
typedef struct {
    uint32_t f_field_mask;   /* bit f set: unknowns of field f are F-points here */
    int32_t frelax;          /* MGR_FRELAX_*                                   */
    int32_t sweeps;          /* F-relaxation sweeps (>= 1)                     */
    double omega;            /* F-relaxation weight                            */
    int32_t restrict_type;   /* MGR_RESTRICT_*                                 */
    int32_t amg_unknown_based; /* MGR_FRELAX_AMG: MGR_AMG_SCALAR, _UNKNOWN or _SEPARATE */
    int32_t amg_agg_levels;  /* MGR_FRELAX_AMG: levels with aggressive coarsening (see mgr_amg_opts) */
} mgr_level_opts;

/* Classical AMG used for the final coarse system and for MGR_FRELAX_AMG. */
typedef struct {
    double theta;            /* strength threshold                             */
    int32_t max_levels;      /* including the coarsest                         */
    int32_t max_coarse;      /* stop coarsening at or below this size          */
    int32_t nu_pre, nu_post; /* L1-Jacobi sweeps                               */
    int32_t unknown_based;   /* coarse AMG: strength/interpolation per field   */
    int32_t interp;          /* MGR_INTERP_DIRECT or MGR_INTERP_EXT_I          */
    int32_t smoother;        /* MGR_SMOOTH_L1_JACOBI or MGR_SMOOTH_HYBRID_GS   */
    int32_t gs_chunk;        /* rows per chunk of the hybrid smoother (1..128) */
    int32_t agg_levels;      /* coarse AMG: the first agg_levels levels coarsen
                                aggressively (Sec. 4.1, the mechanics block: a
                                second PMIS on the graph of first-pass C-points
                                one or two strong connections apart) and
                                interpolate by multiple passes of direct
                                interpolation (Stueben 2001)                   */
    uint64_t seed;           /* PMIS random weights (splitmix64)                */
} mgr_amg_opts;

typedef struct {
    int32_t apply_precision; /* 64: FP64 MGR apply; 32: FP32 storage + accumulation inside the apply */
    int32_t restart;         /* FGMRES restart length m (1..63)                */
    int32_t maxiter;         /* total FGMRES iterations                        */
    double rtol;             /* stop when ||b - A x|| <= rtol ||b|| (x0 = 0)    */
    int32_t ortho;           /* MGR_ORTHO_CGS2                                 */
    mgr_amg_opts amg;
} mgr_opts;

typedef struct {
    int32_t status;          /* MGR_OK or MGR_NOT_CONVERGED                     */
    int32_t iterations;
    int32_t restarts;
    double rel_res_est;      /* Arnoldi estimate |g_{k+1}| / ||b||             */
    double rel_res_true;     /* ||b - A x|| / ||b|| recomputed in FP64         */
} mgr_solve_info;

/* Defaults: apply_precision 64, restart 50, maxiter 1000, rtol 1e-8, CGS2,
 * theta 0.25, max_levels 25, max_coarse 128, V(1,1), direct interpolation,
 * L1-Jacobi smoothing (gs_chunk 32 for the hybrid smoother), no aggressive
 * coarsening, seed 12345.  (host) */
void mgr_default_opts(mgr_opts *o);

/* Device memory provider of a handle (for instance a framework's caching
 * allocator).  alloc returns `bytes` of device memory that work ordered on
 * `stream` may use (NULL on failure); free gives such a pointer back (the
 * library has synchronised `stream` before it frees).  ctx is passed through. */
typedef void *(*mgr_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*mgr_free_fn)(void *p, void *stream, void *ctx);

/* Create a handle bound to a HIP stream (NULL = the null stream) on the
 * current device.  o (host) may be NULL for the defaults.  alloc / free_ /
 * alloc_ctx: the provider of every device array of the handle, or both NULL
 * for the library's own stream-ordered allocations (hipMallocAsync).  Either
 * way the handle keeps freed arrays in a cache of its own (by size class) and
 * hands them out again to later requests on its stream; everything goes back
 * to the provider in mgr_destroy.  Pinned host buffers (a few KB) are the
 * library's own.  Errors: ARG (h NULL, invalid options, only one of alloc and
 * free_ given), OOM, HIP. */
int mgr_create(mgr_handle *h, const mgr_opts *o, void *hip_stream, mgr_alloc_fn alloc, mgr_free_fn free_,
               void *alloc_ctx);

/* Replace the solver options (restart, maxiter, rtol, ortho, apply precision)
 * of an existing handle; AMG options take effect at the next mgr_setup. (host o) */
int mgr_set_opts(mgr_handle h, const mgr_opts *o);

/* Build the MGR hierarchy for A (Sec. 2): for level l the F-points are the
 * unknowns whose field f has bit f set in lvl[l].f_field_mask; P~ = [-M A_FC; I]
 * (Jacobi interpolation, eq. (4), ideal when A_FF is (block-)diagonal, eq. (3)),
 * R~ by lvl[l].restrict_type, coarse operator R~ A P~; then AMG on the last
 * coarse system.  field_of_dof: n labels in [0, 32).  lvl: (host) nlevels.
 * block_of_dof: n group ids for MGR_FRELAX_BLOCK_JACOBI, or NULL for the block
 * row of the input layout (i / b); on every level a block is a maximal run of
 * consecutive F-points (in the order of the unknowns) with one id, so a group
 * should hold consecutive unknowns (the F-points of a b = 1 input's cell, for
 * instance); a block of more than 4 F-points is UNSUPPORTED.  Copied; kept for
 * mgr_update_values.
 * The handle owns all the device memory of the hierarchy; operators with
 * short, nearly uniform rows (at least 32768 rows of at most 16 entries) also
 * get a sliced ELL copy for their SpMVs, made on first use, when it exceeds
 * their entries by at most 15%.
 * Errors: ARG, BAD_LABELS (empty F or C set, label out of range), ZERO_PIVOT,
 * UNSUPPORTED (block of more than 4 F-points, a_ii <= 0 in AMG, coarsest AMG
 * level above 2048 unknowns, an extended+i interpolatory set above 256
 * points), OOM, HIP. */
int mgr_setup(mgr_handle h, const mgr_matrix *A, const int32_t *field_of_dof, int32_t nlevels,
              const mgr_level_opts *lvl, const int32_t *block_of_dof);

/* Setup reuse for a new matrix on the same pattern, as between the Newton
 * solves of a simulation (AMG data reuse, Sec. 3.3 and Sec. 4.4).  values:
 * device pointer, nnzb*b*b doubles in the block layout (row pointers and
 * columns) of the last mgr_setup; copied.  The MGR levels are formed again
 * from the new values.  Every AMG hierarchy keeps its C/F splits and
 * interpolation and forms its Galerkin products, L1 diagonals and coarsest
 * inverse anew; with flags = MGR_REUSE_KEEP_FRELAX_AMG the hierarchies used as
 * F-relaxation are kept whole instead (the caller's A_FF of those levels is
 * unchanged, like the mechanics block of the fracturing case).  Errors: ARG
 * (no setup yet, null values, unknown flags), ZERO_PIVOT, UNSUPPORTED, OOM,
 * HIP; after an error the handle needs a new mgr_setup. */
#define MGR_REUSE_KEEP_FRELAX_AMG 1
int mgr_update_values(mgr_handle h, const double *values, int32_t flags);

/* z = M^{-1} r: one MGR V-cycle (Algorithm 1) from z = 0, no global
 * relaxation.  r, z: n doubles; may not alias.  Asynchronous. */
int mgr_apply(mgr_handle h, const double *r, double *z);

/* z = M^{-1} r exactly as mgr_apply computes it (the same kernels on the same
 * operators, so the same result), for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  It calls no allocating routine: its work vectors live in
 * one static device array per GPU of MGR_NOALLOC_SCRATCH_BYTES (128 MiB), held
 * from the library's first handle on that GPU until the process ends.  Every
 * call on a GPU shares that array, so calls that overlap on one GPU (other
 * streams, other handles, other threads) race; the array keeps the last call's
 * contents, and every value the apply reads from it is written by the same
 * call first.  Requires one mgr_apply or mgr_solve on the current hierarchy
 * beforehand (it makes the operator copies the apply reads; after mgr_setup,
 * mgr_update_values or a change of apply precision, again).  r, z: n doubles;
 * may not alias.  Asynchronous.  Errors: ARG (no setup, no earlier apply, null
 * vector), UNSUPPORTED (the hierarchy's work vectors, each rounded up to 256
 * bytes, exceed the scratch size). */
#define MGR_NOALLOC_SCRATCH_BYTES (128u << 20)
int mgr_apply_noalloc(mgr_handle h, const double *r, double *z);

/* z = M^{-T} r, the exact transpose of mgr_apply (requires sweeps == 1 on
 * every level).  Asynchronous. */
int mgr_apply_transpose(mgr_handle h, const double *r, double *z);

/* y = A x (trans = 0) or y = A^T x (trans = 1) in FP64.  Asynchronous. */
int mgr_matvec(mgr_handle h, int32_t trans, const double *x, double *y);

/* Solve A X = B by FGMRES(m) right-preconditioned with MGR (Sec. 4.1).
 * B, X: n x nrhs column-major; x0 = 0.  info: (host) nrhs entries or NULL.
 * Returns MGR_OK if every column converged, MGR_NOT_CONVERGED otherwise. */
int mgr_solve(mgr_handle h, int32_t nrhs, const double *B, double *X, mgr_solve_info *info);

/* Solve A^T X = B with FGMRES right-preconditioned by M^{-T} (the adjoint
 * solve used for gradients). */
int mgr_solve_transpose(mgr_handle h, int32_t nrhs, const double *B, double *X, mgr_solve_info *info);

/* Gradient of a loss with respect to the stored values of A, given the adjoint
 * solutions Lam (A^T Lam = dL/dX) and the solutions X:
 * dvalues[p*b*b + r*b + c] = -sum_k Lam_k[I*b + r] * X_k[J*b + c] for block p = (I, J).
 * Lam, X: n x nrhs column-major.  dvalues is overwritten.  Asynchronous. */
int mgr_grad_values(mgr_handle h, int32_t nrhs, const double *Lam, const double *X, double *dvalues);

/* Hierarchy sizes (host out, cap entries): out[0] = MGR levels, out[1] = AMG
 * levels, then per MGR level (n, nF, nC, nnz of the coarse operator), then per
 * AMG level (n, nnz).  Returns the number of entries written or an error. */
int mgr_hierarchy_info(mgr_handle h, int64_t *out, int32_t cap);

/* Copy a piece of the hierarchy to host buffers (all host pointers; pass NULL
 * buffers to query sizes only).  kind 0 = MGR level `level`: what 0 = C/F
 * flags (int32, 1 = C, 0 = F), 1 = coarse operator, 2 = P_F, 3 = R_F, 4 = A_FF,
 * 5 = F-relaxation operator M, 6 = R_J = [-omega A_CF M | I] and 7 = P_J =
 * [P_F | omega M ; I | 0] (the two operators of the one-sweep apply with
 * injection, global numbering, columns of P_J: coarse then fine; ARG for a
 * level applied in general form), 8 = A_FC, 9 = A_CF, 10 = A_CC.  kind 1 =
 * coarse AMG level `level`, kind 2 =
 * the F-relaxation AMG of MGR level `sub`: what 0 = C/F (+1 = C, -1 = F), 1 =
 * A_k, 2 = P_k, 3 = the dense inverse of the coarsest level (level = last; n x
 * n row-major doubles in b2), 4 = G = R - (R A) D^-1 and 5 = [W | Q] (W = 2D^-1
 * - D^-1 A D^-1, Q = P - D^-1 A P) of a level applied in composed form (ARG
 * otherwise), 6 = the dense cycle operator W + Q C^-1 G of the composed level
 * above the coarsest, when its cycle is applied as one GEMV (n x n row-major
 * doubles in b2; ARG for any other level), 7 and 8 = the slot tables of the
 * hybrid Gauss-Seidel sweeps on A_k (7: forward, each row's entries left of
 * its diagonal inside its chunk; 8: backward, right of it): sizes = (chunk
 * positions x table chunks, slots per row, their product); slot k of position
 * t of chunk c at (t W + k) nchunks + c, b1 = its column relative to the chunk
 * start (int32), b2 = its value (0 in padding slots); ARG without the hybrid
 * smoother.  sizes[0..2] = rows, cols, nnz (vector length in sizes[0]);
 * b0 = row_ptr (or the C/F vector), b1 = col_idx, b2 = values (double). */
int mgr_export(mgr_handle h, int32_t kind, int32_t level, int32_t what, int32_t sub, int64_t *sizes,
               void *b0, void *b1, void *b2);

/* Message of the last error on this handle (host string, owned by the handle). */
const char *mgr_last_error(mgr_handle h);

/* Free every buffer of the handle (synchronises its stream). */
void mgr_destroy(mgr_handle h);

#ifdef __cplusplus
}
#endif

#endif /* MGR_H */
