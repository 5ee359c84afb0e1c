/*
 * gsr.h -- C interface of libgsr, an MI355X (gfx950) implementation of the
 * hot path of the Gaia AVU-GSR solver (Cesare et al., "The Gaia AVU-GSR
 * solver: a CPU + GPU parallel code toward Exascale systems").
 *
 * The library solves the overdetermined system A x = b of Sec. 2, Eq. (1),
 * with preconditioned LSQR (Paige & Saunders 1982), computing per iteration
 * the two products of Eq. (2) and Eq. (3), the variances, and the
 * covariances of Eq. (4) for a selected set of unknowns.
 *
 * Matrix form (Sec. 2): A is held as a "dense" [m][24] coefficient array with
 * N_Astro = 5, N_Att = 12, N_Instr = 6 and N_Glob = 1 values per row.
 *   slot  0..4   astrometric: columns 5*s .. 5*s+4 of the row's star s
 *   slot  5..16  attitude: axis a = (k-5)/4 uses column
 *                N_A + a*n_att + att_start[r] + (k-5)%4   (N_A = 5*n_stars)
 *   slot 17..22  instrumental: column N_A + 3*n_att + instr_col[r][k-17]
 *   slot 23      global: column N_A + 3*n_att + n_instr  (ignored if n_glob = 0)
 * Unknowns: [astrometric, star-major][attitude, axis-major][instrumental][global],
 * n = 5*n_stars + 3*n_att + n_instr + n_glob.  Rows are sorted by star: star s
 * owns rows star_row_ptr[s] .. star_row_ptr[s+1]-1.
 *
 * Conventions for every entry point:
 *  - Return 0 (GSR_OK) or a negative GSR_E* code; gsr_last_error() then gives
 *    a message (thread-local).  LSQR convergence outcomes are not errors:
 *    they come back in gsr_lsqr_result.istop.
 *  - Pointers marked "device" must be device memory of the current HIP
 *    device (e.g. from hipMalloc or a PyTorch tensor); "host" pointers are
 *    ordinary host memory.  Arrays are dense and C-ordered.
 *  - The system arrays are BORROWED by the handle: the caller keeps them
 *    alive and unchanged until gsr_destroy.  A handle made by
 *    gsr_create_packed holds no copy of the coefficients at all.  A handle
 *    made by gsr_create over rows in star order makes, at the first solve
 *    that needs it, a library-owned copy of the rows regrouped by attitude
 *    window (about the bytes of A; see gsr_set_blocked) and, for star-order
 *    passes, further row-level copies (see gsr_create).  The library
 *    allocates and frees its own workspaces (vectors of the solve, scalars,
 *    partial sums, covariance buffers, index records).
 *  - `stream` is a hipStream_t (NULL: the null stream).  Calls are
 *    asynchronous on it unless stated otherwise.  A handle is not
 *    thread-safe and its calls must be ordered on one stream; separate
 *    handles are independent.
 */
#ifndef GSR_H
#define GSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsr_system gsr_system;
typedef struct gsr_layout gsr_layout;
typedef struct gsr_mlp gsr_mlp;
typedef void *gsr_stream; /* hipStream_t */

enum {
    GSR_OK = 0,
    GSR_EINVAL = -1, /* bad argument, bad index data, unknown handle */
    GSR_ENOMEM = -2, /* device allocation failed */
    GSR_EHIP = -3,   /* a HIP runtime call failed */
    GSR_ESTATE = -4  /* call out of order (e.g. iterate without begin) */
};

enum { GSR_F64 = 0, GSR_F32 = 1 };          /* storage type of the coefficients */
enum { GSR_PROD_F64 = 0, GSR_PROD_F32 = 1 }; /* how a product a*x is formed */

typedef struct {
    int64_t n_stars; /* >= 0 */
    int64_t m;       /* rows (observations), >= 0 */
    int64_t n_att;   /* attitude spline coefficients per axis, >= 4 */
    int64_t n_instr; /* instrumental unknowns, >= 6 */
    int32_t n_glob;  /* 0 or 1 */
    int32_t value_type; /* GSR_F64 or GSR_F32 */
} gsr_dims;

/* n = 5*n_stars + 3*n_att + n_instr + n_glob, or -1 for invalid dims. */
int64_t gsr_num_unknowns(const gsr_dims *d);
const char *gsr_last_error(void);
const char *gsr_version(void);

/*
 * Create a handle over a system (Sec. 2, Eq. 1; the 24-slot form above).
 *   vals          device, [m][24] double (GSR_F64) or float (GSR_F32), 16-byte aligned
 *   star_row_ptr  device, [n_stars+1] int64, star_row_ptr[0] = 0, nondecreasing,
 *                 star_row_ptr[n_stars] = m
 *   att_start     device, [m] int32 in [0, n_att-4]
 *   instr_col     device, [m][6] int32 in [0, n_instr), 8-byte aligned
 * The index arrays are validated on the device; the first offending row or
 * star is reported with GSR_EINVAL.  Synchronous.  *out is set on success.
 */
int gsr_create(gsr_system **out, const gsr_dims *d, const void *vals, const int64_t *star_row_ptr,
               const int32_t *att_start, const int32_t *instr_col, gsr_stream stream);
/* gsr_create also packs the instrumental columns and attitude start of each
 * row (16 bytes per row) for the one-pass iteration.  When 3*n_att + n_instr +
 * n_glob exceeds 2048 (the attitude block does not fit in LDS) the handle makes
 * further library-owned COPIES OF THE COEFFICIENTS at their first use: the
 * rows regrouped by attitude window for LSQR solves and gsr_aprod12 (192
 * bytes per FP64 row plus 28 of indices; gsr_set_blocked), and, for
 * gsr_aprod2 and solves not on that copy, the 12 attitude coefficients of
 * every row grouped by attitude start plus the other 12 in row order (about
 * 200 bytes per FP64 row), so that aprod 2 needs no global atomics.  If an
 * allocation fails the handle falls back to the star-order passes, or to
 * atomics.  To solve without any copy of A, place the rows yourself
 * (gsr_layout_plan / gsr_layout_pack / gsr_create_packed). */
/* Free the handle's workspaces (synchronises the device first).  NULL is a no-op. */
int gsr_destroy(gsr_system *sys);

/*
 * aprod 1 (Sec. 2, Eq. 2): y <- scale_y * y + A x.
 *   x device [n], y device [m] (must not overlap).  scale_y = 1 gives the
 *   paper's "b += A x"; scale_y = 0 overwrites y without reading it.
 *   product GSR_PROD_F32 (FP32 systems only) forms each a*x in FP32 from
 *   fl32(x); sums are always FP64.  The attitude part of x is first copied
 *   into a handle workspace of window records (16 n_att doubles: for each
 *   attitude start the 12 values of its window, one 128-byte line), from
 *   which each tile's windows are loaded together.
 */
int gsr_aprod1(gsr_system *sys, const double *x, double *y, double scale_y, int32_t product,
               gsr_stream stream);
/*
 * gsr_aprod1 without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as gsr_aprod1, on
 * handles made by gsr_create.  Its workspace, the attitude window records
 * of x (16 values per attitude start), lives in a static device array of
 * 16 MiB per GPU held until the process ends: 16 * n_att must not exceed
 * 2,097,152, i.e. n_att <= 131,072 (GSR_EINVAL otherwise).
 * The handle's device must be current.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (other streams, other threads,
 * other handles) race and must be ordered by the caller.
 */
int gsr_aprod1_noalloc(gsr_system *sys, const double *x, double *y, double scale_y, int32_t product,
                       gsr_stream stream);
/*
 * aprod 2 (Sec. 2, Eq. 3): x <- scale_x * x + A^T y.
 *   y device [m], x device [n] (must not overlap).  Same conventions as
 *   gsr_aprod1.  Attitude / instrumental / global sums use FP64 atomics, so
 *   their summation order (and last bits) may vary between calls.
 */
int gsr_aprod2(gsr_system *sys, const double *y, double *x, double scale_x, int32_t product,
               gsr_stream stream);
/*
 * Column scaling used by the preconditioner (Sec. 2, solver step 2; read as
 * diagonal column scaling): scale[j] = 1/||a_j||_2 (1 for an empty column).
 * Computed once per handle and cached.  scale_out device [n] or NULL.
 */
int gsr_column_scale(gsr_system *sys, double *scale_out, gsr_stream stream);

typedef struct {
    double damp;      /* >= 0: minimise ||A x - b||^2 + damp^2 ||S^-1 (x - x0)||^2 */
    double atol, btol; /* Paige-Saunders tolerances, >= 0 */
    double conlim;    /* > 0: stop when cond(A S) estimate exceeds it; 0 = off */
    int64_t itmax;    /* >= 0 */
    int32_t precond;  /* 1: column scaling S = diag(1/||a_j||); 0: S = I */
    int32_t product;  /* GSR_PROD_F64 or GSR_PROD_F32 (FP32 systems) for the iteration products */
    int32_t outer_max;  /* gsr_lsqr_refine only: maximum outer steps (>= 1) */
    double outer_tol;   /* gsr_lsqr_refine only: stop when ||dx|| <= outer_tol ||x||, or when
                           the next correction predicted from the last two,
                           ||dx_k||^2 / ||dx_k-1||, is at most outer_tol ||x|| */
} gsr_lsqr_opts;

typedef struct {
    int32_t istop;      /* 0: x0 solves it (b - A x0 = 0 or A^T(b - A x0) = 0); 1: compatible
                           system solved to atol/btol; 2: least-squares solution to atol;
                           3: conlim reached; 4-6: as 1-3 at machine precision; 7: itmax */
    int32_t outer_steps; /* gsr_lsqr_refine: outer steps taken */
    int64_t itn;        /* iterations (refine: inner iterations of the last step) */
    int64_t inner_total; /* refine: inner iterations summed over the outer steps */
    double rnorm, arnorm, anorm, acond, xnorm, bnorm; /* Paige-Saunders estimates; xnorm = ||y||
                           of the scaled problem, computed directly */
} gsr_lsqr_result;

/*
 * Preconditioned LSQR (Sec. 2 solver outline): precondition, initial
 * conditions with aprod 2, iterate aprod 1 / aprod 2 / variances /
 * covariance vectors, de-precondition.  Returns x = x0 + S y where y solves
 * min ||[A S; damp I] y - [b - A x0; 0]||, and the variances
 * var_j = s_j^2 sum_i d_i[j]^2 (d_i = w_i / rho_i).
 *   b device [m]; x0 device [n] or NULL (zero start); x device [n] (output);
 *   var device [n] or NULL; opts host; res host or NULL.
 * Every iteration runs on the device without host round trips; the call
 * returns once the solve has stopped (synchronous).
 */
int gsr_lsqr_solve(gsr_system *sys, const double *b, const double *x0, double *x, double *var,
                   const gsr_lsqr_opts *opts, gsr_lsqr_result *res, gsr_stream stream);

/* The same solve in steps: begin (asynchronous), iterate n more iterations
 * (asynchronous; iterations after a stop are no-ops), status (synchronises
 * and reads the scalars), peek (current x = x0 + S y into device [n]),
 * end (flush covariances, write x / var, read the result; synchronous).
 * b and x0 must stay valid until end.  A begin while a solve is in progress
 * drops that solve and starts a new one. */
int gsr_lsqr_begin(gsr_system *sys, const double *b, const double *x0, const gsr_lsqr_opts *opts,
                   gsr_stream stream);
int gsr_lsqr_iterate(gsr_system *sys, int64_t n_iter, gsr_stream stream);
int gsr_lsqr_status(gsr_system *sys, gsr_lsqr_result *res, gsr_stream stream);
int gsr_lsqr_peek(gsr_system *sys, double *x, gsr_stream stream);
int gsr_lsqr_end(gsr_system *sys, double *x, double *var, gsr_lsqr_result *res, gsr_stream stream);

/*
 * FP32 form with FP64 iterative refinement (FP32 systems).  Each outer step
 * forms r = b - A x with FP64 products on the FP32 coefficients (exact
 * upcast), solves A dx ~ r with LSQR using `inner` (normally
 * product = GSR_PROD_F32 and loose atol/btol), and updates x += dx, until
 * the correction, or the next one predicted from the contraction between the
 * last two, is at most outer_tol ||x||, or outer_max steps.  Arguments as
 * gsr_lsqr_solve, except that damp must be 0 (GSR_EINVAL otherwise): each
 * inner solve would damp its correction towards zero rather than x towards
 * x0, so the outer loop would not converge to the damped solution.
 */
int gsr_lsqr_refine(gsr_system *sys, const double *b, const double *x0, double *x,
                    const gsr_lsqr_opts *inner, gsr_lsqr_result *res, gsr_stream stream);

/*
 * Constraint equations (Sec. 2: a set of them makes the solution unique):
 * ncon sparse rows C under A, with right-hand sides c, so that the LSQR
 * solves of this handle minimise ||[A; C] x - [b; c]||.  Host arrays, copied:
 *   ptr [ncon+1] (ptr[0] = 0), col [ptr[ncon]] in [0, n) strictly increasing
 *   within a row, val [ptr[ncon]], rhs [ncon].  ncon = 0 removes them.
 * They enter the LSQR products, norms, variances and covariances and the
 * column scaling (norms of the columns of [A; C]); gsr_aprod1 / gsr_aprod2
 * keep computing with A alone.  Solves with constraints run the fused
 * iteration (FP64 products; see gsr_set_fused) and gsr_lsqr_refine refuses
 * them.  Rows may be long (e.g. a condition over every star): each is cut
 * into tiles of 8192 entries reduced by one workgroup each.
 */
int gsr_set_constraints(gsr_system *sys, int64_t ncon, const int64_t *ptr, const int64_t *col, const double *val,
                        const double *rhs);

/*
 * Covariances of Eq. (4) for a selected set of unknowns, read as
 * C = S_sel (sum_i d_i[sel] d_i[sel]^T) S_sel with d_i = w_i / rho_i.
 * gsr_cov_request attaches the selection to the handle for the next solves:
 *   sel host [k] in [0, n) (k = 0 detaches), block in [1, 1024]: iterations
 *   buffered on the device (d_i[sel] gathered every iteration, as the
 *   x_Cycle buffer of Sec. 2.2 with itnCovCP = block) before each FP64 MFMA
 *   SYRK update C += D D^T.  Synchronous.
 * gsr_cov_get writes C of the last solve: device [k][k], full symmetric,
 * diagonal = var[sel].
 * gsr_cov_bytes: bytes of the per-cycle buffer of the two pipeline
 * versions of Sec. 2.2 (Eq. 5: version 1, 8*itn_cov_cp*n_unk; Eq. 6:
 * version 2, 8*itn_cov_cp*n_indexes), or -1 for bad arguments.
 */
int gsr_cov_request(gsr_system *sys, const int64_t *sel, int64_t k, int32_t block);
int gsr_cov_get(gsr_system *sys, double *C, gsr_stream stream);
int64_t gsr_cov_bytes(int32_t version, int64_t itn_cov_cp, int64_t count);

/*
 * Covariances for a list of index pairs instead of a dense block (version 2
 * of the covariance pipeline, Sec. 2.2, whose files hold the x_Cycle entries
 * of the indexes j1, j2 of Eq. (4)):
 *   gsr_cov_request_pairs attaches pairs host [P][2] of unknowns in [0, n)
 *   (repeats allowed; (j, j) gives var[j]) for the next solves.  Their
 *   distinct indexes are buffered per iteration as by gsr_cov_request and,
 *   every `block` iterations, C_p += sum_i d_i[j1_p] d_i[j2_p] is formed by a
 *   dot-product kernel (16 lanes per pair); block in [1, 1024].  Replaces a
 *   dense request (and vice versa); P = 0 detaches.
 *   gsr_cov_get_pairs writes out device [P]: C_p = s_j1 s_j2 sum_i ... of the
 *   last solve.
 *   gsr_cov_pairs_from_export forms the same values from blocks written by
 *   gsr_cov_export (arguments as gsr_cov_from_export; pairs host [P][2];
 *   out device [P]).
 */
int gsr_cov_request_pairs(gsr_system *sys, const int64_t *pairs, int64_t P, int32_t block);
int gsr_cov_get_pairs(gsr_system *sys, double *out, gsr_stream stream);
int gsr_cov_pairs_from_export(const double *blocks, int64_t n, int32_t block, int64_t nblocks, int32_t last_cols,
                              const int64_t *pairs, int64_t P, const double *S, double *out, gsr_stream stream);

/*
 * Export of the whole per-iteration vectors d_i = w_i / rho_i (all n
 * unknowns, in the preconditioned variable of the solve) for covariances
 * chosen after the run: version 1 of the covariance pipeline of Sec. 2.2,
 * whose per-cycle size is Eq. (5) (gsr_cov_bytes(1, block, n)).
 *   gsr_cov_export attaches, for the next solves, the caller's host buffer
 *   host [max_blocks][block][n] doubles (pinned memory from hipHostMalloc
 *   lets the copies overlap the solve; pageable memory works but stalls it).
 *   Every `block` iterations the block's vectors are copied asynchronously
 *   from a device ring of 2*block*n doubles on a copy stream of the handle;
 *   gsr_lsqr_end / gsr_lsqr_solve return once all copies have landed.  Block
 *   b holds iterations b*block+1 .. (b+1)*block; blocks past max_blocks are
 *   not stored.  block in [1, 1024]; block = 0 detaches.  Graph replay is
 *   not used while exporting.
 *   gsr_cov_export_status: blocks of the last solve and the vectors in its
 *   last block (itn = (blocks-1)*block + last_cols).
 * gsr_cov_from_export forms C = S_sel (sum_i d_i[sel] d_i[sel]^T) S_sel from
 * such blocks (the covariances program of Sec. 2.2): blocks host
 * [nblocks][block][n], the last holding last_cols vectors; sel host [k] in
 * [0, n); S device [n], the column scaling the solve used (NULL if none);
 * C device [k][k], full symmetric.  Synchronous on `stream`.
 */
int gsr_cov_export(gsr_system *sys, double *host, int64_t max_blocks, int32_t block);
int gsr_cov_export_status(gsr_system *sys, int64_t *blocks, int32_t *last_cols);
int gsr_cov_from_export(const double *blocks, int64_t n, int32_t block, int64_t nblocks, int32_t last_cols,
                        const int64_t *sel, int64_t k, const double *S, double *C, gsr_stream stream);

/*
 * One covariance update C += D[:, :cols] D[:, :cols]^T (Eq. 4 over a block of
 * buffered vectors) on the upper triangle of 32x32 tiles of C.
 *   D device [k][ldd] (cols <= ldd), C device [k][k]; lower-triangle tiles
 *   are not written.
 */
int gsr_syrk(const double *D, int64_t k, int64_t cols, int64_t ldd, double *C, gsr_stream stream);

/* Launch tuning of the star-order row-streaming kernels: waves per CU
 * (1..256), and, when the attitude block does not fit in LDS, att_atomics = 1
 * to sum the attitude part of aprod 2 with device-scope FP64 atomics instead
 * of the attitude-bucketed pass (for comparison; much slower).  Results are
 * unchanged up to the order of FP64 additions. */
int gsr_set_tuning(gsr_system *sys, int32_t waves_per_cu, int32_t att_atomics);

/* Replay of captured HIP graphs for blocks of LSQR iterations (16, or the
 * covariance block), on by default; per-kernel timing disables it.  The
 * graphs run on a stream of the handle, ordered with the caller's stream by
 * events. */
int gsr_set_graphs(gsr_system *sys, int32_t on);

/* One pass over the rows per LSQR iteration (on by default).  An iteration
 * needs A v_i - alpha_i u_i and then A^T u_{i+1} (Sec. 2, Eq. 2 and Eq. 3);
 * with u kept unnormalised, A^T u_{i+1} = A^T(beta_{i+1} u_{i+1}) / beta_{i+1},
 * so both products read each row once and 1/beta_{i+1} is applied
 * afterwards.  Used when the attitude columns are summed in LDS, by the
 * regrouped copy (gsr_set_blocked) or by the bucketed pass; off, or
 * otherwise, an iteration runs gsr_aprod1 and gsr_aprod2 as separate passes.
 * Results agree up to the rounding of the 1/beta scaling (with FP32
 * products: the FP32 operand of A^T u is the unnormalised u). */
int gsr_set_fused(gsr_system *sys, int32_t on);

/* Rows regrouped by attitude window (on by default; used by fused solves
 * when the attitude block does not fit in LDS).
 * At the first such solve the handle makes a device copy of the rows grouped
 * by block g = att_start / Wb, star order inside a block, padded to 64-row
 * tiles, with Wb the widest window whose 3 x (Wb + 3) sums fit in LDS (at
 * most 8192 starts; max_window > 0 caps it, >= 4).  Each iteration is then
 * one pass over that copy: A v, the attitude sums in the LDS window, and the
 * star sums as per-segment partials added by the tail.  The copy takes about
 * the bytes of A plus 28 bytes per row and is kept until gsr_destroy or a
 * change of max_window.  Without memory for it, solves use the bucketed
 * pass.  Results agree with the other forms up to summation order.  Fails
 * with GSR_ESTATE during a solve.  On a handle from gsr_create_packed the
 * layout is fixed: only on = 1 with max_window = 0 is accepted. */
int gsr_set_blocked(gsr_system *sys, int32_t on, int32_t max_window);

typedef struct {
    int32_t active;       /* 1 once the handle's regrouped rows exist */
    int32_t workgroups;   /* of its pass */
    int64_t window;       /* Wb: attitude starts per block */
    int64_t blocks;
    int64_t padded_rows;  /* rows including the padding to 64-row tiles */
    int64_t segments;     /* star segments (astrometric partial sums per pass) */
    int64_t bytes;        /* device bytes the library holds for the layout besides the
                             coefficients: row records (12 B per row), positions, segment
                             lists and sums, workgroup windows, u in this order */
    int64_t value_bytes;  /* coefficient bytes of the regrouped rows (padding included):
                             padded_rows * 24 * sizeof(value) */
    int32_t values_owned; /* 1: the coefficients are the library's copy (gsr_create);
                             0: the caller's buffer (gsr_create_packed) */
    int32_t reserved;
} gsr_blocked_layout;
int gsr_blocked_info(gsr_system *sys, gsr_blocked_layout *info);

/*
 * Rows placed by the caller in the regrouped order (no library copy of A).
 * The one-pass iteration streams the rows grouped by attitude window (block
 * g = att_start / Wb, star order inside a block, 64-row tiles stored
 * chunk-major, blocks padded with zero rows to whole tiles): Sec. 2's
 * products (Eq. 2 and Eq. 3) then read each coefficient once per iteration.
 * Since GPU memory bounds the system one GPU can hold (Sec. 2.1), a caller
 * with a large system computes the layout from its index data, places its
 * coefficients there once while loading them, and hands the buffer over:
 *
 * gsr_layout_plan: the layout of a system from its index arrays (device
 *   pointers, as for gsr_create; validated the same way); max_window > 0
 *   caps Wb (>= 4), 0 takes the widest window that fits in LDS.  Needs
 *   m > 0, n_att >= 8 and n_instr <= 2047.  The caller may free its index
 *   arrays afterwards: the layout keeps 12-byte records per row (star,
 *   attitude start, instrumental columns).  Synchronous.
 * gsr_layout_info: sizes of the layout (active = 0, values_owned = 0); the
 *   caller allocates value_bytes of device memory for the packed rows
 *   (16-byte aligned).
 * gsr_layout_pack: rows row0 .. row0+count-1 (caller's star order), given as
 *   device [count][24] coefficients of the dims' value type, into their
 *   places in packed.  Any chunking and order of calls; every row must be
 *   placed once before gsr_create_packed.  Asynchronous on `stream`.
 * gsr_create_packed: a handle over the packed rows.  The handle borrows
 *   `packed` (kept alive and, apart from the padding rows, which this call
 *   zeroes, unchanged until gsr_destroy) and takes the layout over: on
 *   success the layout is consumed (not to be used or destroyed again); on
 *   failure it stays with the caller.  Every product, solve, covariance and
 *   constraint call works on such a handle, with vectors in the caller's
 *   row order; LSQR always runs the one-pass iteration (gsr_set_fused(0) and
 *   gsr_set_blocked(0) are refused), the standalone products run the same
 *   pass (one pass reads every coefficient) and fail with GSR_ESTATE while a
 *   solve is in progress; gsr_features and gsr_aprod1_noalloc, which read
 *   rows in star order, are refused.  Synchronous.
 * gsr_layout_destroy: frees a layout that was not consumed (NULL: no-op).
 */
int gsr_layout_plan(gsr_layout **out, const gsr_dims *d, const int64_t *star_row_ptr, const int32_t *att_start,
                    const int32_t *instr_col, int32_t max_window, gsr_stream stream);
int gsr_layout_info(gsr_layout *layout, gsr_blocked_layout *info);
int gsr_layout_pack(gsr_layout *layout, const void *rows, int64_t row0, int64_t count, void *packed,
                    gsr_stream stream);
int gsr_create_packed(gsr_system **out, gsr_layout *layout, void *packed, gsr_stream stream);
int gsr_layout_destroy(gsr_layout *layout);

/*
 * Both products of an LSQR iteration in one pass over the regrouped rows
 * (Sec. 2, Eq. 2 then Eq. 3 on the updated vector):
 *   u <- scale_u * u + A v,   then   x <- scale_x * x + A^T u  (the new u).
 *   v device [n], u device [m] (caller's row order), x device [n]; v and x must
 *   not overlap.  product as for gsr_aprod1.  This is the pass the LSQR
 *   iteration runs every step, exposed with plain vectors.  On a handle from
 *   gsr_create it builds the library's regrouped copy at first use
 *   (GSR_ENOMEM without memory for it).  A^T u sums use FP64 LDS atomics and
 *   per-segment partials, so their order (last bits) may vary between calls.
 *   Fails with GSR_ESTATE while a solve is in progress and with GSR_EINVAL
 *   when constraint equations are attached.
 */
int gsr_aprod12(gsr_system *sys, const double *v, double *u, double scale_u, double *x, double scale_x,
                int32_t product, gsr_stream stream);

/* Per-kernel timing with HIP events on the solve's stream (off by default).
 * gsr_timing_get synchronises, returns the totals since the last get and
 * resets them. */
typedef struct {
    double aprod1_ms, aprod2_ms, tail_ms, update_ms, syrk_ms;
    int64_t aprod1_n, aprod2_n, tail_n, update_n, syrk_n;
} gsr_timing;
int gsr_timing_enable(gsr_system *sys, int32_t on);
int gsr_timing_get(gsr_system *sys, gsr_timing *t);

/*
 * Learned warm start.  Not part of the paper's method: a per-star regression
 * from system features to the 5 astrometric unknowns, used only to choose
 * x0 for gsr_lsqr_solve (LSQR from x0 converges to the same solution).
 *
 * gsr_features: F device [n_stars][28] FP64 per star s:
 *   [0..14] upper triangle (row-major) of A_s^T A_s, A_s = the star's rows on its
 *   5 astrometric columns; [15..19] A_s^T bt, bt = b - A_other x_other (the known
 *   terms minus the attitude / instrumental / global part at x_other);
 *   [20] rows; [21] mean(att_start)/n_att; [22] population std of att_start/n_att;
 *   [23] rms attitude coefficient; [24] rms instrumental; [25] rms global (0 if none);
 *   [26] ||bt_s||/sqrt(rows); [27] sum_r a_glob bt_r / rows.
 *   b device [m], x_other device [n - 5*n_stars].
 * gsr_mean_rows: out[j] = mean_i X[i][j]; X device [k][len], out device [len].
 */
int gsr_features(gsr_system *sys, const double *b, const double *x_other, double *F, gsr_stream stream);
int gsr_mean_rows(const double *X, int64_t k, int64_t len, double *out, gsr_stream stream);

/*
 * FP32 network n_in -> n_hidden -> n_hidden -> n_out with ReLU on the hidden
 * layers.  params (host, FP64, copied and rounded to FP32):
 * W1 [n_hidden][n_in], b1, W2 [n_hidden][n_hidden], b2, W3 [n_out][n_hidden], b3.
 * Inputs and targets are standardised with the column mean / population
 * standard deviation set by gsr_mlp_fit_norm (identity until then).
 *   forward: X device [N][n_in] FP64 -> Y device [N][n_out] FP64 (de-standardised).
 *   grad: mean squared error on the standardised targets and its gradient with
 *         respect to every parameter (device FP32 [param count], same order as
 *         params) without updating; loss to *loss_host.  Synchronous.
 *   train: `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8,
 *          learning rate lr); final loss to *loss_host.  Synchronous.
 *   get_params: host FP64 copy of the current parameters.
 */
int gsr_mlp_create(gsr_mlp **out, int32_t n_in, int32_t n_hidden, int32_t n_out, const double *params);
int gsr_mlp_destroy(gsr_mlp *net);
int gsr_mlp_get_params(gsr_mlp *net, double *params);
int gsr_mlp_fit_norm(gsr_mlp *net, const double *X, const double *T, int64_t N, gsr_stream stream);
int gsr_mlp_forward(gsr_mlp *net, const double *X, int64_t N, double *Y, gsr_stream stream);
int gsr_mlp_grad(gsr_mlp *net, const double *X, const double *T, int64_t N, double *loss_host, float *grads,
                 gsr_stream stream);
int gsr_mlp_train(gsr_mlp *net, const double *X, const double *T, int64_t N, int32_t steps, double lr,
                  double *loss_host, gsr_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
