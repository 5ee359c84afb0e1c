// Internal declarations shared by the HIP kernels and the C-ABI layer.
// Not installed; the public interface is include/gsr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsr.h"

namespace gsr {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlock = 256;        // threads per workgroup (4 waves)
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kSlots = 24;         // coefficients per row: 5 astro, 12 attitude, 6 instr, 1 global
constexpr int kMaxPartials = 4096; // upper bound on workgroups of most reducing launches
constexpr int kPartialSlots = 16384; // partial slots in Work (the segment-reducing tail takes up to this many)
constexpr int kLdsTailMax = 2048;   // tail columns accumulated in LDS when they fit (16 KB)
constexpr int kXcds = 8;            // XCDs; workgroup b is dispatched to XCD b mod 8

// Device-resident LSQR state.  Written only by the single "last" workgroup of
// a launch (ticket pattern) or by the host before a solve; every other
// workgroup reads it at kernel entry.
struct Scalars {
  // bidiagonalisation
  double alpha, beta;        // alpha_i, beta_i (beta also the scale of the stored u)
  double u_scale;            // -alpha_i / beta_i : aprod1 multiplier of the stored u
  double inv_beta;           // 1 / beta_{i+1}    : aprod2 multiplier of u
  double v_scale;            // -beta_{i+1}       : aprod2 multiplier of v_i
  double inv_alpha;          // 1 / alpha_{i+1}   : update-pass normaliser of v
  // rotations
  double rhobar, phibar;
  double t1, t2, t3;         // phi/rho, -theta/rho, 1/rho
  // estimates
  double anorm2, ddnorm, res2, xnorm, rnorm, arnorm, acond, bnorm;
  // options
  double damp, atol, btol, ctol;
  double con_sumsq;          // sum of squares of the constraint rows of u (added to beta^2)
  int64_t itn, itmax;
  int32_t istop;             // Paige-Saunders stop code
  int32_t done;              // 1 once the solve has stopped (any reason)
  int32_t do_v;              // 1 if aprod2 runs this iteration (beta_{i+1} > 0)
  int32_t dcount;            // covariance columns buffered since the last SYRK flush
  int32_t raw;               // 1: a standalone product pass; the epilogues only record beta / alpha
  int64_t dblock;            // columns per covariance block
  int64_t nsel;              // selected unknowns (0: no covariances)
};

// Reduction workspace: per-launch workgroup partials and tickets.
struct Work {
  double* part_a;            // [kPartialSlots] partial sums of a reducing launch
  double* part_b;            // [kPartialSlots] second set (astro part of ||v||^2)
  double* part_c;            // [kPartialSlots] third set (sum of d^2 in the update pass)
  unsigned* tickets;         // [8] last-workgroup tickets, one per kernel kind
};

enum Ticket {
  T_APROD1 = 0, T_APROD2 = 1, T_TAIL = 2, T_UPDATE = 3, T_INIT = 4, T_SYRK = 5, T_VALID = 6, T_GATHER = 7,
  T_CON = 8,
  kTickets = 16
};

// A borrowed view of the caller's system arrays plus the sizes derived from them.
struct SysView {
  int64_t n_stars, m, n_att, n_instr;
  int32_t n_glob, value_type;
  int64_t n_astro, tail_len, n;
  const void* vals;
  const int64_t* row_ptr;
  const int32_t* att_start;
  const int32_t* instr_col;
  int32_t has_empty_stars;
};

// Launch shape of the row-streaming kernels: each wave owns a contiguous range
// of whole stars holding about m / waves rows.
struct StreamShape {
  int blocks;
  int waves;
};
StreamShape stream_shape(const SysView& s, int cus, int waves_per_cu);

// Attitude-bucketed view of the system, built once per handle when the
// attitude block does not fit in LDS.  Rows are grouped by bucket
// b = att_start / Wb (Wb consecutive attitude starts per bucket); inside a
// bucket they keep star order, chunk by chunk (chunks of K consecutive rows).
// The attitude part of aprod 2 then reads the 12 attitude coefficients of
// each row in bucket order (batt) together with u permuted into the same
// order (ub, written each product by the partition pass) and accumulates the
// bucket's window of Wb + 3 columns per axis in LDS.
struct AttView {
  int ready;            // 1 once built
  int64_t Wb, nb;       // bucket width, buckets
  int64_t K, nchunks;   // partition chunk rows, chunks
  int32_t* count;       // [nchunks][nb] rows of chunk c in bucket b
  int32_t* cbase;       // [nchunks][nb] bucket-order position of the first such row
  int32_t* lst;         // [nchunks][nb+1] rows of chunk c in buckets before b
  uint16_t* lpos;       // [m] position of row r in its chunk's bucket-grouped order
  void* batt;           // [m][12] attitude coefficients in bucket order (value type)
  uint16_t* bst;        // [m] att_start - b*Wb in bucket order
  int32_t nsub;         // workgroup ranges of the attitude pass
  int64_t* sub_lo;      // [nsub+1] bucket-order row ranges
  int32_t* sub_b;       // [nsub] bucket of each range
  int32_t* bsub;        // [nb+1] first range of each bucket
  double* Q;            // [nsub][3][Wb+3] window partial sums
  double* ub;           // [m] u in bucket order
  void* sv;             // [m][12] astrometric, instrumental, global coefficients in row order (value type)
};

// Rows regrouped by attitude window for the one-pass iteration when the
// attitude block does not fit in LDS: a library-owned copy of the caller's
// rows, or a buffer the caller filled in this order itself (gsr_layout_pack).  Rows are grouped
// by block g = att_start / Wb and keep star order inside a block; each block
// is padded with zero rows to whole 64-row tiles.  A tile's coefficients are
// stored chunk-major (chunk j of its 64 rows is 1 KB), so a wave loads its
// rows coalesced straight into registers.  Each workgroup streams a tile range
// of one block with that block's attitude window (3 x (Wb + 3) sums) in LDS;
// a star's rows inside one wave's range form a segment whose five
// astrometric sums go to P, and the tail adds the segments of each star.
struct BlkView {
  int ready;            // 1 once built
  int64_t Wb, nb;       // attitude starts per block, blocks
  int64_t ntiles, mp;   // 64-row tiles, rows including the padding (64 * ntiles)
  int32_t G;            // workgroups of the pass (kBlkWaves waves each)
  int64_t nseg;         // star segments
  size_t lds;           // dynamic LDS bytes of the pass
  void* T;              // [ntiles][CPR][64] 16-byte chunks of the coefficients
  int t_owned;          // 1: T is the library's copy (freed with the view); 0: the caller's buffer
  int32_t value_type;   // GSR_F64 or GSR_F32
  uint32_t* R;          // [mp][3] row records (12 bytes): attitude offset in the window, end bit, the
                        // 6 instrumental columns and the star's offset from its tile's first star
  uint32_t* tstar;      // [mp / 64] star of each tile's first row
  int64_t m;            // rows of the system
  int32_t* ipos;        // [m] position of each original row
  int32_t* pad;         // [npad] padding positions
  int64_t npad;
  int32_t* wg_block;    // [G] block of each workgroup
  int32_t* wave_tile;   // [kBlkWaves*G + 1] first tile of each wave
  int32_t* seg_base;    // [kBlkWaves*G] segments before each wave's range
  int32_t* bsub;        // [nb + 1] first workgroup of each block
  int64_t ngroups;      // groups of 64 consecutive stars
  int64_t nlist;        // entries of grp_list
  int64_t* grp_base;    // [ngroups + 1] start of each group's ids in grp_list
  int32_t* grp_cnt;     // [ngroups] columns of the group's list (windows touched + a star's extra segments)
  int32_t* grp_list;    // segment ids, per group [grp_cnt][64] (star = lane), aligned by window, padded with nseg
  double* P;            // [nseg + 1][5] astrometric sums of each segment (the last entry stays zero)
  double* Q;            // [G][3][Wb + 3] attitude window sums of each workgroup
  double* ub;           // [mp] u in this order
  double* dummy;        // [kBlkWaves*G][128] per-wave store targets of lanes with nothing to store
};
constexpr int kBlkWaves = 8;  // waves per workgroup of the regrouped pass
// Values per attitude window record (12 used: 4 starts x 3 axes; 128 bytes in FP64).
constexpr int kAttRec = 16;
// Stars a row record can lie past its tile's first star (16-bit offsets).
constexpr int64_t kStarSpan = 65536;
constexpr int kBlkDummy = 128; // doubles per wave in BlkView::dummy: 64 for u, 64 for the segment sums

// LSQR epilogue arguments of the tail pass.
struct TailLsqr {
  int lsqr_stage;       // 0 init, 1 iteration
  int astro_parts;      // partials written by the aprod2 launch
  const double* gA;     // fused iteration: raw astrometric column sums (scaled here by 1/beta); else null
};

// ---- launchers (all asynchronous on `st`) ---------------------------------
// y <- scale*y + ax * A x (or with the LSQR scalars: scale = sc->u_scale, ax = 1,
// and the last workgroup forms beta_{i+1}); mode: 0 FP64 products, 1 FP32 products.
// x3w: kAttRec n_att doubles of workspace, which first takes the attitude window
// records of x (the kernel loads each row's 12 values as one window).
hipError_t launch_aprod1(const SysView& s, StreamShape sh, const double* x, double* x3w, double* y, double scale,
                         double ax, int pmode, Scalars* sc, Work w, int lsqr_stage, hipStream_t st);
// astro part of x <- scale*x + S*(A^T (inv_beta*y)); tail part accumulated in acc
// (attitude part by the bucketed pass when att_mode == 3).
hipError_t launch_aprod2(const SysView& s, StreamShape sh, int att_mode, const void* sv, const double* y,
                         double* x, double* acc, const double* S, double scale, double inv_beta, int pmode, int square,
                         Scalars* sc, Work w, hipStream_t st);
// tail part: x_t <- scale*x_t + S_t * (acc_t or window sums), acc cleared; LSQR epilogue when sc != nullptr.
hipError_t launch_tail(const SysView& s, const AttView& av, int att_mode, double* x, double* acc, const double* S,
                       double scale, Scalars* sc, Work w, int lsqr_stage, int astro_parts, hipStream_t st);
int att_mode_of(const SysView& s, const AttView& av, int force_atomics);
// bucketed attitude pass (attitude.hip)
int att_build(const SysView& s, AttView* av, int cus, char* err, size_t errlen, hipStream_t st);
void att_free(AttView* av);
hipError_t launch_partition(const SysView& s, const AttView& av, const double* u, Scalars* sc, hipStream_t st);
// raw = 1: sums of the stored u as they are (the fused iteration's tail divides by beta)
hipError_t launch_att_pass(const SysView& s, const AttView& av, double inv_beta, int pmode, int square,
                           Scalars* sc, hipStream_t st, int raw = 0);
// One LSQR iteration's pass over the rows (FP64 products, attitude mode 0 or 3):
// u <- u_scale*u + A vg (beta_{i+1} by the last workgroup) and, from the same
// rows, the astrometric, instrumental and global parts of A^T u on the
// unnormalised u (astrometric sums to gA, the others into acc; mode 0 also
// the attitude part).
// Constraint equations: ncon sparse rows C (CSR, entries sorted by row) under A.
// Work is split into tiles of at most kConTile entries of one row.
struct ConView {
  int64_t ncon;
  const int64_t* ptr;     // [ncon+1]
  const int64_t* col;     // [nnz]
  const double* val;      // [nnz]
  int64_t ntiles;
  const int64_t* tile_e;  // [ntiles+1] first entry of each tile
  const int64_t* tile_r;  // [ntiles] row of each tile
  double* tmp;            // [ncon] row sums (zero between uses)
};
constexpr int64_t kConTile = 8192;
// y_C <- scale*y_C + ax*C x (sc != null: scale = sc->u_scale, skipped once done, and the
// last workgroup stores sum(y_C^2) in sc->con_sumsq)
hipError_t launch_con_aprod1(const ConView& c, const double* x, double* yc, double scale, double ax, Scalars* sc,
                             Work w, hipStream_t st);
// raw[j] += sum_i C_ij yc_i into gA (j < n_astro) or acc (j - n_astro), as the fused row pass does
hipError_t launch_con_aprod2(const ConView& c, int64_t n_astro, const double* yc, double* gA, double* acc,
                             Scalars* sc, hipStream_t st);
// sq[j] += sum_i C_ij^2 (column norms of [A; C])
hipError_t launch_con_sq(const ConView& c, double* sq, hipStream_t st);

// rix: packed row indices from launch_pack_rows (required).
// init = 1: the solve's first pass (u_scale = 1 and vg = 0 give u' = u; beta_1 with its init step)
hipError_t launch_fused(const SysView& s, StreamShape sh, int att_mode, int pmode, const double* vg, const double* x3,
                        const void* rix, double* u, double* gA, double* acc, Scalars* sc, Work w, hipStream_t st,
                        int init = 0);
// rix[r] <- {att_start[r], instr_col[r][0..5] as 16-bit pairs} (16 bytes per row; needs n_instr <= 65536)
hipError_t launch_pack_rows(const SysView& s, void* rix, hipStream_t st);
// xr [n_att][kAttRec] <- the attitude window of every start (the row passes' copy of
// the attitude x), and the same rounded to FP32 into xrf when it is not null
hipError_t launch_att_records(const SysView& s, const double* x, double* xr, hipStream_t st, float* xrf = nullptr);
// Tail of the fused iteration: every column x_j <- v_scale*x_j + S_j * raw_j / beta (raw_j from gA, acc
// or the attitude windows), then alpha_{i+1} and the rotations, as launch_tail.
hipError_t launch_tail_fused(const SysView& s, const AttView& av, int att_mode, double* x, double* acc,
                             const double* S, const double* gA, Scalars* sc, Work w, hipStream_t st,
                             int lsqr_stage = 1);
// The same after the regrouped pass: attitude sums from its workgroup windows (gA from launch_seg_reduce).
hipError_t launch_tail_blk(const SysView& s, const BlkView& bv, double* x, double* acc, const double* S,
                           const double* gA, Scalars* sc, Work w, hipStream_t st, int lsqr_stage = 1);
// The tail after the regrouped pass with the segment reduction folded in (no gA): every column
// x_j <- v_scale*x_j + S_j * raw_j / beta, astrometric raw sums from the star's segments, then
// alpha and the rotations (sc required; sc->raw for a standalone product)
hipError_t launch_tail_seg(const SysView& s, const BlkView& bv, double* x, double* acc, const double* S, Scalars* sc,
                           Work w, hipStream_t st, int lsqr_stage = 1);
// gA[5s + k] <- sum of star s's segment sums P[seg][k] (block order); skipped once the solve has stopped
hipError_t launch_seg_reduce(const SysView& s, const BlkView& bv, double* gA, Scalars* sc, hipStream_t st);

// Regrouped one-pass iteration (blocked.hip).  blk_build makes the copy
// (max_window > 0 caps Wb; lds_max: the device's LDS bytes per workgroup);
// GSR_EINVAL if the system does not qualify, GSR_ENOMEM without memory for it.
int blk_build(const SysView& s, BlkView* bv, int cus, int max_window, int lds_max, char* err, size_t errlen,
              hipStream_t st);
// The layout alone (records, positions, segments, workspaces; T left null):
// what a caller needs to place its rows in the regrouped order itself.
int blk_plan(const SysView& s, BlkView* bv, int cus, int max_window, int lds_max, char* err, size_t errlen,
             hipStream_t st);
void blk_free(BlkView* bv);
size_t blk_value_bytes(const BlkView& bv);  // coefficient bytes of the layout (padding included)
size_t blk_index_bytes(const BlkView& bv);  // device bytes of everything else the view holds
// rows (the caller's [count][24] coefficients of rows row0 .. row0+count-1) into T
hipError_t launch_blk_pack(const BlkView& bv, const void* rows, int64_t row0, int64_t count, void* T, hipStream_t st);
// zero coefficients on T's padding positions
hipError_t launch_blk_zero_pad(const BlkView& bv, void* T, hipStream_t st);
// ub <- src (rows in the caller's order) permuted to the regrouped order, zero on padding
hipError_t launch_blk_permute(const BlkView& bv, const double* src, hipStream_t st);
// dst (rows in the caller's order) <- ub
hipError_t launch_blk_unpermute(const BlkView& bv, double* dst, hipStream_t st);
// The iteration's pass as launch_fused, on the regrouped copy (u in bv.ub).
// xr / xrf: the attitude window records of vg (launch_att_records) and their FP32
// rounding, the latter required with pmode 1.
// square = 1: column sums of squares (pmode 0; u taken as 1, the sums as for A^T u).
hipError_t launch_fblk(const SysView& s, const BlkView& bv, int pmode, const double* vg, const double* xr,
                       const float* xrf, double* acc, Scalars* sc, Work w, hipStream_t st, int init = 0,
                       int square = 0);
// Covariance column of the iteration: D[p][dcount] = w[sel[p]] / rho_i for p < nsel (after the tail);
// the last workgroup advances dcount.  Skipped once the solve has stopped or the block is full.
hipError_t launch_cov_gather(int64_t nsel, const int64_t* sel, const double* w, double* D, Scalars* sc, Work wk,
                             hipStream_t st);
// bad[0] <- first row with an out-of-range index, bad[1] <- first bad star, bad[2] <- 1 if a star is empty
hipError_t launch_validate(const SysView& s, unsigned long long* bad, hipStream_t st);
hipError_t launch_scale_from_sq(int64_t n, double* S, hipStream_t st);

// LSQR vector kernels
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st);
hipError_t launch_norm_init(const double* u, int64_t m, Scalars* sc, Work w, hipStream_t st);
hipError_t launch_init_vectors(int64_t n, double* v, double* vg, double* w, double* y, double* var,
                               const double* S, Scalars* sc, hipStream_t st);
// dring: export ring of 2*eblock rows of n (d_i stored in row itn mod 2*eblock), or null
hipError_t launch_update(int64_t n, double* v, double* vg, double* w, double* y, double* var,
                         const double* S, Scalars* sc, Work w_, hipStream_t st, double* dring = nullptr,
                         int64_t eblock = 1);
hipError_t launch_finish(int64_t n, const double* y, const double* var, const double* S, const double* x0,
                         double* x_out, double* var_out, hipStream_t st);
hipError_t launch_syrk(const double* D, int64_t k, int64_t ldd, double* C, Scalars* sc, Work w,
                       int64_t fixed_cols, hipStream_t st);
// Cp[p] += sum_{c<cols} D[pa[p]][c] D[pb[p]][c] (cols = fixed_cols, or sc->dcount then reset to 0)
hipError_t launch_pairdot(const double* D, int64_t ldd, const int32_t* pa, const int32_t* pb, int64_t P, double* Cp,
                          Scalars* sc, Work w, int64_t fixed_cols, hipStream_t st);
// out[p] = S[sel[pa[p]]] S[sel[pb[p]]] Cp[p] (S may be null)
hipError_t launch_pair_out(const double* Cp, int64_t P, const int32_t* pa, const int32_t* pb, const double* S,
                           const int64_t* sel, double* out, hipStream_t st);
hipError_t launch_cov_out(const double* C, int64_t k, const double* S, const int64_t* sel, double* out,
                          hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
// sc <- the scalars of a standalone product pass (raw = 1): u_scale, v_scale, inv_beta = 1, do_v = 1
hipError_t launch_raw_scalars(Scalars* sc, double u_scale, double v_scale, hipStream_t st);
hipError_t launch_step_norms(int64_t n, const double* xn, double* x, double* out2, Work w, hipStream_t st);
hipError_t launch_scaled_copy(const double* src, double* dst, int64_t n, double s, hipStream_t st);

// learned warm start (mlp.hip)
hipError_t launch_features(const SysView& s, const double* b, const double* xo, double* F, hipStream_t st);
hipError_t launch_mean_rows(const double* X, int64_t k, int64_t len, double* out, hipStream_t st);
// Strided FP32 GEMM: C(m,n) = sum_k A(m,k) B(k,n) [+bias] [ReLU] [*(mask>0)]
struct GemmArgs {
  int M, N, K;
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbk, sbn;
  float* C;
  int64_t ldc;
  const float* bias;
  int relu;
  float* Zout;
  const float* mask;
};
hipError_t mlp_col_stats(const double* X, int64_t N, int C, double* mu, double* sd, hipStream_t st);
hipError_t mlp_standardize(const double* X, int64_t N, int C, const double* mu, const double* sd, float* Xs,
                           hipStream_t st);
hipError_t mlp_destandardize(const float* Ys, int64_t N, int C, const double* mu, const double* sd, double* Y,
                             hipStream_t st);
hipError_t mlp_gemm(const GemmArgs& g, int splits, hipStream_t st);
hipError_t mlp_mse(const float* Y, const float* T, int64_t total, float* dY, double* loss, hipStream_t st);
hipError_t mlp_colsum(const float* dZ, int64_t M, int N, float* db, hipStream_t st);
hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t st);
hipError_t mlp_fill(float* p, int64_t n, float val, hipStream_t st);

// number of compute units of the current device (cached)
int device_cus();

}  // namespace gsr
