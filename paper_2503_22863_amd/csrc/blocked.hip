// One pass over the rows per LSQR iteration when the attitude block does not
// fit in LDS (Sec. 2, Eq. 2 and Eq. 3 on the bidiagonalisation of Paige &
// Saunders).
//
// A row touches five columns of its star and twelve attitude columns (three
// axes, four consecutive starts from att_start).  In star order the star
// columns are local and the attitude columns random; the bucketed attitude
// pass pays for that with a second read of the attitude coefficients every
// iteration.  Here the library keeps one copy of the rows regrouped by
// attitude block g = att_start / Wb, star order inside a block, with Wb chosen
// so that a block's window of 3 x (Wb + 3) sums fits in LDS.  Every
// workgroup streams a tile range of one block: A v and u' = u_scale u + A v,
// then a_r u'_r into the window (LDS atomics), the instrumental and global
// sums, and the star sums.  A star's rows inside a wave's range are
// consecutive (a segment); each segment's five sums are written once to P
// and a reduction pass adds the segments of each star (about one per block).
// The attitude windows go to Q and the tail adds the windows that cover a
// column.
//
// The copy stores each 64-row tile chunk-major: 16-byte chunk j of the 64 rows
// is one contiguous kilobyte, so the wave's load of chunk j puts row `lane`'s
// chunk j straight into lane `lane` (no LDS transposition).  Blocks are
// padded with zero rows to whole tiles, so every tile is full.
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "row_tiles.h"

namespace gsr {

constexpr int kBlkThreads = kBlkWaves * kWave;
// static LDS of the pass: the attitude-window regroup buffers and the reduction slots
constexpr size_t kBlkStaticLds = sizeof(double) * 2 * kBlkWaves * (kWave / 2) * 7 + sizeof(double) * kBlkWaves + 64;

// Row records, 12 bytes: word 0 = attitude start within the block's window (13
// bits) | end-of-segment bit << 13 | instrumental column 0 (11 bits) << 14 | the
// low 7 bits of the star's offset d from its tile's first star << 25; words 1-2
// (64 bits) = instrumental columns 1..5 (11 bits each) | the high 9 bits of d << 55.
__device__ __forceinline__ void rec_pack(uint32_t* R, int64_t pos, uint32_t d, uint32_t off, const int* ic,
                                         uint32_t end) {
  const uint32_t w0 = off | (end << 13) | ((uint32_t)ic[0] << 14) | ((d & 0x7Fu) << 25);
  const uint64_t B = (uint64_t)ic[1] | ((uint64_t)ic[2] << 11) | ((uint64_t)ic[3] << 22) | ((uint64_t)ic[4] << 33) |
                     ((uint64_t)ic[5] << 44) | ((uint64_t)(d >> 7) << 55);
  R[3 * pos] = w0;
  R[3 * pos + 1] = (uint32_t)B;
  R[3 * pos + 2] = (uint32_t)(B >> 32);
}

// Row records of every position: for original row r at ipos[r] its star, the
// attitude start within the block's window and the instrumental columns; for
// a padding position the star it repeats and zero columns; and the star of
// every tile's first position.  se[pos]: star | end << 31.
__global__ void k_blk_records(SysView s, BlkView bv, const uint32_t* __restrict__ se) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bv.m + bv.npad;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pos = i < bv.m ? bv.ipos[i] : bv.pad[i - bv.m];
    int ic[6] = {0, 0, 0, 0, 0, 0};
    uint32_t off = 0;
    if (i < bv.m) {
      off = (uint32_t)(s.att_start[i] % bv.Wb);
#pragma unroll
      for (int q = 0; q < 6; ++q) ic[q] = s.instr_col[6 * i + q];
    }
    const uint32_t e = se[pos];
    const uint32_t first = se[(pos / kWave) * kWave] & 0x7FFFFFFFu;
    if (pos % kWave == 0) bv.tstar[pos / kWave] = first;
    rec_pack(bv.R, pos, (e & 0x7FFFFFFFu) - first, off, ic, e >> 31);
  }
}

// Rows row0 .. row0+count-1 of the caller's order (src: their [count][24]
// coefficients) into the chunk-major tiles of T, one row per thread: the rows
// of one block keep their order, so a wave's 16-byte stores of chunk j fall
// in runs of consecutive lanes of a tile.
template <typename VT>
__global__ void k_blk_pack(BlkView bv, const u4* __restrict__ src, int64_t row0, int64_t count, u4* __restrict__ T) {
  constexpr int CPR = Geo<VT>::CPR;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pos = bv.ipos[row0 + i];
    const int64_t tile = pos / kWave, lane = pos - tile * kWave;
    u4 v[CPR];
#pragma unroll
    for (int j = 0; j < CPR; ++j) v[j] = src[i * CPR + j];
    u4* dst = T + tile * CPR * kWave + lane;
#pragma unroll
    for (int j = 0; j < CPR; ++j) dst[j * kWave] = v[j];
  }
}

// Zero coefficients on every padding position of T.
template <typename VT>
__global__ void k_blk_zero_pad(BlkView bv, u4* __restrict__ T) {
  constexpr int CPR = Geo<VT>::CPR;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bv.npad; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pos = bv.pad[i];
    const int64_t tile = pos / kWave, lane = pos - tile * kWave;
    u4* dst = T + tile * CPR * kWave + lane;
#pragma unroll
    for (int j = 0; j < CPR; ++j) dst[j * kWave] = u4{0u, 0u, 0u, 0u};
  }
}

// ub <- src in the regrouped order: coalesced reads of src, and each wave's
// writes fall in runs of consecutive positions (the rows of one block keep
// their order); the padding positions are cleared.
__global__ void k_blk_permute(BlkView bv, const double* __restrict__ src) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < bv.m + bv.npad;
       r += (int64_t)gridDim.x * blockDim.x) {
    if (r < bv.m)
      bv.ub[bv.ipos[r]] = src[r];
    else
      bv.ub[bv.pad[r - bv.m]] = 0.0;
  }
}

// dst (rows in the caller's order) <- ub, the inverse of k_blk_permute.
__global__ void k_blk_unpermute(BlkView bv, double* __restrict__ dst) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < bv.m; r += (int64_t)gridDim.x * blockDim.x)
    dst[r] = bv.ub[bv.ipos[r]];
}

// Logical workgroup of physical workgroup b out of G.  Workgroups are dispatched
// to the chip's 8 XCDs round-robin (b on XCD b % 8); numbering them so that XCD x
// takes a contiguous eighth of the logical workgroups (which run in tile order)
// keeps each XCD's L2 on the attitude window records of about one block.
__device__ __forceinline__ int64_t xcd_logical(int64_t b, int64_t G) {
  const int64_t q = G / 8, r = G % 8, x = b % 8;
  return x * q + min<int64_t>(x, r) + b / 8;
}

// The iteration's pass.  Logical workgroup b streams tiles of block wg_block[b]; its
// waves take consecutive sub-ranges.  Per tile a wave waits for the tile's
// record, chunks and u (loaded one tile ahead) and for its x gathers (issued
// during the previous tile), issues the next tile's loads, forms A x, issues
// the next tile's gathers once this tile's windows sit in LDS, stores the
// previous tile's u and segment sums, and forms the A^T u' parts.
// SQ = 1: the column sums of squares instead (every row value taken as 1 and
// each term a^2 in FP64), for the column norms of the preconditioner.
template <typename VT, int PM, int SQ>
__global__ void __launch_bounds__(kBlkThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_fblk(SysView s, BlkView bv, const double* __restrict__ x, const double* __restrict__ xr,
       const float* __restrict__ xrf, double* __restrict__ acc, Scalars* sc, Work wk, int init) {
  constexpr int CPR = Geo<VT>::CPR;
  __shared__ dd2u rg[kBlkWaves][(kWave / 2) * 7];
  __shared__ double red[kBlkWaves];
  __shared__ int flag;
  extern __shared__ double dyn[];  // window [3][W3], instrumental + global sums, instrumental x
  if (sc->done) return;
  const double scale = sc->u_scale;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t W3 = bv.Wb + 3;
  const int64_t ntl = s.n_instr + s.n_glob;
  double* win = dyn;
  double* tl = dyn + 3 * W3;
  double* xil = tl + ntl;
  const int64_t NI = s.n_astro + 3 * s.n_att;
  for (int64_t j = threadIdx.x; j < 3 * W3 + ntl; j += kBlkThreads) dyn[j] = 0.0;
  for (int64_t j = threadIdx.x; j < s.n_instr; j += kBlkThreads) xil[j] = x[NI + j];
  __syncthreads();

  const int64_t lb = xcd_logical(blockIdx.x, gridDim.x);
  const int64_t g = bv.wg_block[lb];
  const double* xw = xr + kAttRec * g * bv.Wb;   // window records of the block's starts
  const float* xwf = xrf + kAttRec * g * bv.Wb;  // the same rounded to FP32 (FP32 products only)
  const int64_t w = lb * kBlkWaves + wid;
  const int64_t T0 = bv.wave_tile[w], T1 = bv.wave_tile[w + 1];
  double sumsq = 0.0, gsum = 0.0;
  if (T0 < T1) {
    const double xg = s.n_glob ? x[NI + s.n_instr] : 0.0;
    const int64_t xa_last = 5 * s.n_stars - 1;
    const u4* cb = reinterpret_cast<const u4*>(bv.T);
    const uint32_t* rb = bv.R;
    u4 tmp[CPR];
    u4 rec;  // x, y, z: the row's record; w: the star of the tile's first row
    double uo;
    // the record first: the next tile's gathers need only it
    auto fetch = [&](int64_t t) {
      const int64_t tt = min(t, T1 - 1);  // past the range: re-read its last tile (the registers are not used)
      {
        const uint32_t* rr = rb + 3 * (tt * kWave + lane);  // three 4-byte loads, merged into one
        rec.x = __builtin_nontemporal_load(rr);
        rec.y = __builtin_nontemporal_load(rr + 1);
        rec.z = __builtin_nontemporal_load(rr + 2);
        rec.w = bv.tstar[tt];
      }
      const u4* base = cb + tt * CPR * kWave + lane;
#pragma unroll
      for (int j = 0; j < CPR; ++j) tmp[j] = ld_stream(base + j * kWave);
      uo = bv.ub[tt * kWave + lane];
    };
    // x for the tile whose record is in `rec`: the astrometric x of the 12.8
    // stars from its first (one contiguous load, shuffled per row later) and
    // its 64 attitude windows of 96 bytes, each the first 96 bytes of one
    // 128-byte record line, loaded cooperatively (piece j*64 + lane of the
    // tile's windows in cw[j]; consecutive lanes take consecutive 16-byte
    // pieces of one window) and regrouped through LDS.  Issued a tile ahead,
    // in the middle of the previous tile.  With FP32 products the windows come
    // from the FP32 records: 48 bytes each, 3 pieces of 16 bytes (the products
    // round x to FP32 anyway, so the arithmetic is the same).
    constexpr int NP = PM == 1 ? 3 : 6;  // 16-byte pieces per window
    double xs, xs2;
    dd2u cw[NP];
    auto gathers = [&]() {
      const int64_t st0 = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)rec.w, 0);
      xs = x[min(5 * st0 + lane, xa_last)];
      xs2 = x[min(5 * st0 + kWave + lane, xa_last)];
      const int ao_l = (int)(rec.x & 0x1FFFu);
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const int c = j * kWave + lane, i = c / NP, q = c - NP * i;
        const int ao = __shfl(ao_l, i, kWave);
        if constexpr (PM == 1) {
          const f4u v = *reinterpret_cast<const f4u*>(xwf + kAttRec * ao + 4 * q);
          __builtin_memcpy(&cw[j], &v, sizeof v);
        } else {
          cw[j] = *reinterpret_cast<const dd2u*>(xw + kAttRec * ao + 2 * q);
        }
      }
    };
    double carry[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int carry_valid = 0;
    int64_t nstart = bv.seg_base[w];  // segments begun before the current tile
    // Targets of the previous tile's stores.  Every lane stores on every tile, so
    // that the in-order memory counter can be tracked exactly (a conditional
    // store makes the compiler wait for everything at the next use of a load);
    // before the first tile the u targets, and for lanes past the tile's segment
    // sums the P targets, are this wave's dummy slots, one per lane (lanes storing
    // to one address are taken one at a time).  The segment sums of a tile are
    // compacted through LDS into one contiguous run of 5 x (segments closed)
    // values; g0 holds values 0..63 of the run, stored with the next tile.  A tile
    // closing more than 12 segments (rare) stores values 64..127 at once, and one
    // closing more than 25 the rest directly from the end lanes.
    double* const du = bv.dummy + w * kBlkDummy;
    double* u_dst = du + lane;
    double u_out = 0.0;
    double g0 = 0.0;
    double* pbase = bv.P;
    int pn = 0;  // segments the previous tile closed
    auto store_sums = [&]() { *(lane < 5 * pn ? pbase + lane : du + kWave + lane) = g0; };
    fetch(T0);
    gathers();
#pragma unroll 1
    for (int64_t t = T0; t < T1; ++t) {
      const uint32_t w0 = rec.x;
      const uint64_t B = (uint64_t)rec.y | ((uint64_t)rec.z << 32);
      const int64_t star = (int64_t)(rec.w + ((w0 >> 25) | ((uint32_t)(B >> 55) << 7)));
      const int aoff = (int)(w0 & 0x1FFFu);
      const int ic[6] = {(int)((w0 >> 14) & 0x7FFu), (int)(B & 0x7FFu),         (int)((B >> 11) & 0x7FFu),
                         (int)((B >> 22) & 0x7FFu),  (int)((B >> 33) & 0x7FFu), (int)((B >> 44) & 0x7FFu)};
      const bool end = ((w0 >> 13) & 1u) != 0;
      const double uo_c = (scale == 0.0) ? 0.0 : scale * uo;
      const int64_t s0 = lane_read(star, 0);
      const int64_t ds = star - s0;
      // more than 12 stars in the tile: the second shuffle window too; more than 25:
      // per-lane gathers for the lanes past it
      const bool far = __ballot(ds >= 12) != 0;
      const bool farther = __ballot(ds >= 25) != 0;
      u4 cur[CPR];
#pragma unroll
      for (int j = 0; j < CPR; ++j) cur[j] = tmp[j];
      order_point();
      fetch(t + 1);
      order_point();
      VT a[kSlots];
      __builtin_memcpy(a, cur, sizeof(a));
      // u'_r = u_scale * u_r + (A x)_r
      double ax = 0.0;
      {
        // every lane takes its star's x from the shuffle windows (stars st0 ..
        // st0+12 in xs, the next 12.8 in xs2; both loads are issued for every
        // tile, so they stay where they were issued); lanes whose star lies past
        // both windows gather per lane, consumed inside the branch: a load still
        // pending where the paths join would make the compiler wait for the next
        // tile's loads too
        const int base = 5 * (int)min<int64_t>(ds, 24);
        double axa = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int idx = base + k;
          double xv = __shfl(xs, idx & (kWave - 1), kWave);
          if (far) {
            const double hi = __shfl(xs2, idx & (kWave - 1), kWave);
            xv = idx >= kWave ? hi : xv;
          }
          axa += prod<PM>(a[k], xv);
        }
        if (farther && ds >= 25) {
          double xa5[5];
#pragma unroll
          for (int k = 0; k < 5; ++k) xa5[k] = x[5 * star + k];
          axa = 0.0;
#pragma unroll
          for (int k = 0; k < 5; ++k) axa += prod<PM>(a[k], xa5[k]);
        }
        ax += axa;
      }
      if constexpr (PM == 1) {
        // FP32 windows: all 64 rows in one round (piece c = 3 row + q, a row
        // stride of 3 pieces: 8 consecutive rows fall on distinct banks);
        // element e = 3j + axis is column start+j of that axis, taken in the
        // same order as below
        dd2u* wl = rg[wid];
#pragma unroll
        for (int j = 0; j < NP; ++j) wl[j * kWave + lane] = cw[j];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const dd2u pq = wl[lane * NP + q];
          float f[4];
          __builtin_memcpy(f, &pq, sizeof f);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int e = 4 * q + k;
            ax += prod<PM>(a[5 + 4 * (e % 3) + e / 3], (double)f[k]);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      } else {
        // regroup the attitude windows per row through LDS, 32 rows per round
        // (pieces 0..191 hold rows 0..31, pieces 192..383 rows 32..63; a padded
        // row stride of 7 pieces keeps the row reads free of bank conflicts);
        // element e = 3j + axis is column start+j of that axis
        dd2u* wl = rg[wid];
        const int half = lane >> 5, rl = lane & 31;
        double axh = ax;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int j = 3 * h; j < 3 * h + 3; ++j) {
            const int c = j * kWave + lane, ri = c / 6, q = c - 6 * ri;
            wl[(ri - 32 * h) * 7 + q] = cw[j];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          double d = ax;
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const dd2u pq = wl[rl * 7 + q];
            const int e0 = 2 * q, e1 = 2 * q + 1;
            d += prod<PM>(a[5 + 4 * (e0 % 3) + e0 / 3], pq.x);
            d += prod<PM>(a[5 + 4 * (e1 % 3) + e1 / 3], pq.y);
          }
          if (half == h) axh = d;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
        ax = axh;
      }
      // this tile's x is in LDS and registers: the next tile's gathers (its
      // record arrived with the loads issued at the top) overlap the rest of it
      gathers();
      // the previous tile's stores, issued once this tile's gathers are in (vector
      // memory counts stores and loads in one in-order counter): here they have
      // this tile's arithmetic to complete
      order_point();
      *u_dst = u_out;
      store_sums();
#pragma unroll
      for (int q = 0; q < 6; ++q) ax += prod<PM>(a[17 + q], xil[ic[q]]);
      if (s.n_glob) ax += prod<PM>(a[23], xg);
      const double un = SQ ? 1.0 : uo_c + ax;
      u_dst = bv.ub + t * kWave + lane;
      u_out = un;
      sumsq += un * un;
      // a_r * u'_r into the window, the instrumental and global sums, and the star sums
#pragma unroll
      for (int axs = 0; axs < 3; ++axs)
#pragma unroll
        for (int j = 0; j < 4; ++j) atomicAdd(win + axs * W3 + aoff + j, tprod<PM, SQ>(a[5 + 4 * axs + j], un));
#pragma unroll
      for (int q = 0; q < 6; ++q) atomicAdd(tl + ic[q], tprod<PM, SQ>(a[17 + q], un));
      if (s.n_glob) gsum += tprod<PM, SQ>(a[23], un);
      double p[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) p[k] = tprod<PM, SQ>(a[k], un);
      if (carry_valid && lane == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] += carry[k];
      }
      // segment starts: lane 0 unless the previous tile's last segment goes on, else after an end
      const uint64_t ends = __ballot(end);
      const bool prev_end = lane > 0 && ((ends >> (lane - 1)) & 1ull);
      const bool start = (lane == 0) ? !carry_valid : prev_end;
      const uint64_t starts = __ballot(start);
      const uint64_t le = (lane == kWave - 1) ? ~0ull : ((2ull << lane) - 1);
      const uint64_t mine = starts & le;
      const int seg0 = mine ? 63 - __clzll(mine) : 0;
      seg_scan(p, lane, seg0);
      const int64_t sidx = nstart - 1 + __popcll(mine);
      // compaction: the end lane of rank r (ends below it) puts its five sums at
      // 5r .. 5r+4 of the wave's LDS buffer (free between the attitude regroups);
      // the other lanes at slots of their own past 128
      const int nend = __popcll(ends);
      const int rank = __popcll(ends & ((1ull << lane) - 1));
      {
        double* cl = reinterpret_cast<double*>(rg[wid]);
        const int slot = (end && rank < 25) ? 5 * rank : 128 + 5 * lane;
#pragma unroll
        for (int k = 0; k < 5; ++k) cl[slot + k] = p[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        g0 = cl[lane];
        pbase = bv.P + (nend ? 5 * lane_read(sidx, nend ? __builtin_ctzll(ends) : 0) : 0);
        pn = nend;
        if (nend > 12) {
          const double g1 = cl[kWave + lane];
          if (kWave + lane < 5 * min(nend, 25)) pbase[kWave + lane] = g1;  // ranks past 24 store their own
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      if (nend > 25 && end && rank >= 25) {
#pragma unroll
        for (int k = 0; k < 5; ++k) bv.P[5 * sidx + k] = p[k];
      }
      nstart += __popcll(starts);
      const int lend = (int)(ends >> 63);
#pragma unroll
      for (int k = 0; k < 5; ++k) carry[k] = lane_read(p[k], kWave - 1);
      carry_valid = !lend;
    }
    *u_dst = u_out;
    store_sums();
  }
  if (s.n_glob) {
    const double gs = wave_sum(gsum);
    if (lane == 0) atomicAdd(tl + s.n_instr, gs);
  }
  __syncthreads();
  double* q = bv.Q + lb * 3 * W3;
  for (int64_t k = threadIdx.x; k < 3 * W3; k += kBlkThreads) q[k] = win[k];
  for (int64_t j = threadIdx.x; j < ntl; j += kBlkThreads) {
    const double v = tl[j];
    if (v != 0.0) atomicAdd(acc + 3 * s.n_att + j, v);
  }
  const double bs = block_sum<kBlkThreads>(sumsq, red);
  if (threadIdx.x == 0) publish(wk.part_a + blockIdx.x, bs);
  if (last_block(wk.tickets + T_APROD1, &flag)) {
    const double tot = sum_partials<kBlkThreads>(wk.part_a, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_beta(sc, tot + sc->con_sumsq, init);
      ticket_reset(wk.tickets + T_APROD1);
    }
  }
}

hipError_t launch_fblk(const SysView& s, const BlkView& bv, int pmode, const double* vg, const double* xr,
                       const float* xrf, double* acc, Scalars* sc, Work w, hipStream_t st, int init, int square) {
  if (!bv.ready || bv.G < 1 || bv.G > kMaxPartials) return hipErrorInvalidValue;
  if (xr == nullptr || (pmode == 1 && (s.value_type != GSR_F32 || xrf == nullptr))) return hipErrorInvalidValue;
  const dim3 g(bv.G), b(kBlkThreads);
  if (square) {
    if (pmode != 0) return hipErrorInvalidValue;
    if (s.value_type == GSR_F32)
      hipLaunchKernelGGL((k_fblk<float, 0, 1>), g, b, bv.lds, st, s, bv, vg, xr, xrf, acc, sc, w, init);
    else
      hipLaunchKernelGGL((k_fblk<double, 0, 1>), g, b, bv.lds, st, s, bv, vg, xr, xrf, acc, sc, w, init);
  } else if (s.value_type == GSR_F32 && pmode == 1) {
    hipLaunchKernelGGL((k_fblk<float, 1, 0>), g, b, bv.lds, st, s, bv, vg, xr, xrf, acc, sc, w, init);
  } else if (s.value_type == GSR_F32) {
    hipLaunchKernelGGL((k_fblk<float, 0, 0>), g, b, bv.lds, st, s, bv, vg, xr, xrf, acc, sc, w, init);
  } else {
    hipLaunchKernelGGL((k_fblk<double, 0, 0>), g, b, bv.lds, st, s, bv, vg, xr, xrf, acc, sc, w, init);
  }
  return hipGetLastError();
}

hipError_t launch_blk_unpermute(const BlkView& bv, double* dst, hipStream_t st) {
  if (bv.ipos == nullptr) return hipErrorInvalidValue;
  if (bv.m == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(8192, (bv.m + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_blk_unpermute, dim3(blocks), dim3(kBlock), 0, st, bv, dst);
  return hipGetLastError();
}

hipError_t launch_blk_permute(const BlkView& bv, const double* src, hipStream_t st) {
  if (bv.ipos == nullptr) return hipErrorInvalidValue;
  const int blocks = (int)std::min<int64_t>(8192, (bv.m + bv.npad + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_blk_permute, dim3(std::max(blocks, 1)), dim3(kBlock), 0, st, bv, src);
  return hipGetLastError();
}

void blk_free(BlkView* bv) {
  if (bv->t_owned && bv->T) (void)hipFree(bv->T);
  for (void* p : {(void*)bv->R, (void*)bv->tstar, (void*)bv->ipos, (void*)bv->pad, (void*)bv->wg_block, (void*)bv->wave_tile,
                  (void*)bv->seg_base, (void*)bv->bsub, (void*)bv->grp_base, (void*)bv->grp_cnt,
                  (void*)bv->grp_list, (void*)bv->P, (void*)bv->Q, (void*)bv->ub, (void*)bv->dummy})
    if (p) (void)hipFree(p);
  *bv = BlkView{};
}

// ------------------------------------------------------------------ build
// The regrouping (positions, workgroup and wave ranges, segments) is laid out
// on the host from att_start and star_row_ptr; the records are made on the
// device.  The coefficients are placed separately: blk_copy_values from the
// caller's rows in star order, or launch_blk_pack chunk by chunk into a
// buffer the caller owns.
int blk_plan(const SysView& s, BlkView* bv, int cus, int max_window, int lds_max, char* err, size_t errlen,
             hipStream_t st) {
  *bv = BlkView{};
  auto failed = [&](int code, const char* what) {
    snprintf(err, errlen, "%s", what);
    blk_free(bv);
    return code;
  };
  const int64_t m = s.m, S = s.n_stars;
  if (m <= 0 || s.n_att < 8 || s.n_instr > 2047 || S >= ((int64_t)1 << 31) || m >= ((int64_t)1 << 31))
    return failed(GSR_EINVAL, "system outside the regrouped pass's limits");
  // window width: the largest that fits the LDS budget (at most 8192 starts: 13-bit offsets)
  const int64_t budget = (int64_t)lds_max - (int64_t)kBlkStaticLds - 8 * (2 * s.n_instr + s.n_glob);
  int64_t wmax = std::min<int64_t>(budget / 24 - 3, 8192);
  if (max_window > 0) wmax = std::min<int64_t>(wmax, max_window);
  if (wmax < 4) return failed(GSR_EINVAL, "not enough LDS for an attitude window");
  const int64_t nstarts = s.n_att - 3;
  const int64_t nb = (nstarts + wmax - 1) / wmax;
  const int64_t Wb = (nstarts + nb - 1) / nb;
  bv->Wb = Wb;
  bv->nb = nb;
  bv->lds = sizeof(double) * (size_t)(3 * (Wb + 3) + 2 * s.n_instr + s.n_glob);
  bv->value_type = s.value_type;

  std::vector<int32_t> att((size_t)m);
  std::vector<int64_t> rp((size_t)S + 1);
  if (hipMemcpy(att.data(), s.att_start, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(rp.data(), s.row_ptr, sizeof(int64_t) * (size_t)(S + 1), hipMemcpyDeviceToHost) != hipSuccess)
    return failed(GSR_EHIP, "reading the row indices failed");
  // Positions per block, star order inside a block.  A row record holds its star
  // as an offset below kStarSpan from the star of its tile's first row, so a row
  // whose star lies that far past it starts a new tile: the rest of the current
  // tile is padding.  The walk below is repeated to place the rows.
  auto walk = [&](auto&& place, auto&& pad) {
    std::vector<int64_t> k((size_t)nb, 0), first((size_t)nb, 0);
    for (int64_t st_ = 0; st_ < S; ++st_)
      for (int64_t r = rp[(size_t)st_]; r < rp[(size_t)st_ + 1]; ++r) {
        const int64_t g = att[(size_t)r] / Wb;
        int64_t& kg = k[(size_t)g];
        if (kg % kWave != 0 && st_ - first[(size_t)g] >= kStarSpan)
          for (; kg % kWave != 0; ++kg) pad(g, kg);
        if (kg % kWave == 0) first[(size_t)g] = st_;
        place(g, kg++, r, st_);
      }
    return k;
  };
  std::vector<int64_t> tb((size_t)nb + 1, 0);
  {
    const std::vector<int64_t> cnt = walk([](int64_t, int64_t, int64_t, int64_t) {}, [](int64_t, int64_t) {});
    for (int64_t g = 0; g < nb; ++g) tb[(size_t)g + 1] = tb[(size_t)g] + (cnt[(size_t)g] + kWave - 1) / kWave;
  }
  const int64_t ntiles = tb[(size_t)nb], mp = ntiles * kWave;
  if (mp >= ((int64_t)1 << 31)) return failed(GSR_EINVAL, "too many rows for the regrouped pass");
  bv->ntiles = ntiles;
  bv->mp = mp;
  bv->m = m;

  // positions: block-major, star order inside a block; a padding position repeats
  // the star of the position before it
  std::vector<int32_t> ipos((size_t)m);
  std::vector<int32_t> pads;
  std::vector<uint32_t> se((size_t)mp, 0);
  {
    const std::vector<int64_t> used = walk(
        [&](int64_t g, int64_t kg, int64_t r, int64_t st_) {
          const int64_t pos = tb[(size_t)g] * kWave + kg;
          ipos[(size_t)r] = (int32_t)pos;
          se[(size_t)pos] = (uint32_t)st_;
        },
        [&](int64_t g, int64_t kg) {
          const int64_t pos = tb[(size_t)g] * kWave + kg;
          se[(size_t)pos] = se[(size_t)pos - 1];
          pads.push_back((int32_t)pos);
        });
    for (int64_t g = 0; g < nb; ++g)
      for (int64_t pos = tb[(size_t)g] * kWave + used[(size_t)g]; pos < tb[(size_t)g + 1] * kWave; ++pos) {
        se[(size_t)pos] = se[(size_t)pos - 1];
        pads.push_back((int32_t)pos);
      }
  }
  bv->npad = (int64_t)pads.size();

  // workgroups per block in proportion to its tiles (at least one per non-empty block)
  const int64_t gt = std::max<int64_t>(1, 2 * (int64_t)cus);
  std::vector<int32_t> wg_block, bsub((size_t)nb + 1, 0), wave_tile;
  for (int64_t g = 0; g < nb; ++g) {
    const int64_t Tg = tb[(size_t)g + 1] - tb[(size_t)g];
    int64_t Gg = Tg > 0 ? std::max<int64_t>(1, (gt * Tg + ntiles / 2) / ntiles) : 0;
    Gg = std::min(Gg, Tg);
    bsub[(size_t)g] = (int32_t)wg_block.size();
    for (int64_t k = 0; k < Gg; ++k) {
      const int64_t a = tb[(size_t)g] + Tg * k / Gg, b = tb[(size_t)g] + Tg * (k + 1) / Gg;
      wg_block.push_back((int32_t)g);
      for (int i = 0; i < kBlkWaves; ++i) wave_tile.push_back((int32_t)(a + (b - a) * i / kBlkWaves));
    }
  }
  bsub[(size_t)nb] = (int32_t)wg_block.size();
  wave_tile.push_back((int32_t)ntiles);
  const int64_t G = (int64_t)wg_block.size();
  if (G < 1 || G > kMaxPartials) return failed(GSR_EINVAL, "workgroup count outside the partial slots");
  bv->G = (int32_t)G;

  // segments: maximal runs of one star inside a wave's range
  const int64_t W = G * kBlkWaves;
  std::vector<int32_t> seg_base((size_t)W);
  std::vector<int32_t> seg_star;
  for (int64_t w = 0; w < W; ++w) {
    seg_base[(size_t)w] = (int32_t)seg_star.size();
    const int64_t p0 = (int64_t)wave_tile[(size_t)w] * kWave, p1 = (int64_t)wave_tile[(size_t)w + 1] * kWave;
    for (int64_t pos = p0; pos < p1; ++pos) {
      const uint32_t sp = se[(size_t)pos];
      if (pos == p0 || sp != (se[(size_t)pos - 1] & 0x7FFFFFFFu)) {
        seg_star.push_back((int32_t)sp);
        if (seg_star.size() >= ((size_t)1 << 31) / 5) return failed(GSR_EINVAL, "too many star segments");
      }
      const bool end = pos == p1 - 1 || se[(size_t)pos + 1] != sp;
      if (end) se[(size_t)pos] = sp | 0x80000000u;
    }
  }
  const int64_t nseg = (int64_t)seg_star.size();
  bv->nseg = nseg;
  // Per group of 64 stars, the segment ids of its stars as entries [column][lane]
  // (lane l: star 64g+l), aligned by window: one column per window that some star
  // of the group has rows in (in window order), then columns for a star's second
  // and later segments inside one window (a wave boundary inside the star's rows);
  // empty slots hold nseg (the zero entry of P).  Neighbouring stars' segments in
  // one window are consecutive in P, so each column's loads are contiguous.
  std::vector<int32_t> seg_blk((size_t)nseg);
  for (int64_t w = 0; w < W; ++w) {
    const int64_t q1 = w + 1 < W ? seg_base[(size_t)w + 1] : nseg;
    for (int64_t q = seg_base[(size_t)w]; q < q1; ++q) seg_blk[(size_t)q] = wg_block[(size_t)(w / kBlkWaves)];
  }
  // each star's segments in id order (window order: ids are numbered block-major)
  std::vector<int64_t> sptr((size_t)S + 1, 0);
  for (int64_t q = 0; q < nseg; ++q) ++sptr[(size_t)seg_star[(size_t)q] + 1];
  for (int64_t st_ = 0; st_ < S; ++st_) sptr[(size_t)st_ + 1] += sptr[(size_t)st_];
  std::vector<int32_t> ssegs((size_t)std::max<int64_t>(nseg, 1));
  {
    std::vector<int64_t> fill(sptr.begin(), sptr.end() - 1);
    for (int64_t q = 0; q < nseg; ++q) ssegs[(size_t)fill[(size_t)seg_star[(size_t)q]]++] = (int32_t)q;
  }
  const int64_t ngroups = (S + kWave - 1) / kWave;
  bv->ngroups = ngroups;
  std::vector<int64_t> grp_base((size_t)ngroups + 1, 0);
  std::vector<int32_t> grp_cnt((size_t)ngroups, 0);
  std::vector<int32_t> col_of((size_t)nb, -1);
  std::vector<int32_t> ncols_prim((size_t)ngroups, 0);
  for (int64_t g = 0; g < ngroups; ++g) {
    const int64_t s0 = g * kWave, s1 = std::min<int64_t>(S, (g + 1) * kWave);
    std::vector<char> touched((size_t)nb, 0);
    int32_t extra = 0;
    for (int64_t st_ = s0; st_ < s1; ++st_) {
      int32_t e = 0;
      for (int64_t i = sptr[(size_t)st_]; i < sptr[(size_t)st_ + 1]; ++i) {
        const int32_t b = seg_blk[(size_t)ssegs[(size_t)i]];
        if (i > sptr[(size_t)st_] && b == seg_blk[(size_t)ssegs[(size_t)i - 1]])
          ++e;
        else
          touched[(size_t)b] = 1;
      }
      extra = std::max(extra, e);
    }
    int32_t t = 0;
    for (int64_t b = 0; b < nb; ++b) t += touched[(size_t)b];
    ncols_prim[(size_t)g] = t;
    grp_cnt[(size_t)g] = t + extra;
    grp_base[(size_t)g + 1] = grp_base[(size_t)g] + (int64_t)(t + extra) * kWave;
  }
  bv->nlist = grp_base[(size_t)ngroups];
  std::vector<int32_t> grp_list((size_t)std::max<int64_t>(bv->nlist, 1), (int32_t)nseg);
  for (int64_t g = 0; g < ngroups; ++g) {
    const int64_t s0 = g * kWave, s1 = std::min<int64_t>(S, (g + 1) * kWave);
    std::fill(col_of.begin(), col_of.end(), -1);
    for (int64_t st_ = s0; st_ < s1; ++st_)
      for (int64_t i = sptr[(size_t)st_]; i < sptr[(size_t)st_ + 1]; ++i) col_of[(size_t)seg_blk[(size_t)ssegs[(size_t)i]]] = 0;
    int32_t c = 0;
    for (int64_t b = 0; b < nb; ++b)
      if (col_of[(size_t)b] == 0) col_of[(size_t)b] = c++;
    for (int64_t st_ = s0; st_ < s1; ++st_) {
      int32_t e = 0;
      for (int64_t i = sptr[(size_t)st_]; i < sptr[(size_t)st_ + 1]; ++i) {
        const int32_t q = ssegs[(size_t)i], b = seg_blk[(size_t)q];
        const bool again = i > sptr[(size_t)st_] && b == seg_blk[(size_t)ssegs[(size_t)i - 1]];
        const int64_t col = again ? ncols_prim[(size_t)g] + e++ : col_of[(size_t)b];
        grp_list[(size_t)(grp_base[(size_t)g] + col * kWave + (st_ - s0))] = q;
      }
    }
  }

  uint32_t* se_d = nullptr;
  auto dalloc_ = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 16)) == hipSuccess; };
  if (!dalloc_((void**)&bv->R, (size_t)mp * 12) || !dalloc_((void**)&bv->tstar, (size_t)ntiles * 4) || !dalloc_((void**)&bv->ipos, (size_t)m * 4) ||
      !dalloc_((void**)&bv->pad, pads.size() * 4) || !dalloc_((void**)&bv->wg_block, (size_t)G * 4) ||
      !dalloc_((void**)&bv->wave_tile, (size_t)(W + 1) * 4) || !dalloc_((void**)&bv->seg_base, (size_t)W * 4) ||
      !dalloc_((void**)&bv->bsub, (size_t)(nb + 1) * 4) ||
      !dalloc_((void**)&bv->grp_base, (size_t)(ngroups + 1) * 8) ||
      !dalloc_((void**)&bv->grp_cnt, (size_t)ngroups * 4) || !dalloc_((void**)&bv->grp_list, grp_list.size() * 4) ||
      !dalloc_((void**)&bv->P, (size_t)(nseg + 1) * 40) ||
      !dalloc_((void**)&bv->Q, (size_t)G * 3 * (Wb + 3) * 8) || !dalloc_((void**)&bv->ub, (size_t)mp * 8) ||
      !dalloc_((void**)&bv->dummy, (size_t)W * kBlkDummy * 8) ||
      !dalloc_((void**)&se_d, (size_t)mp * 4)) {
    (void)hipGetLastError();
    if (se_d) (void)hipFree(se_d);
    return failed(GSR_ENOMEM, "device memory for the regrouped layout");
  }
  bool ok = hipMemcpyAsync(bv->ipos, ipos.data(), (size_t)m * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            (pads.empty() ||
             hipMemcpyAsync(bv->pad, pads.data(), pads.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess) &&
            hipMemcpyAsync(se_d, se.data(), (size_t)mp * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(bv->wg_block, wg_block.data(), (size_t)G * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(bv->wave_tile, wave_tile.data(), (size_t)(W + 1) * 4, hipMemcpyHostToDevice, st) ==
                hipSuccess &&
            hipMemcpyAsync(bv->seg_base, seg_base.data(), (size_t)W * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(bv->bsub, bsub.data(), (size_t)(nb + 1) * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(bv->grp_base, grp_base.data(), (size_t)(ngroups + 1) * 8, hipMemcpyHostToDevice, st) ==
                hipSuccess &&
            hipMemcpyAsync(bv->grp_cnt, grp_cnt.data(), (size_t)ngroups * 4, hipMemcpyHostToDevice, st) ==
                hipSuccess &&
            hipMemcpyAsync(bv->grp_list, grp_list.data(), grp_list.size() * 4, hipMemcpyHostToDevice, st) ==
                hipSuccess &&
            hipMemsetAsync(bv->P + 5 * nseg, 0, 40, st) == hipSuccess &&
            hipMemsetAsync(bv->ub, 0, (size_t)mp * 8, st) == hipSuccess;
  if (ok) {
    const int blocks = (int)std::min<int64_t>(8192, (m + bv->npad + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_blk_records, dim3(blocks), dim3(kBlock), 0, st, s, *bv, se_d);
    ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
  }
  (void)hipFree(se_d);
  if (!ok) return failed(GSR_EHIP, "building the regrouped layout failed");
  // allow the dynamic LDS size beyond 64 KB (where the runtime asks for it)
  (void)hipFuncSetAttribute((const void*)k_fblk<double, 0, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bv->lds);
  (void)hipFuncSetAttribute((const void*)k_fblk<double, 0, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bv->lds);
  (void)hipFuncSetAttribute((const void*)k_fblk<float, 0, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bv->lds);
  (void)hipFuncSetAttribute((const void*)k_fblk<float, 0, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bv->lds);
  (void)hipFuncSetAttribute((const void*)k_fblk<float, 1, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bv->lds);
  (void)hipGetLastError();
  return GSR_OK;
}

size_t blk_value_bytes(const BlkView& bv) {
  return (size_t)bv.mp * (bv.value_type == GSR_F32 ? Geo<float>::CPR : Geo<double>::CPR) * 16;
}

size_t blk_index_bytes(const BlkView& bv) {
  const int64_t W = (int64_t)bv.G * kBlkWaves;
  return (size_t)bv.mp * 12 + (size_t)bv.ntiles * 4 + (size_t)bv.m * 4 + (size_t)bv.npad * 4 + (size_t)bv.G * 4 + (size_t)(W + 1) * 4 +
         (size_t)W * 4 + (size_t)(bv.nb + 1) * 4 + (size_t)(bv.ngroups + 1) * 8 + (size_t)bv.ngroups * 4 +
         (size_t)std::max<int64_t>(bv.nlist, 1) * 4 + (size_t)(bv.nseg + 1) * 40 +
         (size_t)bv.G * 3 * (bv.Wb + 3) * 8 + (size_t)bv.mp * 8 + (size_t)W * kBlkDummy * 8;
}

hipError_t launch_blk_pack(const BlkView& bv, const void* rows, int64_t row0, int64_t count, void* T,
                           hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (row0 < 0 || row0 + count > bv.m || bv.ipos == nullptr) return hipErrorInvalidValue;
  const int blocks = (int)std::min<int64_t>(8192, (count + kBlock - 1) / kBlock);
  if (bv.value_type == GSR_F32)
    hipLaunchKernelGGL(k_blk_pack<float>, dim3(blocks), dim3(kBlock), 0, st, bv, (const u4*)rows, row0, count,
                       (u4*)T);
  else
    hipLaunchKernelGGL(k_blk_pack<double>, dim3(blocks), dim3(kBlock), 0, st, bv, (const u4*)rows, row0, count,
                       (u4*)T);
  return hipGetLastError();
}

hipError_t launch_blk_zero_pad(const BlkView& bv, void* T, hipStream_t st) {
  if (bv.npad == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(8192, (bv.npad + kBlock - 1) / kBlock);
  if (bv.value_type == GSR_F32)
    hipLaunchKernelGGL(k_blk_zero_pad<float>, dim3(blocks), dim3(kBlock), 0, st, bv, (u4*)T);
  else
    hipLaunchKernelGGL(k_blk_zero_pad<double>, dim3(blocks), dim3(kBlock), 0, st, bv, (u4*)T);
  return hipGetLastError();
}

// The library-owned copy for a handle over rows in star order: the layout, then
// every row placed from the caller's array.
int blk_build(const SysView& s, BlkView* bv, int cus, int max_window, int lds_max, char* err, size_t errlen,
              hipStream_t st) {
  int rc = blk_plan(s, bv, cus, max_window, lds_max, err, errlen, st);
  if (rc != GSR_OK) return rc;
  if (hipMalloc(&bv->T, std::max<size_t>(blk_value_bytes(*bv), 16)) != hipSuccess) {
    (void)hipGetLastError();
    bv->T = nullptr;
    snprintf(err, errlen, "device memory for the regrouped copy");
    blk_free(bv);
    return GSR_ENOMEM;
  }
  bv->t_owned = 1;
  if (launch_blk_pack(*bv, s.vals, 0, s.m, bv->T, st) != hipSuccess ||
      launch_blk_zero_pad(*bv, bv->T, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    snprintf(err, errlen, "building the regrouped copy failed");
    blk_free(bv);
    return GSR_EHIP;
  }
  bv->ready = 1;
  return GSR_OK;
}

}  // namespace gsr
