// The two products of every LSQR iteration (Sec. 2, Eq. 2 and Eq. 3) over the
// 24-coefficient row form of the observation matrix, for gfx950.
//
// Both kernels stream the coefficient rows once in row (star) order; a wave
// walks a contiguous range of rows in tiles of 64 (one row per lane).  A
// tile's coefficients (64 x 192 B for FP64) are fetched with contiguous
// 16-byte nontemporal loads (1 KB per wave instruction), staged in LDS with
// one 16-byte pad per row (conflict-free row reads) and read back
// row-per-lane; the next tile's loads are issued as soon as the current one
// sits in LDS.  The star of each row comes from the tile's 64 star
// boundaries, loaded in one coalesced access and searched in LDS.
//
// aprod1: y_r <- scale*y_r + ax * sum_k a_rk x[col(r,k)].  Wave ranges are
//   whole 64-row tiles, so each tile's 512-byte store of y covers whole
//   64-byte sectors (a partly written sector costs the memory a
//   read-modify-write; with unaligned tiles those stores took a quarter of
//   the kernel's time).  x is gathered per tile: the astrometric x of the
//   tile's stars in one contiguous load, spread to the rows by lane shuffles;
//   the attitude windows with 16-byte loads; the instrumental x from LDS.
// aprod2 (this file: astrometric, instrumental, global; and the attitude
//   block when it fits in LDS): work is split by whole stars (wave w owns
//   the stars whose rows start in [w*m/W, (w+1)*m/W)), so every astrometric
//   unknown is produced by exactly one wave.  Astrometric columns by a
//   segmented scan over the star runs of a tile, carried across tiles;
//   instrumental and global columns LDS-private per workgroup, flushed with
//   one atomic per column per workgroup.  Larger attitude blocks are summed
//   by the bucketed pass in attitude.hip; this pass then reads the row-order
//   copy that holds only the other twelve coefficients (half the bytes).
#include <algorithm>

#include "row_tiles.h"

namespace gsr {

// ---------------------------------------------------------------- aprod1
//
// Gathers of x per tile: the astrometric x of the tile's stars with one
// contiguous load and lane shuffles (when the tile spans at most 12 stars),
// the three 4-column attitude windows with two 16-byte loads each, and the
// instrumental x from an LDS copy (a system has at most kLdsTailMax - 1
// instrumental columns).
// Every global load and store of the steady-state loop is unconditional or
// issued before the next tile's prefetch (y of a tile is stored at the start
// of the next one), so the waits before the compute cover only this tile's
// gathers.
template <typename VT, int PM>
__global__ void __launch_bounds__(kBlock) k_aprod1(SysView s, int waves, const double* __restrict__ x,
                                                   const double* __restrict__ x3, double* __restrict__ y,
                                                   double scale, double ax, Scalars* sc, Work wk, int lsqr_stage) {
  constexpr int CPR = Geo<VT>::CPR;
  __shared__ u4 slabs[kWavesPerBlock][kWave * (CPR + 1)];
  __shared__ int64_t bnds[kWavesPerBlock][kWave];
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  extern __shared__ double xil[];  // instrumental x
  if (sc) {
    if (sc->done) return;
    scale = sc->u_scale;
  }
  const int64_t NI = s.n_astro + 3 * s.n_att;
  for (int64_t j = threadIdx.x; j < s.n_instr; j += kBlock) xil[j] = x[NI + j];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  double sumsq = 0.0;
  if (w < waves) {
    // rows [R0, R1): a contiguous range of whole 64-row tiles, so that every
    // tile (and its 512-byte store of y) is aligned
    const int64_t T = (s.m + kWave - 1) / kWave;
    const int64_t R0 = kWave * (T * w / waves), R1 = min(s.m, kWave * (T * (w + 1) / waves));
    const double xg = s.n_glob ? x[NI + s.n_instr] : 0.0;
    // star of row R0: the last star starting at or before it
    int64_t scur = R0 < R1 ? star_lower_bound(s.row_ptr, s.n_stars, R0 + 1) - 1 : 0;
    const int64_t xa_last = 5 * s.n_stars - 1;
    const u4* vbase = reinterpret_cast<const u4*>(s.vals);
    // registers of the prefetched tile
    u4 tmp[CPR];
    int32_t at;
    i2 i01, i23, i45;
    double yo;
    int64_t bv;
    auto fetch = [&](int64_t tt) {
      // past the end of the range: re-read its last row (the registers are not used)
      const int64_t te = min(tt, R1 - 1);
      const int nr = (int)min((int64_t)kWave, R1 - te);
      const int64_t rr = (lane < nr) ? te + lane : R1 - 1;
      issue_chunks<CPR>(vbase + te * CPR, nr, lane, tmp);
      at = __builtin_nontemporal_load(s.att_start + rr);
      const i2* icp = reinterpret_cast<const i2*>(s.instr_col + 6 * rr);
      i01 = __builtin_nontemporal_load(icp);
      i23 = __builtin_nontemporal_load(icp + 1);
      i45 = __builtin_nontemporal_load(icp + 2);
      yo = y[rr];
      bv = bnd_load(s, scur, lane);
    };
    // y of the previous tile, stored at the start of the next one
    double y_out = 0.0;
    int64_t r_out = -1;
    if (R0 < R1) fetch(R0);
#pragma unroll 1
    for (int64_t t0 = R0; t0 < R1; t0 += kWave) {
      const int nrow = (int)min((int64_t)kWave, R1 - t0);
      const bool valid = lane < nrow;
      const int32_t at_c = at;
      const int ic[6] = {i01.x, i01.y, i23.x, i23.y, i45.x, i45.y};
      const double yo_c = (scale == 0.0) ? 0.0 : scale * yo;
      const int64_t bv_c = bv;
      const int64_t sf = scur;  // star of row t0
      // stars of the tile (valid when the last row's star is among the 64 boundaries)
      const int64_t span = __popcll(__ballot(bv_c <= t0 + nrow - 1)) + 1;
      scur = tile_next(s, bv_c, t0, sf);
      // gathers of x for this tile, issued before the next tile's loads: the
      // astrometric x of the tile's first stars, and the tile's 64 attitude
      // windows (96 bytes each, one 128-byte record line) of x3, loaded
      // cooperatively (piece j*64 + lane in cw[j]; consecutive lanes take
      // consecutive 16-byte pieces of one window)
      const double xs = x[min(5 * sf + lane, xa_last)];
      dd2u cw[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const int c = j * kWave + lane, i = c / 6, q = c - 6 * i;
        const int at_i = __shfl(at_c, i, kWave);
        cw[j] = *reinterpret_cast<const dd2u*>(x3 + kAttRec * (int64_t)at_i + 2 * q);
      }
      bnds[wid][lane] = bv_c;
      lds_put<CPR>(tmp, nrow, slabs[wid], lane);
      order_point();
      fetch(t0 + kWave);
      order_point();
      // the previous tile's store, after the next tile's loads: loads and stores
      // share one in-order counter and this store is conditional, so the next wait
      // on loads also waits for it; here the tile's arithmetic covers its latency
      if (r_out >= 0) y[r_out] = y_out;
      u4 mine[CPR];
      lds_get<CPR>(nrow, slabs[wid], lane, mine);
      // the windows regrouped per row through the (now free) slab; window
      // element e = 3j + axis is column at+j of that axis (slot 5 + 4 axis + j)
      double gx[kSlots];
      {
        dd2u* wl = reinterpret_cast<dd2u*>(slabs[wid]);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          const int c = j * kWave + lane, i = c / 6, q = c - 6 * i;
          wl[i * 7 + q] = cw[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const dd2u pq = wl[lane * 7 + q];
          const int e0 = 2 * q, e1 = 2 * q + 1;
          gx[5 + 4 * (e0 % 3) + e0 / 3] = pq.x;
          gx[5 + 4 * (e1 % 3) + e1 / 3] = pq.y;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      const int64_t st = tile_star(s, t0, lane, bnds[wid], sf);
      VT a[kSlots];
      __builtin_memcpy(a, mine, sizeof(a));
#pragma unroll
      for (int q = 0; q < 6; ++q) gx[17 + q] = xil[ic[q]];
      double acc = 0.0;
      {
        // every lane takes its star's x from the shuffle window (used on every
        // path, so the load stays where it was issued); with many short stars in
        // the tile, lanes past the window gather per lane, consumed inside the
        // branch (a load still pending where the paths join would make the
        // compiler wait for the next tile's loads too)
        const int64_t dst = valid ? st - sf : 0;
        const int base = 5 * (int)min<int64_t>(dst, 11);
#pragma unroll
        for (int k = 0; k < 5; ++k) acc += prod<PM>(a[k], __shfl(xs, base + k, kWave));
        if (span > 12 && dst >= 12) {
          double xa5[5];
#pragma unroll
          for (int k = 0; k < 5; ++k) xa5[k] = x[5 * st + k];
          acc = 0.0;
#pragma unroll
          for (int k = 0; k < 5; ++k) acc += prod<PM>(a[k], xa5[k]);
        }
      }
#pragma unroll
      for (int k = 5; k < 23; ++k) acc += prod<PM>(a[k], gx[k]);
      if (s.n_glob) acc += prod<PM>(a[23], xg);
      const double yn = yo_c + ax * acc;
      r_out = valid ? t0 + lane : -1;
      y_out = yn;
      if (valid) sumsq += yn * yn;
    }
    if (r_out >= 0) y[r_out] = y_out;
  }
  if (!sc) return;
  const double bs = block_sum(sumsq, red);
  if (threadIdx.x == 0) publish(wk.part_a + blockIdx.x, bs);
  if (last_block(wk.tickets + T_APROD1, &flag)) {
    const double tot = sum_partials(wk.part_a, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_beta(sc, tot, lsqr_stage == 0);
      ticket_reset(wk.tickets + T_APROD1);
    }
  }
}

// ---------------------------------------------------------------- aprod2
// ATT_MODE 0: the whole tail (attitude, instrumental, global) in LDS.
// ATT_MODE 1: attitude by device-scope FP64 atomics (fallback), instr + global in LDS.
// ATT_MODE 3: attitude summed by the bucketed pass; its sectors are not read here.
// In mode 3 the rows are read from the star-pass copy sv (astrometric,
// instrumental and global coefficients only, half the row).
template <typename VT, int PM, int SQUARE, int ATT_MODE>
__global__ void __launch_bounds__(kBlock) k_aprod2(SysView s, int waves, const void* __restrict__ sv,
                                                   const double* __restrict__ y, double* __restrict__ x,
                                                   double* __restrict__ acc, const double* __restrict__ S,
                                                   double scale, double inv_beta, Scalars* sc, Work wk) {
  constexpr int CPR = (ATT_MODE == 3) ? Geo<VT>::CPR / 2 : Geo<VT>::CPR;
  constexpr int NS = (ATT_MODE == 3) ? 12 : kSlots;  // coefficients per row read here
  constexpr int IN0 = (ATT_MODE == 3) ? 5 : 17;      // first instrumental coefficient
  constexpr int GL = NS - 1;                         // global coefficient
  __shared__ u4 slabs[kWavesPerBlock][kWave * (CPR + 1)];
  __shared__ int64_t bnds[kWavesPerBlock][kWave];
  __shared__ double red[kWavesPerBlock];
  extern __shared__ double hist[];
  if (sc) {
    if (sc->done || !sc->do_v) return;
    scale = sc->v_scale;
    inv_beta = sc->inv_beta;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  // LDS-private tail: [0, 3*n_att) attitude (mode 0 only), then instr, then global
  const int64_t hoff = (ATT_MODE == 0) ? 0 : 3 * s.n_att;  // tail index of hist[0]
  const int64_t hlen = s.tail_len - hoff;
  for (int64_t j = threadIdx.x; j < hlen; j += kBlock) hist[j] = 0.0;
  __syncthreads();

  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  double sumsq = 0.0, gsum = 0.0;
  if (w < waves) {
    int64_t s0, s1;
    wave_stars(s, w, waves, &s0, &s1);
    const int64_t R0 = s.row_ptr[s0], R1 = s.row_ptr[s1];
    int64_t scur = s0;
    while (scur < s1 && s.row_ptr[scur + 1] <= R0) ++scur;
    double carry[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int carry_valid = 0;
    const u4* vbase = reinterpret_cast<const u4*>(ATT_MODE == 3 ? sv : s.vals);
    const int64_t xa_last = 5 * s.n_stars - 1;
    const double* Sx = S ? S : x;  // read unconditionally, ignored when S is null
    u4 tmp[CPR];
    double tv;
    int32_t at;
    i2 i01, i23, i45;
    int64_t bv;
    auto fetch = [&](int64_t tt) {
      // past the end of the range: re-read its last row (the registers are not used)
      const int64_t te = min(tt, R1 - 1);
      const int nr = (int)min((int64_t)kWave, R1 - te);
      const int64_t rr = (lane < nr) ? te + lane : R1 - 1;
      issue_chunks<CPR>(vbase + te * CPR, nr, lane, tmp);
      tv = SQUARE ? 0.0 : __builtin_nontemporal_load(y + rr);
      at = (ATT_MODE == 3) ? 0 : __builtin_nontemporal_load(s.att_start + rr);
      const i2* icp = reinterpret_cast<const i2*>(s.instr_col + 6 * rr);
      i01 = __builtin_nontemporal_load(icp);
      i23 = __builtin_nontemporal_load(icp + 1);
      i45 = __builtin_nontemporal_load(icp + 2);
      bv = bnd_load(s, scur, lane);
    };
    // stars finished in the previous tile, stored at the start of the next one
    int64_t c_out = -1;
    double x_out[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (R0 < R1) fetch(R0);
#pragma unroll 1
    for (int64_t t0 = R0; t0 < R1; t0 += kWave) {
      const int nrow = (int)min((int64_t)kWave, R1 - t0);
      const bool valid = lane < nrow;
      const int64_t r = t0 + (valid ? lane : 0);
      const double t = tv * inv_beta;
      const int32_t at_c = at;
      const int ic[6] = {i01.x, i01.y, i23.x, i23.y, i45.x, i45.y};
      const int64_t bv_c = bv;
      const int64_t sf = scur;  // star of row t0
      // stars of the tile (valid when the last row's star is among the 64 boundaries)
      const int64_t span = __popcll(__ballot(bv_c <= t0 + nrow - 1)) + 1;
      scur = tile_next(s, bv_c, t0, sf);
      // old x and column scales of the tile's stars, one contiguous load each
      const int64_t ia = min(5 * sf + lane, xa_last);
      const double xo_l = x[ia];
      const double so_l = Sx[ia];
      bnds[wid][lane] = bv_c;
      lds_put<CPR>(tmp, nrow, slabs[wid], lane);
      order_point();
      fetch(t0 + kWave);
      order_point();
      // the previous tile's finished star, stored after the next tile's loads (see
      // k_aprod1; it is a star before this tile's, so no load of this tile reads it)
      if (c_out >= 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) x[c_out + k] = x_out[k];
      }
      u4 mine[CPR];
      lds_get<CPR>(nrow, slabs[wid], lane, mine);
      int64_t rbeg, rend;
      const int64_t st = tile_star(s, t0, lane, bnds[wid], sf, &rbeg, &rend);
      VT a[NS];
      __builtin_memcpy(a, mine, sizeof(a));
      const int seg0 = valid ? (int)(max(rbeg, t0) - t0) : lane;
      double p[5];
      if (valid) {
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] = SQUARE ? (double)a[k] * (double)a[k] : prod<PM>(a[k], t);
        if (ATT_MODE != 3) {
#pragma unroll
          for (int axs = 0; axs < 3; ++axs) {
            const int64_t col = axs * s.n_att + at_c;  // tail index
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const VT av = a[5 + 4 * axs + j];
              const double c = SQUARE ? (double)av * (double)av : prod<PM>(av, t);
              if (ATT_MODE == 0)
                atomicAdd(hist + col + j, c);
              else
                atomicAdd(acc + col + j, c);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const VT av = a[IN0 + q];
          const double c = SQUARE ? (double)av * (double)av : prod<PM>(av, t);
          atomicAdd(hist + (3 * s.n_att - hoff) + ic[q], c);
        }
        if (s.n_glob) gsum += SQUARE ? (double)a[GL] * (double)a[GL] : prod<PM>(a[GL], t);
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] = 0.0;
      }
      // partial sums carried from the star that began in an earlier tile
      if (carry_valid && lane == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] += carry[k];
      }
      // inclusive segmented scan over the star runs of this tile
      seg_scan(p, lane, seg0);
      const bool ends_here = valid && (r == rend - 1);
      // new x of the lane's star from its old x and scale: from the shuffle window
      // (used on every path), or, with many short stars in the tile, from per-lane
      // loads consumed inside the branch (see k_aprod1)
      double xn[5];
      {
        const int64_t dst = valid ? st - sf : 0;
        const int base = 5 * (int)min<int64_t>(dst, 11);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const double xo = __shfl(xo_l, base + k, kWave), so = __shfl(so_l, base + k, kWave);
          xn[k] = ((scale == 0.0) ? 0.0 : scale * xo) + (S ? so : 1.0) * p[k];
        }
        if (span > 12 && dst >= 12) {
          double xo[5], so[5];
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            xo[k] = x[5 * st + k];
            so[k] = Sx[5 * st + k];
          }
#pragma unroll
          for (int k = 0; k < 5; ++k) xn[k] = ((scale == 0.0) ? 0.0 : scale * xo[k]) + (S ? so[k] : 1.0) * p[k];
        }
      }
      c_out = ends_here ? 5 * st : -1;
      if (ends_here) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          x_out[k] = xn[k];
          sumsq += xn[k] * xn[k];
        }
      }
      // carry the last run of the tile if its star continues
      const int last = nrow - 1;
      const int lend = (int)((__ballot(ends_here) >> last) & 1ull);
#pragma unroll
      for (int k = 0; k < 5; ++k) carry[k] = lane_read(p[k], last);
      carry_valid = !lend;
    }
    if (c_out >= 0) {
#pragma unroll
      for (int k = 0; k < 5; ++k) x[c_out + k] = x_out[k];
    }
    // stars without rows: x <- scale*x
    if (s.has_empty_stars) {
      for (int64_t e = s0 + lane; e < s1; e += kWave) {
        if (s.row_ptr[e] == s.row_ptr[e + 1]) {
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            const int64_t c = 5 * e + k;
            const double xn = (scale == 0.0) ? 0.0 : scale * x[c];
            x[c] = xn;
            sumsq += xn * xn;
          }
        }
      }
    }
  }
  // global column: one LDS atomic per wave
  if (s.n_glob) {
    const double g = wave_sum(gsum);
    if (lane == 0) atomicAdd(hist + (hlen - 1), g);
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < hlen; j += kBlock) {
    const double v = hist[j];
    if (v != 0.0) atomicAdd(acc + hoff + j, v);
  }
  if (sc) {
    const double bs = block_sum(sumsq, red);
    if (threadIdx.x == 0) publish(wk.part_b + blockIdx.x, bs);
  }
}

// ------------------------------------------------------------------ tail
// x_t <- scale*x_t + S_t * (sum of the tail contributions) for the attitude,
// instrumental and global unknowns; acc is cleared for the next product.  With
// the bucketed attitude pass, attitude column c of axis a adds the window
// partials Q[sub][a][c - b*Wb] of the (at most two) buckets b whose window
// [b*Wb, b*Wb + Wb + 3) covers c.  In an LSQR solve the last workgroup forms
// alpha_{i+1}, applies the plane rotations of the iteration and buffers
// d_i[sel] = w_i[sel] / rho_i as one covariance column.
__global__ void __launch_bounds__(kBlock) k_tail(SysView s, AttView av, int att_mode, double* __restrict__ x,
                                                 double* __restrict__ acc, const double* __restrict__ S, double scale,
                                                 Scalars* sc, Work wk, TailLsqr L) {
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  int work = 1;
  if (sc) {
    if (sc->done) return;
    work = sc->do_v;
    scale = sc->v_scale;
  }
  double sumsq = 0.0;
  if (work) {
    const int64_t natt = 3 * s.n_att;
    const int64_t win = av.Wb + 3;
    // fused iteration: the astrometric columns too, and every raw sum times 1/beta
    const int64_t j0 = L.gA ? -s.n_astro : 0;
    const double f = L.gA ? sc->inv_beta : 1.0;
    for (int64_t j = j0 + (int64_t)blockIdx.x * kBlock + threadIdx.x; j < s.tail_len;
         j += (int64_t)gridDim.x * kBlock) {
      double a;
      if (j < 0) {
        a = L.gA[s.n_astro + j];
      } else if (att_mode == 3 && j < natt) {
        const int64_t axs = j / s.n_att, c = j - axs * s.n_att;
        a = 0.0;
        const int64_t bhi = min(c / av.Wb, av.nb - 1);
        for (int64_t b = max<int64_t>(bhi - 1, 0); b <= bhi; ++b) {
          const int64_t off = c - b * av.Wb;
          if (off < 0 || off >= win) continue;
          // sixteen windows at a time (independent loads in flight together: a
          // block has tens of workgroups), added in workgroup order
          const double* qp = av.Q + axs * win + off;
          const int64_t qs = 3 * win;
          int32_t q = av.bsub[b];
          for (; q + 16 <= av.bsub[b + 1]; q += 16) {
            double v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = qp[(q + i) * qs];
#pragma unroll
            for (int i = 0; i < 16; ++i) a += v[i];
          }
          for (; q + 4 <= av.bsub[b + 1]; q += 4) {
            const double q0 = qp[q * qs], q1 = qp[(q + 1) * qs], q2 = qp[(q + 2) * qs], q3 = qp[(q + 3) * qs];
            a += q0;
            a += q1;
            a += q2;
            a += q3;
          }
          for (; q < av.bsub[b + 1]; ++q) a += qp[q * qs];
        }
        a += acc[j];  // constraint rows, if any
        acc[j] = 0.0;
      } else {
        a = acc[j];
        acc[j] = 0.0;
      }
      const int64_t c = s.n_astro + j;
      const double xo = (scale == 0.0) ? 0.0 : scale * x[c];
      const double xn = xo + (S ? S[c] : 1.0) * (f * a);
      x[c] = xn;
      sumsq += xn * xn;
    }
  }
  if (!sc) return;
  const double bs = block_sum(sumsq, red);
  if (threadIdx.x == 0) publish(wk.part_a + blockIdx.x, bs);
  if (last_block(wk.tickets + T_TAIL, &flag)) {
    double tot = sum_partials(wk.part_b, L.astro_parts, red);
    tot += sum_partials(wk.part_a, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_alpha(sc, tot, L.lsqr_stage == 0);
      ticket_reset(wk.tickets + T_TAIL);
    }
  }
}

// --------------------------------------------------------------- checks
__global__ void k_validate(SysView s, unsigned long long* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < s.m; r += stride) {
    const int32_t at = s.att_start[r];
    bool ok = at >= 0 && (int64_t)at <= s.n_att - 4;
    for (int q = 0; q < 6; ++q) {
      const int32_t c = s.instr_col[6 * r + q];
      ok = ok && c >= 0 && (int64_t)c < s.n_instr;
    }
    if (!ok) atomicMin(bad, (unsigned long long)r);
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n_stars; i += stride) {
    const int64_t a = s.row_ptr[i], b = s.row_ptr[i + 1];
    if (b < a || (i == 0 && a != 0) || (i == s.n_stars - 1 && b != s.m)) atomicMin(bad + 1, (unsigned long long)i);
    if (a == b) atomicMax(bad + 2, 1ull);
  }
}

__global__ void k_scale_from_sq(int64_t n, double* S) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const double q = S[j];
    S[j] = q > 0.0 ? 1.0 / sqrt(q) : 1.0;
  }
}

// ------------------------------------------------------------ launchers
StreamShape stream_shape(const SysView& s, int cus, int waves_per_cu) {
  // never more waves than stars or row tiles, never more blocks than partial slots
  int64_t waves = (int64_t)cus * waves_per_cu;
  waves = std::min(waves, (int64_t)kMaxPartials * kWavesPerBlock);
  waves = std::min(waves, std::max<int64_t>(1, s.n_stars));
  waves = std::min(waves, std::max<int64_t>(1, (s.m + kWave - 1) / kWave));
  waves = std::max<int64_t>(waves, 1);
  StreamShape sh;
  sh.waves = (int)waves;
  sh.blocks = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  return sh;
}

hipError_t launch_aprod1(const SysView& s, StreamShape sh, const double* x, double* x3w, double* y, double scale,
                         double ax, int pmode, Scalars* sc, Work w, int lsqr_stage, hipStream_t st) {
  if (x3w == nullptr) return hipErrorInvalidValue;
  const hipError_t e = launch_att_records(s, x, x3w, st);
  if (e != hipSuccess) return e;
  const dim3 g(sh.blocks), b(kBlock);
  const size_t lb = sizeof(double) * (size_t)std::max<int64_t>(s.n_instr, 1);
  if (s.value_type == GSR_F32 && pmode == 1)
    hipLaunchKernelGGL((k_aprod1<float, 1>), g, b, lb, st, s, sh.waves, x, x3w, y, scale, ax, sc, w, lsqr_stage);
  else if (s.value_type == GSR_F32)
    hipLaunchKernelGGL((k_aprod1<float, 0>), g, b, lb, st, s, sh.waves, x, x3w, y, scale, ax, sc, w, lsqr_stage);
  else
    hipLaunchKernelGGL((k_aprod1<double, 0>), g, b, lb, st, s, sh.waves, x, x3w, y, scale, ax, sc, w, lsqr_stage);
  return hipGetLastError();
}

int att_mode_of(const SysView& s, const AttView& av, int force_atomics) {
  if (s.tail_len <= kLdsTailMax) return 0;
  if (force_atomics || !av.ready) return 1;
  return 3;
}

template <typename VT, int PM, int SQ>
static void aprod2_mode(int mode, const SysView& s, StreamShape sh, const void* sv, const double* y, double* x,
                        double* acc,
                        const double* S, double scale, double inv_beta, size_t hb, Scalars* sc, Work w,
                        hipStream_t st) {
  const dim3 g(sh.blocks), b(kBlock);
  if (mode == 0)
    hipLaunchKernelGGL((k_aprod2<VT, PM, SQ, 0>), g, b, hb, st, s, sh.waves, sv, y, x, acc, S, scale, inv_beta, sc, w);
  else if (mode == 1)
    hipLaunchKernelGGL((k_aprod2<VT, PM, SQ, 1>), g, b, hb, st, s, sh.waves, sv, y, x, acc, S, scale, inv_beta, sc, w);
  else
    hipLaunchKernelGGL((k_aprod2<VT, PM, SQ, 3>), g, b, hb, st, s, sh.waves, sv, y, x, acc, S, scale, inv_beta, sc, w);
}

hipError_t launch_aprod2(const SysView& s, StreamShape sh, int att_mode, const void* sv, const double* y, double* x,
                         double* acc,
                         const double* S, double scale, double inv_beta, int pmode, int square, Scalars* sc, Work w,
                         hipStream_t st) {
  const size_t hb = sizeof(double) * (size_t)(att_mode == 0 ? s.tail_len : s.tail_len - 3 * s.n_att);
  if (square) {
    if (s.value_type == GSR_F32)
      aprod2_mode<float, 0, 1>(att_mode, s, sh, sv, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
    else
      aprod2_mode<double, 0, 1>(att_mode, s, sh, sv, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  } else if (s.value_type == GSR_F32 && pmode == 1) {
    aprod2_mode<float, 1, 0>(att_mode, s, sh, sv, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  } else if (s.value_type == GSR_F32) {
    aprod2_mode<float, 0, 0>(att_mode, s, sh, sv, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  } else {
    aprod2_mode<double, 0, 0>(att_mode, s, sh, sv, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  }
  return hipGetLastError();
}

hipError_t launch_tail(const SysView& s, const AttView& av, int att_mode, double* x, double* acc, const double* S,
                       double scale, Scalars* sc, Work w, int lsqr_stage, int astro_parts, hipStream_t st) {
  int blocks = (int)std::min<int64_t>(512, std::max<int64_t>(1, (s.tail_len + kBlock - 1) / kBlock));
  TailLsqr L{lsqr_stage, astro_parts, nullptr};
  hipLaunchKernelGGL(k_tail, dim3(blocks), dim3(kBlock), 0, st, s, av, att_mode, x, acc, S, scale, sc, w, L);
  return hipGetLastError();
}

hipError_t launch_tail_fused(const SysView& s, const AttView& av, int att_mode, double* x, double* acc,
                             const double* S, const double* gA, Scalars* sc, Work w, hipStream_t st, int lsqr_stage) {
  const int64_t cols = s.n_astro + s.tail_len;
  int blocks = (int)std::min<int64_t>(kMaxPartials, std::max<int64_t>(1, (cols + kBlock - 1) / kBlock));
  TailLsqr L{lsqr_stage, 0, gA};
  hipLaunchKernelGGL(k_tail, dim3(blocks), dim3(kBlock), 0, st, s, av, att_mode, x, acc, S, 0.0, sc, w, L);
  return hipGetLastError();
}

hipError_t launch_tail_blk(const SysView& s, const BlkView& bv, double* x, double* acc, const double* S,
                           const double* gA, Scalars* sc, Work w, hipStream_t st, int lsqr_stage) {
  const int64_t cols = s.n_astro + s.tail_len;
  int blocks = (int)std::min<int64_t>(kMaxPartials, std::max<int64_t>(1, (cols + kBlock - 1) / kBlock));
  // the workgroup windows take the place of the bucketed pass's windows
  AttView av{};
  av.Wb = bv.Wb;
  av.nb = bv.nb;
  av.bsub = bv.bsub;
  av.Q = bv.Q;
  TailLsqr L{lsqr_stage, 0, gA};
  hipLaunchKernelGGL(k_tail, dim3(blocks), dim3(kBlock), 0, st, s, av, 3, x, acc, S, 0.0, sc, w, L);
  return hipGetLastError();
}

hipError_t launch_validate(const SysView& s, unsigned long long* bad, hipStream_t st) {
  int64_t n = std::max(s.m, s.n_stars);
  int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(kBlock), 0, st, s, bad);
  return hipGetLastError();
}

hipError_t launch_scale_from_sq(int64_t n, double* S, hipStream_t st) {
  int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_scale_from_sq, dim3(blocks), dim3(kBlock), 0, st, n, S);
  return hipGetLastError();
}

}  // namespace gsr
