// The two products of every LSQR iteration (Sec. 2, Eq. 2 and Eq. 3) over the
// 24-coefficient row form of the observation matrix, for gfx950.
//
// Both kernels stream the coefficient rows once in star order.  Work is split
// by whole stars: wave w of W owns the stars whose rows start in
// [w*m/W, (w+1)*m/W), so every astrometric unknown is produced by exactly one
// wave.  A wave walks its rows in tiles of 64 (one row per lane).  A tile's
// coefficients (64 x 192 B for FP64) are fetched with contiguous 16-byte
// nontemporal loads (1 KB per wave instruction), staged in LDS with one
// 16-byte pad per row (conflict-free row reads) and read back row-per-lane.
// The star of each row comes from the tile's 64 star boundaries, loaded in
// one coalesced access and searched in LDS.
//
// aprod1: y_r <- scale*y_r + ax * sum_k a_rk x[col(r,k)]; the x gathers hit
//   L1/L2 (astrometric x is shared by the 20-90 rows of a star, the
//   attitude block is a few MB at most).
// aprod2 (this file: astrometric, instrumental, global; and the attitude
//   block when it fits in LDS): astrometric columns by a segmented scan over
//   the star runs of a tile, carried across tiles and written once by the
//   owning wave; instrumental and global columns LDS-private per workgroup,
//   flushed with one atomic per column per workgroup.  Larger attitude
//   blocks are summed by the bucketed pass in attitude.hip; this pass then
//   skips the 64-byte sectors that hold only attitude coefficients.
#include <algorithm>

#include "device_common.h"

namespace gsr {

template <typename VT>
struct Geo;
template <>
struct Geo<double> {
  static constexpr int CPR = 12;                // 16-byte chunks per row
  static constexpr unsigned ATT_ONLY = 0x0F8u;  // chunks 3..7: bytes 48..127, attitude only
};
template <>
struct Geo<float> {
  static constexpr int CPR = 6;
  static constexpr unsigned ATT_ONLY = 0x00Cu;  // chunks 2..3: bytes 32..63, attitude only
};

// smallest s in [0, S] with row_ptr[s] >= target
__device__ inline int64_t star_lower_bound(const int64_t* rp, int64_t S, int64_t target) {
  int64_t lo = 0, hi = S;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rp[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Star range [s0, s1) of wave w out of W.
__device__ inline void wave_stars(const SysView& s, int64_t w, int64_t W, int64_t* s0, int64_t* s1) {
  const int64_t t0 = (s.m * w + W - 1) / W;
  const int64_t t1 = (s.m * (w + 1) + W - 1) / W;
  *s0 = (w == 0) ? 0 : star_lower_bound(s.row_ptr, s.n_stars, t0);
  *s1 = (w == W - 1) ? s.n_stars : star_lower_bound(s.row_ptr, s.n_stars, t1);
}

template <int PM, typename VT>
__device__ __forceinline__ double prod(VT a, double x) {
  if (PM == 1) return (double)((float)a * (float)x);
  return (double)a * x;
}

// Star boundaries for a tile whose first row is in star scur: lane i holds
// row_ptr[scur + 1 + i] (the end row of star scur + i), clamped at n_stars.
__device__ __forceinline__ int64_t bnd_load(const SysView& s, int64_t scur, int lane) {
  return s.row_ptr[min(scur + 1 + lane, s.n_stars)];
}

// Stars of the tile's rows from the loaded boundaries b (searched in this
// wave's LDS bnd[64]).  Returns the lane's star and advances scur to the star
// of row t0 + 64.
__device__ __forceinline__ int64_t tile_stars(const SysView& s, int64_t b, int64_t t0, int lane, int64_t* bnd,
                                              int64_t& scur, int64_t* rbeg = nullptr, int64_t* rend = nullptr) {
  bnd[lane] = b;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int64_t r = t0 + lane;
  // lo = #{i : bnd[i] <= r}, bnd ascending
  int lo = 0, hi = kWave;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (bnd[mid] <= r)
      lo = mid + 1;
    else
      hi = mid;
  }
  int64_t st = scur + lo;
  if (lo == kWave) {  // more than 64 stars end inside this tile (empty or one-row stars)
    while (st < s.n_stars - 1 && s.row_ptr[st + 1] <= r) ++st;
    if (rbeg) *rbeg = s.row_ptr[st];
    if (rend) *rend = s.row_ptr[st + 1];
  } else {
    // star st = scur + lo spans rows [row_ptr[st], row_ptr[st+1]) = [bnd[lo-1], bnd[lo]);
    // for lo = 0 it began at or before t0
    if (rbeg) *rbeg = lo > 0 ? bnd[lo - 1] : t0;
    if (rend) *rend = bnd[lo];
  }
  const uint64_t adv = __ballot(b <= t0 + kWave);
  int64_t nxt = scur + __popcll(adv);
  if (__popcll(adv) == kWave)
    while (nxt < s.n_stars - 1 && s.row_ptr[nxt + 1] <= t0 + kWave) ++nxt;
  nxt = min(nxt, max<int64_t>(s.n_stars - 1, 0));
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  scur = nxt;
  return st;
}

// ---------------------------------------------------------------- aprod1
template <typename VT, int PM>
__global__ void __launch_bounds__(kBlock) k_aprod1(SysView s, int waves, const double* __restrict__ x,
                                                   double* __restrict__ y, double scale, double ax, Scalars* sc,
                                                   Work wk, int lsqr_stage) {
  constexpr int CPR = Geo<VT>::CPR;
  __shared__ u4 slabs[kWavesPerBlock][kWave * (CPR + 1)];
  __shared__ int64_t bnds[kWavesPerBlock][kWave];
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  if (sc) {
    if (sc->done) return;
    scale = sc->u_scale;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  double sumsq = 0.0;
  if (w < waves) {
    int64_t s0, s1;
    wave_stars(s, w, waves, &s0, &s1);
    const int64_t R0 = s.row_ptr[s0], R1 = s.row_ptr[s1];
    const int64_t NI = s.n_astro + 3 * s.n_att;
    const double xg = s.n_glob ? x[NI + s.n_instr] : 0.0;
    int64_t scur = s0;
    while (scur < s1 && s.row_ptr[scur + 1] <= R0) ++scur;  // leading empty stars
    const u4* vbase = reinterpret_cast<const u4*>(s.vals);
    // registers of the prefetched tile
    u4 tmp[CPR];
    int32_t at;
    i2 i01, i23, i45;
    double yo;
    int64_t bv;
    auto fetch = [&](int64_t tt) {
      const int nr = (int)max<int64_t>(0, min((int64_t)kWave, R1 - tt));
      const int64_t rr = (lane < nr) ? tt + lane : R1 - 1;  // always a valid row
      issue_chunks<CPR, 0u>(vbase + tt * CPR, nr, lane, tmp);
      at = __builtin_nontemporal_load(s.att_start + rr);
      const i2* icp = reinterpret_cast<const i2*>(s.instr_col + 6 * rr);
      i01 = __builtin_nontemporal_load(icp);
      i23 = __builtin_nontemporal_load(icp + 1);
      i45 = __builtin_nontemporal_load(icp + 2);
      yo = (scale == 0.0) ? 0.0 : y[rr];
      bv = bnd_load(s, scur, lane);
    };
    if (R0 < R1) fetch(R0);
#pragma unroll 1
    for (int64_t t0 = R0; t0 < R1; t0 += kWave) {
      const int nrow = (int)min((int64_t)kWave, R1 - t0);
      const bool valid = lane < nrow;
      const int64_t r = t0 + (valid ? lane : 0);
      const int32_t at_c = at;
      const int ic[6] = {i01.x, i01.y, i23.x, i23.y, i45.x, i45.y};
      const double yo_c = yo;
      u4 mine[CPR];
      lds_rows<CPR, 0u>(tmp, nrow, slabs[wid], lane, mine);
      const int64_t st = tile_stars(s, bv, t0, lane, bnds[wid], scur);
      VT a[kSlots];
      __builtin_memcpy(a, mine, sizeof(a));
      // gathers of x for this tile, then the next tile's loads
      double gx[kSlots];
      const double* xa = x + 5 * st;
#pragma unroll
      for (int k = 0; k < 5; ++k) gx[k] = xa[k];
#pragma unroll
      for (int axs = 0; axs < 3; ++axs) {
        const double* xt = x + s.n_astro + axs * s.n_att + at_c;
#pragma unroll
        for (int j = 0; j < 4; ++j) gx[5 + 4 * axs + j] = xt[j];
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) gx[17 + q] = x[NI + ic[q]];
      order_point();
      fetch(t0 + kWave);  // past the end: chunk loads off, index loads from a valid row
      order_point();
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 23; ++k) acc += prod<PM>(a[k], gx[k]);
      if (s.n_glob) acc += prod<PM>(a[23], xg);
      if (valid) {
        const double yn = scale * yo_c + ax * acc;
        y[r] = yn;
        sumsq += yn * yn;
      }
    }
  }
  if (!sc) return;
  const double bs = block_sum(sumsq, red);
  if (threadIdx.x == 0) wk.part_a[blockIdx.x] = bs;
  if (last_block(wk.tickets + T_APROD1, &flag)) {
    const double tot = sum_partials(wk.part_a, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_beta(sc, tot, lsqr_stage == 0);
      wk.tickets[T_APROD1] = 0;
    }
  }
}

// ---------------------------------------------------------------- aprod2
// ATT_MODE 0: the whole tail (attitude, instrumental, global) in LDS.
// ATT_MODE 1: attitude by device-scope FP64 atomics (fallback), instr + global in LDS.
// ATT_MODE 3: attitude summed by the bucketed pass; its sectors are not read here.
template <typename VT, int PM, int SQUARE, int ATT_MODE>
__global__ void __launch_bounds__(kBlock) k_aprod2(SysView s, int waves, const double* __restrict__ y,
                                                   double* __restrict__ x, double* __restrict__ acc,
                                                   const double* __restrict__ S, double scale, double inv_beta,
                                                   Scalars* sc, Work wk) {
  constexpr int CPR = Geo<VT>::CPR;
  constexpr unsigned SKIP = (ATT_MODE == 3) ? Geo<VT>::ATT_ONLY : 0u;
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
    const u4* vbase = reinterpret_cast<const u4*>(s.vals);
    u4 tmp[CPR];
    double tv;
    int32_t at;
    i2 i01, i23, i45;
    int64_t bv;
    auto fetch = [&](int64_t tt) {
      const int nr = (int)max<int64_t>(0, min((int64_t)kWave, R1 - tt));
      const int64_t rr = (lane < nr) ? tt + lane : R1 - 1;  // always a valid row
      issue_chunks<CPR, SKIP>(vbase + tt * CPR, nr, lane, tmp);
      tv = SQUARE ? 0.0 : __builtin_nontemporal_load(y + rr);
      at = (ATT_MODE == 3) ? 0 : __builtin_nontemporal_load(s.att_start + rr);
      const i2* icp = reinterpret_cast<const i2*>(s.instr_col + 6 * rr);
      i01 = __builtin_nontemporal_load(icp);
      i23 = __builtin_nontemporal_load(icp + 1);
      i45 = __builtin_nontemporal_load(icp + 2);
      bv = bnd_load(s, scur, lane);
    };
    if (R0 < R1) fetch(R0);
#pragma unroll 1
    for (int64_t t0 = R0; t0 < R1; t0 += kWave) {
      const int nrow = (int)min((int64_t)kWave, R1 - t0);
      const bool valid = lane < nrow;
      const int64_t r = t0 + (valid ? lane : 0);
      const double t = tv * inv_beta;
      const int32_t at_c = at;
      const int ic[6] = {i01.x, i01.y, i23.x, i23.y, i45.x, i45.y};
      u4 mine[CPR];
      lds_rows<CPR, SKIP>(tmp, nrow, slabs[wid], lane, mine);
      int64_t rbeg, rend;
      const int64_t st = tile_stars(s, bv, t0, lane, bnds[wid], scur, &rbeg, &rend);
      order_point();
      fetch(t0 + kWave);  // past the end: chunk loads off, index loads from a valid row
      order_point();
      VT a[kSlots];
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
          const VT av = a[17 + q];
          const double c = SQUARE ? (double)av * (double)av : prod<PM>(av, t);
          atomicAdd(hist + (3 * s.n_att - hoff) + ic[q], c);
        }
        if (s.n_glob) gsum += SQUARE ? (double)a[23] * (double)a[23] : prod<PM>(a[23], t);
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
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const double o = __shfl_up(p[k], off, kWave);
          if (lane - off >= seg0) p[k] += o;
        }
      }
      const bool ends_here = valid && (r == rend - 1);
      if (ends_here) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int64_t c = 5 * st + k;
          const double xo = (scale == 0.0) ? 0.0 : scale * x[c];
          const double xn = xo + (S ? S[c] : 1.0) * p[k];
          x[c] = xn;
          sumsq += xn * xn;
        }
      }
      // carry the last run of the tile if its star continues
      const int last = nrow - 1;
      const int lend = __shfl(ends_here ? 1 : 0, last, kWave);
#pragma unroll
      for (int k = 0; k < 5; ++k) carry[k] = __shfl(p[k], last, kWave);
      carry_valid = !lend;
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
    if (threadIdx.x == 0) wk.part_b[blockIdx.x] = bs;
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
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < s.tail_len; j += (int64_t)gridDim.x * kBlock) {
      double a;
      if (att_mode == 3 && j < natt) {
        const int64_t axs = j / s.n_att, c = j - axs * s.n_att;
        a = 0.0;
        const int64_t bhi = min(c / av.Wb, av.nb - 1);
        for (int64_t b = max<int64_t>(bhi - 1, 0); b <= bhi; ++b) {
          const int64_t off = c - b * av.Wb;
          if (off < 0 || off >= win) continue;
          for (int32_t q = av.bsub[b]; q < av.bsub[b + 1]; ++q) a += av.Q[((int64_t)q * 3 + axs) * win + off];
        }
      } else {
        a = acc[j];
        acc[j] = 0.0;
      }
      const int64_t c = s.n_astro + j;
      const double xo = (scale == 0.0) ? 0.0 : scale * x[c];
      const double xn = xo + (S ? S[c] : 1.0) * a;
      x[c] = xn;
      sumsq += xn * xn;
    }
  }
  if (!sc) return;
  const double bs = block_sum(sumsq, red);
  if (threadIdx.x == 0) wk.part_a[blockIdx.x] = bs;
  if (last_block(wk.tickets + T_TAIL, &flag)) {
    double tot = sum_partials(wk.part_b, L.astro_parts, red);
    tot += sum_partials(wk.part_a, gridDim.x, red);
    __shared__ double t3s;
    __shared__ int64_t cols;
    if (threadIdx.x == 0) {
      epi_alpha(sc, tot, L.lsqr_stage == 0);
      t3s = sc->t3;
      cols = sc->dcount;
      wk.tickets[T_TAIL] = 0;
    }
    __syncthreads();
    if (L.lsqr_stage != 0 && sc->nsel > 0) {
      const int64_t ld = sc->dblock;
      if (cols < ld) {
        for (int64_t p = threadIdx.x; p < sc->nsel; p += kBlock) L.D[p * ld + cols] = t3s * L.w[L.sel[p]];
        if (threadIdx.x == 0) sc->dcount = (int32_t)(cols + 1);
      }
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

hipError_t launch_aprod1(const SysView& s, StreamShape sh, const double* x, double* y, double scale, double ax,
                         int pmode, Scalars* sc, Work w, int lsqr_stage, hipStream_t st) {
  const dim3 g(sh.blocks), b(kBlock);
  if (s.value_type == GSR_F32 && pmode == 1)
    hipLaunchKernelGGL((k_aprod1<float, 1>), g, b, 0, st, s, sh.waves, x, y, scale, ax, sc, w, lsqr_stage);
  else if (s.value_type == GSR_F32)
    hipLaunchKernelGGL((k_aprod1<float, 0>), g, b, 0, st, s, sh.waves, x, y, scale, ax, sc, w, lsqr_stage);
  else
    hipLaunchKernelGGL((k_aprod1<double, 0>), g, b, 0, st, s, sh.waves, x, y, scale, ax, sc, w, lsqr_stage);
  return hipGetLastError();
}

int att_mode_of(const SysView& s, const AttView& av, int force_atomics) {
  if (s.tail_len <= kLdsTailMax) return 0;
  if (force_atomics || !av.ready) return 1;
  return 3;
}

template <typename VT, int PM, int SQ>
static void aprod2_mode(int mode, const SysView& s, StreamShape sh, const double* y, double* x, double* acc,
                        const double* S, double scale, double inv_beta, size_t hb, Scalars* sc, Work w,
                        hipStream_t st) {
  const dim3 g(sh.blocks), b(kBlock);
  if (mode == 0)
    hipLaunchKernelGGL((k_aprod2<VT, PM, SQ, 0>), g, b, hb, st, s, sh.waves, y, x, acc, S, scale, inv_beta, sc, w);
  else if (mode == 1)
    hipLaunchKernelGGL((k_aprod2<VT, PM, SQ, 1>), g, b, hb, st, s, sh.waves, y, x, acc, S, scale, inv_beta, sc, w);
  else
    hipLaunchKernelGGL((k_aprod2<VT, PM, SQ, 3>), g, b, hb, st, s, sh.waves, y, x, acc, S, scale, inv_beta, sc, w);
}

hipError_t launch_aprod2(const SysView& s, StreamShape sh, int att_mode, const double* y, double* x, double* acc,
                         const double* S, double scale, double inv_beta, int pmode, int square, Scalars* sc, Work w,
                         hipStream_t st) {
  const size_t hb = sizeof(double) * (size_t)(att_mode == 0 ? s.tail_len : s.tail_len - 3 * s.n_att);
  if (square) {
    if (s.value_type == GSR_F32)
      aprod2_mode<float, 0, 1>(att_mode, s, sh, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
    else
      aprod2_mode<double, 0, 1>(att_mode, s, sh, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  } else if (s.value_type == GSR_F32 && pmode == 1) {
    aprod2_mode<float, 1, 0>(att_mode, s, sh, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  } else if (s.value_type == GSR_F32) {
    aprod2_mode<float, 0, 0>(att_mode, s, sh, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  } else {
    aprod2_mode<double, 0, 0>(att_mode, s, sh, y, x, acc, S, scale, inv_beta, hb, sc, w, st);
  }
  return hipGetLastError();
}

hipError_t launch_tail(const SysView& s, const AttView& av, int att_mode, double* x, double* acc, const double* S,
                       double scale, Scalars* sc, Work w, int lsqr_stage, int astro_parts, const int64_t* sel,
                       const double* wv, double* D, hipStream_t st) {
  int blocks = (int)std::min<int64_t>(512, std::max<int64_t>(1, (s.tail_len + kBlock - 1) / kBlock));
  TailLsqr L{lsqr_stage, astro_parts, sel, wv, D};
  hipLaunchKernelGGL(k_tail, dim3(blocks), dim3(kBlock), 0, st, s, av, att_mode, x, acc, S, scale, sc, w, L);
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
