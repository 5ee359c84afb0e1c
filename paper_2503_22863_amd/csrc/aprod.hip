// The two products of every LSQR iteration (Sec. 2, Eq. 2 and Eq. 3) over the
// 24-coefficient row form of the observation matrix, for gfx950.
//
// Both kernels stream the coefficient rows once.  Work is split by whole
// stars: wave w of W owns the stars whose rows start in [w*m/W, (w+1)*m/W),
// so every astrometric unknown is produced by exactly one wave.  A wave
// walks its rows in tiles of 64 (one row per lane); each tile's coefficients
// (64 x 192 B for FP64) are fetched with contiguous 16-byte loads, staged in
// LDS with one 16-byte pad per row (conflict-free row reads), and then read
// back row-per-lane.
//
// aprod1: y_r <- scale*y_r + ax * sum_k a_rk x[col(r,k)]; the x gathers hit
//   L1/L2 (astro x is shared by the ~20-90 rows of a star, the attitude
//   block is a few MB at most).
// aprod2: astrometric columns by a segmented scan over the star runs of a
//   tile (carried across tiles), written once by the owning wave; attitude
//   columns by FP64 atomics (LDS-private when the whole tail fits, otherwise
//   device-scope); instrumental and global columns LDS-private per workgroup,
//   flushed with one atomic per column per workgroup.
#include <algorithm>

#include "device_common.h"

namespace gsr {

template <typename VT>
struct Geo;
template <>
struct Geo<double> {
  static constexpr int CPR = 12;  // 16-byte chunks per row
};
template <>
struct Geo<float> {
  static constexpr int CPR = 6;
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

template <typename VT>
__device__ __forceinline__ double prod(VT a, double x, int pmode) {
  if (pmode == 1) return (double)((float)a * (float)x);
  return (double)a * x;
}

// Stage one tile of `nrow` rows starting at row t0 into this wave's LDS slab
// and return the lane's row as 24 values.
template <typename VT, int STAGE>
__device__ __forceinline__ void load_tile_row(const SysView& s, int64_t t0, int nrow, u4* slab, int lane,
                                              VT* a) {
  constexpr int CPR = Geo<VT>::CPR;
  const u4* g = reinterpret_cast<const u4*>(s.vals) + t0 * CPR;
  if (STAGE == 0) {
    u4 mine[CPR];
#pragma unroll
    for (int j = 0; j < CPR; ++j) mine[j] = (lane < nrow) ? ld_stream(g + lane * CPR + j) : u4{0u, 0u, 0u, 0u};
    __builtin_memcpy(a, mine, sizeof(VT) * kSlots);
    return;
  }
  const int nch = nrow * CPR;
  u4 tmp[CPR];
#pragma unroll
  for (int j = 0; j < CPR; ++j) {
    const int c = j * kWave + lane;
    if (c < nch) tmp[j] = ld_stream(g + c);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < CPR; ++j) {
    const int c = j * kWave + lane;
    if (c < nch) {
      const int r = c / CPR, q = c - r * CPR;
      slab[r * (CPR + 1) + q] = tmp[j];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  u4 mine[CPR];
  if (lane < nrow) {
#pragma unroll
    for (int j = 0; j < CPR; ++j) mine[j] = slab[lane * (CPR + 1) + j];
  } else {
#pragma unroll
    for (int j = 0; j < CPR; ++j) mine[j] = u4{0u, 0u, 0u, 0u};
  }
  __builtin_memcpy(a, mine, sizeof(VT) * kSlots);
}

// Star of row r, scanning forward from s_hint (rows are sorted by star).
__device__ __forceinline__ int64_t star_of(const int64_t* rp, int64_t s_hint, int64_t r) {
  int64_t st = s_hint;
  while (rp[st + 1] <= r) ++st;
  return st;
}

// ---------------------------------------------------------------- aprod1
template <typename VT, int STAGE>
__global__ void __launch_bounds__(kBlock) k_aprod1(SysView s, int waves, const double* __restrict__ x,
                                                   double* __restrict__ y, double scale, double ax, int pmode,
                                                   Scalars* sc, Work wk, int lsqr_stage) {
  constexpr int CPR = Geo<VT>::CPR;
  __shared__ u4 slabs[kWavesPerBlock][STAGE ? kWave * (CPR + 1) : 1];
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
    for (int64_t t0 = R0; t0 < R1; t0 += kWave) {
      const int nrow = (int)min((int64_t)kWave, R1 - t0);
      // the tile's first star
      while (s.row_ptr[scur + 1] <= t0) ++scur;
      VT a[kSlots];
      load_tile_row<VT, STAGE>(s, t0, nrow, slabs[wid], lane, a);
      if (lane < nrow) {
        const int64_t r = t0 + lane;
        const int64_t st = star_of(s.row_ptr, scur, r);
        const int32_t at = __builtin_nontemporal_load(s.att_start + r);
        const i2* icp = reinterpret_cast<const i2*>(s.instr_col + 6 * r);
        const i2 i01 = __builtin_nontemporal_load(icp), i23 = __builtin_nontemporal_load(icp + 1),
                 i45 = __builtin_nontemporal_load(icp + 2);
        const int ic[6] = {i01.x, i01.y, i23.x, i23.y, i45.x, i45.y};
        double acc = 0.0;
        const double* xa = x + 5 * st;
#pragma unroll
        for (int k = 0; k < 5; ++k) acc += prod<VT>(a[k], xa[k], pmode);
#pragma unroll
        for (int axs = 0; axs < 3; ++axs) {
          const double* xt = x + s.n_astro + axs * s.n_att + at;
#pragma unroll
          for (int j = 0; j < 4; ++j) acc += prod<VT>(a[5 + 4 * axs + j], xt[j], pmode);
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) acc += prod<VT>(a[17 + p], x[NI + ic[p]], pmode);
        if (s.n_glob) acc += prod<VT>(a[23], xg, pmode);
        const double yo = (scale == 0.0) ? 0.0 : scale * y[r];
        const double yn = yo + ax * acc;
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
// tail_mode 0: the whole tail (attitude, instrumental, global) in LDS.
// tail_mode 1: attitude by device-scope atomics, instrumental + global in LDS.
// tail_mode 2: attitude by atomics into a private copy per XCD (each XCD has
//   its own L2; the copy of XCD x is only touched by waves running on x, so
//   the atomics stay in that L2), instrumental + global in LDS.  The tail
//   pass adds the copies.
template <typename VT, int STAGE>
__global__ void __launch_bounds__(kBlock) k_aprod2(SysView s, int waves, const double* __restrict__ y,
                                                   double* __restrict__ x, double* __restrict__ acc,
                                                   const double* __restrict__ S, double scale, double inv_beta,
                                                   int pmode, int square, int tail_mode, Scalars* sc, Work wk) {
  constexpr int CPR = Geo<VT>::CPR;
  __shared__ u4 slabs[kWavesPerBlock][STAGE ? kWave * (CPR + 1) : 1];
  __shared__ double red[kWavesPerBlock];
  extern __shared__ double hist[];
  if (sc) {
    if (sc->done || !sc->do_v) return;
    scale = sc->v_scale;
    inv_beta = sc->inv_beta;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  // LDS-private tail: [0, 3*n_att) attitude (mode 0 only), then instr, then global
  const int64_t hoff = (tail_mode == 0) ? 0 : 3 * s.n_att;  // tail index of hist[0]
  const int64_t hlen = s.tail_len - hoff;
  double* acc_att = acc;
  if (tail_mode == 2) acc_att = acc + s.tail_len + (int64_t)xcc_id() * 3 * s.n_att;
  for (int64_t j = threadIdx.x; j < hlen; j += kBlock) hist[j] = 0.0;
  __syncthreads();

  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  double sumsq = 0.0, gsum = 0.0;
  if (w < waves) {
    int64_t s0, s1;
    wave_stars(s, w, waves, &s0, &s1);
    const int64_t R0 = s.row_ptr[s0], R1 = s.row_ptr[s1];
    int64_t scur = s0;
    double carry[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int carry_valid = 0;
    for (int64_t t0 = R0; t0 < R1; t0 += kWave) {
      const int nrow = (int)min((int64_t)kWave, R1 - t0);
      while (s.row_ptr[scur + 1] <= t0) ++scur;
      VT a[kSlots];
      load_tile_row<VT, STAGE>(s, t0, nrow, slabs[wid], lane, a);
      const bool valid = lane < nrow;
      const int64_t r = t0 + (valid ? lane : 0);
      const int64_t st = valid ? star_of(s.row_ptr, scur, r) : scur;
      const int64_t rbeg = s.row_ptr[st], rend = s.row_ptr[st + 1];
      const int seg0 = valid ? (int)(max(rbeg, t0) - t0) : lane;
      double p[5];
      if (valid) {
        const double t = square ? 0.0 : __builtin_nontemporal_load(y + r) * inv_beta;
        const int32_t at = __builtin_nontemporal_load(s.att_start + r);
        const i2* icp = reinterpret_cast<const i2*>(s.instr_col + 6 * r);
        const i2 i01 = __builtin_nontemporal_load(icp), i23 = __builtin_nontemporal_load(icp + 1),
                 i45 = __builtin_nontemporal_load(icp + 2);
        const int ic[6] = {i01.x, i01.y, i23.x, i23.y, i45.x, i45.y};
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] = square ? (double)a[k] * (double)a[k] : prod<VT>(a[k], t, pmode);
#pragma unroll
        for (int axs = 0; axs < 3; ++axs) {
          const int64_t col = axs * s.n_att + at;  // tail index
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const VT av = a[5 + 4 * axs + j];
            const double c = square ? (double)av * (double)av : prod<VT>(av, t, pmode);
            if (tail_mode == 0)
              atomicAdd(hist + col + j, c);
            else if (tail_mode == 1)
              atomicAdd(acc_att + col + j, c);
            else
              __hip_atomic_fetch_add(acc_att + col + j, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const VT av = a[17 + q];
          const double c = square ? (double)av * (double)av : prod<VT>(av, t, pmode);
          atomicAdd(hist + (3 * s.n_att - hoff) + ic[q], c);
        }
        if (s.n_glob) gsum += square ? (double)a[23] * (double)a[23] : prod<VT>(a[23], t, pmode);
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] = 0.0;
      }
      // carried partial sums of a star that began in an earlier tile
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
// x_t <- scale*x_t + S_t * acc_t for the attitude, instrumental and global
// unknowns; acc is cleared for the next product.  In an LSQR solve the last
// workgroup forms alpha_{i+1}, applies the rotations of the iteration and
// buffers d_i[sel] = w_i[sel] / rho_i as one covariance column.
struct TailLsqr {
  int lsqr_stage;       // 0 init, 1 iteration
  int astro_parts;      // partials written by the aprod2 launch
  const int64_t* sel;   // selected unknowns (nsel = sc->nsel)
  const double* w;      // search direction w_i
  double* D;            // [nsel][dblock]
};

__global__ void __launch_bounds__(kBlock) k_tail(SysView s, double* __restrict__ x, double* __restrict__ acc,
                                                 const double* __restrict__ S, double scale, Scalars* sc, Work wk,
                                                 TailLsqr L, int xcd_copies) {
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
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < s.tail_len; j += (int64_t)gridDim.x * kBlock) {
      double a = acc[j];
      acc[j] = 0.0;
      if (xcd_copies && j < natt) {
#pragma unroll
        for (int x = 0; x < kXcds; ++x) {
          double* q = acc + s.tail_len + x * natt + j;
          a += *q;
          *q = 0.0;
        }
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
StreamShape stream_shape(const SysView& s, int cus, int waves_per_cu, int stage, int xcd_copies) {
  // never more waves than stars or row tiles, never more blocks than partial slots
  int64_t waves = (int64_t)cus * waves_per_cu;
  waves = std::min(waves, (int64_t)kMaxPartials * kWavesPerBlock);
  waves = std::min(waves, std::max<int64_t>(1, s.n_stars));
  waves = std::min(waves, std::max<int64_t>(1, (s.m + kWave - 1) / kWave));
  waves = std::max<int64_t>(waves, 1);
  StreamShape sh;
  sh.waves = (int)waves;
  sh.blocks = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  sh.stage = stage;
  sh.xcd_copies = xcd_copies;
  return sh;
}

template <int STAGE>
static void aprod1_go(const SysView& s, StreamShape sh, const double* x, double* y, double scale, double ax,
                      int pmode, Scalars* sc, Work w, int lsqr_stage, hipStream_t st) {
  if (s.value_type == GSR_F32)
    hipLaunchKernelGGL((k_aprod1<float, STAGE>), dim3(sh.blocks), dim3(kBlock), 0, st, s, sh.waves, x, y, scale, ax,
                       pmode, sc, w, lsqr_stage);
  else
    hipLaunchKernelGGL((k_aprod1<double, STAGE>), dim3(sh.blocks), dim3(kBlock), 0, st, s, sh.waves, x, y, scale,
                       ax, 0, sc, w, lsqr_stage);
}

hipError_t launch_aprod1(const SysView& s, StreamShape sh, const double* x, double* y, double scale, double ax,
                         int pmode, Scalars* sc, Work w, int lsqr_stage, hipStream_t st) {
  if (sh.stage)
    aprod1_go<1>(s, sh, x, y, scale, ax, pmode, sc, w, lsqr_stage, st);
  else
    aprod1_go<0>(s, sh, x, y, scale, ax, pmode, sc, w, lsqr_stage, st);
  return hipGetLastError();
}

int tail_mode_of(const SysView& s, int xcd_copies) {
  if (s.tail_len <= kLdsTailMax) return 0;
  return xcd_copies ? 2 : 1;
}

template <int STAGE>
static void aprod2_go(const SysView& s, StreamShape sh, const double* y, double* x, double* acc, const double* S,
                      double scale, double inv_beta, int pmode, int square, int tm, size_t hbytes, Scalars* sc,
                      Work w, hipStream_t st) {
  if (s.value_type == GSR_F32)
    hipLaunchKernelGGL((k_aprod2<float, STAGE>), dim3(sh.blocks), dim3(kBlock), hbytes, st, s, sh.waves, y, x, acc,
                       S, scale, inv_beta, pmode, square, tm, sc, w);
  else
    hipLaunchKernelGGL((k_aprod2<double, STAGE>), dim3(sh.blocks), dim3(kBlock), hbytes, st, s, sh.waves, y, x,
                       acc, S, scale, inv_beta, 0, square, tm, sc, w);
}

hipError_t launch_aprod2(const SysView& s, StreamShape sh, const double* y, double* x, double* acc, const double* S,
                         double scale, double inv_beta, int pmode, int square, Scalars* sc, Work w,
                         hipStream_t st) {
  const int tm = tail_mode_of(s, sh.xcd_copies);
  const size_t hbytes = sizeof(double) * (size_t)(tm == 0 ? s.tail_len : s.tail_len - 3 * s.n_att);
  if (sh.stage)
    aprod2_go<1>(s, sh, y, x, acc, S, scale, inv_beta, pmode, square, tm, hbytes, sc, w, st);
  else
    aprod2_go<0>(s, sh, y, x, acc, S, scale, inv_beta, pmode, square, tm, hbytes, sc, w, st);
  return hipGetLastError();
}

hipError_t launch_tail(const SysView& s, double* x, double* acc, const double* S, double scale, int square,
                       Scalars* sc, Work w, int lsqr_stage, int astro_parts, const int64_t* sel, const double* wv,
                       double* D, int xcd_copies, hipStream_t st) {
  (void)square;
  int blocks = (int)std::min<int64_t>(256, std::max<int64_t>(1, (s.tail_len + kBlock - 1) / kBlock));
  TailLsqr L{lsqr_stage, astro_parts, sel, wv, D};
  hipLaunchKernelGGL(k_tail, dim3(blocks), dim3(kBlock), 0, st, s, x, acc, S, scale, sc, w, L,
                     tail_mode_of(s, xcd_copies) == 2 ? 1 : 0);
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
