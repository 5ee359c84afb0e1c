// One pass over the rows per LSQR iteration (Sec. 2, Eq. 2 and Eq. 3 on the
// bidiagonalisation of Paige & Saunders).
//
// The iteration needs u_{i+1} = (A v_i - alpha_i u_i) / beta_{i+1} and then
// A^T u_{i+1}.  Both are linear in the unnormalised u' = A v_i - alpha_i u_i,
// so A^T u_{i+1} = (A^T u') / beta_{i+1}: one streaming pass forms u'_r for
// each row and, from the same registers, adds a_r * u'_r to the
// astrometric, instrumental and global columns; beta_{i+1} is known at the end
// of the pass and the tail pass applies 1/beta_{i+1} when it forms v_{i+1}.
// The coefficients are read once per iteration instead of twice.  (Mixing
// even a few percent of stores into a read stream lowers the HBM rate
// markedly on this chip, so a separate aprod 1 pass, which writes u, and
// star pass, which reads the rows again, cost far more than their bytes.)
// The attitude columns are summed afterwards by the bucketed pass on u'
// (or, when the tail fits in LDS, in the same pass).
//
// Work split and tile mechanics as in aprod.hip: wave w owns whole stars,
// 64-row tiles staged through LDS, the next tile's loads issued as soon as
// the current one is in LDS, stores of a tile issued at the start of the next.
#include <algorithm>

#include "row_tiles.h"

namespace gsr {

// Row index record of the fused pass (when every instrumental column fits in
// 16 bits): the attitude start and the six instrumental columns in 16 bytes,
// fetched with one load instead of four (28 bytes).
__global__ void k_pack_rows(SysView s, u4* __restrict__ rix) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < s.m; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t* ic = s.instr_col + 6 * r;
    rix[r] = u4{(unsigned)s.att_start[r], (unsigned)ic[0] | ((unsigned)ic[1] << 16),
                (unsigned)ic[2] | ((unsigned)ic[3] << 16), (unsigned)ic[4] | ((unsigned)ic[5] << 16)};
  }
}

// Attitude window records, the copy of x that every row pass reads its
// attitude x from: record a holds the 12 attitude x of
// starts a .. a+3 (element 3j + axis: axis `axis` at start a+j), padded to
// kAttRec = 16 values, so that the window a row reads is one 128-byte cache
// line (64 bytes in the FP32 copy) instead of 96 bytes at a 24-byte stride,
// which straddles two lines for 11 of every 16 starts.  Written once per
// iteration (16 n_att values).
__global__ void k_att_records(SysView s, const double* __restrict__ x, double* __restrict__ xr,
                              float* __restrict__ xrf) {
  const int64_t nr = kAttRec * s.n_att;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nr; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / kAttRec;
    const int k = (int)(e - a * kAttRec), j = k / 3, axs = k - 3 * j;
    const double v = (k < 12 && a + j < s.n_att) ? x[s.n_astro + axs * s.n_att + a + j] : 0.0;
    xr[e] = v;
    if (xrf) xrf[e] = (float)v;
  }
}

// The attitude windows of a tile are loaded cooperatively: the tile's 64
// windows of 96 bytes are 384 16-byte pieces, loaded as 6 wave instructions
// in which consecutive lanes take consecutive pieces of the same window (a
// row-per-lane load would touch a separate cache line in every lane), then
// regrouped per row through LDS.
// Row indices come from the packed records; the instrumental x (at most
// kLdsTailMax - 1 columns) from an LDS copy.
// Two waves per SIMD: the register budget is held to 256 (it fits without spills).
// PM = 1 (FP32 systems): each product a * x is formed in FP32 and summed in
// FP64, the inner products of the FP32 form.
template <typename VT, int ATT_MODE, int PM>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) k_fused(SysView s, int waves, const double* __restrict__ x,
                                                  const double* __restrict__ x3, const u4* __restrict__ rix,
                                                  double* __restrict__ u, double* __restrict__ gA,
                                                  double* __restrict__ acc, Scalars* sc, Work wk, int init) {
  constexpr int CPR = Geo<VT>::CPR;
  __shared__ u4 slabs[kWavesPerBlock][kWave * (CPR + 1)];
  __shared__ int64_t bnds[kWavesPerBlock][kWave];
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  extern __shared__ double dyn[];  // tail histogram, then the instrumental x
  if (sc->done) return;
  const double scale = sc->u_scale;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t hoff = (ATT_MODE == 0) ? 0 : 3 * s.n_att;  // tail index of hist[0]
  const int64_t hlen = s.tail_len - hoff;
  double* hist = dyn;
  double* xil = dyn + hlen;
  const int64_t NI = s.n_astro + 3 * s.n_att;
  for (int64_t j = threadIdx.x; j < hlen; j += kBlock) hist[j] = 0.0;
  for (int64_t j = threadIdx.x; j < s.n_instr; j += kBlock) xil[j] = x[NI + j];
  __syncthreads();

  const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  double sumsq = 0.0, gsum = 0.0;
  if (w < waves) {
    int64_t s0, s1;
    wave_stars(s, w, waves, &s0, &s1);
    const int64_t R0 = s.row_ptr[s0], R1 = s.row_ptr[s1];
    int64_t scur = s0;
    while (scur < s1 && s.row_ptr[scur + 1] <= R0) ++scur;  // leading empty stars
    const double xg = s.n_glob ? x[NI + s.n_instr] : 0.0;
    const int64_t xa_last = 5 * s.n_stars - 1;
    const u4* vbase = reinterpret_cast<const u4*>(s.vals);
    u4 tmp[CPR];
    u4 ri;
    double uo;
    int64_t bv;
    auto fetch = [&](int64_t tt) {
      // past the end of the range: re-read its last row (the registers are not used)
      const int64_t te = min(tt, R1 - 1);
      const int nr = (int)min((int64_t)kWave, R1 - te);
      const int64_t rr = (lane < nr) ? te + lane : R1 - 1;
      issue_chunks<CPR>(vbase + te * CPR, nr, lane, tmp);
      ri = __builtin_nontemporal_load(rix + rr);
      uo = u[rr];
      bv = bnd_load(s, scur, lane);
    };
    double carry[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int carry_valid = 0;
    // results of the previous tile, stored at the start of the next one
    int64_t r_out = -1, c_out = -1;
    double u_out = 0.0;
    double g_out[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (R0 < R1) fetch(R0);
#pragma unroll 1
    for (int64_t t0 = R0; t0 < R1; t0 += kWave) {
      const int nrow = (int)min((int64_t)kWave, R1 - t0);
      const bool valid = lane < nrow;
      const int64_t r = t0 + (valid ? lane : 0);
      const int32_t at_c = (int32_t)ri.x;
      const int ic[6] = {(int)(ri.y & 0xFFFFu), (int)(ri.y >> 16), (int)(ri.z & 0xFFFFu),
                         (int)(ri.z >> 16),     (int)(ri.w & 0xFFFFu), (int)(ri.w >> 16)};
      const double uo_c = (scale == 0.0) ? 0.0 : scale * uo;
      const int64_t bv_c = bv;
      const int64_t sf = scur;  // star of row t0
      const int64_t span = __popcll(__ballot(bv_c <= t0 + nrow - 1)) + 1;
      scur = tile_next(s, bv_c, t0, sf);
      if (r_out >= 0) u[r_out] = u_out;
      if (c_out >= 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) gA[c_out + k] = g_out[k];
      }
      // gathers of x for this tile, issued before the next tile's loads
      const double xs = x[min(5 * sf + lane, xa_last)];
      dd2u cw[6];  // piece j*64 + lane of the tile's attitude windows
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
      u4 mine[CPR];
      lds_get<CPR>(nrow, slabs[wid], lane, mine);
      int64_t rbeg, rend;
      const int64_t st = tile_star(s, t0, lane, bnds[wid], sf, &rbeg, &rend);
      VT a[kSlots];
      __builtin_memcpy(a, mine, sizeof(a));
      // u'_r = u_scale * u_r + (A x)_r, each gathered x consumed as it is formed
      double ax = 0.0;
      {
        // every lane takes its star's x from the shuffle window (used on every
        // path, so the load stays where it was issued); with many short stars
        // in the tile, lanes past the window gather per lane, consumed inside
        // the branch (a load still pending where the paths join would make the
        // compiler wait for the next tile's loads too)
        const int64_t dst = valid ? st - sf : 0;
        const int base = 5 * (int)min<int64_t>(dst, 11);
        double axa = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) axa += prod<PM>(a[k], __shfl(xs, base + k, kWave));
        if (span > 12 && dst >= 12) {
          double xa5[5];
#pragma unroll
          for (int k = 0; k < 5; ++k) xa5[k] = x[5 * st + k];
          axa = 0.0;
#pragma unroll
          for (int k = 0; k < 5; ++k) axa += prod<PM>(a[k], xa5[k]);
        }
        ax += axa;
      }
      {
        // regroup the attitude windows per row through the (now free) slab;
        // window element e = 3j + axis is column at+j of that axis
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
          ax += prod<PM>(a[5 + 4 * (e0 % 3) + e0 / 3], pq.x);
          ax += prod<PM>(a[5 + 4 * (e1 % 3) + e1 / 3], pq.y);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) ax += prod<PM>(a[17 + q], xil[ic[q]]);
      if (s.n_glob) ax += prod<PM>(a[23], xg);
      const double un = uo_c + ax;
      r_out = valid ? r : -1;
      u_out = un;
      // a_r * u'_r into the star's, the instrumental and the global columns
      const double t = valid ? un : 0.0;
      sumsq += t * t;
      double p[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) p[k] = prod<PM>(a[k], t);
      if (valid) {
        if (ATT_MODE == 0) {
#pragma unroll
          for (int axs = 0; axs < 3; ++axs)
#pragma unroll
            for (int j = 0; j < 4; ++j) atomicAdd(hist + axs * s.n_att + at_c + j, prod<PM>(a[5 + 4 * axs + j], t));
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) atomicAdd(hist + (3 * s.n_att - hoff) + ic[q], prod<PM>(a[17 + q], t));
        if (s.n_glob) gsum += prod<PM>(a[23], t);
      }
      if (carry_valid && lane == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] += carry[k];
      }
      const int seg0 = valid ? (int)(max(rbeg, t0) - t0) : lane;
      seg_scan(p, lane, seg0);
      const bool ends_here = valid && (r == rend - 1);
      c_out = ends_here ? 5 * st : -1;
#pragma unroll
      for (int k = 0; k < 5; ++k) g_out[k] = p[k];
      const int last = nrow - 1;
      const int lend = (int)((__ballot(ends_here) >> last) & 1ull);
#pragma unroll
      for (int k = 0; k < 5; ++k) carry[k] = lane_read(p[k], last);
      carry_valid = !lend;
    }
    if (r_out >= 0) u[r_out] = u_out;
    if (c_out >= 0) {
#pragma unroll
      for (int k = 0; k < 5; ++k) gA[c_out + k] = g_out[k];
    }
    // stars without rows contribute nothing to A^T u
    if (s.has_empty_stars) {
      for (int64_t e = s0 + lane; e < s1; e += kWave)
        if (s.row_ptr[e] == s.row_ptr[e + 1]) {
#pragma unroll
          for (int k = 0; k < 5; ++k) gA[5 * e + k] = 0.0;
        }
    }
  }
  if (s.n_glob) {
    const double g = wave_sum(gsum);
    if (lane == 0) atomicAdd(hist + (hlen - 1), g);
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < hlen; j += kBlock) {
    const double v = hist[j];
    if (v != 0.0) atomicAdd(acc + hoff + j, v);
  }
  const double bs = block_sum(sumsq, red);
  if (threadIdx.x == 0) publish(wk.part_a + blockIdx.x, bs);
  if (last_block(wk.tickets + T_APROD1, &flag)) {
    const double tot = sum_partials(wk.part_a, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_beta(sc, tot + sc->con_sumsq, init);
      ticket_reset(wk.tickets + T_APROD1);
    }
  }
}

hipError_t launch_fused(const SysView& s, StreamShape sh, int att_mode, int pmode, const double* vg, const double* x3,
                        const void* rix, double* u, double* gA, double* acc, Scalars* sc, Work w, hipStream_t st,
                        int init) {
  if ((att_mode != 0 && att_mode != 3) || !rix || s.n_instr + 1 > kLdsTailMax) return hipErrorInvalidValue;
  if (pmode == 1 && s.value_type != GSR_F32) return hipErrorInvalidValue;
  const int64_t hlen = att_mode == 0 ? s.tail_len : s.tail_len - 3 * s.n_att;
  const size_t lds = sizeof(double) * (size_t)(hlen + s.n_instr);
  const dim3 g(sh.blocks), b(kBlock);
  const u4* rx = reinterpret_cast<const u4*>(rix);
  if (s.value_type == GSR_F32 && pmode == 1) {
    if (att_mode == 0)
      hipLaunchKernelGGL((k_fused<float, 0, 1>), g, b, lds, st, s, sh.waves, vg, x3, rx, u, gA, acc, sc, w, init);
    else
      hipLaunchKernelGGL((k_fused<float, 3, 1>), g, b, lds, st, s, sh.waves, vg, x3, rx, u, gA, acc, sc, w, init);
  } else if (s.value_type == GSR_F32) {
    if (att_mode == 0)
      hipLaunchKernelGGL((k_fused<float, 0, 0>), g, b, lds, st, s, sh.waves, vg, x3, rx, u, gA, acc, sc, w, init);
    else
      hipLaunchKernelGGL((k_fused<float, 3, 0>), g, b, lds, st, s, sh.waves, vg, x3, rx, u, gA, acc, sc, w, init);
  } else {
    if (att_mode == 0)
      hipLaunchKernelGGL((k_fused<double, 0, 0>), g, b, lds, st, s, sh.waves, vg, x3, rx, u, gA, acc, sc, w, init);
    else
      hipLaunchKernelGGL((k_fused<double, 3, 0>), g, b, lds, st, s, sh.waves, vg, x3, rx, u, gA, acc, sc, w, init);
  }
  return hipGetLastError();
}

hipError_t launch_pack_rows(const SysView& s, void* rix, hipStream_t st) {
  if (s.m == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(8192, (s.m + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pack_rows, dim3(blocks), dim3(kBlock), 0, st, s, reinterpret_cast<u4*>(rix));
  return hipGetLastError();
}

hipError_t launch_att_records(const SysView& s, const double* x, double* xr, hipStream_t st, float* xrf) {
  const int64_t nr = kAttRec * s.n_att;
  if (nr == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(2048, (nr + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_att_records, dim3(blocks), dim3(kBlock), 0, st, s, x, xr, xrf);
  return hipGetLastError();
}


}  // namespace gsr
