// Star sums of the regrouped row pass.  That pass writes, for every star
// segment (a star's rows inside one wave's tile range), the five partial sums
// of a_r u'_r on the star's astrometric columns; these kernels add each star's
// segments.  k_tail_seg also forms the new v of every column (the tail of the
// iteration, Sec. 2, Eq. 3 then the normalisation of Paige and Saunders'
// bidiagonalisation), k_seg_reduce only the raw star sums (used when constraint
// rows are added between the two).
#include <algorithm>

#include "row_tiles.h"

namespace gsr {

// One wave per group of 64 consecutive stars, one star per lane: entry i of
// the group's list holds, lane by lane, the id of each star's i-th segment
// (block order; padding points at the zero entry P[nseg]).  Neighbouring stars'
// i-th segments are neighbours in P (same block), so both the id loads and the
// P loads of a wave are contiguous; ids are taken four entries at a time so
// that the two dependent loads overlap across entries.
__global__ void __launch_bounds__(kBlock) k_seg_reduce(SysView s, BlkView bv, double* __restrict__ gA, Scalars* sc) {
  if (sc && (sc->done || !sc->do_v)) return;
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; grp < bv.ngroups;
       grp += (int64_t)gridDim.x * blockDim.x / kWave) {
    const int32_t* L = bv.grp_list + bv.grp_base[grp] + lane;
    const int32_t cnt = bv.grp_cnt[grp];
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int32_t i = 0;
    for (; i + 4 <= cnt; i += 4) {
      int32_t id[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) id[e] = L[(int64_t)(i + e) * kWave];
      double v[4][5];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int k = 0; k < 5; ++k) v[e][k] = bv.P[5 * (int64_t)id[e] + k];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int k = 0; k < 5; ++k) a[k] += v[e][k];
    }
    for (; i < cnt; ++i) {
      const int32_t id = L[(int64_t)i * kWave];
#pragma unroll
      for (int k = 0; k < 5; ++k) a[k] += bv.P[5 * (int64_t)id + k];
    }
    const int64_t st = grp * kWave + lane;
    if (st < s.n_stars) {
#pragma unroll
      for (int k = 0; k < 5; ++k) gA[5 * st + k] = a[k];
    }
  }
}

// The tail of the regrouped iteration with the segment reduction folded in: the
// five astrometric sums of each star are added from its segments' partials (one
// wave per group of 64 consecutive stars, one star per lane, as k_seg_reduce),
// staged in LDS and turned into the group's 320 new v entries with coalesced
// loads and stores; the attitude, instrumental and global columns come from the
// workgroup windows and the accumulators (as k_tail).  Every column:
// x_j <- v_scale x_j + S_j raw_j / beta.  The last workgroup forms alpha and the
// rotations.
__global__ void __launch_bounds__(kBlock) k_tail_seg(SysView s, BlkView bv, double* __restrict__ x,
                                                     double* __restrict__ acc, const double* __restrict__ S,
                                                     Scalars* sc, Work wk, int lsqr_stage) {
  __shared__ double red[kWavesPerBlock];
  __shared__ double stage[kWavesPerBlock][5 * kWave];
  __shared__ int flag;
  if (sc->done) return;
  const double scale = sc->v_scale, f = sc->inv_beta;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  double sumsq = 0.0;
  if (sc->do_v) {
    double* sg = stage[wid];
    for (int64_t grp = (int64_t)blockIdx.x * kWavesPerBlock + wid; grp < bv.ngroups;
         grp += (int64_t)gridDim.x * kWavesPerBlock) {
      const int32_t* L = bv.grp_list + bv.grp_base[grp] + lane;
      const int32_t cnt = bv.grp_cnt[grp];
      double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      int32_t i = 0;
      for (; i + 4 <= cnt; i += 4) {
        int32_t id[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) id[e] = L[(int64_t)(i + e) * kWave];
        double v[4][5];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int k = 0; k < 5; ++k) v[e][k] = bv.P[5 * (int64_t)id[e] + k];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int k = 0; k < 5; ++k) a[k] += v[e][k];
      }
      for (; i < cnt; ++i) {
        const int32_t id = L[(int64_t)i * kWave];
#pragma unroll
        for (int k = 0; k < 5; ++k) a[k] += bv.P[5 * (int64_t)id + k];
      }
      // the group's 320 columns: element e = 5 (star - 64 grp) + k
#pragma unroll
      for (int k = 0; k < 5; ++k) sg[5 * lane + k] = a[k];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int64_t c0 = 5 * kWave * grp;
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        const int e = r * kWave + lane;
        const int64_t c = c0 + e;
        if (c < s.n_astro) {
          const double xo = (scale == 0.0) ? 0.0 : scale * x[c];
          const double xn = xo + (S ? S[c] : 1.0) * (f * sg[e]);
          x[c] = xn;
          sumsq += xn * xn;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    const int64_t natt = 3 * s.n_att, win = bv.Wb + 3;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < s.tail_len; j += (int64_t)gridDim.x * kBlock) {
      double r = 0.0;
      if (j < natt) {
        // the (at most two) blocks whose window covers column c of axis axs, their
        // workgroups' sums added in workgroup order, sixteen loads in flight
        const int64_t axs = j / s.n_att, c = j - axs * s.n_att;
        const int64_t bhi = min(c / bv.Wb, bv.nb - 1);
        for (int64_t b = max<int64_t>(bhi - 1, 0); b <= bhi; ++b) {
          const int64_t off = c - b * bv.Wb;
          if (off < 0 || off >= win) continue;
          const double* qp = bv.Q + axs * win + off;
          const int64_t qs = 3 * win;
          int32_t q = bv.bsub[b];
          for (; q + 16 <= bv.bsub[b + 1]; q += 16) {
            double v[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = qp[(q + e) * qs];
#pragma unroll
            for (int e = 0; e < 16; ++e) r += v[e];
          }
          for (; q < bv.bsub[b + 1]; ++q) r += qp[q * qs];
        }
      } else {
        r = acc[j];
        acc[j] = 0.0;
      }
      const int64_t c = s.n_astro + j;
      const double xo = (scale == 0.0) ? 0.0 : scale * x[c];
      const double xn = xo + (S ? S[c] : 1.0) * (f * r);
      x[c] = xn;
      sumsq += xn * xn;
    }
  }
  const double bs = block_sum(sumsq, red);
  if (threadIdx.x == 0) publish(wk.part_a + blockIdx.x, bs);
  if (last_block(wk.tickets + T_TAIL, &flag)) {
    const double tot = sum_partials(wk.part_a, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_alpha(sc, tot, lsqr_stage == 0);
      ticket_reset(wk.tickets + T_TAIL);
    }
  }
}

hipError_t launch_tail_seg(const SysView& s, const BlkView& bv, double* x, double* acc, const double* S, Scalars* sc,
                           Work w, hipStream_t st, int lsqr_stage) {
  if (sc == nullptr) return hipErrorInvalidValue;
  // every wave of the grid takes about one group of stars (the segment sums are a
  // chain of dependent loads: many waves keep them in flight), and the tail
  // columns are shared out too
  const int64_t want = std::max<int64_t>((bv.ngroups + kWavesPerBlock - 1) / kWavesPerBlock,
                                         (s.tail_len + kBlock - 1) / kBlock);
  const int blocks = (int)std::min<int64_t>(kPartialSlots, std::max<int64_t>(1, want));
  hipLaunchKernelGGL(k_tail_seg, dim3(blocks), dim3(kBlock), 0, st, s, bv, x, acc, S, sc, w, lsqr_stage);
  return hipGetLastError();
}

hipError_t launch_seg_reduce(const SysView& s, const BlkView& bv, double* gA, Scalars* sc, hipStream_t st) {
  if (s.n_stars == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(16384, (bv.ngroups * kWave + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_seg_reduce, dim3(blocks), dim3(kBlock), 0, st, s, bv, gA, sc);
  return hipGetLastError();
}

}  // namespace gsr
