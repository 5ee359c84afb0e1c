// Constraint equations (Sec. 2: a set of them makes the solution unique): a
// few sparse rows C appended under A, each possibly touching millions of
// unknowns (e.g. a condition over every star).  The rows are cut into tiles
// of at most kConTile entries of one row; a workgroup per tile reduces its
// entries and adds one partial per tile, so a row is summed by many
// workgroups without contention on its accumulator.
#include <algorithm>

#include "device_common.h"

namespace gsr {

// tmp[row] += sum over the tile of val[e] * x[col[e]]
__global__ void __launch_bounds__(kBlock) k_con_dot(ConView c, const double* __restrict__ x, Scalars* sc) {
  __shared__ double red[kWavesPerBlock];
  if (sc && sc->done) return;
  const int64_t t = blockIdx.x;
  const int64_t e0 = c.tile_e[t], e1 = c.tile_e[t + 1];
  double acc = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kBlock) acc += c.val[e] * x[c.col[e]];
  const double bs = block_sum(acc, red);
  if (threadIdx.x == 0) atomicAdd(c.tmp + c.tile_r[t], bs);
}

// y_C <- scale*y_C + ax*tmp; tmp <- 0; the last workgroup stores sum(y_C^2).
__global__ void __launch_bounds__(kBlock) k_con_fin(ConView c, double* __restrict__ yc, double scale, double ax,
                                                    Scalars* sc, Work wk) {
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  if (sc) {
    if (sc->done) return;
    scale = sc->u_scale;
  }
  double ss = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < c.ncon; i += (int64_t)gridDim.x * kBlock) {
    const double y = ((scale == 0.0) ? 0.0 : scale * yc[i]) + ax * c.tmp[i];
    c.tmp[i] = 0.0;
    yc[i] = y;
    ss += y * y;
  }
  if (!sc) return;
  const double bs = block_sum(ss, red);
  if (threadIdx.x == 0) publish(wk.part_c + blockIdx.x, bs);
  if (last_block(wk.tickets + T_CON, &flag)) {
    const double tot = sum_partials(wk.part_c, gridDim.x, red);
    if (threadIdx.x == 0) {
      sc->con_sumsq = tot;
      ticket_reset(wk.tickets + T_CON);
    }
  }
}

// raw[col[e]] += val[e] * yc[row]: the entries of a row are distinct and sorted,
// so the atomics of a wave hit consecutive addresses.
__global__ void __launch_bounds__(kBlock) k_con_scatter(ConView c, int64_t n_astro, const double* __restrict__ yc,
                                                        double* __restrict__ gA, double* __restrict__ acc,
                                                        Scalars* sc, int square) {
  if (sc && (sc->done || !sc->do_v)) return;
  const int64_t t = blockIdx.x;
  const int64_t e0 = c.tile_e[t], e1 = c.tile_e[t + 1];
  const double y = square ? 0.0 : yc[c.tile_r[t]];
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const int64_t j = c.col[e];
    const double v = square ? c.val[e] * c.val[e] : c.val[e] * y;
    if (j < n_astro)
      atomicAdd(gA + j, v);
    else
      atomicAdd(acc + (j - n_astro), v);
  }
}

hipError_t launch_con_aprod1(const ConView& c, const double* x, double* yc, double scale, double ax, Scalars* sc,
                             Work w, hipStream_t st) {
  if (c.ncon == 0) return hipSuccess;
  if (c.ntiles > 0) hipLaunchKernelGGL(k_con_dot, dim3((unsigned)c.ntiles), dim3(kBlock), 0, st, c, x, sc);
  const int blocks = (int)std::min<int64_t>(kMaxPartials, (c.ncon + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_con_fin, dim3(blocks), dim3(kBlock), 0, st, c, yc, scale, ax, sc, w);
  return hipGetLastError();
}

hipError_t launch_con_aprod2(const ConView& c, int64_t n_astro, const double* yc, double* gA, double* acc,
                             Scalars* sc, hipStream_t st) {
  if (c.ncon == 0 || c.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_con_scatter, dim3((unsigned)c.ntiles), dim3(kBlock), 0, st, c, n_astro, yc, gA, acc, sc, 0);
  return hipGetLastError();
}

hipError_t launch_con_sq(const ConView& c, double* sq, hipStream_t st) {
  if (c.ncon == 0 || c.ntiles == 0) return hipSuccess;
  // every column into one array: n_astro = 0 sends all entries to `acc` = sq
  hipLaunchKernelGGL(k_con_scatter, dim3((unsigned)c.ntiles), dim3(kBlock), 0, st, c, (int64_t)0, nullptr, nullptr,
                     sq, nullptr, 1);
  return hipGetLastError();
}

}  // namespace gsr
