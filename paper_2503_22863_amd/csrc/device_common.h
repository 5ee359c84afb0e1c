// Device helpers shared by the kernels: 16-byte streaming loads, wave and
// workgroup reductions, the last-workgroup ticket, and the LSQR scalar
// recurrences (Paige & Saunders 1982) run by that last workgroup.
#pragma once

#include "internal.h"

namespace gsr {

typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef int i2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u4 ld_stream(const u4* p) { return __builtin_nontemporal_load(p); }


// Row tiles are moved in three steps so that the next tile's loads are in
// flight while the current tile is processed:
//   issue_chunks: the tile's nrow (>= 1) rows of CPR 16-byte chunks (starting
//     at chunk pointer g) as contiguous 16-byte nontemporal loads, chunk
//     j*64+lane in register j.  Lanes past the tile's last chunk re-read that
//     chunk, so every load is issued unconditionally: with no branches around
//     them the compiler can count outstanding loads exactly and wait for just
//     the ones it needs (a data-dependent branch makes it wait for all);
//   lds_put: writes those registers to this wave's LDS slab (row stride CPR+1
//     chunks, so that row-per-lane reads are free of bank conflicts); the
//     registers may then take the next tile's loads;
//   lds_get: reads back the lane's own row (zeros past the tile's rows).
template <int CPR>
__device__ __forceinline__ void issue_chunks(const u4* __restrict__ g, int nrow, int lane, u4* tmp) {
  const int last = nrow * CPR - 1;
#pragma unroll
  for (int j = 0; j < CPR; ++j) tmp[j] = ld_stream(g + min(j * kWave + lane, last));
}

template <int CPR>
__device__ __forceinline__ void lds_put(const u4* tmp, int nrow, u4* slab, int lane) {
  const int nch = nrow * CPR;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < CPR; ++j) {
    const int c = j * kWave + lane;
    const int r = c / CPR, q = c - r * CPR;
    if (c < nch) slab[r * (CPR + 1) + q] = tmp[j];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int CPR>
__device__ __forceinline__ void lds_get(int nrow, const u4* slab, int lane, u4* mine) {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int j = 0; j < CPR; ++j) mine[j] = lane < nrow ? slab[lane * (CPR + 1) + j] : u4{0u, 0u, 0u, 0u};
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int CPR>
__device__ __forceinline__ void lds_rows(const u4* tmp, int nrow, u4* slab, int lane, u4* mine) {
  lds_put<CPR>(tmp, nrow, slab, lane);
  lds_get<CPR>(nrow, slab, lane, mine);
}

// Keeps the compiler from moving memory operations across this point (used to
// issue the current tile's gathers before the next tile's prefetch: vector
// loads complete in order, so a later wait on the gathers must not also wait
// on the prefetch).
__device__ __forceinline__ void order_point() { __builtin_amdgcn_sched_barrier(0); }

// Cross-lane moves that bypass the LDS crossbar.  dpp0: a DPP move (GFX9
// controls: row_shr:n = 0x110 + n shifts within rows of 16 lanes; row_bcast:15 =
// 0x142 sends lane 15 of each row to the next row; row_bcast:31 = 0x143 sends
// lane 31 to rows 2 and 3); lanes whose source lies outside their row, and the
// rows left out of ROW_MASK, get 0.  lane_read: the value of lane l (uniform l).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp0(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_read(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t lane_read(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Segmented inclusive sums over the wave: lane l ends with the sum of p over
// lanes seg0(l)..l, where seg0(l) <= l is the first lane of l's segment.  Four
// shifts within rows of 16 lanes, then the row totals: lane 15 into row 1 and
// lane 47 into row 3, lane 31 into rows 2 and 3 (Hillis-Steele over the row
// structure of DPP); a term is added only when its source lane lies in l's
// segment, so every partial stays inside one segment.
template <int OFF, int K>
__device__ __forceinline__ void seg_shift_row(double (&p)[K], bool take) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double o = dpp0<0x110 + OFF, 0xF>(p[k]);
    if (take) p[k] += o;
  }
}

template <int K>
__device__ __forceinline__ void seg_scan(double (&p)[K], int lane, int seg0) {
  seg_shift_row<1>(p, lane - 1 >= seg0);
  seg_shift_row<2>(p, lane - 2 >= seg0);
  seg_shift_row<4>(p, lane - 4 >= seg0);
  seg_shift_row<8>(p, lane - 8 >= seg0);
  const bool t15 = (lane & ~15) - 1 >= seg0, t31 = 31 >= seg0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double o = dpp0<0x142, 0xA>(p[k]);
    if (t15) p[k] += o;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double o = dpp0<0x143, 0xC>(p[k]);
    if (t31) p[k] += o;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum of one double per thread over an NT-thread workgroup, fixed order.
// Every thread gets the result.  Uses `red` (NT / 64 doubles of LDS).
template <int NT = kBlock>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) t += red[i];
  return t;
}

// Cross-workgroup reductions without cache maintenance.  Thread 0 of each
// workgroup publishes its partials with write-through stores (coherent at
// device scope), waits until they are acknowledged, and then draws a ticket;
// the workgroup drawing the last ticket reads all partials with device-coherent
// loads.  Nothing else written in the launch is read by that workgroup, so no
// device-scope fence is needed: on this chip such a fence writes back and
// invalidates the XCD's whole L2, and one per workgroup stalls every wave on it.
__device__ __forceinline__ void publish(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void ticket_reset(unsigned* ticket) {
  __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in the single workgroup that finishes last.  Only thread 0 may
// have published partials before the call.
__device__ __forceinline__ bool last_block(unsigned* ticket, int* flag_lds) {
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's stores are acknowledged
    const unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *flag_lds = (t == gridDim.x - 1);
  }
  __syncthreads();
  return *flag_lds != 0;
}

// Fixed-order sum of `n` partials by the whole (NT-thread) workgroup.
template <int NT = kBlock>
__device__ __forceinline__ double sum_partials(const double* p, int n, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) v += __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return block_sum<NT>(v, red);
}

// ---- LSQR scalar steps (run by one thread) --------------------------------

// beta_{i+1} = ||A v_i - alpha_i u_i|| (or beta_1 = ||b - A x0|| at init).
__device__ inline void epi_beta(Scalars* sc, double sumsq, int init) {
  const double beta = sqrt(sumsq);
  sc->beta = beta;
  if (sc->raw) return;  // standalone product: u_scale, inv_beta and v_scale stay as set
  if (init) {
    sc->bnorm = beta;
    sc->rnorm = beta;
    sc->v_scale = 0.0;  // no previous v
    sc->inv_beta = beta > 0.0 ? 1.0 / beta : 0.0;
    sc->do_v = beta > 0.0;
    if (!(beta > 0.0)) {
      sc->alpha = 0.0;
      sc->arnorm = 0.0;
      sc->istop = 0;
      sc->done = 1;
    }
    return;
  }
  if (beta > 0.0) {
    const double a = sc->alpha;
    sc->anorm2 = sc->anorm2 + a * a + beta * beta + sc->damp * sc->damp;
    sc->inv_beta = 1.0 / beta;
    sc->v_scale = -beta;
    sc->do_v = 1;
  } else {
    sc->do_v = 0;
  }
}

// alpha_{i+1} and the two plane rotations of iteration i.
__device__ inline void epi_alpha(Scalars* sc, double sumsq, int init) {
  if (sc->raw) {  // standalone product: ||x'|| only
    sc->alpha = sqrt(sumsq);
    return;
  }
  if (init) {
    const double alpha = sqrt(sumsq);
    sc->alpha = alpha;
    sc->inv_alpha = alpha > 0.0 ? 1.0 / alpha : 1.0;
    sc->rhobar = alpha;
    sc->phibar = sc->beta;
    sc->arnorm = alpha * sc->beta;
    sc->u_scale = sc->beta > 0.0 ? -alpha / sc->beta : 0.0;
    if (sc->arnorm == 0.0) {
      sc->istop = 0;
      sc->done = 1;
    }
    return;
  }
  if (sc->do_v) {
    const double alpha = sqrt(sumsq);
    sc->alpha = alpha;
    sc->inv_alpha = alpha > 0.0 ? 1.0 / alpha : 1.0;
  } else {
    sc->inv_alpha = 1.0;  // v untouched this iteration
  }
  const double alpha = sc->alpha, beta = sc->beta, damp = sc->damp;
  double rhobar = sc->rhobar, phibar = sc->phibar;
  double rhobar1, psi;
  if (damp > 0.0) {
    rhobar1 = sqrt(rhobar * rhobar + damp * damp);
    const double cs1 = rhobar / rhobar1, sn1 = damp / rhobar1;
    psi = sn1 * phibar;
    phibar = cs1 * phibar;
  } else {
    rhobar1 = rhobar;
    psi = 0.0;
  }
  const double rho = sqrt(rhobar1 * rhobar1 + beta * beta);
  const double cs = rhobar1 / rho, sn = beta / rho;
  const double theta = sn * alpha;
  rhobar = -cs * alpha;
  const double phi = cs * phibar;
  phibar = sn * phibar;
  const double tau = sn * phi;
  sc->rhobar = rhobar;
  sc->phibar = phibar;
  sc->t1 = phi / rho;
  sc->t2 = -theta / rho;
  sc->t3 = 1.0 / rho;
  sc->res2 = sc->res2 + psi * psi;
  sc->rnorm = sqrt(phibar * phibar + sc->res2);
  sc->arnorm = alpha * fabs(tau);
  sc->u_scale = beta > 0.0 ? -alpha / beta : 0.0;
}

// Estimates and stopping tests after the x / w update of iteration i.
__device__ inline void epi_update(Scalars* sc, double xsq, double ddsq) {
  sc->itn = sc->itn + 1;
  sc->xnorm = sqrt(xsq);
  sc->ddnorm = sc->ddnorm + ddsq;
  const double anorm = sqrt(sc->anorm2);
  sc->acond = anorm * sqrt(sc->ddnorm);
  const double bnorm = sc->bnorm, rnorm = sc->rnorm, xnorm = sc->xnorm;
  const double test1 = rnorm / bnorm;
  const double test2 = (anorm * rnorm > 0.0) ? sc->arnorm / (anorm * rnorm) : 0.0;
  const double test3 = (sc->acond > 0.0) ? 1.0 / sc->acond : __builtin_inf();
  const double tt1 = test1 / (1.0 + anorm * xnorm / bnorm);
  const double rtol = sc->btol + sc->atol * anorm * xnorm / bnorm;
  int istop = 0;
  if (sc->itn >= sc->itmax) istop = 7;
  if (1.0 + test3 <= 1.0) istop = 6;
  if (1.0 + test2 <= 1.0) istop = 5;
  if (1.0 + tt1 <= 1.0) istop = 4;
  if (test3 <= sc->ctol) istop = 3;
  if (test2 <= sc->atol) istop = 2;
  if (test1 <= rtol) istop = 1;
  if (istop) {
    sc->istop = istop;
    sc->done = 1;
  }
}

}  // namespace gsr
