// n-sized LSQR passes (initial vectors, the per-iteration x / w / variance
// update, de-preconditioning), the covariance SYRK on FP64 MFMA, and small
// utility kernels.  Scalar recurrences run in the last workgroup of each
// reducing launch (device_common.h), so the host never waits inside a solve.
#include <algorithm>

#include "row_tiles.h"

namespace gsr {

static int blocks_for(int64_t n, int cap = 2048) {
  return (int)std::min<int64_t>(cap, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) p[j] = v;
}

// The scalars of a standalone product pass: u' = u_scale u + A v, then
// x = v_scale x + A^T u' (inv_beta = 1); the epilogues record ||u'|| and ||x|| only.
__global__ void k_raw_scalars(Scalars* sc, double u_scale, double v_scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Scalars h = {};
  h.raw = 1;
  h.u_scale = u_scale;
  h.v_scale = v_scale;
  h.inv_beta = 1.0;
  h.do_v = 1;
  *sc = h;
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) b[j] = a[j];
}

// beta_1 = ||u|| for u = b (or b - A x0); the last workgroup starts the recurrences.
__global__ void __launch_bounds__(kBlock) k_norm_init(const double* __restrict__ u, int64_t m, Scalars* sc, Work wk) {
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  double s = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m; j += (int64_t)gridDim.x * kBlock) {
    const double v = u[j];
    s += v * v;
  }
  const double bs = block_sum(s, red);
  if (threadIdx.x == 0) publish(wk.part_a + blockIdx.x, bs);
  if (last_block(wk.tickets + T_INIT, &flag)) {
    const double tot = sum_partials(wk.part_a, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_beta(sc, tot, 1);
      ticket_reset(wk.tickets + T_INIT);
    }
  }
}

// v_1 = (S A^T u_1) / alpha_1, its scaled copy for the gathers of aprod 1,
// w_1 = v_1, y = 0, var = 0.
__global__ void k_init_vectors(int64_t n, double* __restrict__ v, double* __restrict__ vg, double* __restrict__ w,
                               double* __restrict__ y, double* __restrict__ var, const double* __restrict__ S,
                               const Scalars* sc) {
  const double ia = sc->do_v ? sc->inv_alpha : 1.0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
    const double vj = sc->do_v ? v[j] * ia : 0.0;
    v[j] = vj;
    if (S) vg[j] = S[j] * vj;
    w[j] = vj;
    y[j] = 0.0;
    var[j] = 0.0;
  }
}

// Iteration i, after alpha_{i+1} and the rotations are known:
//   v <- v / alpha_{i+1};  d = w / rho;  y += (phi/rho) w;  var += d^2;
//   w <- v - (theta/rho) w;  partial sums of ||y||^2 and ||d||^2.
// The last workgroup evaluates the stopping tests.
// With an export ring (dring != null, 2*eblock rows of n): d_i is also stored
// whole, in row i mod 2*eblock, where i = sc->itn is read before this launch's
// last workgroup advances it.
__global__ void __launch_bounds__(kBlock) k_update(int64_t n, double* __restrict__ v, double* __restrict__ vg,
                                                   double* __restrict__ w, double* __restrict__ y,
                                                   double* __restrict__ var, const double* __restrict__ S,
                                                   Scalars* sc, Work wk, double* __restrict__ dring,
                                                   int64_t eblock) {
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  if (sc->done) return;
  const double ia = sc->inv_alpha, t1 = sc->t1, t2 = sc->t2, t3 = sc->t3;
  double* drow = dring ? dring + (sc->itn % (2 * eblock)) * n : nullptr;
  double xs = 0.0, ds = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
    const double vj = v[j] * ia;
    v[j] = vj;
    if (S) vg[j] = S[j] * vj;
    const double wj = w[j];
    const double d = t3 * wj;
    if (drow) drow[j] = d;
    const double yj = y[j] + t1 * wj;
    y[j] = yj;
    var[j] = var[j] + d * d;
    w[j] = vj + t2 * wj;
    xs += yj * yj;
    ds += d * d;
  }
  const double bx = block_sum(xs, red);
  const double bd = block_sum(ds, red);
  if (threadIdx.x == 0) {
    publish(wk.part_a + blockIdx.x, bx);
    publish(wk.part_c + blockIdx.x, bd);
  }
  if (last_block(wk.tickets + T_UPDATE, &flag)) {
    const double tx = sum_partials(wk.part_a, gridDim.x, red);
    const double td = sum_partials(wk.part_c, gridDim.x, red);
    if (threadIdx.x == 0) {
      epi_update(sc, tx, td);
      ticket_reset(wk.tickets + T_UPDATE);
    }
  }
}

// x = x0 + S y, var_out = S^2 var (de-preconditioning, the solver's last step).
__global__ void k_finish(int64_t n, const double* __restrict__ y, const double* __restrict__ var,
                         const double* __restrict__ S, const double* __restrict__ x0, double* __restrict__ x,
                         double* __restrict__ vo) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
    const double s = S ? S[j] : 1.0;
    if (x) x[j] = (x0 ? x0[j] : 0.0) + s * y[j];
    if (vo) vo[j] = (s * s) * var[j];
  }
}

// ---------------------------------------------------------------- SYRK
// C += D D^T over the first `cols` columns of D ([k][ldd], row-major), on the
// upper triangle of 32 x 32 tiles of C ([k][k], row-major).  A workgroup owns
// a 64 x 64 tile of C (upper tiles only); its four waves each hold a 32 x 32
// quadrant in 2 x 2 accumulators of v_mfma_f64_16x16x4f64.  The accumulators
// start from the quadrant's C values, loaded before anything else, so the
// read of C from HBM overlaps the staging of D and the MFMA work (C is the
// bulk of the traffic: 2 k^2 / 2 doubles read and written per call, D only
// 2 k cols).  D is staged 32 columns at a time: the 64 rows of the tile's row
// panel and of its column panel go to LDS (row pitch 34 doubles: conflict-free
// 16-byte reads), the next stage's panels are prefetched into registers
// meanwhile (16-byte loads when the row pitch is even).  Inside each
// 16-column half of a stage the k index of MFMA step s for lane group g is
// 4g + s, so each lane reads 4 consecutive doubles of a row; A and B use the
// same order, so the contraction is unchanged.  Four waves per SIMD (the
// register budget is held to 128).
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double dd2 __attribute__((ext_vector_type(2)));  // 16-byte aligned pair (LDS)
constexpr int kSyT = 64;  // C tile per workgroup
constexpr int kSyK = 32;  // D columns per stage
constexpr int kSyP = 34;  // LDS row pitch (doubles)

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_syrk(const double* __restrict__ D, int64_t k, int64_t ldd,
                                                 double* __restrict__ C, Scalars* sc, Work wk, int64_t fixed_cols,
                                                 int64_t T, int64_t ntiles) {
  __shared__ __align__(16) double pa[kSyT * kSyP];
  __shared__ __align__(16) double pb[kSyT * kSyP];
  __shared__ int flag;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t cols = fixed_cols >= 0 ? fixed_cols : (int64_t)sc->dcount;
  const int64_t tile = blockIdx.x;
  if (tile < ntiles && cols > 0) {
    int64_t ti = 0, rem = tile;
    while (rem >= T - ti) {
      rem -= T - ti;
      ++ti;
    }
    const int64_t tj = ti + rem;
    const int64_t r0 = ti * kSyT, c0 = tj * kSyT;
    const int qi = wid >> 1, qj = wid & 1;  // this wave's 32 x 32 quadrant
    const int i16 = lane & 15, g = lane >> 4;
    const bool pairs = (ldd & 1) == 0;  // 16-byte aligned pairs of D (D itself is 256-byte aligned)
    // global -> register staging: thread t moves 16-byte pieces t + 256 h of
    // each 64 x kSyK panel (kSyK / 2 pieces per row)
    constexpr int kPieces = kSyT * kSyK / 2 / kBlock, kRowPieces = kSyK / 2;
    dd2 ra[kPieces], rb[kPieces];
    auto fetch = [&](int64_t kk) {
#pragma unroll
      for (int h = 0; h < kPieces; ++h) {
        const int c = (int)threadIdx.x + h * kBlock, row = c / kRowPieces, part = c % kRowPieces;
        const int64_t col = kk + 2 * part;
        const int64_t ga = r0 + row, gb = c0 + row;
        dd2 va = {0.0, 0.0}, vb = {0.0, 0.0};
        if (pairs && col + 1 < cols) {
          if (ga < k) va = *reinterpret_cast<const dd2*>(D + ga * ldd + col);
          if (gb < k) vb = *reinterpret_cast<const dd2*>(D + gb * ldd + col);
        } else {
          if (ga < k) {
            if (col < cols) va.x = D[ga * ldd + col];
            if (col + 1 < cols) va.y = D[ga * ldd + col + 1];
          }
          if (gb < k) {
            if (col < cols) vb.x = D[gb * ldd + col];
            if (col + 1 < cols) vb.y = D[gb * ldd + col + 1];
          }
        }
        ra[h] = va;
        rb[h] = vb;
      }
    };
    // accumulator layout of the 16x16 f64 result: element e of lane l is row (l/16) + 4e,
    // column l%16.  Only 32 x 32 tiles on or above the diagonal are read and written.
    const int64_t row32 = r0 + 32 * qi, col32 = c0 + 32 * qj;
    const bool mine = row32 <= col32;
    const bool inner = row32 + 32 <= k && col32 + 32 <= k;
    double* cq = C + (row32 + g) * k + col32 + i16;
    d4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
    if (mine && inner) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[bi][bj][e] = cq[(int64_t)(16 * bi + 4 * e) * k + 16 * bj];
    } else if (mine) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row32 + g + 16 * bi + 4 * e < k && col32 + i16 + 16 * bj < k)
              acc[bi][bj][e] = cq[(int64_t)(16 * bi + 4 * e) * k + 16 * bj];
    }
    // the stores below recompute their addresses from here rather than keep the
    // 16 load addresses live across the MFMA loop
    __asm__ volatile("" : "+v"(cq));
    fetch(0);
    for (int64_t kk = 0; kk < cols; kk += kSyK) {
      __syncthreads();  // the previous stage's reads are done
#pragma unroll
      for (int h = 0; h < kPieces; ++h) {
        const int c = (int)threadIdx.x + h * kBlock, row = c / kRowPieces, part = c % kRowPieces;
        *reinterpret_cast<dd2*>(pa + row * kSyP + 2 * part) = ra[h];
        *reinterpret_cast<dd2*>(pb + row * kSyP + 2 * part) = rb[h];
      }
      __syncthreads();
      if (kk + kSyK < cols) fetch(kk + kSyK);
#pragma unroll
      for (int hh = 0; hh < kSyK / 16; ++hh) {
      double av[2][4], bv[2][4];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const double* a = pa + (32 * qi + 16 * bi + i16) * kSyP + 16 * hh + 4 * g;
        const double* b = pb + (32 * qj + 16 * bi + i16) * kSyP + 16 * hh + 4 * g;
        const dd2 a01 = *reinterpret_cast<const dd2*>(a), a23 = *reinterpret_cast<const dd2*>(a + 2);
        const dd2 b01 = *reinterpret_cast<const dd2*>(b), b23 = *reinterpret_cast<const dd2*>(b + 2);
        av[bi][0] = a01.x;
        av[bi][1] = a01.y;
        av[bi][2] = a23.x;
        av[bi][3] = a23.y;
        bv[bi][0] = b01.x;
        bv[bi][1] = b01.y;
        bv[bi][2] = b23.x;
        bv[bi][3] = b23.y;
      }
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi][st], bv[bj][st], acc[bi][bj], 0, 0, 0);
      }
    }
    if (mine) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (inner || (row32 + g + 16 * bi + 4 * e < k && col32 + i16 + 16 * bj < k))
              cq[(int64_t)(16 * bi + 4 * e) * k + 16 * bj] = acc[bi][bj][e];
    }
  }
  if (fixed_cols < 0) {
    if (last_block(wk.tickets + T_SYRK, &flag) && threadIdx.x == 0) {
      sc->dcount = 0;
      ticket_reset(wk.tickets + T_SYRK);
    }
  }
}

// d_i[sel] = w_i[sel] / rho_i as column dcount of D ([nsel][dblock]).
__global__ void __launch_bounds__(kBlock) k_cov_gather(int64_t nsel, const int64_t* __restrict__ sel,
                                                       const double* __restrict__ w, double* __restrict__ D,
                                                       Scalars* sc, Work wk) {
  __shared__ int flag;
  if (sc->done) return;
  const int64_t cols = sc->dcount, ld = sc->dblock;
  if (cols >= ld) return;
  const double t3 = sc->t3;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nsel; p += (int64_t)gridDim.x * kBlock)
    D[p * ld + cols] = t3 * w[sel[p]];
  if (last_block(wk.tickets + T_GATHER, &flag) && threadIdx.x == 0) {
    sc->dcount = (int32_t)(cols + 1);
    ticket_reset(wk.tickets + T_GATHER);
  }
}

// Covariances for a list of pairs (version 2 of the covariance pipeline,
// Sec. 2.2: (j1, j2) index pairs rather than a dense block):
// Cp[p] += sum_{c < cols} D[a_p][c] D[b_p][c], 16 lanes per pair.
__global__ void __launch_bounds__(kBlock) k_pairdot(const double* __restrict__ D, int64_t ldd,
                                                    const int32_t* __restrict__ pa, const int32_t* __restrict__ pb,
                                                    int64_t P, double* __restrict__ Cp, Scalars* sc, Work wk,
                                                    int64_t fixed_cols) {
  __shared__ int flag;
  const int64_t cols = fixed_cols >= 0 ? fixed_cols : (int64_t)sc->dcount;
  const int l = threadIdx.x & 15;
  constexpr int kPerBlock = kBlock / 16;
  if (cols > 0) {
    for (int64_t p0 = (int64_t)blockIdx.x * kPerBlock; p0 < P; p0 += (int64_t)gridDim.x * kPerBlock) {
      const int64_t p = p0 + threadIdx.x / 16;
      double acc = 0.0;
      if (p < P) {
        const double* da = D + (int64_t)pa[p] * ldd;
        const double* db = D + (int64_t)pb[p] * ldd;
        for (int64_t c = l; c < cols; c += 16) acc += da[c] * db[c];
      }
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 16);
      if (p < P && l == 0) Cp[p] += acc;
    }
  }
  if (fixed_cols < 0) {
    if (last_block(wk.tickets + T_SYRK, &flag) && threadIdx.x == 0) {
      sc->dcount = 0;
      ticket_reset(wk.tickets + T_SYRK);
    }
  }
}

// out[p] = s_{sel[a_p]} s_{sel[b_p]} Cp[p]
__global__ void k_pair_out(const double* __restrict__ Cp, int64_t P, const int32_t* __restrict__ pa,
                           const int32_t* __restrict__ pb, const double* __restrict__ S,
                           const int64_t* __restrict__ sel, double* __restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P; p += (int64_t)gridDim.x * kBlock)
    out[p] = (S ? S[sel[pa[p]]] * S[sel[pb[p]]] : 1.0) * Cp[p];
}

// out[p][q] = s_p s_q C[min(p,q)][max(p,q)], s = column scaling at the selected unknowns.
__global__ void k_cov_out(const double* __restrict__ C, int64_t k, const double* __restrict__ S,
                          const int64_t* __restrict__ sel, double* __restrict__ out) {
  const int64_t n = k * k;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
    const int64_t p = e / k, q = e - p * k;
    const double c = (p <= q) ? C[p * k + q] : C[q * k + p];
    const double s = S ? S[sel[p]] * S[sel[q]] : 1.0;
    out[e] = s * c;
  }
}

// End of an outer refinement step: x <- x_new, partial ||x_new - x||^2 and ||x_new||^2.
__global__ void __launch_bounds__(kBlock) k_step_norms(int64_t n, const double* __restrict__ xn,
                                                       double* __restrict__ x, double* out2, Work wk) {
  __shared__ double red[kWavesPerBlock];
  __shared__ int flag;
  double a = 0.0, b = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
    const double v = xn[j];
    const double d = v - x[j];
    x[j] = v;
    a += d * d;
    b += v * v;
  }
  const double ba = block_sum(a, red);
  const double bb = block_sum(b, red);
  if (threadIdx.x == 0) {
    publish(wk.part_a + blockIdx.x, ba);
    publish(wk.part_c + blockIdx.x, bb);
  }
  if (last_block(wk.tickets + T_VALID, &flag)) {
    const double ta = sum_partials(wk.part_a, gridDim.x, red);
    const double tb = sum_partials(wk.part_c, gridDim.x, red);
    if (threadIdx.x == 0) {
      out2[0] = ta;
      out2[1] = tb;
      ticket_reset(wk.tickets + T_VALID);
    }
  }
}

__global__ void k_scaled_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n, double s) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) b[j] = s * a[j];
}

// ------------------------------------------------------------ launchers
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_raw_scalars(Scalars* sc, double u_scale, double v_scale, hipStream_t st) {
  hipLaunchKernelGGL(k_raw_scalars, dim3(1), dim3(64), 0, st, sc, u_scale, v_scale);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(kBlock), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_norm_init(const double* u, int64_t m, Scalars* sc, Work w, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_init, dim3(blocks_for(m)), dim3(kBlock), 0, st, u, m, sc, w);
  return hipGetLastError();
}

hipError_t launch_init_vectors(int64_t n, double* v, double* vg, double* w, double* y, double* var, const double* S,
                               Scalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_init_vectors, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, v, vg, w, y, var, S, sc);
  return hipGetLastError();
}

hipError_t launch_update(int64_t n, double* v, double* vg, double* w, double* y, double* var, const double* S,
                         Scalars* sc, Work w_, hipStream_t st, double* dring, int64_t eblock) {
  hipLaunchKernelGGL(k_update, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, v, vg, w, y, var, S, sc, w_, dring,
                     eblock);
  return hipGetLastError();
}

hipError_t launch_finish(int64_t n, const double* y, const double* var, const double* S, const double* x0,
                         double* x_out, double* var_out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finish, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, y, var, S, x0, x_out, var_out);
  return hipGetLastError();
}

hipError_t launch_syrk(const double* D, int64_t k, int64_t ldd, double* C, Scalars* sc, Work w, int64_t fixed_cols,
                       hipStream_t st) {
  const int64_t T = (k + kSyT - 1) / kSyT;
  const int64_t ntiles = T * (T + 1) / 2;
  const int64_t blocks = std::max<int64_t>(1, ntiles);
  hipLaunchKernelGGL(k_syrk, dim3((unsigned)blocks), dim3(kBlock), 0, st, D, k, ldd, C, sc, w, fixed_cols, T,
                     ntiles);
  return hipGetLastError();
}

hipError_t launch_cov_gather(int64_t nsel, const int64_t* sel, const double* w, double* D, Scalars* sc, Work wk,
                             hipStream_t st) {
  if (nsel <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cov_gather, dim3(blocks_for(nsel)), dim3(kBlock), 0, st, nsel, sel, w, D, sc, wk);
  return hipGetLastError();
}

hipError_t launch_pairdot(const double* D, int64_t ldd, const int32_t* pa, const int32_t* pb, int64_t P, double* Cp,
                          Scalars* sc, Work w, int64_t fixed_cols, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>(kMaxPartials, std::max<int64_t>(1, (P + kBlock / 16 - 1) / (kBlock / 16)));
  hipLaunchKernelGGL(k_pairdot, dim3((unsigned)blocks), dim3(kBlock), 0, st, D, ldd, pa, pb, P, Cp, sc, w,
                     fixed_cols);
  return hipGetLastError();
}

hipError_t launch_pair_out(const double* Cp, int64_t P, const int32_t* pa, const int32_t* pb, const double* S,
                           const int64_t* sel, double* out, hipStream_t st) {
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_out, dim3(blocks_for(P)), dim3(kBlock), 0, st, Cp, P, pa, pb, S, sel, out);
  return hipGetLastError();
}

hipError_t launch_cov_out(const double* C, int64_t k, const double* S, const int64_t* sel, double* out,
                          hipStream_t st) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cov_out, dim3(blocks_for(k * k)), dim3(kBlock), 0, st, C, k, S, sel, out);
  return hipGetLastError();
}

hipError_t launch_step_norms(int64_t n, const double* xn, double* x, double* out2, Work w, hipStream_t st) {
  hipLaunchKernelGGL(k_step_norms, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, xn, x, out2, w);
  return hipGetLastError();
}

hipError_t launch_scaled_copy(const double* src, double* dst, int64_t n, double s, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scaled_copy, dim3(blocks_for(n)), dim3(kBlock), 0, st, src, dst, n, s);
  return hipGetLastError();
}

}  // namespace gsr
