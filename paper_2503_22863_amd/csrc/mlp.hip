// Learned warm start: per-star features of an observation system and a small
// FP32 MLP (two ReLU hidden layers) trained with full-batch Adam, all on the
// device.  The network maps the features of a star (its 5x5 normal-matrix
// block, the projected known terms, summary statistics of its rows) to the
// star's 5 astrometric unknowns, giving x0 for a warm-started LSQR.
#include <algorithm>

#include "device_common.h"

namespace gsr {

constexpr int kFeat = 28;

// ---------------------------------------------------------------- features
// One thread per star (features are computed once per system).  FP64.
//   [0..14] upper triangle of A_s^T A_s (row-major), A_s = the star's rows on its
//           5 astrometric columns; [15..19] A_s^T bt with bt = b - A_other xo;
//   [20] rows; [21] mean(att_start)/n_att; [22] std(att_start/n_att);
//   [23] rms attitude coefficient; [24] rms instrumental; [25] rms global;
//   [26] ||bt_s|| / sqrt(rows); [27] sum(a_glob * bt) / rows.
template <typename VT>
__global__ void k_features(SysView s, const double* __restrict__ b, const double* __restrict__ xo,
                           double* __restrict__ F) {
  const int64_t st = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (st >= s.n_stars) return;
  const VT* V = reinterpret_cast<const VT*>(s.vals);
  double f[kFeat];
#pragma unroll
  for (int i = 0; i < kFeat; ++i) f[i] = 0.0;
  const int64_t r0 = s.row_ptr[st], r1 = s.row_ptr[st + 1];
  const double rows = (double)(r1 - r0);
  double* out = F + kFeat * st;
  if (r1 <= r0) {
    for (int i = 0; i < kFeat; ++i) out[i] = 0.0;
    return;
  }
  const double inv_natt = 1.0 / (double)s.n_att;
  double mean_att = 0.0;
  for (int64_t r = r0; r < r1; ++r) mean_att += (double)s.att_start[r] * inv_natt;
  mean_att /= rows;
  const int64_t tin = 3 * s.n_att;  // instrumental offset inside xo
  double var_att = 0.0, sq_att = 0.0, sq_ins = 0.0, sq_glb = 0.0, sq_bt = 0.0, gb = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    double a[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) a[k] = (double)V[kSlots * r + k];
    const int32_t at = s.att_start[r];
    double bt = b[r];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int j = 0; j < 4; ++j) bt -= a[5 + 4 * ax + j] * xo[ax * s.n_att + at + j];
#pragma unroll
    for (int q = 0; q < 6; ++q) bt -= a[17 + q] * xo[tin + s.instr_col[6 * r + q]];
    if (s.n_glob) bt -= a[23] * xo[tin + s.n_instr];
    int q = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int l = k; l < 5; ++l) f[q++] += a[k] * a[l];
#pragma unroll
    for (int k = 0; k < 5; ++k) f[15 + k] += a[k] * bt;
    const double da = (double)at * inv_natt - mean_att;
    var_att += da * da;
#pragma unroll
    for (int k = 5; k < 17; ++k) sq_att += a[k] * a[k];
#pragma unroll
    for (int k = 17; k < 23; ++k) sq_ins += a[k] * a[k];
    if (s.n_glob) {
      sq_glb += a[23] * a[23];
      gb += a[23] * bt;
    }
    sq_bt += bt * bt;
  }
  f[20] = rows;
  f[21] = mean_att;
  f[22] = sqrt(var_att / rows);
  f[23] = sqrt(sq_att / (12.0 * rows));
  f[24] = sqrt(sq_ins / (6.0 * rows));
  f[25] = sqrt(sq_glb / rows);
  f[26] = sqrt(sq_bt / rows);
  f[27] = gb / rows;
  for (int i = 0; i < kFeat; ++i) out[i] = f[i];
}

hipError_t launch_features(const SysView& s, const double* b, const double* xo, double* F, hipStream_t st) {
  if (s.n_stars == 0) return hipSuccess;
  const int blocks = (int)((s.n_stars + kBlock - 1) / kBlock);
  if (s.value_type == GSR_F32)
    hipLaunchKernelGGL(k_features<float>, dim3(blocks), dim3(kBlock), 0, st, s, b, xo, F);
  else
    hipLaunchKernelGGL(k_features<double>, dim3(blocks), dim3(kBlock), 0, st, s, b, xo, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------- MLP
// Column mean and population standard deviation (1 where it is 0) of a
// [N][C] FP64 matrix; one thread per column (C is small).
__global__ void k_col_stats(const double* __restrict__ X, int64_t N, int C, double* __restrict__ mu,
                            double* __restrict__ sd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double m = 0.0;
  for (int64_t i = 0; i < N; ++i) m += X[i * C + c];
  m = N > 0 ? m / (double)N : 0.0;
  double v = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const double d = X[i * C + c] - m;
    v += d * d;
  }
  v = N > 0 ? sqrt(v / (double)N) : 0.0;
  mu[c] = m;
  sd[c] = v > 0.0 ? v : 1.0;
}

// Xs = fl32((X - mu) / sd)
__global__ void k_standardize(const double* __restrict__ X, int64_t N, int C, const double* __restrict__ mu,
                              const double* __restrict__ sd, float* __restrict__ Xs) {
  const int64_t total = N * C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    Xs[e] = (float)((X[e] - mu[c]) / sd[c]);
  }
}

// Y = Ys * sd + mu, written to FP64.
__global__ void k_destandardize(const float* __restrict__ Ys, int64_t N, int C, const double* __restrict__ mu,
                                const double* __restrict__ sd, double* __restrict__ Y) {
  const int64_t total = N * C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    Y[e] = (double)Ys[e] * sd[c] + mu[c];
  }
}

// Tiled FP32 GEMM with strided operands, on the matrix cores:
//   C(m, n) = sum_k A(m, k) B(k, n) [+ bias(n)] [then ReLU] [times (mask(m, n) > 0)]
// A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn], C row-major with ldc.
// A 64 x 64 tile per 256-thread workgroup, K in steps of 16 through LDS; each
// wave holds a 32 x 32 quadrant in 2 x 2 accumulators of v_mfma_f32_16x16x4f32
// (per instruction lane l gives A(row l%16, k l/16) and B(k l/16, column l%16);
// element r of the result is row 4 (l/16) + r, column l%16).  gridDim.z > 1
// splits K; partial tiles are added with atomics into a C cleared beforehand.
typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int qi = wid >> 1, qj = wid & 1, i16 = lane & 15, grp = lane >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int splits = gridDim.z;
  const int kper = ((g.K + splits - 1) / splits + 15) / 16 * 16;
  const int kbeg = blockIdx.z * kper, kend = min(g.K, kbeg + kper);
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    // 1024 elements of each tile, 4 per thread
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int kk = idx >> 6, mm = idx & 63;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < g.M && gk < kend) ? g.A[(int64_t)gm * g.sam + (int64_t)gk * g.sak] : 0.f;
      const int gn = n0 + mm;
      Bs[kk][mm] = (gn < g.N && gk < kend) ? g.B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kk = 4 * s4 + grp;
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk][32 * qi + 16 * i + i16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][32 * qj + 16 * j + i16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + 32 * qi + 16 * i + 4 * grp + r;
      if (gm >= g.M) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gn = n0 + 32 * qj + 16 * j + i16;
        if (gn >= g.N) continue;
        const int64_t o = (int64_t)gm * g.ldc + gn;
        if (splits > 1) {
          atomicAdd(g.C + o, acc[i][j][r]);
          continue;
        }
        float z = acc[i][j][r] + (g.bias ? g.bias[gn] : 0.f);
        if (g.Zout) g.Zout[o] = z;
        if (g.relu) z = fmaxf(z, 0.f);
        if (g.mask) z = g.mask[o] > 0.f ? z : 0.f;
        g.C[o] = z;
      }
    }
}

// dY = 2 (Y - T) / (N*O) and the loss mean((Y - T)^2) (loss accumulated in FP64).
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t total, float* __restrict__ dY,
                      double* loss) {
  __shared__ double red[kWavesPerBlock];
  double s = 0.0;
  const float scale = 2.0f / (float)total;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    const float d = Y[e] - T[e];
    dY[e] = scale * d;
    s += (double)d * (double)d;
  }
  const double bs = block_sum(s, red);
  if (threadIdx.x == 0 && loss) atomicAdd(loss, bs / (double)total);
}

// db(n) = sum_m dZ(m, n)
__global__ void k_colsum(const float* __restrict__ dZ, int64_t M, int N, float* __restrict__ db) {
  const int n = blockIdx.x;
  float s = 0.f;
  for (int64_t m = threadIdx.x; m < M; m += blockDim.x) s += dZ[m * N + n];
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[n] = red[0];
}

// Adam with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_fill_f(float* __restrict__ p, int64_t n, float val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void k_mean_rows(const double* __restrict__ X, int64_t k, int64_t len, double* __restrict__ out) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < len; j += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) s += X[i * len + j];
    out[j] = s / (double)k;
  }
}

// ------------------------------------------------------------ launchers
static int grid_for(int64_t n) { return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

hipError_t mlp_col_stats(const double* X, int64_t N, int C, double* mu, double* sd, hipStream_t st) {
  hipLaunchKernelGGL(k_col_stats, dim3((C + 63) / 64), dim3(64), 0, st, X, N, C, mu, sd);
  return hipGetLastError();
}
hipError_t mlp_standardize(const double* X, int64_t N, int C, const double* mu, const double* sd, float* Xs,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_standardize, dim3(grid_for(N * C)), dim3(256), 0, st, X, N, C, mu, sd, Xs);
  return hipGetLastError();
}
hipError_t mlp_destandardize(const float* Ys, int64_t N, int C, const double* mu, const double* sd, double* Y,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_destandardize, dim3(grid_for(N * C)), dim3(256), 0, st, Ys, N, C, mu, sd, Y);
  return hipGetLastError();
}
hipError_t mlp_gemm(const GemmArgs& g, int splits, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (splits > 1)
    hipLaunchKernelGGL(k_fill_f, dim3(grid_for((int64_t)g.M * g.ldc)), dim3(256), 0, st, g.C, (int64_t)g.M * g.ldc,
                       0.f);
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}
hipError_t mlp_mse(const float* Y, const float* T, int64_t total, float* dY, double* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(std::min(grid_for(total), 1024)), dim3(kBlock), 0, st, Y, T, total, dY, loss);
  return hipGetLastError();
}
hipError_t mlp_colsum(const float* dZ, int64_t M, int N, float* db, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3(N), dim3(256), 0, st, dZ, M, N, db);
  return hipGetLastError();
}
hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t mlp_fill(float* p, int64_t n, float val, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f, dim3(grid_for(n)), dim3(256), 0, st, p, n, val);
  return hipGetLastError();
}
hipError_t launch_mean_rows(const double* X, int64_t k, int64_t len, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mean_rows, dim3(grid_for(len)), dim3(256), 0, st, X, k, len, out);
  return hipGetLastError();
}

}  // namespace gsr
