// Memory-system calibration for the row pass (a standalone program, not part
// of libgsr): streams exactly the regrouped pass's per-row bytes — 64-row tiles
// of 12 chunk-major 16-byte chunks (FP64 coefficients; 6 for FP32), a 16-byte
// record and an 8-byte u per row, one tile prefetched (or two), 8 waves per
// workgroup and one workgroup per CU (the pass's LDS footprint) — with the
// per-row u store in several forms, to show what a pass that must write u can
// reach on this chip.
//
//   stream_probe [rows]      (default 70,004,736: the 10^6-star share)
//
// One JSON object per line: {"chunks": ..., "depth": ..., "store": ..., "ms": ...,
// "read_GBps": ...}.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

typedef unsigned u4 __attribute__((ext_vector_type(4)));

#define CHK(x)                                                                        \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      fprintf(stderr, "stream_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      exit(1);                                                                        \
    }                                                                                 \
  } while (0)

constexpr int kMaxChunks = 12;  // 16-byte chunks per row (24 FP64 coefficients; 6 for FP32)
constexpr int kWaves = 8;       // waves per workgroup
constexpr int kStage = 16;      // tiles per burst in the LDS-staged form
constexpr int kSeg = 35;        // values per tile of the second stream (7 segment sums of 5)

// Two tiles ahead: tiles in pairs, each pair's loads issued while the other
// pair member is consumed (no register copy of loads still in flight).
template <int CH, bool STORE>
__global__ void __launch_bounds__(kWaves * 64) k_stream2(const u4* __restrict__ T, const u4* __restrict__ R,
                                                          double* __restrict__ u, double* __restrict__ p, long ntiles,
                                                          double* sink) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long W = (long)gridDim.x * kWaves, w = (long)blockIdx.x * kWaves + wid;
  const long t0 = ntiles * w / W, t1 = ntiles * (w + 1) / W;
  double acc = 0.0;
  if (t0 < t1) {
    struct Buf {
      u4 c[CH];
      u4 rec;
      double uo;
    };
    auto fetch = [&](Buf& b, long t) {
      const long tt = t < t1 ? t : t0;  // past the range: re-read its first tile (unused)
      const u4* base = T + tt * CH * 64 + lane;
#pragma unroll
      for (int j = 0; j < CH; ++j) b.c[j] = __builtin_nontemporal_load(base + j * 64);
      b.rec = __builtin_nontemporal_load(R + tt * 64 + lane);
      b.uo = u[tt * 64 + lane];
    };
    long r_out = -1;
    double u_out = 0.0;
    auto consume = [&](const Buf& b, long t) {
      if (STORE && r_out >= 0) u[r_out] = u_out;
      double s = b.uo + (double)b.rec.x;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const double2 d = *reinterpret_cast<const double2*>(&b.c[j]);
        s += d.x * 1.0000001 + d.y;
      }
      r_out = t * 64 + lane;
      u_out = s;
      acc += s;
    };
    Buf X, Y, cur;
    fetch(X, t0);
    fetch(Y, t0 + 1);
    long t = t0;
    for (; t + 1 < t1; t += 2) {
      cur = X;
      __builtin_amdgcn_sched_barrier(0);
      fetch(X, t + 2);
      __builtin_amdgcn_sched_barrier(0);
      consume(cur, t);
      cur = Y;
      __builtin_amdgcn_sched_barrier(0);
      fetch(Y, t + 3);
      __builtin_amdgcn_sched_barrier(0);
      consume(cur, t + 1);
    }
    if (t < t1) consume(X, t);
    if (STORE && r_out >= 0) u[r_out] = u_out;
  }
  if (acc == 1.2345) sink[0] = acc;  // keeps the sums live
}

// Store forms: 0 none, 1 plain, 2 nontemporal, 3 into a 1 MB wrap-around buffer
// (never reaches HBM), 4 from every fourth wave only, 5 staged in LDS and
// written kStage tiles at a time; with a second stream of kSeg values per tile
// (the size of a tile's segment sums): 6 into a buffer of its own beside u,
// 7 interleaved with u in one buffer (u of a tile, then its kSeg values), so
// that each wave writes one sequential stream of the same bytes as in 6.
template <int kChunks, int STORE>
__global__ void __launch_bounds__(kWaves * 64) k_stream(const u4* __restrict__ T, const u4* __restrict__ R,
                                                         double* __restrict__ u, double* __restrict__ p, long ntiles,
                                                         double* sink) {
  extern __shared__ double lds[];  // sized to leave one workgroup per CU
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long W = (long)gridDim.x * kWaves, w = (long)blockIdx.x * kWaves + wid;
  const long t0 = ntiles * w / W, t1 = ntiles * (w + 1) / W;
  double acc = 0.0;
  if (t0 < t1) {
    u4 tmp[kChunks];
    u4 rec;
    double uo;
    auto fetch = [&](long t) {
      const long tt = t < t1 ? t : t0;  // past the range: re-read its first tile (unused)
      const u4* base = T + tt * kChunks * 64 + lane;
#pragma unroll
      for (int j = 0; j < kChunks; ++j) tmp[j] = __builtin_nontemporal_load(base + j * 64);
      rec = __builtin_nontemporal_load(R + tt * 64 + lane);
      uo = u[tt * 64 + lane];
    };
    fetch(t0);
    long r_out = -1;
    double u_out = 0.0;
    for (long t = t0; t < t1; ++t) {
      u4 cur[kChunks];
#pragma unroll
      for (int j = 0; j < kChunks; ++j) cur[j] = tmp[j];
      const u4 rc = rec;
      const double uc = uo;
      __builtin_amdgcn_sched_barrier(0);
      fetch(t + 1);
      __builtin_amdgcn_sched_barrier(0);
      if (r_out >= 0) {
        if (STORE == 1) u[r_out] = u_out;
        if (STORE == 2) __builtin_nontemporal_store(u_out, u + r_out);
        if (STORE == 3) u[r_out & ((1 << 17) - 1)] = u_out;
        if (STORE == 4 && (w & 3) == 0) u[r_out] = u_out;
        if (STORE == 6) {
          u[r_out] = u_out;
          p[lane < kSeg ? (r_out >> 6) * kSeg + lane : ntiles * kSeg + w * 64 + lane] = u_out;
        }
        if (STORE == 7) {
          constexpr int kRun = 64 + kSeg;
          p[(r_out >> 6) * kRun + lane] = u_out;
          p[lane < kSeg ? (r_out >> 6) * kRun + 64 + lane : ntiles * kRun + w * 64 + lane] = u_out;
        }
        if (STORE == 5) {
          double* st = lds + wid * kStage * 64;
          const long k = (t - 1 - t0) % kStage;
          st[k * 64 + lane] = u_out;
          if (k == kStage - 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const long base = r_out - lane - (kStage - 1) * 64;
#pragma unroll
            for (int q = 0; q < kStage; ++q) u[base + q * 64 + lane] = st[q * 64 + lane];
          }
        }
      }
      double s = uc + (double)rc.x;
#pragma unroll
      for (int j = 0; j < kChunks; ++j) {
        const double2 d = *reinterpret_cast<const double2*>(&cur[j]);
        s += d.x * 1.0000001 + d.y;
      }
      r_out = t * 64 + lane;
      u_out = s;
      acc += s;
    }
    if ((STORE == 1 || STORE == 2) && r_out >= 0) u[r_out] = u_out;
  }
  if (acc == 1.2345) sink[0] = acc;  // keeps the sums live
}

template <typename K>
static void run(K kernel, int chunks, int depth, const char* name, const u4* T, const u4* R, double* u, double* p,
                long ntiles, double* sink, int blocks, size_t lds) {
  (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  hipEvent_t a, b;
  CHK(hipEventCreate(&a));
  CHK(hipEventCreate(&b));
  for (int i = 0; i < 2; ++i)
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kWaves * 64), lds, 0, T, R, u, p, ntiles, sink);
  CHK(hipGetLastError());
  const int reps = 10;
  CHK(hipEventRecord(a));
  for (int i = 0; i < reps; ++i)
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kWaves * 64), lds, 0, T, R, u, p, ntiles, sink);
  CHK(hipEventRecord(b));
  CHK(hipEventSynchronize(b));
  float ms = 0.0f;
  CHK(hipEventElapsedTime(&ms, a, b));
  ms /= reps;
  const double read = (double)ntiles * 64 * (chunks * 16 + 16 + 8);
  printf("{\"chunks\": %d, \"depth\": %d, \"store\": \"%s\", \"rows\": %ld, \"ms\": %.4f, \"read_GBps\": %.1f}\n",
         chunks, depth, name, ntiles * 64, ms, read / (ms * 1e-3) / 1e9);
  fflush(stdout);
  CHK(hipEventDestroy(a));
  CHK(hipEventDestroy(b));
}

int main(int argc, char** argv) {
  const long rows = argc > 1 ? atol(argv[1]) : 70004736L;
  const long ntiles = (rows + 63) / 64;
  if (ntiles < 1) return 1;
  int dev = 0, cus = 256, lmax = 65536;
  CHK(hipGetDevice(&dev));
  CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  CHK(hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // more than half of a CU's LDS per workgroup: one workgroup of 8 waves per CU
  const size_t lds = (size_t)lmax * 3 / 4;
  if (lds < sizeof(double) * kWaves * kStage * 64) return 1;
  u4 *T, *R;
  double *u, *p, *sink;
  const int blocks = 2 * cus;
  const size_t pn = (size_t)ntiles * (64 + kSeg) + (size_t)blocks * kWaves * 64;  // forms 6 and 7
  CHK(hipMalloc(&T, (size_t)ntiles * 64 * kMaxChunks * 16));
  CHK(hipMalloc(&R, (size_t)ntiles * 64 * 16));
  CHK(hipMalloc(&u, (size_t)ntiles * 64 * 8));
  CHK(hipMalloc(&p, pn * 8));
  CHK(hipMemset(p, 0, pn * 8));
  CHK(hipMalloc(&sink, 64));
  CHK(hipMemset(T, 0, (size_t)ntiles * 64 * kMaxChunks * 16));
  CHK(hipMemset(R, 0, (size_t)ntiles * 64 * 16));
  CHK(hipMemset(u, 0, (size_t)ntiles * 64 * 8));
  CHK(hipDeviceSynchronize());
  // FP64 rows, one tile ahead, every store form
  run(k_stream<12, 0>, 12, 1, "none", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<12, 1>, 12, 1, "plain", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<12, 2>, 12, 1, "nontemporal", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<12, 3>, 12, 1, "1 MB wrap-around buffer", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<12, 4>, 12, 1, "every fourth wave only", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<12, 5>, 12, 1, "LDS-staged, 16 tiles per burst", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<12, 6>, 12, 1, "u + 35 values per tile, two streams", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<12, 7>, 12, 1, "u + 35 values per tile, one merged stream", T, R, u, p, ntiles, sink, blocks, lds);
  // two tiles ahead; FP32 rows one and two tiles ahead
  run(k_stream2<12, true>, 12, 2, "plain", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<6, 0>, 6, 1, "none", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream<6, 1>, 6, 1, "plain", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream2<6, false>, 6, 2, "none", T, R, u, p, ntiles, sink, blocks, lds);
  run(k_stream2<6, true>, 6, 2, "plain", T, R, u, p, ntiles, sink, blocks, lds);
  CHK(hipFree(T));
  CHK(hipFree(R));
  CHK(hipFree(u));
  CHK(hipFree(p));
  CHK(hipFree(sink));
  return 0;
}
