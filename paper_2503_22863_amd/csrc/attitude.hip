// Attitude part of aprod 2 (Sec. 2, Eq. 3) without global atomics.
//
// Rows are stored in star order, and the 12 attitude coefficients of a row
// land on 3 x 4 consecutive columns starting at a random att_start, so a
// star-ordered pass would need 12 scattered FP64 atomics per row (measured on
// MI355X at ~2e10 atomics/s, far below the HBM stream).  Instead the handle
// keeps, once per system, a copy of the attitude coefficients grouped by
// attitude bucket b = att_start / Wb, and a row-order copy of the other twelve
// coefficients for the star pass of aprod 2 (which then streams half a row).
// Each product then
//   1. permutes u into the same order (partition pass: one workgroup per
//      chunk of K rows stages the chunk's u in LDS by bucket and writes one
//      contiguous run per bucket), and
//   2. sums, per workgroup, a bucket range of rows into an LDS window of
//      3 x (Wb + 3) columns (ds_add_f64) and stores the window once.
// The tail pass adds the (at most two) windows that cover each column.
#include <algorithm>
#include <vector>

#include "device_common.h"

namespace gsr {

template <typename VT>
struct AttGeo;
template <>
struct AttGeo<double> {
  static constexpr int CPR = 6;  // 12 doubles = 96 B = 6 chunks
};
template <>
struct AttGeo<float> {
  static constexpr int CPR = 3;  // 12 floats = 48 B
};

// ------------------------------------------------------------------ build
__global__ void k_bk_count(SysView s, AttView av) {
  extern __shared__ int hist_i[];
  const int64_t c = blockIdx.x;
  for (int64_t b = threadIdx.x; b < av.nb; b += blockDim.x) hist_i[b] = 0;
  __syncthreads();
  const int64_t r0 = c * av.K, r1 = min(s.m, r0 + av.K);
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) atomicAdd(hist_i + s.att_start[r] / av.Wb, 1);
  __syncthreads();
  for (int64_t b = threadIdx.x; b < av.nb; b += blockDim.x) av.count[c * av.nb + b] = hist_i[b];
}

// lst[c][b] = rows of chunk c in buckets before b (local start of bucket b's run)
__global__ void k_bk_lstart(AttView av) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= av.nchunks) return;
  int32_t run = 0;
  for (int64_t b = 0; b < av.nb; ++b) {
    av.lst[c * (av.nb + 1) + b] = run;
    run += av.count[c * av.nb + b];
  }
  av.lst[c * (av.nb + 1) + av.nb] = run;
}

// cbase[c][b] = rows of bucket b in chunks before c; btot[b] = rows of bucket b
__global__ void k_bk_colscan(AttView av, int32_t* btot) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= av.nb) return;
  int32_t run = 0;
  for (int64_t c = 0; c < av.nchunks; ++c) {
    av.cbase[c * av.nb + b] = run;
    run += av.count[c * av.nb + b];
  }
  btot[b] = run;
}

__global__ void k_bk_addbase(AttView av, const int64_t* bptr) {
  const int64_t total = av.nchunks * av.nb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    av.cbase[e] += (int32_t)bptr[e % av.nb];
}

// Stable ranking inside each chunk: one wave per chunk, 64 rows at a time.
__global__ void __launch_bounds__(kWave) k_bk_rank(SysView s, AttView av, int32_t* dest) {
  extern __shared__ int lds_i[];
  int* lstart = lds_i;         // [nb] local start of each bucket run
  int* cur = lds_i + av.nb;    // [nb] rows of each bucket placed so far
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  for (int64_t b = lane; b < av.nb; b += kWave) {
    lstart[b] = av.lst[c * (av.nb + 1) + b];
    cur[b] = 0;
  }
  __syncthreads();
  const int64_t r0 = c * av.K, r1 = min(s.m, r0 + av.K);
  for (int64_t t0 = r0; t0 < r1; t0 += kWave) {
    const int64_t r = t0 + lane;
    const bool valid = r < r1;
    const int b = valid ? (int)(s.att_start[r] / av.Wb) : -1 - lane;
    int rank = 0, later = 0;
    for (int j = 0; j < kWave; ++j) {
      const int bj = __shfl(b, j, kWave);
      rank += (j < lane && bj == b);
      later += (j > lane && bj == b);
    }
    if (valid) {
      const int k = cur[b] + rank;
      av.lpos[r] = (uint16_t)(lstart[b] + k);
      dest[r] = av.cbase[c * av.nb + b] + k;
    }
    __syncthreads();
    if (valid && later == 0) cur[b] += rank + 1;
    __syncthreads();
  }
}

// One pass over the rows (64-row tiles per wave, staged through LDS): the
// attitude coefficients go to their bucket-order slot dest[r] in batt, the
// other twelve (astrometric, instrumental, global) to row r of sv.
template <typename VT>
__global__ void __launch_bounds__(kBlock) k_bk_split(SysView s, AttView av, const int32_t* __restrict__ dest) {
  constexpr int HC = AttGeo<VT>::CPR;  // chunks per half row
  constexpr int RC = 2 * HC;           // chunks per row
  __shared__ u4 slabs[kWavesPerBlock][kWave * (RC + 1)];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t W = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t ntiles = (s.m + kWave - 1) / kWave;
  const u4* vb = reinterpret_cast<const u4*>(s.vals);
  u4* svp = reinterpret_cast<u4*>(av.sv);
  u4* bap = reinterpret_cast<u4*>(av.batt);
  for (int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wid; t < ntiles; t += W) {
    const int64_t t0 = t * kWave;
    const int nrow = (int)min<int64_t>(kWave, s.m - t0);
    u4 tmp[RC], mine[RC];
    issue_chunks<RC>(vb + t0 * RC, nrow, lane, tmp);
    lds_rows<RC>(tmp, nrow, slabs[wid], lane, mine);
    if (lane < nrow) {
      const int64_t r = t0 + lane;
      VT a[kSlots], sp[12], ap[12];
      __builtin_memcpy(a, mine, sizeof(a));
#pragma unroll
      for (int k = 0; k < 5; ++k) sp[k] = a[k];
#pragma unroll
      for (int k = 0; k < 7; ++k) sp[5 + k] = a[17 + k];
#pragma unroll
      for (int k = 0; k < 12; ++k) ap[k] = a[5 + k];
      u4 so[HC], ao[HC];
      __builtin_memcpy(so, sp, sizeof(so));
      __builtin_memcpy(ao, ap, sizeof(ao));
      const int64_t d = dest[r];
#pragma unroll
      for (int j = 0; j < HC; ++j) {
        svp[r * HC + j] = so[j];
        bap[d * HC + j] = ao[j];
      }
      const int32_t at = s.att_start[r];
      av.bst[d] = (uint16_t)(at - (at / av.Wb) * av.Wb);
    }
  }
}

void att_free(AttView* av) {
  for (void* p : {(void*)av->count, (void*)av->cbase, (void*)av->lst, (void*)av->lpos, av->batt, (void*)av->bst,
                  (void*)av->sub_lo, (void*)av->sub_b, (void*)av->bsub, (void*)av->Q, (void*)av->ub, av->sv})
    if (p) (void)hipFree(p);
  *av = AttView{};
}

#define ATT_CHK(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      snprintf(err, errlen, "%s: %s", #call, hipGetErrorString(e_));                   \
      (void)hipGetLastError();                                                         \
      if (dest) (void)hipFree(dest);                                                   \
      if (btot) (void)hipFree(btot);                                                   \
      if (bptr_d) (void)hipFree(bptr_d);                                               \
      att_free(av);                                                                    \
      return e_ == hipErrorOutOfMemory ? GSR_ENOMEM : GSR_EHIP;                        \
    }                                                                                  \
  } while (0)

int att_build(const SysView& s, AttView* av, int cus, char* err, size_t errlen, hipStream_t st) {
  *av = AttView{};
  int32_t* dest = nullptr;
  int32_t* btot = nullptr;
  int64_t* bptr_d = nullptr;
  if (s.m >= ((int64_t)1 << 31) - 1) {
    snprintf(err, errlen, "bucketed attitude pass needs m < 2^31");
    return GSR_EINVAL;
  }
  const int64_t V = s.n_att - 3;  // distinct attitude starts
  av->K = 2048;
  av->Wb = std::max<int64_t>(32, (V + 127) / 128);
  av->nb = (V + av->Wb - 1) / av->Wb;
  av->nchunks = std::max<int64_t>(1, (s.m + av->K - 1) / av->K);
  const size_t m = (size_t)std::max<int64_t>(s.m, 1);
  const size_t vsz = s.value_type == GSR_F32 ? sizeof(float) : sizeof(double);
  ATT_CHK(hipMalloc((void**)&av->count, sizeof(int32_t) * av->nchunks * av->nb));
  ATT_CHK(hipMalloc((void**)&av->cbase, sizeof(int32_t) * av->nchunks * av->nb));
  ATT_CHK(hipMalloc((void**)&av->lst, sizeof(int32_t) * av->nchunks * (av->nb + 1)));
  ATT_CHK(hipMalloc((void**)&av->lpos, sizeof(uint16_t) * m));
  ATT_CHK(hipMalloc((void**)&av->batt, vsz * 12 * m));
  ATT_CHK(hipMalloc((void**)&av->sv, vsz * 12 * m));
  ATT_CHK(hipMalloc((void**)&av->bst, sizeof(uint16_t) * m));
  ATT_CHK(hipMalloc((void**)&av->ub, sizeof(double) * m));
  ATT_CHK(hipMalloc((void**)&dest, sizeof(int32_t) * m));
  ATT_CHK(hipMalloc((void**)&btot, sizeof(int32_t) * av->nb));
  ATT_CHK(hipMalloc((void**)&bptr_d, sizeof(int64_t) * (av->nb + 1)));
  const int g = (int)std::min<int64_t>(4096, (int64_t)(m + 255) / 256);
  hipLaunchKernelGGL(k_bk_count, dim3((unsigned)av->nchunks), dim3(256), sizeof(int) * av->nb, st, s, *av);
  ATT_CHK(hipGetLastError());
  hipLaunchKernelGGL(k_bk_colscan, dim3((unsigned)((av->nb + 63) / 64)), dim3(64), 0, st, *av, btot);
  ATT_CHK(hipGetLastError());
  hipLaunchKernelGGL(k_bk_lstart, dim3((unsigned)((av->nchunks + 255) / 256)), dim3(256), 0, st, *av);
  ATT_CHK(hipGetLastError());
  std::vector<int32_t> tot(av->nb);
  ATT_CHK(hipMemcpyAsync(tot.data(), btot, sizeof(int32_t) * av->nb, hipMemcpyDeviceToHost, st));
  ATT_CHK(hipStreamSynchronize(st));
  std::vector<int64_t> bptr(av->nb + 1, 0);
  for (int64_t b = 0; b < av->nb; ++b) bptr[b + 1] = bptr[b] + tot[b];
  // workgroup ranges of the attitude pass: about 8 per CU, never across buckets
  const int64_t R = std::max<int64_t>(1024, (s.m + 8 * (int64_t)cus - 1) / (8 * (int64_t)cus));
  std::vector<int64_t> lo;
  std::vector<int32_t> sb, bs(av->nb + 1, 0);
  for (int64_t b = 0; b < av->nb; ++b) {
    bs[b] = (int32_t)lo.size();
    for (int64_t p = bptr[b]; p < bptr[b + 1]; p += R) {
      lo.push_back(p);
      sb.push_back((int32_t)b);
    }
  }
  bs[av->nb] = (int32_t)lo.size();
  av->nsub = (int32_t)lo.size();
  lo.push_back(s.m);
  ATT_CHK(hipMalloc((void**)&av->sub_lo, sizeof(int64_t) * lo.size()));
  ATT_CHK(hipMalloc((void**)&av->sub_b, sizeof(int32_t) * std::max<size_t>(1, sb.size())));
  ATT_CHK(hipMalloc((void**)&av->bsub, sizeof(int32_t) * bs.size()));
  ATT_CHK(hipMalloc((void**)&av->Q, sizeof(double) * std::max<int64_t>(1, av->nsub) * 3 * (av->Wb + 3)));
  ATT_CHK(hipMemcpyAsync(av->sub_lo, lo.data(), sizeof(int64_t) * lo.size(), hipMemcpyHostToDevice, st));
  if (!sb.empty())
    ATT_CHK(hipMemcpyAsync(av->sub_b, sb.data(), sizeof(int32_t) * sb.size(), hipMemcpyHostToDevice, st));
  ATT_CHK(hipMemcpyAsync(av->bsub, bs.data(), sizeof(int32_t) * bs.size(), hipMemcpyHostToDevice, st));
  ATT_CHK(hipMemcpyAsync(bptr_d, bptr.data(), sizeof(int64_t) * bptr.size(), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_bk_addbase, dim3(g), dim3(256), 0, st, *av, bptr_d);
  ATT_CHK(hipGetLastError());
  hipLaunchKernelGGL(k_bk_rank, dim3((unsigned)av->nchunks), dim3(kWave), 2 * sizeof(int) * av->nb, st, s, *av, dest);
  ATT_CHK(hipGetLastError());
  const int gs = (int)std::min<int64_t>(8 * (int64_t)cus, (s.m + 4 * kWave - 1) / (4 * kWave));
  if (s.value_type == GSR_F32)
    hipLaunchKernelGGL(k_bk_split<float>, dim3(std::max(gs, 1)), dim3(kBlock), 0, st, s, *av, dest);
  else
    hipLaunchKernelGGL(k_bk_split<double>, dim3(std::max(gs, 1)), dim3(kBlock), 0, st, s, *av, dest);
  ATT_CHK(hipGetLastError());
  ATT_CHK(hipStreamSynchronize(st));
  (void)hipFree(dest);
  (void)hipFree(btot);
  (void)hipFree(bptr_d);
  av->ready = 1;
  return GSR_OK;
}

// ------------------------------------------------------------- per product
// ub <- u in bucket order.  One workgroup per chunk of K rows.  Consecutive
// chunks run on the same XCD (workgroup b runs on XCD b mod 8): the run of a
// bucket from chunk c ends where the run from chunk c+1 begins, so the 64-byte
// sector they share is completed in one L2 instead of reaching memory as two
// partial writes.
__global__ void __launch_bounds__(kBlock) k_partition(SysView s, AttView av, const double* __restrict__ u,
                                                      Scalars* sc) {
  if (sc && (sc->done || !sc->do_v)) return;
  extern __shared__ double buf[];
  int* ls = reinterpret_cast<int*>(buf + av.K);  // [nb+1]
  const int64_t per = (av.nchunks + kXcds - 1) / kXcds;
  const int64_t c = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  if (c >= av.nchunks) return;
  const int64_t r0 = c * av.K;
  const int n = (int)min(av.K, s.m - r0);
  for (int64_t b = threadIdx.x; b <= av.nb; b += kBlock) ls[b] = av.lst[c * (av.nb + 1) + b];
  for (int i = threadIdx.x; i < n; i += kBlock) buf[av.lpos[r0 + i]] = __builtin_nontemporal_load(u + r0 + i);
  __syncthreads();
  for (int p = threadIdx.x; p < n; p += kBlock) {
    // bucket of local position p: the largest b with ls[b] <= p
    int lo = 0, hi = (int)av.nb - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ls[mid] <= p)
        lo = mid;
      else
        hi = mid - 1;
    }
    av.ub[av.cbase[c * av.nb + lo] + (p - ls[lo])] = buf[p];
  }
}

// Attitude sums of one bucket range per workgroup into its LDS window, then Q.
template <typename VT, int PM, int SQUARE>
__global__ void __launch_bounds__(kBlock) k_att_pass(SysView s, AttView av, double inv_beta, Scalars* sc, int raw) {
  constexpr int CPR = AttGeo<VT>::CPR;
  __shared__ u4 slabs[kWavesPerBlock][kWave * (CPR + 1)];
  extern __shared__ double win[];
  if (sc) {
    if (sc->done || !sc->do_v) return;
    if (!raw) inv_beta = sc->inv_beta;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t W3 = av.Wb + 3;
  for (int64_t k = threadIdx.x; k < 3 * W3; k += kBlock) win[k] = 0.0;
  __syncthreads();
  const int64_t sub = blockIdx.x;
  const int64_t lo = av.sub_lo[sub], hi = av.sub_lo[sub + 1];
  const u4* base = reinterpret_cast<const u4*>(av.batt);
  u4 tmp[CPR];
  double tv;
  int sov;
  auto fetch = [&](int64_t tt) {
    // past the end of the range: re-read its last row (the registers are not used)
    const int64_t te = min(tt, hi - 1);
    const int nr = (int)min((int64_t)kWave, hi - te);
    const int64_t ii = (lane < nr) ? te + lane : hi - 1;
    issue_chunks<CPR>(base + te * CPR, nr, lane, tmp);
    tv = SQUARE ? 0.0 : __builtin_nontemporal_load(av.ub + ii);
    sov = av.bst[ii];
  };
  const int64_t step = (int64_t)kWavesPerBlock * kWave;
  int64_t t0 = lo + (int64_t)wid * kWave;
  if (t0 < hi) fetch(t0);
#pragma unroll 1
  for (; t0 < hi; t0 += step) {
    const int nrow = (int)min((int64_t)kWave, hi - t0);
    const bool valid = lane < nrow;
    const double t = tv * inv_beta;
    const int so = sov;
    lds_put<CPR>(tmp, nrow, slabs[wid], lane);
    order_point();
    fetch(t0 + step);
    order_point();
    u4 mine[CPR];
    lds_get<CPR>(nrow, slabs[wid], lane, mine);
    VT a[12];
    __builtin_memcpy(a, mine, sizeof(a));
    if (valid) {
#pragma unroll
      for (int axs = 0; axs < 3; ++axs)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const VT v = a[4 * axs + j];
          const double cterm = SQUARE ? (double)v * (double)v
                                      : (PM == 1 ? (double)((float)v * (float)t) : (double)v * t);
          atomicAdd(win + axs * W3 + so + j, cterm);
        }
    }
  }
  __syncthreads();
  double* q = av.Q + sub * 3 * W3;
  for (int64_t k = threadIdx.x; k < 3 * W3; k += kBlock) q[k] = win[k];
}

hipError_t launch_partition(const SysView& s, const AttView& av, const double* u, Scalars* sc, hipStream_t st) {
  if (s.m == 0) return hipSuccess;
  const size_t lds = sizeof(double) * av.K + sizeof(int) * (av.nb + 1);
  const int64_t per = (av.nchunks + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(k_partition, dim3((unsigned)(per * kXcds)), dim3(kBlock), lds, st, s, av, u, sc);
  return hipGetLastError();
}

hipError_t launch_att_pass(const SysView& s, const AttView& av, double inv_beta, int pmode, int square, Scalars* sc,
                           hipStream_t st, int raw) {
  if (av.nsub == 0) return hipSuccess;
  const size_t lds = sizeof(double) * 3 * (av.Wb + 3);
  const dim3 g((unsigned)av.nsub), b(kBlock);
  if (s.value_type == GSR_F32) {
    if (square)
      hipLaunchKernelGGL((k_att_pass<float, 0, 1>), g, b, lds, st, s, av, inv_beta, sc, raw);
    else if (pmode == 1)
      hipLaunchKernelGGL((k_att_pass<float, 1, 0>), g, b, lds, st, s, av, inv_beta, sc, raw);
    else
      hipLaunchKernelGGL((k_att_pass<float, 0, 0>), g, b, lds, st, s, av, inv_beta, sc, raw);
  } else {
    if (square)
      hipLaunchKernelGGL((k_att_pass<double, 0, 1>), g, b, lds, st, s, av, inv_beta, sc, raw);
    else
      hipLaunchKernelGGL((k_att_pass<double, 0, 0>), g, b, lds, st, s, av, inv_beta, sc, raw);
  }
  return hipGetLastError();
}

}  // namespace gsr
