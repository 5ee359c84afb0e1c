// Row-tile helpers shared by the streaming passes over the 24-coefficient
// rows: tile geometry, the star of each row of a 64-row tile, and the
// per-coefficient product in FP64 or FP32.
#pragma once

#include "device_common.h"

namespace gsr {

typedef double dd2u __attribute__((ext_vector_type(2), aligned(8)));  // 16-byte load at 8-byte alignment
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));    // 16-byte load at 4-byte alignment

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

template <int PM, typename VT>
__device__ __forceinline__ double prod(VT a, double x) {
  if (PM == 1) return (double)((float)a * (float)x);
  return (double)a * x;
}

// A term of A^T u: a * u as prod forms it, or a^2 in FP64 when summing the
// squares of the columns (SQ = 1).
template <int PM, int SQ, typename VT>
__device__ __forceinline__ double tprod(VT a, double u) {
  if (SQ) return (double)a * (double)a;
  return prod<PM>(a, u);
}

// Star boundaries for a tile whose first row is in star scur: lane i holds
// row_ptr[scur + 1 + i] (the end row of star scur + i), clamped at n_stars.
__device__ __forceinline__ int64_t bnd_load(const SysView& s, int64_t scur, int lane) {
  return s.row_ptr[min(scur + 1 + lane, s.n_stars)];
}

// First star of the next tile (the star of row t0 + 64) from the tile's
// boundaries b (lane i: end row of star scur + i), by one ballot.
__device__ __forceinline__ int64_t tile_next(const SysView& s, int64_t b, int64_t t0, int64_t scur) {
  const int n = __popcll(__ballot(b <= t0 + kWave));
  int64_t nxt = scur + n;
  if (n == kWave)  // more than 64 stars end inside this tile (empty or one-row stars)
    while (nxt < s.n_stars - 1 && s.row_ptr[nxt + 1] <= t0 + kWave) ++nxt;
  return min(nxt, max<int64_t>(s.n_stars - 1, 0));
}

// Star of row t0 + lane (first star sf of the tile, boundaries staged in bnd)
// and optionally that star's row range.
__device__ __forceinline__ int64_t tile_star(const SysView& s, int64_t t0, int lane, const int64_t* bnd, int64_t sf,
                                             int64_t* rbeg = nullptr, int64_t* rend = nullptr) {
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
  int64_t st = sf + lo;
  if (lo == kWave) {
    // more than 64 stars end inside this tile: walk on from star sf + 64.  Every
    // loaded boundary is consumed inside the walk, so no load is left pending
    // past this branch.
    int64_t b0 = bnd[kWave - 1], b1 = s.m;
    if (st >= s.n_stars) {  // only rows past the end
      st = s.n_stars - 1;
      b0 = s.m;
    } else {
      for (; st < s.n_stars - 1; ++st) {
        const int64_t nb = s.row_ptr[st + 1];
        if (nb > r) {
          b1 = nb;
          break;
        }
        b0 = nb;
      }
    }
    if (rbeg) *rbeg = b0;
    if (rend) *rend = b1;
  } else {
    // star st = sf + lo spans rows [row_ptr[st], row_ptr[st+1]) = [bnd[lo-1], bnd[lo]);
    // for lo = 0 it began at or before t0
    if (rbeg) *rbeg = lo > 0 ? bnd[lo - 1] : t0;
    if (rend) *rend = bnd[lo];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  return st;
}

}  // namespace gsr
