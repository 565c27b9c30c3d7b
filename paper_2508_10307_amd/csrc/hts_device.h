// Device-side helpers shared by the HIP kernels.
#pragma once

#include "hts_internal.h"

namespace hts {

// Find the image owning global work item w of kind `kind` in a batched
// launch (largest i with table[i].woff[kind] <= w).
__device__ inline int find_image(const Launch& L, int kind, int w) {
  int lo = 0, hi = L.n_img - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (L.table[mid].woff[kind] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Loop over the work items of one kind assigned to this work group
// (persistent when gridDim.x < total).  `body(desc, local_item)`.
// XCD-aware order: consecutive work groups are dispatched round-robin over
// the 8 XCDs, so group b runs on XCD b % 8.  When the grid is a multiple of
// 8, each XCD gets one contiguous run of the item list (neighbouring tiles
// read the same image rows, which then stay in that XCD's L2).
template <int KIND, typename F>
__device__ __forceinline__ void for_each_item(const Launch& L, F&& body) {
  const int G = gridDim.x, T = L.total;
  int start = blockIdx.x, step = G, end = T;
  if (G >= 8 && (G & 7) == 0) {
    const int chunk = (T + 7) >> 3;
    const int x = blockIdx.x & 7;
    start = x * chunk + (blockIdx.x >> 3);
    step = G >> 3;
    end = min(T, (x + 1) * chunk);
  }
  for (int w = start; w < end; w += step) {
    if (L.table) {
      int i = find_image(L, KIND, w);
      const ImgDesc d = L.table[i];
      body(d, w - d.woff[KIND]);
    } else {
      body(L.one, w);
    }
  }
}

// Reference coordinate along one axis: 0, s, 2s, ... clamped to the last
// valid position (the clamp realises the extra last reference).
__device__ inline int ref_coord(int i, int s, int n_valid) { return min(i * s, n_valid - 1); }

// Guide quantisation: round_half_even(256 v) clamped to +-(2^20 - 1); NaN -> 0.
__device__ inline int quantize(float v) {
  float r = rintf(v * 256.0f);
  if (!(r == r)) return 0;
  r = fminf(fmaxf(r, -(float)QMAX), (float)QMAX);
  return (int)r;
}

__device__ inline unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = __shfl_xor(lo, m, 64);
  hi = __shfl_xor(hi, m, 64);
  return ((unsigned long long)hi << 32) | lo;
}

// Ascending bitonic sort of 64*E keys held E per lane (element index
// e*64 + lane), across one wavefront.
template <int E>
__device__ inline void wave_sort_u64(unsigned long long (&v)[E]) {
  const int lane = threadIdx.x & 63;
  constexpr int N = 64 * E;
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        const int je = j >> 6;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int p = e ^ je;
          if (p > e) {
            int i = e * 64 + lane;
            bool asc = (i & k) == 0;
            unsigned long long a = v[e], b = v[p];
            bool sw = asc ? (a > b) : (a < b);
            v[e] = sw ? b : a;
            v[p] = sw ? a : b;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int i = e * 64 + lane;
          unsigned long long o = shfl_xor_u64(v[e], j);
          bool asc = (i & k) == 0;
          bool lower = (i & j) == 0;
          unsigned long long mn = v[e] < o ? v[e] : o;
          unsigned long long mx = v[e] < o ? o : v[e];
          v[e] = (lower == asc) ? mn : mx;
        }
      }
    }
  }
}

}  // namespace hts
