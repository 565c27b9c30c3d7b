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

// A descriptor read through the constant address space: its fields are
// invariant for the kernel, so the compiler may load each one where it is
// used (scalar loads) instead of holding the whole descriptor in registers.
typedef __attribute__((address_space(4))) const ImgDesc ConstDesc;

// for_each_item for bodies that take the descriptor as `const auto&`: a
// batched launch passes its table entry as a ConstDesc reference (fields
// loaded where used instead of held in registers).
template <int KIND, typename F>
__device__ __forceinline__ void for_each_item_cd(const Launch& L, F&& body);

// Same, with the single-image / batched choice made at compile time
// (BATCH = 1: the launch has a descriptor table, whose entry reaches the
// body as a ConstDesc reference).
template <int KIND, int BATCH, typename F>
__device__ __forceinline__ void for_each_item_t(const Launch& L, F&& body) {
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
    if constexpr (BATCH) {
      const int i = find_image(L, KIND, w);
      ConstDesc& d = ((ConstDesc*)L.table)[i];
      body(d, w - d.woff[KIND]);
    } else {
      body(L.one, w);
    }
  }
}

template <int KIND, typename F>
__device__ __forceinline__ void for_each_item_cd(const Launch& L, F&& body) {
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
      const int i = find_image(L, KIND, w);
      ConstDesc& d = ((ConstDesc*)L.table)[i];
      body(d, w - d.woff[KIND]);
    } else {
      body(L.one, w);
    }
  }
}

// Reference coordinate along one axis: 0, s, 2s, ... clamped to the last
// valid position (the clamp realises the extra last reference).
__device__ inline int ref_coord(int i, int s, int n_valid) { return min(i * s, n_valid - 1); }

// Aggregation accumulates estimates in 64-bit two's-complement fixed point
// with 32 fractional bits: integer additions are exact, so sums do not
// depend on the order in which work groups add them.  fx_from_float is
// exact for |v| < 2^24 up to the 2^-32 step and saturates beyond +-2^31.
// (integer part floor(v) by v_cvt_flr_i32_f32, fraction v - floor(v) by
// v_fract_f32, which keeps it below 1)
__device__ inline unsigned long long fx_from_float(float v) {
  int hi;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(hi) : "v"(v));
  const unsigned lo = (unsigned)(__builtin_amdgcn_fractf(v) * 4294967296.0f);
  return ((unsigned long long)(unsigned)hi << 32) + lo;
}
__device__ inline double fx_to_double(unsigned long long x) {
  return (double)(long long)x * 0x1p-32;
}

// Power-of-two factor applied to the estimates before the fixed-point
// conversion (and divided out at the write-back): it maps the largest input
// magnitude M of the image to [2^11, 2^12), so the 2^-32 step is relative
// to M and per-pixel sums of thousands of estimates of size M stay within
// the 31 integer bits.  1 when the numerator is not fixed point.
template <class Desc>
__device__ inline float fx_scale(const Desc& d) {
  if (!d.num64 || !d.fxmax) return 1.f;
  const int e = (int)((*d.fxmax >> 23) & 0xffu) - 127;   // M in [2^e, 2^(e+1))
  int k = e == 128 ? 0 : 11 - e;                          // inf / NaN: output is NaN anyway
  k = min(max(k, -100), 100);
  return __int_as_float((k + 127) << 23);
}

// Bits of |v| for the magnitude reduction; non-finite values count as 0
// (their groups are poisoned, so they should not set the scale).
__device__ inline uint32_t abs_bits(float v) {
  const uint32_t b = __float_as_uint(v) & 0x7fffffffu;
  return b < 0x7f800000u ? b : 0u;
}

// Folds the max over the calling threads of abs_bits values into *dst (the
// bit pattern of a non-negative float is monotonic).
__device__ inline void absmax_to(uint32_t* dst, uint32_t bits) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t v = (uint32_t)__shfl_xor((int)bits, o, 64);
    bits = v > bits ? v : bits;
  }
  if ((threadIdx.x & 63) == 0 && bits) atomicMax(dst, bits);
}

// Row y and column x of a flattened position pos = y*W + x (rW = 1/W in
// FP32).  The FP32 quotient is within one of the true row while pos/W stays
// below 2^22 (relative error <= 3 * 2^-24), so one correction step is exact;
// callers clamp the result, which keeps out-of-range positions in bounds.
__device__ inline void split_pos(int pos, int W, float rW, int& y, int& x) {
  y = (int)((float)pos * rW);
  x = pos - y * W;
  if (x < 0) { --y; x += W; }
  else if (x >= W) { ++y; x -= W; }
}

// A group that gathered a non-finite pixel or produced a non-finite estimate
// marks every pixel of its K patches: in the poison plane when the
// numerator is fixed point (the write-back turns those pixels into NaN),
// else by adding NaN to the float numerator; its exported estimates become
// NaN.  Called by all 64 lanes of a wavefront; lane = patch pixel.
template <class Desc>
__device__ inline void poison_group(const Desc& d, const int* gidx, int grel, int K, int C,
                                    float rW, int lane) {
  for (int k = 0; k < K; ++k) {
    if (d.group_est)
      for (int c = 0; c < C; ++c)
        d.group_est[(((size_t)grel * K + k) * C + c) * PS2 + lane] = __builtin_nanf("");
    int py, px;
    split_pos(gidx[k], d.W, rW, py, px);
    py = min(max(py, 0), d.Hp - 1);
    px = min(max(px, 0), d.Wp - 1);
    const int pix = (py + (lane >> 3)) * d.W + px + (lane & 7);
    if (d.num64) {
      d.poison[pix] = 1;
    } else {
      for (int c = 0; c < C; ++c) atomicAdd(d.num + c * d.H * d.W + pix, __builtin_nanf(""));
    }
  }
}

// Adds one LDS tile of fixed-point sums into the image numerator (exact
// integer atomics, or float atomics into a float numerator).
// Weighted aggregation: the weight plane (plane C of the tile) holds the
// group weights times 2^16 in the same fixed point.
constexpr float WEIGHT_SCALE = 65536.f;

template <class Desc>
__device__ inline void flush_tile(const Desc& d, const unsigned long long* acc, int C, int RA,
                                  int CA, int AY0, int AX0, int AH, int AW, bool weighted = false) {
  const int HW = d.H * d.W;
  const int NP = C + (weighted ? 1 : 0);
  for (int e = threadIdx.x; e < NP * AH * AW; e += blockDim.x) {
    const int pl = e / (AH * AW), rem = e - pl * (AH * AW);
    const int y = rem / AW, x = rem - y * AW;
    const unsigned long long v = acc[(pl * RA + y) * CA + x];
    if (v != 0ull) {
      const int pix = (AY0 + y) * d.W + AX0 + x;
      if (pl == C) {   // weight sums
        if (d.wsum64) atomicAdd(d.wsum64 + pix, v);
        else if (d.cnt) atomicAdd(d.cnt + pix, (float)(fx_to_double(v) * (1.0 / WEIGHT_SCALE)));
        continue;
      }
      const int gp = pl * HW + pix;
      if (d.num64) atomicAdd(d.num64 + gp, v);
      else atomicAdd(d.num + gp, (float)fx_to_double(v));
    }
  }
}

// Cold path of the fused aggregation: an estimate of a patch that lies
// outside the work group's LDS tile (a caller-given idx entry that is not
// from its reference's search window) is added straight into the image
// numerator, scaled like the tile values (fixed point, or a float numerator
// when d.num64 is null).  pix is the pixel index y * W + x.
template <class Desc>
__device__ inline void add_estimate_global(const Desc& d, int ch, int pix, float v) {
  if (d.num64) atomicAdd(d.num64 + (size_t)ch * d.H * d.W + pix, fx_from_float(v));
  else atomicAdd(d.num + (size_t)ch * d.H * d.W + pix, v);
}
// The weight (fixed point, times WEIGHT_SCALE) of such a patch pixel.
template <class Desc>
__device__ inline void add_weight_global(const Desc& d, int pix, unsigned long long w) {
  if (d.wsum64) atomicAdd(d.wsum64 + pix, w);
  else if (d.cnt) atomicAdd(d.cnt + pix, (float)(fx_to_double(w) * (1.0 / WEIGHT_SCALE)));
}

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
