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

// Aggregation accumulates estimates in 64-bit two's-complement fixed point:
// integer additions are exact, so sums do not depend on the order in which
// work groups add them.  Two encodings (of num64 and of the filters' LDS
// tiles), chosen by fx_int_units:
//  * integer units: the forward c = 1, 3 filters with uniform weights.  Estimates
//    are scaled so that the image's largest input magnitude M lies in
//    [2^23, 2^24) and rounded to integers (fx_from_units: one
//    v_cvt_rpi_i32_f32, then sign extension).  An estimate is at most
//    sqrt(64 K c) M <= 79 M in magnitude (the projection, the Haar
//    transform and their inverses are orthonormal and the threshold only
//    removes coefficients; c = 3 filters take K <= 32, c = 1 K <= 64), so
//    it stays below 79 * 2^24 < 2^31.  The rounding step is at most
//    2^-23 M, the order of FP32 rounding of the estimate itself.
//  * 2^-32 units: the weighted aggregation (whose group weights scale
//    estimates down by up to 1/(64 K c)), the frozen adjoints and the
//    band-count filter (whose groups can reach 724 M).  M lies in [2^11, 2^12), and the integer and
//    fraction parts are converted apart (fx_from_float: integer part
//    floor(v) by v_cvt_flr_i32_f32, fraction v - floor(v) by v_fract_f32,
//    exact for |v| < 2^24 up to the 2^-32 step, saturating beyond 2^31).
// For c = 3 the c = 1, 3 filters add each estimate pixel's channel DFT,
// (F0, Re F1, Im F1) / 3 = ((x0 + x1 + x2) / 3, (2 x0 - x1 - x2) / 6,
// (x2 - x1) / (2 sqrt 3)), and the write-back inverts it (fx_fourier):
// x0 = A0 + 2 A1, x1 = A0 - A1 - sqrt3 A2, x2 = A0 - A1 + sqrt3 A2.
// The frozen adjoints keep 2^-32 units, and the band-count filter adds
// pixel values (fx_int_units and fx_fourier in hts_internal.h).

__device__ inline unsigned long long fx_from_float(float v) {
  int hi;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(hi) : "v"(v));
  const unsigned lo = (unsigned)(__builtin_amdgcn_fractf(v) * 4294967296.0f);
  return ((unsigned long long)(unsigned)hi << 32) + lo;
}
__device__ inline unsigned long long fx_from_units(float v) {
  int i;   // floor(v + 1/2)
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(i) : "v"(v));
  return (unsigned long long)(long long)i;
}
template <bool UNITS>
__device__ inline unsigned long long fx_from(float v) {
  if constexpr (UNITS) return fx_from_units(v);
  else return fx_from_float(v);
}
__device__ inline double fx_to_double(unsigned long long x) {
  return (double)(long long)x * 0x1p-32;
}
__device__ inline double fx_value(unsigned long long x, bool units) {
  return units ? (double)(long long)x : fx_to_double(x);
}

// Power-of-two factor applied to the estimates before the fixed-point
// conversion (and divided out at the write-back): it maps the largest input
// magnitude M of the image (*d.fxmax) to [2^23, 2^24) in integer units, to
// [2^11, 2^12) in 2^-32 units, so that per-pixel sums of thousands of
// estimates stay far inside 64 bits.  1 without a magnitude, and in 2^-32
// units also without a fixed-point numerator (float numerators then take
// the tile sums as they are).
template <class Desc>
__device__ inline float fx_scale(const Desc& d, bool units) {
  if (!d.fxmax || (!units && !d.num64)) return 1.f;
  const int e = (int)((*d.fxmax >> 23) & 0xffu) - 127;   // M in [2^e, 2^(e+1))
  int k = e == 128 ? 0 : (units ? 23 : 11) - e;          // inf / NaN: output is NaN anyway
  k = min(max(k, -100), 100);
  return __int_as_float((k + 127) << 23);
}

// The inverse channel DFT of a fixed-point triple (A0, A1, A2) of fx_fourier.
__device__ inline void fx_idft3(double a0, double a1, double a2, double& x0, double& x1, double& x2) {
  const double r3 = 1.7320508075688772935;
  x0 = a0 + 2.0 * a1;
  x1 = a0 - a1 - r3 * a2;
  x2 = a0 - a1 + r3 * a2;
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

// Adds one LDS tile of fixed-point sums into the image numerator: exact
// integer atomics, or float atomics of the decoded values into a float
// numerator (image units: the tile's scale divided out, and for c = 3 the
// channel DFT inverted).  Weighted aggregation: the weight plane (plane C
// of the tile) holds the group weights times 2^16 in 2^-32 units.
constexpr float WEIGHT_SCALE = 65536.f;

template <class Desc>
__device__ inline void flush_tile(const Desc& d, const unsigned long long* acc, int C, int RA,
                                  int CA, int AY0, int AX0, int AH, int AW, bool units,
                                  float fxs, bool weighted = false) {
  const int HW = d.H * d.W;
  if (d.num64) {
    const int NP = C + (weighted ? 1 : 0);
    for (int e = threadIdx.x; e < NP * AH * AW; e += blockDim.x) {
      const int pl = e / (AH * AW), rem = e - pl * (AH * AW);
      const int y = rem / AW, x = rem - y * AW;
      const unsigned long long v = acc[(pl * RA + y) * CA + x];
      if (v != 0ull) {
        const int pix = (AY0 + y) * d.W + AX0 + x;
        if (pl < C) atomicAdd(d.num64 + pl * HW + pix, v);
        else if (d.wsum64) atomicAdd(d.wsum64 + pix, v);   // weight sums
        else if (d.cnt) atomicAdd(d.cnt + pix, (float)(fx_to_double(v) * (1.0 / WEIGHT_SCALE)));
      }
    }
    return;
  }
  const double rs = 1.0 / (double)fxs;
  for (int e = threadIdx.x; e < AH * AW; e += blockDim.x) {
    const int y = e / AW, x = e - y * AW;
    const int pix = (AY0 + y) * d.W + AX0 + x;
    const int t = y * CA + x;
    if (weighted && d.cnt) {
      const unsigned long long w = acc[C * RA * CA + t];
      if (w != 0ull) atomicAdd(d.cnt + pix, (float)(fx_to_double(w) * (1.0 / WEIGHT_SCALE)));
    }
    if (C == 3) {
      const unsigned long long a0 = acc[t], a1 = acc[RA * CA + t], a2 = acc[2 * RA * CA + t];
      if ((a0 | a1 | a2) == 0ull) continue;
      double x0, x1, x2;
      fx_idft3(fx_value(a0, units) * rs, fx_value(a1, units) * rs, fx_value(a2, units) * rs, x0, x1, x2);
      atomicAdd(d.num + pix, (float)x0);
      atomicAdd(d.num + HW + pix, (float)x1);
      atomicAdd(d.num + 2 * HW + pix, (float)x2);
    } else {
      for (int pl = 0; pl < C; ++pl) {
        const unsigned long long v = acc[pl * RA * CA + t];
        if (v != 0ull) atomicAdd(d.num + pl * HW + pix, (float)(fx_value(v, units) * rs));
      }
    }
  }
}

// Cold path of the fused aggregation: the estimate of one pixel (its C tile
// values: for c = 3 the fx_fourier triple) of a patch that lies outside the
// work group's LDS tile (a caller-given idx entry that is not from its
// reference's search window) goes straight into the image numerator,
// encoded like the tile values, or decoded (scale fxs divided out, channel
// DFT inverted) into a float numerator.  pix is the pixel index y * W + x.
template <bool UNITS, class Desc>
__device__ inline void add_pixel_global(const Desc& d, int C, int pix, const float (&a)[3], float fxs) {
  const size_t HW = (size_t)d.H * d.W;
  if (d.num64) {
    for (int ch = 0; ch < C; ++ch) atomicAdd(d.num64 + ch * HW + pix, fx_from<UNITS>(a[ch]));
  } else if (C == 3) {
    const double rs = 1.0 / (double)fxs;
    double x0, x1, x2;
    fx_idft3((double)a[0] * rs, (double)a[1] * rs, (double)a[2] * rs, x0, x1, x2);
    atomicAdd(d.num + pix, (float)x0);
    atomicAdd(d.num + HW + pix, (float)x1);
    atomicAdd(d.num + 2 * HW + pix, (float)x2);
  } else {
    atomicAdd(d.num + pix, (float)((double)a[0] / (double)fxs));
  }
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
