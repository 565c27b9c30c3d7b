// Element-wise stages: guide quantisation (Eq. 10 inputs), GCP branch per
// reference (Eq. 10), clearing of accumulators and counters, and the
// averaged write-back out = num / cnt (Eq. 2).
#include "hts_device.h"

namespace hts {

// Guide planes from the noisy image: C = 1 -> q; C = 3 -> (qG, qR + qG + qB);
// other C -> the band mean on the same grid, round-half-even(sum q_j / C) in
// exact integer arithmetic.
__global__ __launch_bounds__(256) void k_quant(Launch L) {
  for_each_item<W_PIX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int p0 = item * PIX_CHUNK;
    const int p1 = min(HW, p0 + PIX_CHUNK);
    uint32_t mb = 0;   // bits of max |x| (sets the fixed-point scale of the aggregation)
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
      if (L.count_hist) d.hist[p] = 0;
      if (L.C == 1) {
        const float v = d.img[p];
        d.gplanes[p] = quantize(v);
        mb = max(mb, abs_bits(v));
      } else if (L.C != 3) {
        int sq = 0;   // |sum| <= 256 (2^20 - 1) < 2^28
        for (int j = 0; j < L.C; ++j) {
          const float v = d.img[(size_t)j * HW + p];
          sq += quantize(v);
          mb = max(mb, abs_bits(v));
        }
        // floor division, then half to even
        int fl = sq / L.C, rem = sq - fl * L.C;
        if (rem < 0) { --fl; rem += L.C; }
        if (2 * rem > L.C || (2 * rem == L.C && (fl & 1))) ++fl;
        d.gplanes[p] = fl;
      } else {
        const float r = d.img[p], g = d.img[HW + p], b = d.img[2 * HW + p];
        int qr = quantize(r);
        int qg = quantize(g);
        int qb = quantize(b);
        d.gplanes[p] = qg;
        d.gplanes[HW + p] = qr + qg + qb;
        mb = max(mb, max(abs_bits(r), max(abs_bits(g), abs_bits(b))));
      }
    }
    if (d.fxmax) absmax_to(d.fxmax, mb);
  });
}

// Magnitude reduction of the filter input alone (bits of max |x| over all
// channels into *d.fxmax, zeroed by the caller): the fixed-point scale for
// calls that filter without quantising first.
__global__ __launch_bounds__(256) void k_absmax(Launch L) {
  for_each_item<W_PIX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int p0 = item * PIX_CHUNK;
    const int p1 = min(HW, p0 + PIX_CHUNK);
    uint32_t mb = 0;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x)
      for (int c = 0; c < L.C; ++c) mb = max(mb, abs_bits(d.img[(size_t)c * HW + p]));
    absmax_to(d.fxmax, mb);
  });
}

// Eq. 10 branch of every reference: green guide when
// num^2 |qG|^2 >= den^2 max(|qR|^2, |qB|^2) on the reference patch (exact int64).
__global__ __launch_bounds__(256) void k_gcp(Launch L) {
  for_each_item<W_REF>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int r = item * 256 + threadIdx.x;
    if (r >= d.n_ref) return;
    if (L.C != 3) { d.green[r] = 1; return; }   // one guide plane
    const int ry = ref_coord(r / d.nrx, L.stride, d.Hp);
    const int rx = ref_coord(r % d.nrx, L.stride, d.Wp);
    const int HW = d.H * d.W;
    long long n[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c)
      for (int a = 0; a < PS; ++a)
        for (int b = 0; b < PS; ++b) {
          long long q = quantize(d.img[c * HW + (ry + a) * d.W + rx + b]);
          n[c] += q * q;
        }
    long long lhs = (long long)L.gcp_num * L.gcp_num * n[1];
    long long rhs = (long long)L.gcp_den * L.gcp_den * (n[0] > n[2] ? n[0] : n[2]);
    d.green[r] = lhs >= rhs ? 1 : 0;
  });
}

// Clears the per-image counters: the match fallback list length and the
// input magnitude reduced by k_quant.
__global__ void k_reset_counters(Launch L) {
  if (!L.table) {
    if (threadIdx.x == 0) {
      if (L.one.fb_count) *L.one.fb_count = 0;
      if (L.one.fxmax) *L.one.fxmax = 0;
    }
    return;
  }
  for (int i = threadIdx.x; i < L.n_img; i += blockDim.x) {
    if (L.table[i].fb_count) *L.table[i].fb_count = 0;
    if (L.table[i].fxmax) *L.table[i].fxmax = 0;
  }
}

// Accumulators to zero: the fixed-point numerator (or the float one when
// the descriptor has none), cnt and the poison plane (a fill kernel rather
// than a memset so that the sequence stays valid inside captured graphs).
// The slot histogram is cleared where it is built (k_quant before a match
// that counts, or k_zero_hist).
__global__ __launch_bounds__(256) void k_zero_accum(Launch L) {
  for_each_item<W_PIX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int p0 = item * PIX_CHUNK;
    const int p1 = min(HW, p0 + PIX_CHUNK);
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
      if (d.num64) {
        for (int c = 0; c < L.C; ++c) d.num64[c * HW + p] = 0ull;
      } else {
        for (int c = 0; c < L.C; ++c) d.num[c * HW + p] = 0.0f;
      }
      if (d.cnt && !L.adjoint) d.cnt[p] = 0.0f;   // the adjoint's cnt is the caller's state
      if (d.poison) d.poison[p] = 0;
      if (d.wsum64) d.wsum64[p] = 0ull;
    }
  });
}

// Eq. 2: out = num / cnt (uniform weights) or num / weight sum (weighted
// aggregation, when the descriptor has the weight plane), from the
// fixed-point numerator when the descriptor has one (decoded as its encoding
// says: scales divided out and, for the channel-DFT triples of c = 3, the
// channel DFT inverted, in FP64 with one rounding), else from the float
// numerator.  Without cnt the numerator is converted as it is (the
// adjoint's output).  Pixels marked in the poison plane become NaN.
__global__ __launch_bounds__(256) void k_finalize(Launch L) {
  for_each_item<W_PIX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int p0 = item * PIX_CHUNK;
    const int p1 = min(HW, p0 + PIX_CHUNK);
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
      if (d.num64) {
        const bool units = fx_int_units(L.C, L.flags, d.num_enc);
        const double den = d.wsum64 ? fx_to_double(d.wsum64[p]) * (1.0 / WEIGHT_SCALE)
                                    : (d.cnt && !L.adjoint ? (double)d.cnt[p] : 1.0);
        const double c = den * (double)fx_scale(d, units);
        const bool bad = d.poison && d.poison[p];
        if (fx_fourier(L.C, d.num_enc)) {
          double x0, x1, x2;
          fx_idft3(fx_value(d.num64[p], units), fx_value(d.num64[HW + p], units),
                   fx_value(d.num64[2 * HW + p], units), x0, x1, x2);
          d.out[p] = bad ? __builtin_nanf("") : (float)(x0 / c);
          d.out[HW + p] = bad ? __builtin_nanf("") : (float)(x1 / c);
          d.out[2 * HW + p] = bad ? __builtin_nanf("") : (float)(x2 / c);
        } else {
          for (int ch = 0; ch < L.C; ++ch)
            d.out[ch * HW + p] =
                bad ? __builtin_nanf("") : (float)(fx_value(d.num64[ch * HW + p], units) / c);
        }
      } else {
        const float inv = 1.0f / d.cnt[p];
        for (int ch = 0; ch < L.C; ++ch) d.out[ch * HW + p] = d.num[ch * HW + p] * inv;
      }
    }
  });
}

// Adjoint input: r = g / cnt (and max |r|).  Single image: g = d.img, r into
// the workspace buffer d.num (see hts_denoise_backward).  Batched adjoint
// (L.adjoint): g = d.num (the caller's gradient), r into d.img (the
// workspace buffer the filter then reads).
__global__ __launch_bounds__(256) void k_adjoint_prep(Launch L) {
  for_each_item<W_PIX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int p0 = item * PIX_CHUNK;
    const int p1 = min(HW, p0 + PIX_CHUNK);
    const float* g = L.adjoint ? d.num : d.img;
    float* rr = L.adjoint ? const_cast<float*>(d.img) : d.num;
    uint32_t mb = 0;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
      float inv = 1.0f / d.cnt[p];
      for (int c = 0; c < L.C; ++c) {
        const float r = g[c * HW + p] * inv;
        rr[c * HW + p] = r;
        mb = max(mb, abs_bits(r));
      }
    }
    if (d.fxmax) absmax_to(d.fxmax, mb);
  });
}

// Coverage counts (the Eq. 2 denominator) depend only on the match indices:
// hist[p] = number of (group, slot) patches with top-left corner p, and
// cnt = hist convolved with the 8x8 box (every such patch covers 8x8 pixels).
__global__ __launch_bounds__(256) void k_zero_hist(Launch L) {
  for_each_item<W_PIX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int p0 = item * PIX_CHUNK;
    const int p1 = min(HW, p0 + PIX_CHUNK);
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) d.hist[p] = 0;
  });
}

__global__ __launch_bounds__(256) void k_count_hist(Launch L) {
  for_each_item<W_REF>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int g = item * 256 + threadIdx.x;
    if (g < d.ref_begin || g >= d.ref_begin + d.ref_count) return;
    const int* row = d.idx + (size_t)g * L.K;
    const float rW = 1.0f / (float)d.W;
    for (int k = 0; k < L.K; ++k) {
      // an entry that is not a valid patch corner counts at the nearest
      // one, where the filters aggregate its estimate
      int py, px;
      split_pos(row[k], d.W, rW, py, px);
      py = min(max(py, 0), d.Hp - 1);
      px = min(max(px, 0), d.Wp - 1);
      atomicAdd(d.hist + py * d.W + px, 1);
    }
  });
}

// cnt += 8x8 box sum of hist over valid top-left corners, one
// BOX_TY x BOX_TX output tile per item (vertical then horizontal sums in LDS).
__global__ __launch_bounds__(256) void k_count_box(Launch L) {
  __shared__ int h[BOX_TY + PS - 1][BOX_TX + PS - 1];
  __shared__ int v[BOX_TY][BOX_TX + PS - 1];
  for_each_item<W_BOX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int ntx = (d.W + BOX_TX - 1) / BOX_TX;
    const int y0 = (item / ntx) * BOX_TY, x0 = (item % ntx) * BOX_TX;
    __syncthreads();
    for (int e = threadIdx.x; e < (BOX_TY + PS - 1) * (BOX_TX + PS - 1); e += blockDim.x) {
      const int yy = e / (BOX_TX + PS - 1), xx = e % (BOX_TX + PS - 1);
      const int gy = y0 + yy - (PS - 1), gx = x0 + xx - (PS - 1);
      h[yy][xx] = (gy >= 0 && gy < d.Hp && gx >= 0 && gx < d.Wp) ? d.hist[gy * d.W + gx] : 0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < BOX_TY * (BOX_TX + PS - 1); e += blockDim.x) {
      const int yy = e / (BOX_TX + PS - 1), xx = e % (BOX_TX + PS - 1);
      int a = 0;
#pragma unroll
      for (int k = 0; k < PS; ++k) a += h[yy + k][xx];
      v[yy][xx] = a;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < BOX_TY * BOX_TX; e += blockDim.x) {
      const int yy = e / BOX_TX, xx = e % BOX_TX;
      const int gy = y0 + yy, gx = x0 + xx;
      if (gy < d.H && gx < d.W) {
        int a = 0;
#pragma unroll
        for (int k = 0; k < PS; ++k) a += v[yy][xx + k];
        d.cnt[gy * d.W + gx] += (float)a;
      }
    }
  });
}

static int grid_for(const Launch& L, int grid) { return xcd_grid(grid > 0 && grid < L.total ? grid : L.total); }

hipError_t launch_quant(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quant, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_gcp(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gcp, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_reset_counters(const Launch& L, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_absmax(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_absmax, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_zero_accum(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_accum, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_finalize(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
__global__ void k_fill(float* p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill(float* p, int n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_zero_hist(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_hist, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_count_hist(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_hist, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_count_box(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_box, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_adjoint_prep(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adjoint_prep, dim3(grid_for(L, grid)), dim3(256), 0, s, L);
  return hipGetLastError();
}

}  // namespace hts

namespace hts {

// Deterministic structured test image for the autotuner: smooth pattern plus
// a hashed pseudo-noise whose standard deviation sweeps 5..50 across the
// columns (low noise is the hard case for the distance-tile error bound).
__global__ __launch_bounds__(256) void k_synth(float* img, int C, int H, int W) {
  const int n = C * H * W;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c = i / (H * W), p = i % (H * W), y = p / W, x = p % W;
    unsigned h = (unsigned)i * 2654435761u + 12345u;
    h ^= h >> 15; h *= 2246822519u; h ^= h >> 13; h *= 3266489917u; h ^= h >> 16;
    const float u = (h & 0xFFFFFF) * (1.0f / 16777216.0f) - 0.5f;
    const float sd = 5.f + 45.f * (float)x / (float)W;
    img[i] = 128.f + 60.f * __sinf(x * 0.13f + c) * __cosf(y * 0.09f) + 3.4641f * sd * u;
  }
}

hipError_t launch_synth(float* img, int C, int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(k_synth, dim3(1024), dim3(256), 0, s, img, C, H, W);
  return hipGetLastError();
}

}  // namespace hts
