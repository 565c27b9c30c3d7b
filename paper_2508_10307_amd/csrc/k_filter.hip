// Launches of the vector-ALU filter (kernel template in filter_valu.h):
// uniform or weighted aggregation, real-domain threshold (Eq. 19); the
// channel-Fourier threshold variant is launched from k_filter_ft.hip.
#include "filter_valu.h"
#include "video_internal.h"

namespace hts {

size_t filter_lds_bytes(int C, int K, int stride, int window, int ty, int tx, bool weighted) {
  (void)K;
  const int r = (window - 1) / 2;
  const size_t RA = (size_t)(ty - 1) * stride + 2 * r + PS;
  const size_t CA = (size_t)(tx - 1) * stride + 2 * r + PS;
  const size_t NP = C + (weighted ? 1 : 0);
  return ((2 * NP * RA * CA + 3) / 4 * 4 + 4 * TSCRATCH) * sizeof(float);
}

template <int C, int ADJ, int MASKS, int BATCH, int WT = 0>
static hipError_t launch_filter_c(const Launch& L, int g, size_t lds, hipStream_t s) {
  constexpr int FT = 0;
  switch (L.K) {
    case 2: case 4: case 8:
      hipLaunchKernelGGL((k_filter<C, 1, ADJ, MASKS, BATCH, WT, FT>), dim3(g), dim3(256), lds, s, L); break;
    case 16:
      hipLaunchKernelGGL((k_filter<C, 2, ADJ, MASKS, BATCH, WT, FT>), dim3(g), dim3(256), lds, s, L); break;
    case 32:
      hipLaunchKernelGGL((k_filter<C, 4, ADJ, MASKS, BATCH, WT, FT>), dim3(g), dim3(256), lds, s, L); break;
    case 64:
      if constexpr (C == 1) {
        hipLaunchKernelGGL((k_filter<C, 8, ADJ, MASKS, BATCH, WT, FT>), dim3(g), dim3(256), lds, s, L);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_filter(const Launch& L, int ty, int tx, int adjoint, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  const int g = xcd_grid(grid > 0 && grid < L.total ? grid : L.total);
  const bool wt = !adjoint && (L.flags & HTS_FLAG_WEIGHTED);
  const size_t lds = filter_lds_bytes(L.C, L.K, L.stride, L.window, ty, tx, wt);
  // batched launches (descriptor table) export masks when L.batch_masks is
  // set (uniform weights, Eq. 19 only) and run the adjoint when asked
  const bool batch = L.table != nullptr;
  const bool masks = batch ? L.batch_masks != 0 : L.one.masks != nullptr;
  if (batch && masks && (wt || (L.flags & HTS_FLAG_FOURIER_THRESHOLD))) return hipErrorInvalidValue;
  if (L.C == 3 && !adjoint && (L.flags & HTS_FLAG_FOURIER_THRESHOLD))
    return launch_filter_ft(L, g, lds, batch, masks, wt, s);
  if (wt) {   // weighted aggregation: no adjoint
    if (L.C == 1) {
      if (batch) return launch_filter_c<1, 0, 0, 1, 1>(L, g, lds, s);
      return masks ? launch_filter_c<1, 0, 1, 0, 1>(L, g, lds, s) : launch_filter_c<1, 0, 0, 0, 1>(L, g, lds, s);
    }
    if (batch) return launch_filter_c<3, 0, 0, 1, 1>(L, g, lds, s);
    return masks ? launch_filter_c<3, 0, 1, 0, 1>(L, g, lds, s) : launch_filter_c<3, 0, 0, 0, 1>(L, g, lds, s);
  }
  if (L.C == 1) {
    if (adjoint) return batch ? launch_filter_c<1, 1, 0, 1>(L, g, lds, s) : launch_filter_c<1, 1, 0, 0>(L, g, lds, s);
    if (batch) return masks ? launch_filter_c<1, 0, 1, 1>(L, g, lds, s) : launch_filter_c<1, 0, 0, 1>(L, g, lds, s);
    return masks ? launch_filter_c<1, 0, 1, 0>(L, g, lds, s) : launch_filter_c<1, 0, 0, 0>(L, g, lds, s);
  }
  if (adjoint) return batch ? launch_filter_c<3, 1, 0, 1>(L, g, lds, s) : launch_filter_c<3, 1, 0, 0>(L, g, lds, s);
  if (batch) return masks ? launch_filter_c<3, 0, 1, 1>(L, g, lds, s) : launch_filter_c<3, 0, 0, 1>(L, g, lds, s);
  return masks ? launch_filter_c<3, 0, 1, 0>(L, g, lds, s) : launch_filter_c<3, 0, 0, 0>(L, g, lds, s);
}

// Row projections (the first product of the filter's t-SVD projection,
// hoisted out of the group loop): one thread per output position (row y,
// column start x < Wp), taken in the order of the [H][Wp] output.  The
// row's 8 pixels of every channel go through the channel DFT and the
// products with the V slices in exactly the order the filter used to apply
// them per slot, so every estimate keeps its bits.  A non-finite pixel
// makes all 8 C values of every row window over it non-finite (each V
// column has a non-zero entry), which the filter's poison check sees.
// A work group's 256 consecutive positions have one contiguous output
// range: their values are staged in LDS and written out in 16-byte pieces
// by consecutive lanes (written directly, each lane's 8 C values would
// spread one store instruction over dozens of cache lines).
template <int C>
__global__ __launch_bounds__(256) void k_rowproj(Launch L) {
  constexpr int NF = 8 * C;   // floats per position
  __shared__ __align__(16) float stage[256 * NF];
  for_each_item<W_PIX>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int NQ = d.H * d.Wp;
    const int q0 = item * PIX_CHUNK;
    const int q1 = min(NQ, q0 + PIX_CHUNK);
    const cfloat* fb = uniform_ptr(d.fbasis);
    for (int qb = q0; qb < q1; qb += blockDim.x) {
      const int q = qb + (int)threadIdx.x;
      if (q < q1) {
        const int y = q / d.Wp, x = q - y * d.Wp;
        const float* src = d.img + (size_t)y * d.W + x;
        float* dst = stage + threadIdx.x * NF;
        if (C == 1) {
          float xr[8], yv[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) xr[b] = src[b];
          mv<false>(xr, fb, FB_V0T, 1.f, yv);   // y[b] = sum_t x[t] V[t][b]
#pragma unroll
          for (int b = 0; b < 8; ++b) dst[b] = yv[b];
        } else {
          float f0[8], f1r[8], f1i[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const float q0v = src[b], q1v = src[HW + b], q2v = src[2 * HW + b];
            f0[b] = q0v + q1v + q2v;
            f1r[b] = q0v - 0.5f * (q1v + q2v);
            f1i[b] = HALF_SQRT3 * (q2v - q1v);
          }
          float y0[8], y1r[8], y1i[8];
          mv<false>(f0, fb, FB_V0T, 1.f, y0);
          // y1 = V_F(1)^T P^(1) per row: (V1R + i V1I)^T (f1r + i f1i)
          cmv(f1r, f1i, fb, FB_V1RT, FB_V1IT, 1.f, FB_V1PT, y1r, y1i);
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            dst[b] = y0[b];
            dst[8 + b] = y1r[b];
            dst[16 + b] = y1i[b];
          }
        }
      }
      __syncthreads();
      const int n4 = min((int)blockDim.x, q1 - qb) * (NF / 4);
      const float4* s4 = (const float4*)stage;
      float4* d4 = (float4*)(d.rowp + (size_t)qb * NF);
      for (int i = threadIdx.x; i < n4; i += blockDim.x) d4[i] = s4[i];
      __syncthreads();
    }
  });
}

hipError_t launch_rowproj(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  const int g = xcd_grid(grid > 0 && grid < L.total ? grid : L.total);
  if (L.C == 1) hipLaunchKernelGGL(k_rowproj<1>, dim3(g), dim3(256), 0, s, L);
  else if (L.C == 3) hipLaunchKernelGGL(k_rowproj<3>, dim3(g), dim3(256), 0, s, L);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// Stand-alone aggregation of precomputed group estimates (Eq. 2 numerator
// and denominator): one wavefront per group, lane = slot-row.
__global__ __launch_bounds__(256) void k_scatter_est(Launch L, const float* est, int C) {
  const ImgDesc& d = L.one;
  const int K = L.K;
  const int HW = d.H * d.W;
  const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (gw >= d.ref_count) return;
  const int g = d.ref_begin + gw;
  const float rW = 1.0f / (float)d.W;
  for (int e = lane; e < K * PS; e += 64) {
    const int k = e >> 3, a = e & 7;
    const int pos = d.idx[(size_t)g * K + k];
    // positions come from the caller's idx: clamp to valid patch corners
    int py, px;
    split_pos(pos, d.W, rW, py, px);
    py = min(max(py, 0), d.Hp - 1);
    px = min(max(px, 0), d.Wp - 1);
    for (int ch = 0; ch < C; ++ch)
      for (int b = 0; b < 8; ++b)
        atomicAdd(d.num + ch * HW + (py + a) * d.W + px + b,
                  est[(((size_t)gw * K + k) * C + ch) * PS2 + a * 8 + b]);
    for (int b = 0; b < 8; ++b) atomicAdd(d.cnt + (py + a) * d.W + px + b, 1.0f);
  }
}

hipError_t launch_scatter_est(const Launch& L, hipStream_t s) {
  const int n = L.one.ref_count;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_est, dim3((n + 3) / 4), dim3(256), 0, s, L, L.one.group_est, L.C);
  return hipGetLastError();
}

// Export instantiation (WT = 2): the groups of a tile may reach beyond its
// search windows (the stacked frames of a video), so there is no LDS tile,
// only the transpose scratch; every slot's estimate goes to L.one.group_est
// (fixed-point scaled; k_gather_tiles adds them up).
hipError_t launch_filter_stacked(const Launch& L, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  if (L.table || !L.one.group_est || !L.one.num64 || (L.C != 1 && L.C != 3)) return hipErrorInvalidValue;
  const int g = xcd_grid(L.total);
  const size_t lds = 4 * TSCRATCH * sizeof(float);
  const bool masks = L.one.masks != nullptr;
  if (L.C == 1)
    return masks ? launch_filter_c<1, 0, 1, 0, 2>(L, g, lds, s) : launch_filter_c<1, 0, 0, 0, 2>(L, g, lds, s);
  return masks ? launch_filter_c<3, 0, 1, 0, 2>(L, g, lds, s) : launch_filter_c<3, 0, 0, 0, 2>(L, g, lds, s);
}

}  // namespace hts
