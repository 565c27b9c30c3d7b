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
  // batched launches (descriptor table) never export masks nor run the adjoint
  const bool batch = L.table != nullptr;
  if (batch && adjoint) return hipErrorInvalidValue;
  const bool masks = !batch && L.one.masks;
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
    if (batch) return launch_filter_c<1, 0, 0, 1>(L, g, lds, s);
    if (adjoint) return launch_filter_c<1, 1, 0, 0>(L, g, lds, s);
    return masks ? launch_filter_c<1, 0, 1, 0>(L, g, lds, s) : launch_filter_c<1, 0, 0, 0>(L, g, lds, s);
  }
  if (batch) return launch_filter_c<3, 0, 0, 1>(L, g, lds, s);
  if (adjoint) return launch_filter_c<3, 1, 0, 0>(L, g, lds, s);
  return masks ? launch_filter_c<3, 0, 1, 0>(L, g, lds, s) : launch_filter_c<3, 0, 0, 0>(L, g, lds, s);
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

// Global aggregation (WT = 2): the groups of a tile may reach beyond its
// search windows (the stacked frames of a video), so there is no LDS tile,
// only the transpose scratch; no group estimates.
hipError_t launch_filter_stacked(const Launch& L, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  if (L.table || L.one.group_est || !L.one.num64 || (L.C != 1 && L.C != 3)) return hipErrorInvalidValue;
  const int g = xcd_grid(L.total);
  const size_t lds = 4 * TSCRATCH * sizeof(float);
  const bool masks = L.one.masks != nullptr;
  if (L.C == 1)
    return masks ? launch_filter_c<1, 0, 1, 0, 2>(L, g, lds, s) : launch_filter_c<1, 0, 0, 0, 2>(L, g, lds, s);
  return masks ? launch_filter_c<3, 0, 1, 0, 2>(L, g, lds, s) : launch_filter_c<3, 0, 0, 0, 2>(L, g, lds, s);
}

}  // namespace hts
