// Noise-level adjustment of A-Haar-tSVD (Sec. III-C, Eq. 21-22; Algorithm
// A-Haar-tSVD Step 1), for a caller-supplied sigma_est.
//
// circ(G) circ(G)^T of a group G = (p_1 .. p_K) along its group mode has the
// K nonzero eigenvalues lambda_m = sum over the patch values of
// |DFT_K(p_1 .. p_K)[m]|^2; Eq. 21's lambda-hat (alternating eigenvector) is
// lambda_{K/2}.  Its 1-based ascending rank a = 1 + #{m : lambda_m <
// lambda-hat} votes for sigma_est / beta when a <= gamma (Eq. 22); more than
// half of the sampled groups decide.
//
// One work group per image; each wavefront takes every fourth sampled group.
// Lane = patch pixel (a, b); for every frequency m the lanes form their
// pixel's K-point DFT term in FP64 and the squared moduli are summed across
// the wavefront by a fixed butterfly, so the result does not depend on
// scheduling.  Lane m keeps lambda_m; the rank is one ballot.
#include "hts_device.h"

namespace hts {

template <int K>
__global__ __launch_bounds__(256) void k_vote(Launch L) {
  __shared__ double tw[2][K];   // cos, sin of 2 pi j / K
  __shared__ int votes[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pa = lane >> 3, pb = lane & 7;   // this lane's pixel of the patch
  if (tid < K) {
    double sn, cs;
    sincospi(2.0 * tid / K, &sn, &cs);   // exact at j = 0, K/4, K/2, 3K/4
    tw[0][tid] = cs;
    tw[1][tid] = sn;
  }
  __syncthreads();
  const int nimg = L.table ? L.n_img : 1;
  for (int im = blockIdx.x; im < nimg; im += gridDim.x) {
    const ImgDesc& d = L.table ? L.table[im] : L.one;
    const int ns = d.n_samples;
    if (ns <= 0 || !d.samples || !d.sigma_dev) continue;   // same for the whole block
    const int HW = d.H * d.W;
    const float rW = 1.0f / (float)d.W;
    int myv = 0;
    for (int t = wave; t < ns; t += 4) {
      const int ref = min(max(d.samples[t], 0), d.n_ref - 1);
      const int* gidx = d.idx + (size_t)ref * K;
      int off[K];   // this lane's pixel in patch k (channel 0)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        int py, px;
        split_pos(gidx[k], d.W, rW, py, px);
        py = min(max(py, 0), d.Hp - 1);
        px = min(max(px, 0), d.Wp - 1);
        off[k] = (py + pa) * d.W + px + pb;
      }
      double mine = 0.0;   // lambda_m of lane m
      for (int ch = 0; ch < L.C; ++ch) {
        float x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = d.img[ch * HW + off[k]];
        for (int m = 0; m < K; ++m) {
          double re = 0.0, imv = 0.0;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int j = (k * m) & (K - 1);
            re = fma((double)x[k], tw[0][j], re);
            imv = fma(-(double)x[k], tw[1][j], imv);
          }
          double v = fma(re, re, imv * imv);
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
          if (lane == m) mine += v;
        }
      }
      const double lh = __shfl(mine, K / 2, 64);
      const int below = __popcll(__ballot(lane < K && mine < lh));
      const int rank = 1 + below;
      if (d.ranks && lane == 0) d.ranks[t] = rank;
      myv += rank <= d.gamma ? 1 : 0;
    }
    if (lane == 0) votes[wave] = myv;
    __syncthreads();
    if (tid == 0) {
      const int v = votes[0] + votes[1] + votes[2] + votes[3];
      *d.sigma_dev = 2 * v > ns ? d.sigma / d.beta : d.sigma;
    }
    __syncthreads();
  }
}

hipError_t launch_vote(const Launch& L, hipStream_t s) {
  const int n = L.table ? L.n_img : 1;
  switch (L.K) {
    case 2: hipLaunchKernelGGL(k_vote<2>, dim3(n), dim3(256), 0, s, L); break;
    case 4: hipLaunchKernelGGL(k_vote<4>, dim3(n), dim3(256), 0, s, L); break;
    case 8: hipLaunchKernelGGL(k_vote<8>, dim3(n), dim3(256), 0, s, L); break;
    case 16: hipLaunchKernelGGL(k_vote<16>, dim3(n), dim3(256), 0, s, L); break;
    case 32: hipLaunchKernelGGL(k_vote<32>, dim3(n), dim3(256), 0, s, L); break;
    case 64: hipLaunchKernelGGL(k_vote<64>, dim3(n), dim3(256), 0, s, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hts
