// Noise-level adjustment of A-Haar-tSVD (Sec. III.D, Eq. 21-22; Algorithm
// A-Haar-tSVD Step 1), for a caller-supplied sigma_est.
//
// circ(G) circ(G)^T of a group G = (p_1 .. p_K) along its group mode has the
// K nonzero eigenvalues lambda_m = sum over the patch values of
// |DFT_K(p_1 .. p_K)[m]|^2; Eq. 21's lambda-hat (alternating eigenvector) is
// lambda_{K/2}.  Its 1-based ascending rank a = 1 + #{m : lambda_m <
// lambda-hat} votes for sigma_est / beta when a <= gamma (Eq. 22); more than
// half of the sampled groups decide.
//
// One work group of eight (four) wavefronts per image; each wavefront takes
// every eighth (fourth) sampled group.  Lane = patch pixel (a, b); for every frequency m
// the lanes form their pixel's K-point DFT terms (all channels) in FP64 and
// the squared moduli are summed across the wavefront by a fixed butterfly,
// so the result does not depend on scheduling.  Lane m keeps lambda_m; the
// rank is one ballot.
#include "hts_device.h"

namespace hts {

// wavefronts per work group: eight, or four where a lane's group values
// (C*K doubles) need more than half of the registers of two waves per SIMD
template <int K, int C>
constexpr int vote_waves() { return C * K >= 96 ? 4 : 8; }

template <int K, int C>
__global__ __launch_bounds__((64 * vote_waves<K, C>())) void k_vote(Launch L) {
  constexpr int VOTE_WAVES = vote_waves<K, C>();
  __shared__ double tw[2][K];   // cos, sin of 2 pi j / K
  __shared__ int votes[VOTE_WAVES];
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
    for (int t = wave; t < ns; t += VOTE_WAVES) {
      const int ref = min(max(d.samples[t], 0), d.n_ref - 1);
      const int* gidx = d.idx + (size_t)ref * K;
      double x[C][K];   // this lane's pixel in the K patches, every channel
#pragma unroll
      for (int k = 0; k < K; ++k) {
        int py, px;
        split_pos(gidx[k], d.W, rW, py, px);
        py = min(max(py, 0), d.Hp - 1);
        px = min(max(px, 0), d.Wp - 1);
        const int off = (py + pa) * d.W + px + pb;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) x[ch][k] = (double)d.img[ch * HW + off];
      }
      // lambda_m = lambda_{K-m} for real groups: frequencies 0..K/2 suffice,
      // each m in 1..K/2-1 standing for its pair
      double mine = 0.0;   // lambda_m of lane m (m <= K/2)
      for (int m = 0; m <= K / 2; ++m) {
        double v = 0.0;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          double re = 0.0, imv = 0.0;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int j = (k * m) & (K - 1);
            re = fma(x[ch][k], tw[0][j], re);
            imv = fma(-x[ch][k], tw[1][j], imv);
          }
          v = fma(re, re, fma(imv, imv, v));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == m) mine = v;
      }
      const double lh = __shfl(mine, K / 2, 64);
      const bool lt = lane <= K / 2 && mine < lh;
      const unsigned long long bl = __ballot(lt);
      // lane 0 counts once, lanes 1..K/2-1 twice (their pair K - m)
      const int below = (int)(bl & 1ull) + 2 * __popcll(bl & ~1ull);
      const int rank = 1 + below;
      if (d.ranks && lane == 0) d.ranks[t] = rank;
      myv += rank <= d.gamma ? 1 : 0;
    }
    if (lane == 0) votes[wave] = myv;
    __syncthreads();
    if (tid == 0) {
      int v = 0;
      for (int w = 0; w < VOTE_WAVES; ++w) v += votes[w];
      *d.sigma_dev = 2 * v > ns ? d.sigma / d.beta : d.sigma;
    }
    __syncthreads();
  }
}

template <int C>
static hipError_t launch_vote_c(const Launch& L, int n, hipStream_t s) {
  const dim3 g(n);
  switch (L.K) {
    case 2: hipLaunchKernelGGL((k_vote<2, C>), g, dim3(64 * vote_waves<2, C>()), 0, s, L); break;
    case 4: hipLaunchKernelGGL((k_vote<4, C>), g, dim3(64 * vote_waves<4, C>()), 0, s, L); break;
    case 8: hipLaunchKernelGGL((k_vote<8, C>), g, dim3(64 * vote_waves<8, C>()), 0, s, L); break;
    case 16: hipLaunchKernelGGL((k_vote<16, C>), g, dim3(64 * vote_waves<16, C>()), 0, s, L); break;
    case 32: hipLaunchKernelGGL((k_vote<32, C>), g, dim3(64 * vote_waves<32, C>()), 0, s, L); break;
    case 64:
      if constexpr (C == 1) {   // K = 64 is grey only
        hipLaunchKernelGGL((k_vote<64, 1>), g, dim3(64 * vote_waves<64, 1>()), 0, s, L);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vote(const Launch& L, hipStream_t s) {
  const int n = L.table ? L.n_img : 1;
  return L.C == 1 ? launch_vote_c<1>(L, n, s) : launch_vote_c<3>(L, n, s);
}

}  // namespace hts
