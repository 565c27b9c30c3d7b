// Surrogate derivative of a loss with respect to the threshold (adjoint
// extension; the hard threshold of Eq. 19 has a zero derivative almost
// everywhere).  The keep-mask is relaxed to m(s) = phi((|s| - tau) / eps),
// phi the logistic function; with grouping, basis and coverage count frozen,
//   dL/dtau = sum over groups and coefficients of r * s * (-phi'(u) / eps),
//   s = Q Gather y,  r = Q Gather (g / cnt),  u = (|s| - tau) / eps,
// where Q = orthonormal Haar along the group (Eq. 9) o t-SVD projection
// (Eq. 18) and g = dL/dx_hat.
//
// One wavefront per work group, one group at a time; lane = patch element
// (a, b).  The projections of y and r share LDS tiles and three barriers;
// each lane's element of the K slots' real core tensors of y and of r (C*K
// values each) is parked in LDS, then the Haar transform along the group
// runs in the lane's registers.  Each group's sum (FP64, fixed butterfly across the
// wavefront) goes to partial[g]; k_taugrad_sum adds the partials in order, so
// the result is the same on every run.
#include "group_proj.h"

namespace hts {

template <int K, int C>
__global__ __launch_bounds__(64) void k_taugrad(Launch L, const float* g, double* partial,
                                                 float kappa) {
  __shared__ float PX[4][2][64], PY[4][2][64];   // projection tiles
  __shared__ float core[2][K][C][64];   // real core tensors of y and r, per lane
  const int lane = threadIdx.x;
  const int a = lane >> 3, b = lane & 7;
  const ImgDesc& d = L.one;
  const int HW = d.H * d.W;
  const float rW = 1.0f / (float)d.W;
  const float* fb = d.fbasis;
  const double tau = d.tau, eps = (double)d.sigma * (double)kappa;   // relaxation width
  for (int grp = blockIdx.x; grp < d.n_ref; grp += gridDim.x) {
    const int* gi = d.idx + (size_t)grp * K;
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      int py, px;
      split_pos(gi[k], d.W, rW, py, px);
      py = min(max(py, 0), d.Hp - 1);
      px = min(max(px, 0), d.Wp - 1);
      const int pix = (py + a) * d.W + px + b;
      const float rc = 1.0f / d.cnt[pix];
      float p[2][C], t[2][C];
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        p[0][ch] = d.img[ch * HW + pix];
        p[1][ch] = g[ch * HW + pix] * rc;
      }
      project_pair<C>(PX, PY, lane, fb, p, t);
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        core[0][k][ch][lane] = t[0][ch];
        core[1][k][ch][lane] = t[1][ch];
      }
    }
    // real core tensors of y (ts) and of r = g / cnt (tr): [slot][channel]
    float ts[K][C], tr[K][C];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        ts[k][ch] = core[0][k][ch][lane];
        tr[k][ch] = core[1][k][ch][lane];
      }
    // orthonormal Haar along the group; the coefficient order does not
    // enter the sum below
    haar_forward_slots<K, C>(ts);
    haar_forward_slots<K, C>(tr);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        const double s = ts[k][ch];
        const double u = (fabs(s) - tau) / eps;
        const double ph = 0.5 * (1.0 + tanh(0.5 * u));
        acc = fma((double)tr[k][ch] * s, -ph * (1.0 - ph) / eps, acc);
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) partial[grp] = acc;
  }
}

// out[0] = sigma * sum of the partials (in index order): dL/dlambda.
__global__ __launch_bounds__(256) void k_taugrad_sum(const double* partial, int n, float sigma,
                                                     float* out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  const int per = (n + 255) / 256;
  for (int i = tid * per; i < min(n, (tid + 1) * per); ++i) s += partial[i];
  red[tid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < 256; ++i) t += red[i];
    out[0] = (float)((double)sigma * t);
  }
}

template <int C>
static hipError_t launch_tg(const Launch& L, const float* g, double* partial, float kappa, int grid,
                            hipStream_t s) {
  switch (L.K) {
    case 2: hipLaunchKernelGGL((k_taugrad<2, C>), dim3(grid), dim3(64), 0, s, L, g, partial, kappa); break;
    case 4: hipLaunchKernelGGL((k_taugrad<4, C>), dim3(grid), dim3(64), 0, s, L, g, partial, kappa); break;
    case 8: hipLaunchKernelGGL((k_taugrad<8, C>), dim3(grid), dim3(64), 0, s, L, g, partial, kappa); break;
    case 16: hipLaunchKernelGGL((k_taugrad<16, C>), dim3(grid), dim3(64), 0, s, L, g, partial, kappa); break;
    case 32: hipLaunchKernelGGL((k_taugrad<32, C>), dim3(grid), dim3(64), 0, s, L, g, partial, kappa); break;
    case 64:
      if constexpr (C == 1) {
        hipLaunchKernelGGL((k_taugrad<64, 1>), dim3(grid), dim3(64), 0, s, L, g, partial, kappa);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_taugrad(const Launch& L, const float* g, double* partial, float kappa, float* out,
                          int grid, hipStream_t s) {
  const int n = L.one.n_ref;
  const int gr = min(n, grid > 0 ? grid : 2048);
  const hipError_t e = L.C == 1 ? launch_tg<1>(L, g, partial, kappa, gr, s)
                                 : launch_tg<3>(L, g, partial, kappa, gr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_taugrad_sum, dim3(1), dim3(256), 0, s, partial, n, L.one.sigma, out);
  return hipGetLastError();
}

}  // namespace hts
