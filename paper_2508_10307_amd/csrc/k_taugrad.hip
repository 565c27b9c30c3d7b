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
// (a, b).  The projection's row and column sums go through a small LDS tile;
// each lane's element of the K slots' real core tensors of y and of r (C*K
// values each) is parked in LDS, then the Haar transform along the group
// runs in the lane's registers.  Each group's sum (FP64, fixed butterfly across the
// wavefront) goes to partial[g]; k_taugrad_sum adds the partials in order, so
// the result is the same on every run.
#include "hts_device.h"

namespace hts {

namespace {

constexpr double TG_SQ3_2 = 0.86602540378443864676;   // sqrt(3) / 2

// Y = P V (if right) or Z = U^H P (else) for one 8x8 complex slice held one
// element per lane: element (a, b) of the product from the LDS copy of P.
// B is the basis slice pair (re, im) in row-major [r][c] order (im nullable).
__device__ inline void slice_product(float (*lr)[8], float (*li)[8], int a, int b, const float* Br,
                                     const float* Bi, bool right, double& outr, double& outi) {
  double yr = 0.0, yi = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    // right: sum_t P[a][t] V[t][b];  left: sum_t conj(U[t][a]) P[t][b]
    const double pr = right ? lr[a][t] : lr[t][b];
    const double pi = right ? li[a][t] : li[t][b];
    const double br = right ? Br[t * 8 + b] : Br[t * 8 + a];
    const double bi = Bi ? (right ? Bi[t * 8 + b] : -(double)Bi[t * 8 + a]) : 0.0;
    yr = fma(pr, br, fma(-pi, bi, yr));
    yi = fma(pr, bi, fma(pi, br, yi));
  }
  outr = yr;
  outi = yi;
}

}  // namespace

template <int K, int C>
__global__ __launch_bounds__(64) void k_taugrad(Launch L, const float* g, double* partial,
                                                 float kappa) {
  __shared__ float lr[8][8], li[8][8];
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
#pragma unroll
      for (int which = 0; which < 2; ++which) {
        float p[C];
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
          p[ch] = which == 0 ? d.img[ch * HW + pix] : g[ch * HW + pix] * rc;
        double z0 = 0.0, z1r = 0.0, z1i = 0.0;
        // f = 0 (real) and, for c = 3, f = 1 (complex): Z = U_F^H (P^ V_F)
#pragma unroll
        for (int f = 0; f < (C == 3 ? 2 : 1); ++f) {
          double pr, pi;
          if (C == 1) {
            pr = p[0];
            pi = 0.0;
          } else if (f == 0) {
            pr = (double)p[0] + (double)p[1] + (double)p[2];
            pi = 0.0;
          } else {
            pr = (double)p[0] - 0.5 * ((double)p[1] + (double)p[2]);
            pi = TG_SQ3_2 * ((double)p[2] - (double)p[1]);
          }
          __syncthreads();
          lr[a][b] = (float)pr;
          li[a][b] = (float)pi;
          __syncthreads();
          double yr, yi;
          slice_product(lr, li, a, b, fb + (f ? FB_V1R : FB_V0), f ? fb + FB_V1I : nullptr, true,
                        yr, yi);
          __syncthreads();
          lr[a][b] = (float)yr;
          li[a][b] = (float)yi;
          __syncthreads();
          double zr, zi;
          slice_product(lr, li, a, b, fb + (f ? FB_U1R : FB_U0), f ? fb + FB_U1I : nullptr, false,
                        zr, zi);
          if (f == 0) z0 = zr;
          else { z1r = zr; z1i = zi; }
        }
        // inverse DFT along the channel mode: T_j = (Z_0 + 2 Re(Z_1 e^{2 pi i j / 3})) / 3
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          double t;
          if (C == 1) t = z0;
          else if (ch == 0) t = (z0 + 2.0 * z1r) / 3.0;
          else if (ch == 1) t = (z0 - z1r - 2.0 * TG_SQ3_2 * z1i) / 3.0;
          else t = (z0 - z1r + 2.0 * TG_SQ3_2 * z1i) / 3.0;
          core[which][k][ch][lane] = (float)t;
        }
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
    // orthonormal Haar along the group (pairs of running sums, 1/sqrt 2 per
    // level); the coefficient order does not enter the sum below
#pragma unroll
    for (int st = 1; st < K; st <<= 1)
#pragma unroll
      for (int k = 0; k < K; k += 2 * st)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          const float us = ts[k][ch], vs = ts[k + st][ch];
          ts[k][ch] = (us + vs) * 0.70710678118654752440f;
          ts[k + st][ch] = (us - vs) * 0.70710678118654752440f;
          const float ur = tr[k][ch], vr = tr[k + st][ch];
          tr[k][ch] = (ur + vr) * 0.70710678118654752440f;
          tr[k + st][ch] = (ur - vr) * 0.70710678118654752440f;
        }
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
