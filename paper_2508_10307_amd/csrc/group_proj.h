// Per-element t-SVD projection for the one-wavefront group kernels of the
// adjoint extensions (k_taugrad, k_gbasis): lane = patch element (a, b); the
// 8x8 slice products go through LDS tiles.
#pragma once
#include "hts_device.h"

namespace hts {

constexpr double GP_SQ3_2 = 0.86602540378443864676;   // sqrt(3) / 2

// Real core tensors T = U^T * P * V (t-product, Eq. 18) of two patches at
// this lane's element, from their C channel values p[0], p[1] there: per
// frequency f <= c/2, Z(f) = U_F(f)^H (P^(f) V_F(f)), then the inverse DFT
// along the channel mode, T_j = (Z_0 + 2 Re(Z_1 e^{2 pi i j / 3})) / 3.  Both
// patches and all frequencies share three work-group barriers: X (the DFTs
// of the bands) and Y = X V_F live in LDS tiles [which * NF + f][re/im][64];
// fb holds the Fourier basis slices (FB_* layout).  One wavefront per work
// group.
template <int C>
__device__ inline void project_pair(float (*X)[2][64], float (*Y)[2][64], int lane,
                                    const float* fb, const float (&p)[2][C], float (&t)[2][C]) {
  constexpr int NF = C == 3 ? 2 : 1;
  const int a = lane >> 3, b = lane & 7;
  __syncthreads();   // the previous call's readers of X and Y are done
#pragma unroll
  for (int w = 0; w < 2; ++w)
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      float xr, xi;
      if (C == 1) { xr = p[w][0]; xi = 0.f; }
      else if (f == 0) { xr = (float)((double)p[w][0] + (double)p[w][1] + (double)p[w][2]); xi = 0.f; }
      else {
        xr = (float)((double)p[w][0] - 0.5 * ((double)p[w][1] + (double)p[w][2]));
        xi = (float)(GP_SQ3_2 * ((double)p[w][2] - (double)p[w][1]));
      }
      X[w * NF + f][0][lane] = xr;
      X[w * NF + f][1][lane] = xi;
    }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 2 * NF; ++m) {
    const int f = m % NF;
    const float* Vr = fb + (f ? FB_V1R : FB_V0);
    const float* Vi = f ? fb + FB_V1I : nullptr;
    double yr = 0.0, yi = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {   // sum_q X(a, q) V(q, b)
      const double xr = X[m][0][a * 8 + q], xi = X[m][1][a * 8 + q];
      const double vr = Vr[q * 8 + b], vi = Vi ? Vi[q * 8 + b] : 0.0;
      yr = fma(xr, vr, fma(-xi, vi, yr));
      yi = fma(xr, vi, fma(xi, vr, yi));
    }
    Y[m][0][lane] = (float)yr;
    Y[m][1][lane] = (float)yi;
  }
  __syncthreads();
  double z[2][NF][2];
#pragma unroll
  for (int m = 0; m < 2 * NF; ++m) {
    const int f = m % NF;
    const float* Ur = fb + (f ? FB_U1R : FB_U0);
    const float* Ui = f ? fb + FB_U1I : nullptr;
    double zr = 0.0, zi = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {   // sum_q conj(U(q, a)) Y(q, b)
      const double yr = Y[m][0][q * 8 + b], yi = Y[m][1][q * 8 + b];
      const double ur = Ur[q * 8 + a], ui = Ui ? -(double)Ui[q * 8 + a] : 0.0;
      zr = fma(yr, ur, fma(-yi, ui, zr));
      zi = fma(yr, ui, fma(yi, ur, zi));
    }
    z[m / NF][f][0] = zr;
    z[m / NF][f][1] = zi;
  }
#pragma unroll
  for (int w = 0; w < 2; ++w)
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
      double v;
      if (C == 1) v = z[w][0][0];
      else if (ch == 0) v = (z[w][0][0] + 2.0 * z[w][NF - 1][0]) / 3.0;
      else if (ch == 1) v = (z[w][0][0] - z[w][NF - 1][0] - 2.0 * GP_SQ3_2 * z[w][NF - 1][1]) / 3.0;
      else v = (z[w][0][0] - z[w][NF - 1][0] + 2.0 * GP_SQ3_2 * z[w][NF - 1][1]) / 3.0;
      t[w][ch] = (float)v;
    }
}

// Orthonormal Haar along the group (Eq. 9) on K slots of C values, in
// place: level by level, pairs (k, k + st) become ((u + v), (u - v)) / sqrt 2,
// so slot k > 0 ends holding the coefficient of Haar row
// (K >> l) + (k >> l), l = ctz(k) + 1, and slot 0 the DC row.
template <int K, int C>
__device__ inline void haar_forward_slots(float (*x)[C]) {
#pragma unroll
  for (int st = 1; st < K; st <<= 1)
#pragma unroll
    for (int k = 0; k < K; k += 2 * st)
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        const float u = x[k][ch], v = x[k + st][ch];
        x[k][ch] = (u + v) * 0.70710678118654752440f;
        x[k + st][ch] = (u - v) * 0.70710678118654752440f;
      }
}

// Its inverse (the transpose): the same butterflies, coarsest level first.
template <int K, int C>
__device__ inline void haar_inverse_slots(float (*x)[C]) {
#pragma unroll
  for (int st = K >> 1; st >= 1; st >>= 1)
#pragma unroll
    for (int k = 0; k < K; k += 2 * st)
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        const float u = x[k][ch], v = x[k + st][ch];
        x[k][ch] = (u + v) * 0.70710678118654752440f;
        x[k + st][ch] = (u - v) * 0.70710678118654752440f;
      }
}

// Haar row (Eq. 9 ordering) of the coefficient in slot k after haar_forward_slots.
__host__ __device__ constexpr int haar_slot_row(int k, int K) {
  return k == 0 ? 0 : (K >> (__builtin_ctz(k) + 1)) + (k >> (__builtin_ctz(k) + 1));
}

}  // namespace hts
