// General band counts: the spectral tubes of HSI (a ps x ps x c patch, the
// other parameters unchanged), c other than 1 and 3.  The t-product keeps
// its Fourier-domain form along the channel mode, so for f = 0..floor(c/2)
// (the rest by conjugate symmetry; f = 0 and, for even c, f = c/2 real):
//
//  k_cov_gen       C_U(f) = sum_i P^_i(f) P^_i(f)^H, C_V(f) = sum_i P^_i^H P^_i
//                  (Eq. 11-12), FP64, one partial per reference tile, work
//                  items = (tile, chunk of GEN_FC frequencies); lane = patch
//                  element, P^ = DFT along the channel mode in FP64;
//  k_eig_gen       the partials in order, the 8x8 eigenproblems (parallel
//                  Jacobi, GEN_EIG_M per work group), descending order and
//                  phase convention (largest-modulus entry real positive,
//                  first on ties), into ufg and the eigenvalues;
//  k_tensor_gen    U(:,:,j) = (1/c) sum_f U_F(f) e^{2 pi i f j / c}, real;
//  k_fbasis_gen    float Fourier slices U_F(f) of the (float) real tensors;
//  k_filter_gen    Eq. 18-20 per group (or, with ADJ, the transpose of the
//                  frozen-mask map: the forward masks replace Eq. 19):
//                  per slot and frequency
//                  Z(f) = U_F^H P^(f) V_F (8x8 products through an LDS
//                  tile), the real core tensor by the inverse DFT into the
//                  work group's scratch, Haar along the group and the hard
//                  threshold per channel, then the inverse, aggregated in
//                  fixed point (Eq. 2; float atomics into a float numerator
//                  for hts_filter), optional per-group estimates.
//
// Twiddles come from sincospi (exact at the quarter points).
#include "jacobi8.h"
#include "group_proj.h"
#include "video_internal.h"

namespace hts {

namespace {

// e^{-2 pi i m / c} for m < c: (tc[m], ts[m]) = (cos, -sin).
template <typename T>
__device__ inline void fill_twiddles(T* tc, T* ts, int c) {
  for (int m = threadIdx.x; m < c; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)c, &sn, &cs);
    tc[m] = (T)cs;
    ts[m] = (T)(-sn);
  }
}

}  // namespace

size_t cov_gen_lds_bytes(int C) {
  return (size_t)2 * GEN_FC * 128 * 8 + 2 * 64 * 8 + (size_t)2 * C * 8 + (size_t)C * 64 * 4;
}

// Work item w = tile * nchunk + chunk over n_cov * nchunk items; lane = (a, b).
__global__ __launch_bounds__(64) void k_cov_gen(Launch L) {
  extern __shared__ double gsm[];
  const int C = L.C, NF = n_freq(C);
  const int nchunk = (NF + GEN_FC - 1) / GEN_FC;
  double* acc = gsm;                                  // [2 GEN_FC][re/im][64]
  double* pt = acc + 2 * GEN_FC * 128;                // [re/im][64]: P^(f)
  double* tc = pt + 128;                              // twiddles [C]
  double* ts = tc + C;
  float* pv = (float*)(ts + C);                       // [C][64] the patch's bands
  const int lane = threadIdx.x, a = lane >> 3, b = lane & 7;
  const ImgDesc& d = L.one;
  const int HW = d.H * d.W;
  const int tr = cov_tile(L.stride);
  const int ntx = (d.nrx + tr - 1) / tr;
  const int nel = cov_elems(C);
  fill_twiddles(tc, ts, C);
  __syncthreads();
  for (int w = blockIdx.x; w < L.total; w += gridDim.x) {
    const int tile = w / nchunk, chunk = w - tile * nchunk;
    const int f0 = chunk * GEN_FC, nf = min(GEN_FC, NF - f0);
    const int ty = tile / ntx, tx = tile - ty * ntx;
    for (int e = 0; e < 2 * GEN_FC * 2; ++e) acc[e * 64 + lane] = 0.0;
    for (int iy = ty * tr; iy < min(d.nry, ty * tr + tr); ++iy)
      for (int ix = tx * tr; ix < min(d.nrx, tx * tr + tr); ++ix) {
        const int ry = ref_coord(iy, L.stride, d.Hp), rx = ref_coord(ix, L.stride, d.Wp);
        const int pix = (ry + a) * d.W + rx + b;
        for (int j = 0; j < C; ++j) pv[j * 64 + lane] = d.img[(size_t)j * HW + pix];
        for (int fl = 0; fl < nf; ++fl) {
          const int f = f0 + fl;
          double pr = 0.0, pi = 0.0;
          for (int j = 0, m = 0; j < C; ++j, m = (m + f) % C) {
            const double v = pv[j * 64 + lane];
            pr = fma(v, tc[m], pr);
            pi = fma(v, ts[m], pi);
          }
          __syncthreads();
          pt[lane] = pr;
          pt[64 + lane] = pi;
          __syncthreads();
          // C_U(a,b) += sum_t P^(a,t) conj(P^(b,t));  C_V(a,b) += sum_t conj(P^(t,a)) P^(t,b)
          double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const double xr = pt[a * 8 + t], xi = pt[64 + a * 8 + t];
            const double yr = pt[b * 8 + t], yi = pt[64 + b * 8 + t];
            ur += xr * yr + xi * yi;
            ui += xi * yr - xr * yi;
            const double sr = pt[t * 8 + a], si = pt[64 + t * 8 + a];
            const double qr = pt[t * 8 + b], qi = pt[64 + t * 8 + b];
            vr += sr * qr + si * qi;
            vi += sr * qi - si * qr;
          }
          acc[(fl * 2 + 0) * 64 + lane] += ur;
          acc[(fl * 2 + 1) * 64 + lane] += ui;
          acc[((GEN_FC + fl) * 2 + 0) * 64 + lane] += vr;
          acc[((GEN_FC + fl) * 2 + 1) * 64 + lane] += vi;
        }
      }
    double* o = d.cov_part + (size_t)tile * nel;
    for (int fl = 0; fl < nf; ++fl) {
      const int f = f0 + fl;
      o[(f * 2 + 0) * 64 + lane] = acc[(fl * 2 + 0) * 64 + lane];
      o[(f * 2 + 1) * 64 + lane] = acc[(fl * 2 + 1) * 64 + lane];
      o[((NF + f) * 2 + 0) * 64 + lane] = acc[((GEN_FC + fl) * 2 + 0) * 64 + lane];
      o[((NF + f) * 2 + 1) * 64 + lane] = acc[((GEN_FC + fl) * 2 + 1) * 64 + lane];
    }
  }
}

// Work group w solves eigenproblems m = w * GEN_EIG_M .. (m = uv * NF + f).
__global__ __launch_bounds__(128) void k_eig_gen(Launch L) {
  __shared__ double mr[GEN_EIG_M][8][8], mi[GEN_EIG_M][8][8], vr[GEN_EIG_M][8][8], vi[GEN_EIG_M][8][8];
  const int C = L.C, NF = n_freq(C), NM = 2 * NF;
  const ImgDesc& d = L.one;
  const int nel = cov_elems(C);
  const int m0 = blockIdx.x * GEN_EIG_M, nm = min(GEN_EIG_M, NM - m0);
  const int tid = threadIdx.x;
  // ordered sum of the partials; eight loads in flight
  for (int e = tid; e < nm * 128; e += blockDim.x) {
    const int ml = e >> 7, ri = (e >> 6) & 1, ab = e & 63;
    const int src = (m0 + ml) * 128 + ri * 64 + ab;
    double s = 0.0;
    int j = 0;
    for (; j + 8 <= d.n_cov; j += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = d.cov_part[(size_t)(j + u) * nel + src];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; j < d.n_cov; ++j) s += d.cov_part[(size_t)j * nel + src];
    const int f = (m0 + ml) % NF;
    const bool real_f = f == 0 || 2 * f == C;
    if (ri == 0) mr[ml][ab >> 3][ab & 7] = s;
    else mi[ml][ab >> 3][ab & 7] = real_f ? 0.0 : s;
  }
  __syncthreads();
  jacobi_herm8_group(mr, mi, vr, vi, nm);
  if (tid < nm) {
    const int ml = tid, m = m0 + ml;
    int order[8];
    for (int k = 0; k < 8; ++k) order[k] = k;
    for (int q = 1; q < 8; ++q) {   // descending eigenvalues, stable
      const int key = order[q];
      int p = q - 1;
      while (p >= 0 && mr[ml][order[p]][order[p]] < mr[ml][key][key]) { order[p + 1] = order[p]; --p; }
      order[p + 1] = key;
    }
    double* ev = d.basis64 + 2 * C * 64 + m * 8;
    double* uf = d.ufg + (size_t)m * 128;
    for (int k = 0; k < 8; ++k) {
      const int src = order[k];
      ev[k] = mr[ml][src][src];
      int best = 0;
      double bm = -1.0;
      for (int q = 0; q < 8; ++q) {
        const double mm = vr[ml][q][src] * vr[ml][q][src] + vi[ml][q][src] * vi[ml][q][src];
        if (mm > bm) { bm = mm; best = q; }
      }
      const double nr = sqrt(bm);
      const double pr = vr[ml][best][src] / nr, pi = -vi[ml][best][src] / nr;   // conj(v) / |v|
      for (int q = 0; q < 8; ++q) {
        const double xr = vr[ml][q][src], xi = vi[ml][q][src];
        uf[q * 8 + k] = xr * pr - xi * pi;
        uf[64 + q * 8 + k] = q == best ? 0.0 : xr * pi + xi * pr;
      }
    }
  }
}

// Real tensors U(:,:,j), V(:,:,j) (FP64 and float) from the Fourier slices.
__global__ void k_tensor_gen(Launch L) {
  const int C = L.C, NF = n_freq(C);
  const ImgDesc& d = L.one;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * C * 64) return;
  const int uv = e / (C * 64), rem = e - uv * C * 64, j = rem >> 6, ab = rem & 63;
  double acc = 0.0;
  for (int f = 0; f < NF; ++f) {
    const double* uf = d.ufg + (size_t)(uv * NF + f) * 128;
    double sn, cs;
    sincospi(2.0 * (double)((f * j) % C) / (double)C, &sn, &cs);
    const double re = uf[ab], im = uf[64 + ab];
    const double w = (f == 0 || 2 * f == C) ? 1.0 : 2.0;     // conjugate partner f' = c - f
    acc += w * (re * cs - im * sn);
  }
  const double val = acc / (double)C;
  d.basis64[e] = val;
  d.basis[e] = (float)val;
}

// Covariance partials of one image (d.n_cov tiles from d.cov_part on).
hipError_t launch_cov_gen(const Launch& L, hipStream_t s) {
  const int NF = n_freq(L.C);
  const int nchunk = (NF + GEN_FC - 1) / GEN_FC;
  Launch Lc = L;
  Lc.total = L.one.n_cov * nchunk;
  if (Lc.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cov_gen, dim3(Lc.total), dim3(64), cov_gen_lds_bytes(L.C), s, Lc);
  return hipGetLastError();
}

// Eigen-solves of the d.n_cov partials and the real tensors.
hipError_t launch_eig_gen(const Launch& L, hipStream_t s) {
  const int C = L.C, NF = n_freq(C);
  hipLaunchKernelGGL(k_eig_gen, dim3((2 * NF + GEN_EIG_M - 1) / GEN_EIG_M), dim3(128), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tensor_gen, dim3((2 * C * 64 + 255) / 256), dim3(256), 0, s, L);
  return hipGetLastError();
}

hipError_t launch_basis_gen(const Launch& L, hipStream_t s) {
  const hipError_t e = launch_cov_gen(L, s);
  return e != hipSuccess ? e : launch_eig_gen(L, s);
}

// Float Fourier slices of the float real tensors, FP64 sums:
// fbasis[((uv * NF + f) * 2 + re/im) * 64 + ab].
__global__ void k_fbasis_gen(Launch L) {
  const int C = L.C, NF = n_freq(C);
  const ImgDesc& d = L.one;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * NF * 64) return;
  const int m = e >> 6, ab = e & 63, uv = m / NF, f = m % NF;
  const float* T = d.basis + uv * C * 64;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < C; ++j) {
    double sn, cs;
    sincospi(2.0 * (double)((f * j) % C) / (double)C, &sn, &cs);
    re += (double)T[j * 64 + ab] * cs;
    im -= (double)T[j * 64 + ab] * sn;
  }
  d.fbasis[(m * 2 + 0) * 64 + ab] = (float)re;
  d.fbasis[(m * 2 + 1) * 64 + ab] = (float)im;
}

hipError_t launch_fbasis_gen(const Launch& L, hipStream_t s) {
  const int NF = n_freq(L.C);
  hipLaunchKernelGGL(k_fbasis_gen, dim3((2 * NF * 64 + 255) / 256), dim3(256), 0, s, L);
  return hipGetLastError();
}

size_t filter_gen_lds_bytes(int C) {
  return ((size_t)C + (size_t)2 * n_freq(C) * 64) * sizeof(float2);
}

// One wavefront per work group, groups [ref_begin, ref_begin + ref_count)
// in a grid-stride loop; lane = patch element (a, b).  The work group's
// scratch holds the group's real core tensor [K][C][64].  Per slot, the
// products of all frequencies share two LDS round trips: X(f) (the DFT of
// the bands, lane-private entry) -> Y(f) = X(f) V_F(f) (or X(f) V_F(f)^H)
// -> U_F(f)^H Y(f) (or U_F(f) Y(f)) back into X(f).  Complex values and
// twiddles are float2 (one LDS access per complex operand); the lane's band
// values are parked in the Y area while the DFT reads them.
template <int K, int ADJ>
__global__ __launch_bounds__(64) void k_filter_gen(Launch L) {
  extern __shared__ float2 fsm2[];
  const int C = L.C, NF = n_freq(C);
  float2* tw = fsm2;               // e^{-2 pi i m / c} = (cos, -sin), m < c
  float2* X = tw + C;              // [NF][64]
  float2* Y = X + NF * 64;         // [NF][64]; the band values (float [C][64]) before the products
  float* Yb = (float*)Y;
  const int lane = threadIdx.x, a = lane >> 3, b = lane & 7;
  const ImgDesc& d = L.one;
  const int HW = d.H * d.W;
  const float rW = 1.0f / (float)d.W;
  const float* fb = d.fbasis;
  float* S = d.gscratch + (size_t)blockIdx.x * K * C * 64;
  const float tau = d.tau;
  const float fxs = fx_scale(d, false) / (float)C;   // 2^-32 units
  for (int m = threadIdx.x; m < C; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)C, &sn, &cs);
    tw[m] = make_float2((float)cs, (float)-sn);
  }
  __syncthreads();
  // Bands j and c - j share their cosines and have opposite sines, so the
  // DFTs below work on pairs: JH = floor((c - 1) / 2) pairs, band 0 and, for
  // even c, band c/2 on their own.
  const int JH = (C - 1) / 2;
  const bool even = (C & 1) == 0;
  // X(f) <- DFT of the lane's band values (in Y), f < NF:
  //   X(f) = x_0 + sum_{j <= JH} [(x_j + x_{c-j}) cos - i (x_j - x_{c-j}) sin](2 pi f j / c)
  //          (+ (-1)^f x_{c/2});
  // the band values are first turned into the pair sums (j) and differences
  // (c - j) in place; four frequencies per pass (m_f = f j mod c, kept by
  // adding f).
  auto dft_bands = [&]() {
    for (int j = 1; j <= JH; ++j) {
      const float u = Yb[j * 64 + lane], w = Yb[(C - j) * 64 + lane];
      Yb[j * 64 + lane] = u + w;
      Yb[(C - j) * 64 + lane] = u - w;
    }
    const float x0 = Yb[lane], xh = even ? Yb[(C / 2) * 64 + lane] : 0.f;
    for (int f0 = 0; f0 < NF; f0 += 4) {
      float xr[4], xi[4] = {0.f, 0.f, 0.f, 0.f};
      int m[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xr[u] = x0 + (((f0 + u) & 1) ? -xh : xh);
        m[u] = 0;
      }
#pragma unroll 4
      for (int j = 1; j <= JH; ++j) {
        const float sj = Yb[j * 64 + lane], dj = Yb[(C - j) * 64 + lane];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          m[u] += f0 + u;
          m[u] -= m[u] >= C ? C : 0;
          const float2 w = tw[m[u]];
          xr[u] = fmaf(sj, w.x, xr[u]);
          xi[u] = fmaf(dj, w.y, xi[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (f0 + u < NF) X[(f0 + u) * 64 + lane] = make_float2(xr[u], xi[u]);
    }
  };
  // c x the (1/c) IDFT of the lane's X(f), f < NF, scaled by sc, into band
  // j of dst (stride 64 floats): with A_j = sum_f w_f Re X(f) cos and
  // B_j = -sum_f w_f Im X(f) sin (w_f = 2, 1 at f = c/2),
  // t_j = X(0) + A_j + B_j and t_{c-j} = X(0) + A_j - B_j; four pairs per pass.
  auto idft_bands = [&](float* dst, float sc) {
    const float x0 = X[lane].x;
    float t0 = x0, th = x0;
    for (int f = 1; f < NF; ++f) {
      const float w = 2 * f == C ? 1.f : 2.f;
      const float zr = w * X[f * 64 + lane].x;
      t0 += zr;
      th += (f & 1) ? -zr : zr;
    }
    dst[lane] = t0 * sc;
    if (even) dst[(C / 2) * 64 + lane] = th * sc;
    for (int j0 = 1; j0 <= JH; j0 += 4) {
      float A[4] = {0.f, 0.f, 0.f, 0.f}, B[4] = {0.f, 0.f, 0.f, 0.f};
      int m[4] = {0, 0, 0, 0};
#pragma unroll 4
      for (int f = 1; f < NF; ++f) {
        const float w = 2 * f == C ? 1.f : 2.f;
        const float2 z = X[f * 64 + lane];
        const float zr = w * z.x, zi = w * z.y;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          m[u] += j0 + u;
          m[u] -= m[u] >= C ? C : 0;
          const float2 e = tw[m[u]];
          A[u] = fmaf(zr, e.x, A[u]);
          B[u] = fmaf(zi, e.y, B[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u <= JH) {
          dst[(j0 + u) * 64 + lane] = (x0 + A[u] + B[u]) * sc;
          dst[(C - j0 - u) * 64 + lane] = (x0 + A[u] - B[u]) * sc;
        }
    }
  };
  // X(f) <- U_F(f)^H X(f) V_F(f) (forward) or U_F(f) X(f) V_F(f)^H (inverse)
  auto products = [&](bool inverse) {
    __syncthreads();
    for (int f = 0; f < NF; ++f) {
      const float* Vr = fb + ((NF + f) * 2 + 0) * 64;
      const float* Vi = fb + ((NF + f) * 2 + 1) * 64;
      float yr = 0.f, yi = 0.f;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float2 p = X[f * 64 + a * 8 + t];
        const float vr = inverse ? Vr[b * 8 + t] : Vr[t * 8 + b];     // conj(V(b,t)) or V(t,b)
        const float vi = inverse ? -Vi[b * 8 + t] : Vi[t * 8 + b];
        yr += p.x * vr - p.y * vi;
        yi += p.x * vi + p.y * vr;
      }
      Y[f * 64 + lane] = make_float2(yr, yi);
    }
    __syncthreads();
    for (int f = 0; f < NF; ++f) {
      const float* Ur = fb + (f * 2 + 0) * 64;
      const float* Ui = fb + (f * 2 + 1) * 64;
      float zr = 0.f, zi = 0.f;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float2 p = Y[f * 64 + t * 8 + b];
        const float ur = inverse ? Ur[a * 8 + t] : Ur[t * 8 + a];     // U(a,t) or conj(U(t,a))
        const float ui = inverse ? Ui[a * 8 + t] : -Ui[t * 8 + a];
        zr += ur * p.x - ui * p.y;
        zi += ur * p.y + ui * p.x;
      }
      X[f * 64 + lane] = make_float2(zr, zi);
    }
  };
  for (int gl = blockIdx.x; gl < d.ref_count; gl += gridDim.x) {
    const int grp = d.ref_begin + gl;
    const int* gi = d.idx + (size_t)grp * K;
    bool bad = false;
    // forward projection of every slot into the scratch: T_j, j < c
    for (int k = 0; k < K; ++k) {
      int py, px;
      split_pos(gi[k], d.W, rW, py, px);
      py = min(max(py, 0), d.Hp - 1);
      px = min(max(px, 0), d.Wp - 1);
      const int pix = (py + a) * d.W + px + b;
      __syncthreads();   // Y is read across lanes by the previous slot's products
      for (int j = 0; j < C; ++j) {
        const float v = d.img[(size_t)j * HW + pix];
        bad |= !isfinite(v);
        Yb[j * 64 + lane] = v;
      }
      dft_bands();
      products(false);
      idft_bands(S + (size_t)k * C * 64, 1.0f / (float)C);
    }
    // Haar along the group, hard threshold (Eq. 19), inverse; per band
    for (int j = 0; j < C; ++j) {
      float x[K][1];
#pragma unroll
      for (int k = 0; k < K; ++k) x[k][0] = S[((size_t)k * C + j) * 64 + lane];
      haar_forward_slots<K, 1>(x);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        bool keep;
        if (ADJ) {   // the frozen mask of the forward pass
          const size_t word = ((size_t)gl * K + haar_slot_row(k, K)) * C + j;
          keep = (d.masks_in[2 * word + (lane >> 5)] >> (lane & 31)) & 1u;
        } else {
          keep = fabsf(x[k][0]) >= tau;
        }
        x[k][0] = keep ? x[k][0] : 0.f;
        if (!ADJ && d.masks) {
          const unsigned long long bal = __ballot(keep);
          if (lane == 0) {
            const size_t word = ((size_t)gl * K + haar_slot_row(k, K)) * C + j;
            d.masks[2 * word] = (uint32_t)bal;
            d.masks[2 * word + 1] = (uint32_t)(bal >> 32);
          }
        }
      }
      haar_inverse_slots<K, 1>(x);
#pragma unroll
      for (int k = 0; k < K; ++k) S[((size_t)k * C + j) * 64 + lane] = x[k][0];
    }
    // inverse projection per slot and fixed-point aggregation (Eq. 2)
    for (int k = 0; k < K; ++k) {
      int py, px;
      split_pos(gi[k], d.W, rW, py, px);
      py = min(max(py, 0), d.Hp - 1);
      px = min(max(px, 0), d.Wp - 1);
      const int pix = (py + a) * d.W + px + b;
      __syncthreads();
      for (int j = 0; j < C; ++j) Yb[j * 64 + lane] = S[((size_t)k * C + j) * 64 + lane];
      dft_bands();
      products(true);
      // c x the estimate (the 1/c is in fxs), parked in the slot's scratch
      idft_bands(S + (size_t)k * C * 64, 1.f);
      for (int j = 0; j < C; ++j) bad |= !isfinite(S[((size_t)k * C + j) * 64 + lane]);
      if (__ballot(bad)) break;
      for (int j = 0; j < C; ++j) {
        const float t = S[((size_t)k * C + j) * 64 + lane];
        if (d.num64) atomicAdd(d.num64 + (size_t)j * HW + pix, fx_from_float(t * fxs));
        else atomicAdd(d.num + (size_t)j * HW + pix, t * fxs);   // fxs = 1 / c here
        if (d.group_est) d.group_est[(((size_t)gl * K + k) * C + j) * PS2 + lane] = t * (1.0f / (float)C);
      }
    }
    if (__ballot(bad)) poison_group(d, gi, gl, K, C, rW, lane);
  }
}

template <int ADJ>
static hipError_t launch_fg(const Launch& L, int grid, hipStream_t s) {
  const size_t lds = filter_gen_lds_bytes(L.C);
  const int g = grid > 0 ? grid : 1;
  switch (L.K) {
    case 2: hipLaunchKernelGGL((k_filter_gen<2, ADJ>), dim3(g), dim3(64), lds, s, L); break;
    case 4: hipLaunchKernelGGL((k_filter_gen<4, ADJ>), dim3(g), dim3(64), lds, s, L); break;
    case 8: hipLaunchKernelGGL((k_filter_gen<8, ADJ>), dim3(g), dim3(64), lds, s, L); break;
    case 16: hipLaunchKernelGGL((k_filter_gen<16, ADJ>), dim3(g), dim3(64), lds, s, L); break;
    case 32: hipLaunchKernelGGL((k_filter_gen<32, ADJ>), dim3(g), dim3(64), lds, s, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_filter_gen(const Launch& L, int grid, hipStream_t s) { return launch_fg<0>(L, grid, s); }

// The transpose of the frozen-mask map (the adjoint): the masks of the
// forward pass (d.masks_in) replace the threshold.
hipError_t launch_filter_gen_adj(const Launch& L, int grid, hipStream_t s) {
  return launch_fg<1>(L, grid, s);
}

}  // namespace hts
