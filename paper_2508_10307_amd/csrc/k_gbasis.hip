// Derivative of the denoiser through its learned basis (adjoint extension).
// Alg. 1 Step 2(1) learns U, V from the noisy image itself (the per-frequency
// eigenproblems of the patch second moments, Eq. 11-12); with grouping,
// keep-masks and coverage count frozen, dL/dy gains a term through U(y),
// V(y).  Three stages:
//
//  k_gbasis_acc    per group slot, with P / R the slot's patch of y / of
//                  r = g / cnt, T' = H^T M H (U^T * P * V) and
//                  D = H^T M H (U^T * R * V) (Haar H along the group, Eq. 9;
//                  frozen mask M), the Fourier-domain cotangents of the
//                  real basis tensors, per frequency f <= c/2:
//                    A_U(f) += R^ V_F T'^^H + P^ V_F D^^H
//                    A_V(f) += R^^H U_F T'^ + P^^H U_F D^
//                  (FP32 per group, FP64 per work group, one partial per
//                  work group);
//  k_gbasis_eig    one work group: the partials in order, then per
//                  eigenproblem (U or V, f) the first-order eigenvector
//                  perturbation with the phase convention's gauge term:
//                    G = (w_f / c) A, G[m_k][k] += i Im<G_k, u_k> / u_m
//                    (m_k the pivot: first entry of largest modulus),
//                    Cbar = U (F o (U^H G)) U^H, F_jk = 1 / (l_k - l_j),
//                    M = Cbar + Cbar^H   (= 2 x its Hermitian part);
//  k_gbasis_place  per pixel: dL/dP^_i(f) = M_U(f) P^_i(f) + P^_i(f) M_V(f)
//                  for every reference patch i over the pixel, back to the
//                  channels (Re(. e^{2 pi i f j / c})) and added into grad.
//                  Entry (a, b) of M_U P^ reads column b of the patch (the
//                  pixel's image column), entry (a, b) of P^ M_V row a (its
//                  image row), so the sum over the ny x nx references over
//                  the pixel splits into nx * (column sums over their rows)
//                  + ny * (row sums over their columns).
//
// Every sum runs in a fixed order: the result is the same on every run.
#include "group_proj.h"

namespace hts {

namespace {

// Complex 8x8 tiles in LDS, entry (r, c) at [re/im][r * 8 + c].
using Tile = float[2][64];

__device__ inline void put(Tile& t, int lane, float re, float im) {
  t[0][lane] = re;
  t[1][lane] = im;
}

}  // namespace

// Partials: [work group][2 * NF matrices (U: f, then V: f)][re/im][64].
template <int K, int C>
__global__ __launch_bounds__(64) void k_gbasis_acc(Launch L, const float* g, double* partial) {
  constexpr int NF = C / 2 + 1;
  // eight complex 8x8 tiles: the projections' X and Y, then the cotangent
  // products' operands (the two uses never overlap)
  __shared__ Tile tl[8];
  __shared__ float core[2][K][C][64];   // T' and D per slot, per lane
  float (*PX)[2][64] = tl, (*PY)[2][64] = tl + 4;
  const int lane = threadIdx.x;
  const int a = lane >> 3, b = lane & 7;
  const ImgDesc& d = L.one;
  const int HW = d.H * d.W;
  const float rW = 1.0f / (float)d.W;
  const float* fb = d.fbasis;
  double accU[NF][2], accV[NF][2];
#pragma unroll
  for (int f = 0; f < NF; ++f) accU[f][0] = accU[f][1] = accV[f][0] = accV[f][1] = 0.0;
  for (int grp = blockIdx.x; grp < d.n_ref; grp += gridDim.x) {
    const int* gi = d.idx + (size_t)grp * K;
    // core tensors of the slots' patches of y (0) and of r (1)
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
    // Haar along the group, frozen mask, inverse: T' and D (lane-private)
    {
      float ts[K][C], tr[K][C];
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          ts[k][ch] = core[0][k][ch][lane];
          tr[k][ch] = core[1][k][ch][lane];
        }
      haar_forward_slots<K, C>(ts);
      haar_forward_slots<K, C>(tr);
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          const size_t word = ((size_t)grp * K + haar_slot_row(k, K)) * C + ch;   // 64-bit word
          const uint32_t w = d.masks_in[2 * word + (lane >> 5)];
          const bool keep = (w >> (lane & 31)) & 1u;
          ts[k][ch] = keep ? ts[k][ch] : 0.f;
          tr[k][ch] = keep ? tr[k][ch] : 0.f;
        }
      haar_inverse_slots<K, C>(ts);
      haar_inverse_slots<K, C>(tr);
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          core[0][k][ch][lane] = ts[k][ch];
          core[1][k][ch][lane] = tr[k][ch];
        }
    }
    // per slot and frequency: the cotangent products
    float gU[NF][2], gV[NF][2];
#pragma unroll
    for (int f = 0; f < NF; ++f) gU[f][0] = gU[f][1] = gV[f][0] = gV[f][1] = 0.f;
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      int py, px;
      split_pos(gi[k], d.W, rW, py, px);
      py = min(max(py, 0), d.Hp - 1);
      px = min(max(px, 0), d.Wp - 1);
      const int pix = (py + a) * d.W + px + b;
      const float rc = 1.0f / d.cnt[pix];
      float p[C], r[C], tp[C], dd[C];
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        p[ch] = d.img[ch * HW + pix];
        r[ch] = g[ch * HW + pix] * rc;
        tp[ch] = core[0][k][ch][lane];
        dd[ch] = core[1][k][ch][lane];
      }
      // channel DFT at f: X^(f) = sum_j X_j e^{-2 pi i f j / 3}
      auto dft = [&](const float* x, int f, float& re, float& im) {
        if (C == 1) { re = x[0]; im = 0.f; }
        else if (f == 0) { re = x[0] + x[1] + x[2]; im = 0.f; }
        else { re = x[0] - 0.5f * (x[1] + x[2]); im = (float)GP_SQ3_2 * (x[2] - x[1]); }
      };
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        float rr, ri, pr, pi, tr_, ti, dr, di;
        dft(r, f, rr, ri);
        dft(p, f, pr, pi);
        dft(tp, f, tr_, ti);
        dft(dd, f, dr, di);
        __syncthreads();   // the previous readers of the tiles are done
        put(tl[0], lane, rr, ri);   // R^
        put(tl[1], lane, pr, pi);   // P^
        put(tl[2], lane, tr_, ti);  // T'^
        put(tl[3], lane, dr, di);   // D^
        __syncthreads();
        const float* Ur = fb + (f ? FB_U1R : FB_U0);
        const float* Vr = fb + (f ? FB_V1R : FB_V0);
        const float* Ui = f ? fb + FB_U1I : nullptr;
        const float* Vi = f ? fb + FB_V1I : nullptr;
        // X1 = R^ V_F, X2 = P^ V_F, Y1 = U_F T'^, Y2 = U_F D^ at (a, b)
        float x1r = 0.f, x1i = 0.f, x2r = 0.f, x2i = 0.f, y1r = 0.f, y1i = 0.f, y2r = 0.f, y2i = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float vr = Vr[t * 8 + b], ur = Ur[a * 8 + t];
          const float vi = Vi ? Vi[t * 8 + b] : 0.f, ui = Ui ? Ui[a * 8 + t] : 0.f;
          const float Rr = tl[0][0][a * 8 + t], Ri = tl[0][1][a * 8 + t];
          const float Pr = tl[1][0][a * 8 + t], Pi = tl[1][1][a * 8 + t];
          const float Tr = tl[2][0][t * 8 + b], Ti = tl[2][1][t * 8 + b];
          const float Dr = tl[3][0][t * 8 + b], Di = tl[3][1][t * 8 + b];
          x1r += Rr * vr - Ri * vi;  x1i += Rr * vi + Ri * vr;
          x2r += Pr * vr - Pi * vi;  x2i += Pr * vi + Pi * vr;
          y1r += ur * Tr - ui * Ti;  y1i += ur * Ti + ui * Tr;
          y2r += ur * Dr - ui * Di;  y2i += ur * Di + ui * Dr;
        }
        put(tl[4], lane, x1r, x1i);
        put(tl[5], lane, x2r, x2i);
        put(tl[6], lane, y1r, y1i);
        put(tl[7], lane, y2r, y2i);
        __syncthreads();
        // A_U(a, b) += sum_t X1(a,t) conj(T'^(b,t)) + X2(a,t) conj(D^(b,t))
        // A_V(a, b) += sum_t conj(R^(t,a)) Y1(t,b) + conj(P^(t,a)) Y2(t,b)
        float ur_ = 0.f, ui_ = 0.f, vr_ = 0.f, vi_ = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float X1r = tl[4][0][a * 8 + t], X1i = tl[4][1][a * 8 + t];
          const float X2r = tl[5][0][a * 8 + t], X2i = tl[5][1][a * 8 + t];
          const float Tr = tl[2][0][b * 8 + t], Ti = tl[2][1][b * 8 + t];
          const float Dr = tl[3][0][b * 8 + t], Di = tl[3][1][b * 8 + t];
          ur_ += X1r * Tr + X1i * Ti + X2r * Dr + X2i * Di;
          ui_ += X1i * Tr - X1r * Ti + X2i * Dr - X2r * Di;
          const float Rr = tl[0][0][t * 8 + a], Ri = tl[0][1][t * 8 + a];
          const float Pr = tl[1][0][t * 8 + a], Pi = tl[1][1][t * 8 + a];
          const float Y1r = tl[6][0][t * 8 + b], Y1i = tl[6][1][t * 8 + b];
          const float Y2r = tl[7][0][t * 8 + b], Y2i = tl[7][1][t * 8 + b];
          vr_ += Rr * Y1r + Ri * Y1i + Pr * Y2r + Pi * Y2i;
          vi_ += Rr * Y1i - Ri * Y1r + Pr * Y2i - Pi * Y2r;
        }
        gU[f][0] += ur_;
        gU[f][1] += ui_;
        gV[f][0] += vr_;
        gV[f][1] += vi_;
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      accU[f][0] += gU[f][0];
      accU[f][1] += gU[f][1];
      accV[f][0] += gV[f][0];
      accV[f][1] += gV[f][1];
    }
  }
  double* o = partial + (size_t)blockIdx.x * (2 * NF * 128);
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    o[(f * 2 + 0) * 64 + lane] = accU[f][0];
    o[(f * 2 + 1) * 64 + lane] = accU[f][1];
    o[((NF + f) * 2 + 0) * 64 + lane] = accV[f][0];
    o[((NF + f) * 2 + 1) * 64 + lane] = accV[f][1];
  }
}

// One work group of 256 threads.  U64, V64: the real basis tensors
// [C][8][8] (FP64); eig: [2][NF][8] descending eigenvalues; M out:
// [2 * NF][re/im][64] (FP64).
template <int C>
__global__ __launch_bounds__(256) void k_gbasis_eig(const double* partial, int nblk,
                                                    const double* U64, const double* V64,
                                                    const double* eig, double* M) {
  constexpr int NF = C / 2 + 1, NM = 2 * NF;
  __shared__ double G[NM][2][64], B[NM][2][64], Wt[NM][2][64];
  const int tid = threadIdx.x;
  // ordered sum of the partials, scaled to dL/dU_F(f) = (w_f / c) A(f)
  for (int e = tid; e < NM * 128; e += 256) {
    double s = 0.0;
    int j = 0;
    for (; j + 8 <= nblk; j += 8) {   // eight loads in flight, added in order
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(j + u) * NM * 128 + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; j < nblk; ++j) s += partial[(size_t)j * NM * 128 + e];
    const int f = (e >> 7) % NF;
    const double wf = C == 1 ? 1.0 : (f == 0 ? 1.0 / 3.0 : 2.0 / 3.0);
    (&G[0][0][0])[e] = wf * s;
  }
  // Fourier slices U_F(f) (DFT of the real tensor along the channel mode)
  for (int e = tid; e < NM * 64; e += 256) {
    const int m = e >> 6, ab = e & 63, uv = m / NF, f = m % NF;
    const double* T = uv ? V64 : U64;
    double re, im;
    if (C == 1) { re = T[ab]; im = 0.0; }
    else if (f == 0) { re = T[ab] + T[64 + ab] + T[128 + ab]; im = 0.0; }
    else { re = T[ab] - 0.5 * (T[64 + ab] + T[128 + ab]); im = GP_SQ3_2 * (T[128 + ab] - T[64 + ab]); }
    B[m][0][ab] = re;
    B[m][1][ab] = im;
  }
  __syncthreads();
  // gauge term: column k keeps its pivot entry real
  if (tid < NM * 8) {
    const int m = tid >> 3, k = tid & 7;
    int piv = 0;
    double best = -1.0, s = 0.0;
    for (int t = 0; t < 8; ++t) {
      const double ur = B[m][0][t * 8 + k], ui = B[m][1][t * 8 + k];
      const double mm = ur * ur + ui * ui;
      if (mm > best) { best = mm; piv = t; }
      s += G[m][0][t * 8 + k] * ui - G[m][1][t * 8 + k] * ur;   // Im(conj(G) u)
    }
    G[m][1][piv * 8 + k] += s / B[m][0][piv * 8 + k];
  }
  __syncthreads();
  // W = F o (U^H G)
  const int m = tid >> 6, ab = tid & 63, j = ab >> 3, k = ab & 7;
  const int uv = m / NF, f = m % NF;
  const bool act = m < NM;
  if (act) {
    double wr = 0.0, wi = 0.0;
    for (int t = 0; t < 8; ++t) {
      const double ur = B[m][0][t * 8 + j], ui = B[m][1][t * 8 + j];
      const double gr = G[m][0][t * 8 + k], gi = G[m][1][t * 8 + k];
      wr += ur * gr + ui * gi;
      wi += ur * gi - ui * gr;
    }
    const double* ev = eig + (uv * NF + f) * 8;
    const double F = j == k ? 0.0 : 1.0 / (ev[k] - ev[j]);
    Wt[m][0][ab] = F * wr;
    Wt[m][1][ab] = F * wi;
  }
  __syncthreads();
  // Y = W U^H (into G)
  if (act) {
    double yr = 0.0, yi = 0.0;
    for (int t = 0; t < 8; ++t) {
      const double wr = Wt[m][0][j * 8 + t], wi = Wt[m][1][j * 8 + t];
      const double ur = B[m][0][k * 8 + t], ui = -B[m][1][k * 8 + t];
      yr += wr * ur - wi * ui;
      yi += wr * ui + wi * ur;
    }
    G[m][0][ab] = yr;
    G[m][1][ab] = yi;
  }
  __syncthreads();
  // Cbar = U Y (into Wt)
  if (act) {
    double cr = 0.0, ci = 0.0;
    for (int t = 0; t < 8; ++t) {
      const double ur = B[m][0][j * 8 + t], ui = B[m][1][j * 8 + t];
      const double yr = G[m][0][t * 8 + k], yi = G[m][1][t * 8 + k];
      cr += ur * yr - ui * yi;
      ci += ur * yi + ui * yr;
    }
    Wt[m][0][ab] = cr;
    Wt[m][1][ab] = ci;
  }
  __syncthreads();
  // M = Cbar + Cbar^H
  if (act) {
    M[(m * 2 + 0) * 64 + ab] = Wt[m][0][ab] + Wt[m][0][k * 8 + j];
    M[(m * 2 + 1) * 64 + ab] = Wt[m][1][ab] - Wt[m][1][k * 8 + j];
  }
}

// Covering reference coordinates of pixel coordinate y along one axis (grid
// of ref_coord), in increasing order; returns their count (<= 8).
__device__ inline int covering_refs(int y, int s, int nr, int n_valid, int* out) {
  int n = 0;
  for (int i = max(0, (y - 7 + s - 1) / s); i < nr; ++i) {
    const int r = ref_coord(i, s, n_valid);
    if (r > y) break;
    if (r + 7 >= y) out[n++] = r;
  }
  return n;
}

// grad[ch][y][x] += the basis term at every pixel; M as k_gbasis_eig writes it.
template <int C>
__global__ __launch_bounds__(256) void k_gbasis_place(Launch L, const double* M, float* grad) {
  constexpr int NF = C / 2 + 1, NM = 2 * NF;
  __shared__ float Ms[NM][2][64];
  for (int e = threadIdx.x; e < NM * 128; e += blockDim.x) (&Ms[0][0][0])[e] = (float)M[e];
  __syncthreads();
  const ImgDesc& d = L.one;
  const int HW = d.H * d.W;
  const int s = L.stride;
  for (int pix = blockIdx.x * blockDim.x + threadIdx.x; pix < HW; pix += gridDim.x * blockDim.x) {
    const int y = pix / d.W, x = pix - y * d.W;
    int ry[8], rx[8];
    const int ny = covering_refs(y, s, d.nry, d.Hp, ry);
    const int nx = covering_refs(x, s, d.nrx, d.Wp, rx);
    // column sums: sum over ry of sum_t M_U(f)[y - ry][t] P^(f)(ry + t, x)
    // row sums:    sum over rx of sum_t P^(f)(y, rx + t) M_V(f)[t][x - rx]
    float cs[NF][2], rs[NF][2];
#pragma unroll
    for (int f = 0; f < NF; ++f) cs[f][0] = cs[f][1] = rs[f][0] = rs[f][1] = 0.f;
    for (int q = 0; q < ny; ++q) {
      const int a = y - ry[q];
      for (int t = 0; t < 8; ++t) {
        const int src = (ry[q] + t) * d.W + x;
        float v[C];
#pragma unroll
        for (int ch = 0; ch < C; ++ch) v[ch] = d.img[ch * HW + src];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          float pr, pi;
          if (C == 1) { pr = v[0]; pi = 0.f; }
          else if (f == 0) { pr = v[0] + v[1] + v[2]; pi = 0.f; }
          else { pr = v[0] - 0.5f * (v[1] + v[2]); pi = (float)GP_SQ3_2 * (v[2] - v[1]); }
          const float mr = Ms[f][0][a * 8 + t], mi = Ms[f][1][a * 8 + t];
          cs[f][0] += mr * pr - mi * pi;
          cs[f][1] += mr * pi + mi * pr;
        }
      }
    }
    for (int q = 0; q < nx; ++q) {
      const int b = x - rx[q];
      for (int t = 0; t < 8; ++t) {
        const int src = y * d.W + rx[q] + t;
        float v[C];
#pragma unroll
        for (int ch = 0; ch < C; ++ch) v[ch] = d.img[ch * HW + src];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          float pr, pi;
          if (C == 1) { pr = v[0]; pi = 0.f; }
          else if (f == 0) { pr = v[0] + v[1] + v[2]; pi = 0.f; }
          else { pr = v[0] - 0.5f * (v[1] + v[2]); pi = (float)GP_SQ3_2 * (v[2] - v[1]); }
          const float mr = Ms[NF + f][0][t * 8 + b], mi = Ms[NF + f][1][t * 8 + b];
          rs[f][0] += pr * mr - pi * mi;
          rs[f][1] += pr * mi + pi * mr;
        }
      }
    }
    // dL/dP_j = sum_f Re(G_f e^{2 pi i f j / c}), G_f = nx * cs + ny * rs
    float G[NF][2];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      G[f][0] = (float)nx * cs[f][0] + (float)ny * rs[f][0];
      G[f][1] = (float)nx * cs[f][1] + (float)ny * rs[f][1];
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
      float v;
      if (C == 1) v = G[0][0];
      else if (ch == 0) v = G[0][0] + G[1][0];
      else if (ch == 1) v = G[0][0] - 0.5f * G[1][0] - (float)GP_SQ3_2 * G[1][1];
      else v = G[0][0] - 0.5f * G[1][0] + (float)GP_SQ3_2 * G[1][1];
      grad[ch * HW + pix] += v;
    }
  }
}

// The FP64 basis as the float tensors and Fourier slices the group kernel reads.
__global__ void k_gbasis_prep(const double* U64, const double* V64, float* basis, int n) {
  for (int e = threadIdx.x; e < 2 * n; e += blockDim.x) basis[e] = (float)(e < n ? U64[e] : V64[e - n]);
}

template <int C>
static hipError_t launch_gb_acc(const Launch& L, const float* g, double* partial, int grid,
                                hipStream_t s) {
  switch (L.K) {
    case 2: hipLaunchKernelGGL((k_gbasis_acc<2, C>), dim3(grid), dim3(64), 0, s, L, g, partial); break;
    case 4: hipLaunchKernelGGL((k_gbasis_acc<4, C>), dim3(grid), dim3(64), 0, s, L, g, partial); break;
    case 8: hipLaunchKernelGGL((k_gbasis_acc<8, C>), dim3(grid), dim3(64), 0, s, L, g, partial); break;
    case 16: hipLaunchKernelGGL((k_gbasis_acc<16, C>), dim3(grid), dim3(64), 0, s, L, g, partial); break;
    case 32: hipLaunchKernelGGL((k_gbasis_acc<32, C>), dim3(grid), dim3(64), 0, s, L, g, partial); break;
    case 64:
      if constexpr (C == 1) {
        hipLaunchKernelGGL((k_gbasis_acc<64, 1>), dim3(grid), dim3(64), 0, s, L, g, partial);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gbasis(const Launch& L, const float* g, const double* U64, const double* V64,
                         const double* eig, double* partial, int grid, double* M, float* grad,
                         hipStream_t s) {
  const ImgDesc& d = L.one;
  hipLaunchKernelGGL(k_gbasis_prep, dim3(1), dim3(256), 0, s, U64, V64, d.basis, L.C * 64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_fbasis(L, nullptr, nullptr, s);
  if (e != hipSuccess) return e;
  e = L.C == 1 ? launch_gb_acc<1>(L, g, partial, grid, s) : launch_gb_acc<3>(L, g, partial, grid, s);
  if (e != hipSuccess) return e;
  if (L.C == 1)
    hipLaunchKernelGGL((k_gbasis_eig<1>), dim3(1), dim3(256), 0, s, partial, grid, U64, V64, eig, M);
  else
    hipLaunchKernelGGL((k_gbasis_eig<3>), dim3(1), dim3(256), 0, s, partial, grid, U64, V64, eig, M);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int HW = d.H * d.W;
  const int pg = min((HW + 255) / 256, 8192);
  if (L.C == 1) hipLaunchKernelGGL((k_gbasis_place<1>), dim3(pg), dim3(256), 0, s, L, M, grad);
  else hipLaunchKernelGGL((k_gbasis_place<3>), dim3(pg), dim3(256), 0, s, L, M, grad);
  return hipGetLastError();
}

}  // namespace hts
