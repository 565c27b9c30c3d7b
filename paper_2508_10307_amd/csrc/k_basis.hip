// Global circulant patch basis (Sec. III.B.1, Eq. 11-12; Alg. 1 Step 2(1)).
//
// In the Fourier domain of the t-product (Eq. 5-6) the basis tensors U, V
// become one unitary 8x8 slice per frequency f of the channel-mode DFT.
// Each slice is the eigenbasis of a second moment of the transformed
// reference patches P^(f) = sum_j P(:,:,j) exp(-2 pi i f j / c):
//   C_U(f) = sum_i P^_i(f) P^_i(f)^H,   C_V(f) = sum_i P^_i(f)^H P^_i(f),
// for f = 0..floor(c/2) (the rest follow by conjugate symmetry).  All of it
// runs in FP64: partial sums per block of references (k_cov), an ordered
// reduction and cyclic complex Jacobi eigen-solves (k_eig), then the real
// tensors U(:,:,j) = (1/c) sum_f U_F(f) exp(+2 pi i f j / c).
#include "jacobi8.h"

namespace hts {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline void dft3(double p0, double p1, double p2, double& f0, double& f1r, double& f1i) {
  // P^(0) = p0 + p1 + p2;  P^(1) = p0 + w p1 + w^2 p2, w = exp(-2 pi i / 3)
  f0 = p0 + p1 + p2;
  f1r = p0 - 0.5 * (p1 + p2);
  f1i = 0.86602540378443864676 * (p2 - p1);
}

// Partial covariances of one tile of cov_tile x cov_tile references
// (item = tile in row-major order over the reference grid): layout per
// item: C_U(0)[8][8], C_V(0)[8][8], then for c = 3 C_U(1), C_V(1) as
// interleaved (re, im) [8][8][2].
//
// Every covariance is a Gram matrix summed over the references, computed
// on FP64 MFMA (v_mfma_f64_16x16x4f64: lane l holds A(l%16, l/16) and
// B(l/16, l%16); D(l/16 + 4v, l%16) in register v).  With one 16 x 8
// operand Z per reference, Z Z^T needs Z both as A and as B^T, which is the
// same register, two k-steps of 4 columns:
//   C_U(1): Z = [Re P^(1); Im P^(1)]   -> Re = G11 + G22, Im = G21 - G12;
//   C_V(1): Z = [Re P^(1)^T; Im P^(1)^T] -> Re = G11 + G22, Im = G12 - G21;
//   C_U(0), C_V(0): Z = [P^(0); P^(0)] (resp. transposed) -> C = G11,
// where Gxy are the 8 x 8 blocks of G = Z Z^T.  The tile's pixel region is
// staged in LDS first (overlapping patches read it many times over); each
// wavefront takes every fourth reference of the tile; the four partial
// Grams are added in LDS in wavefront order.
__global__ __launch_bounds__(256) void k_cov(Launch L) {
  extern __shared__ float px[];         // [C][RH][RW] pixel region of the tile
  __shared__ double red[4][4][4][64];   // [wavefront][gram][register][lane]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4, rr = r16 & 7;
  const bool upper = r16 >= 8;          // rows 8..15 of Z
  const int nel = cov_elems(L.C);
  const int s = L.stride, TR = cov_tile(s);
  for_each_item<W_COV>(L, [&](const ImgDesc& d, int item) __attribute__((always_inline)) {
    const int HW = d.H * d.W;
    const int ntx = (d.nrx + TR - 1) / TR;
    const int iy0 = (item / ntx) * TR, ix0 = (item % ntx) * TR;
    const int ty = min(d.nry - iy0, TR), tx = min(d.nrx - ix0, TR);
    const int Y0 = ref_coord(iy0, s, d.Hp), X0 = ref_coord(ix0, s, d.Wp);
    const int RH = ref_coord(iy0 + ty - 1, s, d.Hp) + PS - Y0;   // <= cov_region(s)
    const int RW = ref_coord(ix0 + tx - 1, s, d.Wp) + PS - X0;
    const int RP = RH * RW;
    __syncthreads();   // the previous item's references still read px
    // eight loads per thread in flight before the first wait (indices past
    // the region repeat its last element and are not stored)
    const int NE = L.C * RP;
    for (int e0 = tid; e0 < NE; e0 += 256 * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(e0 + 256 * u, NE - 1);
        const int ch = e / RP, rem = e - ch * RP, y = rem / RW, x = rem - y * RW;
        v[u] = d.img[ch * HW + (Y0 + y) * d.W + X0 + x];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (e0 + 256 * u < NE) px[e0 + 256 * u] = v[u];
    }
    __syncthreads();
    d4 gu1 = {0.0, 0.0, 0.0, 0.0}, gv1 = gu1, gu0 = gu1, gv0 = gu1;
    const int nt = ty * tx;
    // four references per round: their pixels are read before the MFMAs
    // (a reference past the end reads the last one and contributes zero)
    constexpr int RB = 4;
    for (int t0 = wave; t0 < nt; t0 += 4 * RB) {
      float pu[RB][2][3], pv[RB][2][3];
      double live[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int t = min(t0 + 4 * u, nt - 1);
        live[u] = t0 + 4 * u < nt ? 1.0 : 0.0;
        const int iy = t / tx;
        const int ry = ref_coord(iy0 + iy, s, d.Hp) - Y0;
        const int rx = ref_coord(ix0 + t - iy * tx, s, d.Wp) - X0;
        const float* base = px + ry * RW + rx;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int ou = rr * RW + kq + 4 * c;       // pixel (row rr, column kq + 4c): C_U operands
          const int ov = (kq + 4 * c) * RW + rr;     // pixel (row kq + 4c, column rr): C_V operands
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            pu[u][c][ch] = ch < L.C ? base[ch * RP + ou] : 0.f;
            pv[u][c][ch] = ch < L.C ? base[ch * RP + ov] : 0.f;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (L.C == 1) {
            const double zu = live[u] * (double)pu[u][c][0], zv = live[u] * (double)pv[u][c][0];
            gu0 = __builtin_amdgcn_mfma_f64_16x16x4f64(zu, zu, gu0, 0, 0, 0);
            gv0 = __builtin_amdgcn_mfma_f64_16x16x4f64(zv, zv, gv0, 0, 0, 0);
          } else {
            double f0u, f1ru, f1iu, f0v, f1rv, f1iv;
            dft3(live[u] * pu[u][c][0], live[u] * pu[u][c][1], live[u] * pu[u][c][2], f0u, f1ru, f1iu);
            dft3(live[u] * pv[u][c][0], live[u] * pv[u][c][1], live[u] * pv[u][c][2], f0v, f1rv, f1iv);
            const double zu = upper ? f1iu : f1ru, zv = upper ? f1iv : f1rv;
            gu1 = __builtin_amdgcn_mfma_f64_16x16x4f64(zu, zu, gu1, 0, 0, 0);
            gv1 = __builtin_amdgcn_mfma_f64_16x16x4f64(zv, zv, gv1, 0, 0, 0);
            gu0 = __builtin_amdgcn_mfma_f64_16x16x4f64(f0u, f0u, gu0, 0, 0, 0);
            gv0 = __builtin_amdgcn_mfma_f64_16x16x4f64(f0v, f0v, gv0, 0, 0, 0);
          }
        }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      red[wave][0][v][lane] = gu0[v];
      red[wave][1][v][lane] = gv0[v];
      red[wave][2][v][lane] = gu1[v];
      red[wave][3][v][lane] = gv1[v];
    }
    __syncthreads();
    // G(i, j) of gram g summed over the wavefronts, in wavefront order
    auto G = [&](int g, int i, int j) __attribute__((always_inline)) {
      const int v = i >> 2, l = 16 * (i & 3) + j;
      return ((red[0][g][v][l] + red[1][g][v][l]) + red[2][g][v][l]) + red[3][g][v][l];
    };
    for (int e = tid; e < nel; e += 256) {
      double val;
      if (e < 128) {
        const int g = e < 64 ? 0 : 1, ab = e & 63, a = ab >> 3, b = ab & 7;
        val = G(g, a, b);
      } else {
        const int q = e - 128, g = q < 128 ? 2 : 3, qq = q & 127;
        const int ab = qq >> 1, a = ab >> 3, b = ab & 7;
        if (!(qq & 1)) val = G(g, a, b) + G(g, 8 + a, 8 + b);
        else if (g == 2) val = G(g, 8 + a, b) - G(g, a, 8 + b);
        else val = G(g, a, 8 + b) - G(g, 8 + a, b);
      }
      d.cov_part[(size_t)item * nel + e] = val;
    }
  });
}

// One work group per image: ordered reduction of the partials, eigen-solves
// (eight threads per covariance matrix), descending order, phase convention
// (largest-modulus entry real positive, first on ties), real tensors.
__global__ __launch_bounds__(256) void k_eig(Launch L) {
  __shared__ double cov[384];
  __shared__ double mr[4][8][8], mi[4][8][8], vr[4][8][8], vi[4][8][8];
  __shared__ double UF[2][2][8][8][2];  // [U/V][f][row][col][re/im], sorted + phased
  __shared__ double ev[2][2][8];
  const int tid = threadIdx.x;
  const int nel = cov_elems(L.C);
  const int nm = L.C == 1 ? 2 : 4;
  const int nimg = L.table ? L.n_img : 1;
  for (int im = blockIdx.x; im < nimg; im += gridDim.x) {
    const ImgDesc d = L.table ? L.table[im] : L.one;
    __syncthreads();
    for (int e = tid; e < nel; e += blockDim.x) {
      // partials added in their order; eight loads in flight at a time
      double s = 0.0;
      int j = 0;
      for (; j + 8 <= d.n_cov; j += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = d.cov_part[(size_t)(j + u) * nel + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; j < d.n_cov; ++j) s += d.cov_part[(size_t)j * nel + e];
      cov[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < nm * 64; e += blockDim.x) {
      const int m = e >> 6, a = (e >> 3) & 7, b = e & 7;
      if (m < 2) { mr[m][a][b] = cov[m * 64 + a * 8 + b]; mi[m][a][b] = 0.0; }
      else { const int base = 128 + (m - 2) * 128 + (a * 8 + b) * 2; mr[m][a][b] = cov[base]; mi[m][a][b] = cov[base + 1]; }
    }
    __syncthreads();
    jacobi_herm8_group(mr, mi, vr, vi, nm);
    if (tid < nm) {
      const int m = tid;
      // descending eigenvalues, stable
      int order[8];
      for (int k = 0; k < 8; ++k) order[k] = k;
      for (int a = 1; a < 8; ++a) {
        int key = order[a], b = a - 1;
        while (b >= 0 && mr[m][order[b]][order[b]] < mr[m][key][key]) { order[b + 1] = order[b]; --b; }
        order[b + 1] = key;
      }
      const int uv = m & 1, f = m >> 1;  // m: 0 = C_U(0), 1 = C_V(0), 2 = C_U(1), 3 = C_V(1)
      for (int k = 0; k < 8; ++k) {
        const int src = order[k];
        ev[uv][f][k] = mr[m][src][src];
        int best = 0;
        double bm = -1.0;
        for (int a = 0; a < 8; ++a) {
          const double mm = vr[m][a][src] * vr[m][a][src] + vi[m][a][src] * vi[m][a][src];
          if (mm > bm) { bm = mm; best = a; }
        }
        const double nr = sqrt(bm);
        const double pr = vr[m][best][src] / nr, pi = -vi[m][best][src] / nr;  // conj(v)/|v|
        for (int a = 0; a < 8; ++a) {
          const double xr = vr[m][a][src], xi = vi[m][a][src];
          UF[uv][f][a][k][0] = xr * pr - xi * pi;
          UF[uv][f][a][k][1] = xr * pi + xi * pr;
        }
        UF[uv][f][best][k][1] = 0.0;
      }
    }
    __syncthreads();
    // real tensors: c = 1: U = U_F(0); c = 3: U(:,:,j) = (U_F(0) + 2 Re(U_F(1) e^{2 pi i j/3})) / 3
    for (int e = tid; e < 2 * L.C * 64; e += blockDim.x) {
      const int uv = e / (L.C * 64), rem = e % (L.C * 64), j = rem >> 6, ab = rem & 63;
      const int a = ab >> 3, b = ab & 7;
      double val;
      if (L.C == 1) {
        val = UF[uv][0][a][b][0];
      } else {
        const double c0 = UF[uv][0][a][b][0], r1 = UF[uv][1][a][b][0], i1 = UF[uv][1][a][b][1];
        const double cs = j == 0 ? 1.0 : -0.5;
        const double sn = j == 0 ? 0.0 : (j == 1 ? 0.86602540378443864676 : -0.86602540378443864676);
        val = (c0 + 2.0 * (r1 * cs - i1 * sn)) / 3.0;
      }
      const int off = uv * L.C * 64 + j * 64 + ab;
      d.basis64[off] = val;
      d.basis[off] = (float)val;
    }
    const int nf = L.C / 2 + 1;
    for (int e = tid; e < 2 * nf * 8; e += blockDim.x) {
      const int uv = e / (nf * 8), f = (e / 8) % nf, k = e % 8;
      d.basis64[2 * L.C * 64 + e] = ev[uv][f][k];
    }
  }
}

// Fourier slices (float) of the real basis tensors for the filter:
// U_F(f) = sum_j U(:,:,j) exp(-2 pi i f j / c), evaluated in FP64.
// U_ext / V_ext (single-image launches, nullable) replace the image's own
// basis as the source.  The scaled V slices (FB_V0S...) carry the filters'
// output scale: the fixed-point scale of the image's numerator encoding,
// times 1/3 for c = 3 unless the threshold is the channel-Fourier one.
__global__ void k_fbasis(Launch L, const float* U_ext, const float* V_ext) {
  const int nimg = L.table ? L.n_img : 1;
  for (int im = blockIdx.x; im < nimg; im += gridDim.x) {
    const ImgDesc d = L.table ? L.table[im] : L.one;
    const bool ft = L.C == 3 && (L.flags & HTS_FLAG_FOURIER_THRESHOLD);
    const double osc = (double)fx_scale(d, fx_int_units(L.C, L.flags, d.num_enc)) *
                       (L.C == 3 && !ft ? 1.0 / 3.0 : 1.0);
    for (int e = threadIdx.x; e < 128; e += blockDim.x) {
      const int uv = e >> 6, ab = e & 63;
      const float* ext = uv ? V_ext : U_ext;
      const float* T = ext ? ext : d.basis + uv * L.C * 64;
      const int tr = (ab & 7) * 8 + (ab >> 3);   // position of entry ab in the transpose
      if (L.C == 1) {
        d.fbasis[(uv ? FB_V0 : FB_U0) + ab] = T[ab];
        d.fbasis[(uv ? FB_V0T : FB_U0T) + tr] = T[ab];
        if (uv) d.fbasis[FB_V0S + ab] = (float)(osc * (double)T[ab]);
      } else {
        double f0, f1r, f1i;
        dft3((double)T[ab], (double)T[64 + ab], (double)T[128 + ab], f0, f1r, f1i);
        d.fbasis[(uv ? FB_V0 : FB_U0) + ab] = (float)f0;
        d.fbasis[(uv ? FB_V1R : FB_U1R) + ab] = (float)f1r;
        d.fbasis[(uv ? FB_V1I : FB_U1I) + ab] = (float)f1i;
        // the transposed U slices (the left products of the projection)
        // carry the 1/c of the inverse DFT that follows them
        const double q = uv ? 1.0 : 1.0 / 3.0;
        d.fbasis[(uv ? FB_V0T : FB_U0T) + tr] = (float)(q * f0);
        d.fbasis[(uv ? FB_V1RT : FB_U1RT) + tr] = (float)(q * f1r);
        d.fbasis[(uv ? FB_V1IT : FB_U1IT) + tr] = (float)(q * f1i);
        if (uv) {
          d.fbasis[FB_V1PT + tr] = (float)(f1r + f1i);
          d.fbasis[FB_V1M + ab] = (float)(f1r - f1i);
          d.fbasis[FB_V0S + ab] = (float)(osc * f0);
          d.fbasis[FB_V1RS + ab] = (float)(osc * f1r);
          d.fbasis[FB_V1IS + ab] = (float)(osc * f1i);
          d.fbasis[FB_V1MS + ab] = (float)(osc * (f1r - f1i));
        } else {
          d.fbasis[FB_U1MT + tr] = (float)(q * (f1r - f1i));
          d.fbasis[FB_U1P + ab] = (float)(f1r + f1i);
        }
      }
    }
  }
}

hipError_t launch_cov(const Launch& L, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  const int reg = cov_region(L.stride);
  const size_t lds = (size_t)L.C * reg * reg * sizeof(float);
  hipLaunchKernelGGL(k_cov, dim3(xcd_grid(grid > 0 && grid < L.total ? grid : L.total)), dim3(256), lds, s, L);
  return hipGetLastError();
}
hipError_t launch_eig(const Launch& L, hipStream_t s) {
  const int n = L.table ? L.n_img : 1;
  hipLaunchKernelGGL(k_eig, dim3(n), dim3(256), 0, s, L);
  return hipGetLastError();
}
__global__ void k_copy_basis(Launch L, int to_ext) {
  const int nimg = L.table ? L.n_img : 1;
  const int n = L.C * 64;
  for (int im = blockIdx.x; im < nimg; im += gridDim.x) {
    const ImgDesc& d = L.table ? L.table[im] : L.one;
    for (int e = threadIdx.x; e < 2 * n; e += blockDim.x) {
      float* ext = e < n ? d.U_ext : d.V_ext;
      if (!ext) continue;
      if (to_ext) ext[e % n] = d.basis[e];
      else d.basis[e] = ext[e % n];
    }
  }
}

hipError_t launch_copy_basis(const Launch& L, int to_ext, hipStream_t s) {
  const int n = L.table ? L.n_img : 1;
  hipLaunchKernelGGL(k_copy_basis, dim3(n < 65535 ? n : 65535), dim3(256), 0, s, L, to_ext);
  return hipGetLastError();
}

hipError_t launch_fbasis(const Launch& L, const float* U, const float* V, hipStream_t s) {
  const int n = L.table ? L.n_img : 1;
  hipLaunchKernelGGL(k_fbasis, dim3(n), dim3(128), 0, s, L, U, V);
  return hipGetLastError();
}

}  // namespace hts
