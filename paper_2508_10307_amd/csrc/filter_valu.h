#pragma once
// Collaborative filtering and aggregation (Sec. III.B.2, Eq. 17-20; Eq. 2;
// Alg. 1 Step 2(2)-(4) and Step 3), fused in one kernel.
//
// One work group per tile of references; each wavefront filters one group
// at a time.  Lane = (slot lane kl, patch row a): lane kl*8 + a holds row a
// of the K/8 slots kl*SPL .. kl*SPL+SPL-1 for every channel, so
//  * the right products X V run inside the lane, with the 8x8 basis slices
//    (uniform across the wavefront) as scalar operands;
//  * the left products U^H Y run inside the lane after an 8x8 transpose
//    through LDS;
//  * the channel-mode DFT of the t-product (c = 3) is lane-local;
//  * the Haar transform along the group mode (Eq. 9, fast form: pairwise
//    sums and differences, unnormalised, with the scales moved into the
//    thresholds and a power-of-two weight per kept coefficient) runs first
//    on the slots of a lane, then across lanes with xor shuffles;
//  * thresholding, masks and the inverse transforms follow the same layout;
//  * estimates accumulate, in 64-bit fixed point, into an LDS tile covering
//    every patch the tile's groups can touch, flushed once with atomics
//    (coverage counts depend only on the match indices and come from a
//    separate histogram pass).
// ADJ = 1 applies frozen masks instead of the threshold (adjoint of the
// frozen map, see hts_denoise_backward).
#include "hts_device.h"

namespace hts {

constexpr float SQRT3 = 1.73205080756887729353f;
constexpr float HALF_SQRT3 = 0.86602540378443864676f;
constexpr int TPITCH = 9;                 // transpose scratch pitch (floats)
constexpr int TSCRATCH = 8 * 8 * TPITCH;  // floats per wavefront

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Basis slices are read through the constant address space: they are the
// same for every lane, so they become scalar loads into SGPRs and feed the
// FMAs as scalar operands.
typedef __attribute__((address_space(4))) const float cfloat;

// A pointer known to be the same in every lane, moved to SGPRs.
__device__ inline const cfloat* uniform_ptr(const float* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (const cfloat*)(((unsigned long long)hi << 32) | lo);
}

// The basis pointer is passed through an empty asm before every use so that
// the compiler cannot hoist scalar loads out of the group loop (it would
// then keep the coefficients live and spill SGPRs into VGPR lanes).  Only
// the base is laundered: slice offsets are constants added afterwards, so
// they fold into the loads' immediate offsets and no per-slice pointer
// stays live.
__device__ inline const cfloat* launder(const cfloat* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// y[b] (+)= sgn * sum_t M[b*8 + t] x[t], M = fb + off: one 8x8 row-major
// basis slice, consumed as two blocks of four rows (32 scalar operands live
// at a time).  Each block's four results pass through an empty asm: that
// pins the block's FMAs between its own pointer launder and the next one,
// so the compiler cannot gather the loads of several blocks ahead of their
// FMAs (which would again spill coefficients into VGPR lanes).
template <bool ACC>
__device__ inline void mv(const float (&x)[8], const cfloat* fb, int off, float sgn, float (&y)[8]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const cfloat* M = launder(fb) + off + 32 * h;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int b = 4 * h + bb;
      float s = ACC ? y[b] : 0.f;
#pragma unroll
      for (int t = 0; t < 8; ++t) s = fmaf(sgn * x[t], M[bb * 8 + t], s);
      y[b] = s;
    }
    asm volatile("" : "+v"(y[4 * h]), "+v"(y[4 * h + 1]), "+v"(y[4 * h + 2]), "+v"(y[4 * h + 3]));
  }
}

// Complex product with three real products (Gauss):
// (yr + i yi) = (MR + i MI)(xr + i xi), given the slices MR, MI and
// MP = MR + MI (all row-major, at offsets MR, MI, MP of fb):  A = MR xr,
// B = MI xi, C = MP (xr + xi);
// yr = A - B, yi = C - A - B.  MI may be negated through sgn_i (with MP the
// matching sum) to apply a conjugate.
__device__ inline void cmv(const float (&xr)[8], const float (&xi)[8], const cfloat* fb, int MR,
                           int MI, float sgn_i, int MP, float (&yr)[8], float (&yi)[8]) {
  float a[8], b[8], xs[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) xs[t] = xr[t] + xi[t];
  mv<false>(xr, fb, MR, 1.f, a);
  mv<false>(xi, fb, MI, sgn_i, b);
  mv<false>(xs, fb, MP, 1.f, yi);
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    yr[t] = a[t] - b[t];
    yi[t] = yi[t] - a[t] - b[t];
  }
}

// Transposes through the wavefront's LDS scratch.  Forward: lane (kl, a)
// holds row a of an 8x8 matrix and receives column a.  Backward: holds
// column a and receives row a.
__device__ inline void transpose_rc(float* T, int kl, int a, float (&v)[8]) {
  float* base = T + kl * 8 * TPITCH;
#pragma unroll
  for (int c = 0; c < 8; ++c) base[a * TPITCH + c] = v[c];
  wave_sync();
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = base[r * TPITCH + a];
  wave_sync();
}
__device__ inline void transpose_cr(float* T, int kl, int a, float (&v)[8]) {
  float* base = T + kl * 8 * TPITCH;
#pragma unroll
  for (int r = 0; r < 8; ++r) base[r * TPITCH + a] = v[r];
  wave_sync();
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = base[a * TPITCH + c];
  wave_sync();
}

// One Haar butterfly across slot lanes kl and kl ^ m (lanes l and l ^ 8m):
// the lower lane keeps x_lo + x_hi, the upper x_lo - x_hi (sg = +1 / -1).
// m = 1: the partner by a DPP rotation by 8 within each 16-lane row.
// m = 2, 4: v_permlane16_swap / v_permlane32_swap of the value with itself
// leaves, in every lane of the pair, the lower lane's value in the first
// result and the upper lane's in the second, with no trip through LDS.
// Both lanes of a pair are active or inactive together.
__device__ inline float haar_xlane(float x, int m, float sg) {
  if (m == 1) {
    const float o = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128 /* row_ror:8 */,
                                                               0xF, 0xF, false));
    return fmaf(sg, x, o);
  }
  const unsigned b = __float_as_uint(x);
  const auto r = m == 2 ? __builtin_amdgcn_permlane16_swap(b, b, false, false)
                        : __builtin_amdgcn_permlane32_swap(b, b, false, false);
  return fmaf(sg, __uint_as_float(r[1]), __uint_as_float(r[0]));
}

// Haar row (Eq. 9 ordering) of the coefficient produced for group slot k.
__device__ inline int haar_row(int k, int K) {
  if (k == 0) return 0;
  const int L = __builtin_ctz(k) + 1;
  return (K >> L) + (k >> L);
}

// The butterflies run unnormalised ((u + v, u - v), no 1/sqrt 2): the
// forward transform is D H (H orthonormal, D = diag 2^(l/2), l = the level
// of the coefficient left in slot k: ctz(k) + 1, log2 K for the DC row in
// slot 0), so a coefficient is compared with tau 2^(l/2).  The unscaled
// inverse butterflies apply H^T D; scaling each kept coefficient by 2^-l
// (a power of two) first makes it H^T D^-1, the exact inverse.
__device__ inline int haar_level(int k, int K) {
  return k == 0 ? __builtin_ctz(K) : __builtin_ctz(k) + 1;
}
__device__ inline float haar_scale(int k, int K) {
  const int l = haar_level(k, K);
  const float p = (float)(1 << (l >> 1));
  return (l & 1) ? p * 1.41421356237309504880f : p;
}
__device__ inline float haar_unscale(int k, int K) {
  return 1.f / (float)(1 << haar_level(k, K));
}

// MASKS = 1 exports the keep-masks (when d.masks is set).
// WT = 1: weighted aggregation (a separate instantiation, so that the
// uniform one keeps its register budget).
// WT = 2: uniform weights without the LDS tile, for groups whose patches
// may lie anywhere in the image (the stacked frames of a video): every slot's
// estimate, scaled for the fixed-point conversion, is exported to its record
// d.group_est[(g K + k) C + ch][row][col], and the aggregation gathers them
// per output tile afterwards (k_gather_tiles).
// FT = 1 (c = 3): threshold in the channel-Fourier domain (whole conjugate
// pairs by their orthonormal magnitude) instead of Eq. 19 on the real core:
// the channel IDFT after the projection and the DFT before the inverse are
// skipped, since the Haar transform along the group commutes with them.
template <int C, int SPL, int ADJ, int MASKS, int BATCH, int WT, int FT>
__global__ __launch_bounds__(256, 2) void k_filter(Launch L) {
  extern __shared__ __align__(16) float fsm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kl = lane >> 3, a = lane & 7;
  const int K = L.K;
  const int NL = SPL > 1 ? 8 : (K < 8 ? K : 8);   // slot lanes in use (all eight for K >= 16)
  const bool active = SPL > 1 || kl < NL;   // K >= 16 keeps every lane busy
  const int r = (L.window - 1) / 2;
  const int s = L.stride;
  const int TY = L.fty, TX = L.ftx;
  const int RA = (TY - 1) * s + 2 * r + PS, CA = (TX - 1) * s + 2 * r + PS;
  // weighted aggregation (Eq. 2 with w_g = 1 / max(1, kept coefficients)):
  // one more tile plane for the weight sums
  constexpr bool wtd = WT == 1 && !ADJ;
  constexpr bool glob = WT == 2 && !ADJ;
  constexpr bool ft = FT != 0 && C == 3 && !ADJ;
  constexpr int NP = C + (wtd ? 1 : 0);
  constexpr bool units = WT != 1 && !ADJ;   // integer-unit numerator (fx_int_units)
  unsigned long long* acc = (unsigned long long*)fsm;          // [NP][RA][CA] fixed point
  float* T = fsm + (glob ? 0 : (2 * NP * RA * CA + 3) / 4 * 4) + wave * TSCRATCH;   // transpose scratch

  for_each_item_t<W_FILT, BATCH>(L, [&](const auto& d, int item) __attribute__((always_inline)) {
    const int ntx = (d.nrx + TX - 1) / TX;
    const int iy0 = (item / ntx) * TY, ix0 = (item % ntx) * TX;
    const int iy1 = min(d.nry, iy0 + TY) - 1, ix1 = min(d.nrx, ix0 + TX) - 1;
    const int AY0 = max(0, ref_coord(iy0, s, d.Hp) - r);
    const int AY1 = min(d.Hp - 1, ref_coord(iy1, s, d.Hp) + r) + PS - 1;
    const int AX0 = max(0, ref_coord(ix0, s, d.Wp) - r);
    const int AX1 = min(d.Wp - 1, ref_coord(ix1, s, d.Wp) + r) + PS - 1;
    const int AW = AX1 - AX0 + 1, AH = AY1 - AY0 + 1;
    const int HW = d.H * d.W;
    const cfloat* fb = uniform_ptr(d.fbasis);
    // adjusted noise level (A-Haar-tSVD) when the descriptor carries one
    const float tau = d.sigma_dev ? L.tau_mult * *d.sigma_dev : d.tau;
    const float rW = 1.0f / (float)d.W;
    const float fxs = fx_scale(d, units);          // fixed-point scale of the estimates
    const float rfxs = 1.f / fxs;
    float tauj[SPL], wj[SPL];                      // thresholds and inverse weights of this lane's slots
    float tq0[SPL], tq1[SPL];                      // FT: squared thresholds of f = 0 and of the f = 1 pair
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      tauj[j] = tau * haar_scale(kl * SPL + j, K);
      // the lanes hold Fourier coefficients / 3 (the U slices carry 1/3):
      // |F_0| / sqrt 3 >= t  <=>  (F_0/3)^2 >= t^2 / 3;
      // sqrt(2/3) |F_1| >= t  <=>  |F_1/3|^2 >= t^2 / 6
      tq0[j] = tauj[j] * tauj[j] * (1.f / 3.f);
      tq1[j] = tauj[j] * tauj[j] * (1.f / 6.f);
      wj[j] = haar_unscale(kl * SPL + j, K);
    }

    if (!glob) {
      __syncthreads();
      for (int e = tid; e < NP * RA * CA; e += 256) acc[e] = 0ull;
      __syncthreads();
    }

    const int ngroups = (iy1 - iy0 + 1) * (ix1 - ix0 + 1);
    const int gw = ix1 - ix0 + 1;
    auto group_of = [&](int gl) __attribute__((always_inline)) {
      return (iy0 + gl / gw) * d.nrx + ix0 + gl % gw;
    };
    // the idx entries of the wavefront's next group are loaded one group
    // ahead (inactive lanes, K < 8, read slot 0 and drop it)
    auto load_pos = [&](int gl, int (&pos)[SPL]) __attribute__((always_inline)) {
      const int gn = gl < ngroups ? group_of(gl) : -1;
      const bool ok = gn >= d.ref_begin && gn < d.ref_begin + d.ref_count;
#pragma unroll
      for (int j = 0; j < SPL; ++j)
        pos[j] = ok ? d.idx[(size_t)gn * K + (active ? kl * SPL + j : 0)] : 0;
    };
    int pos_next[SPL];
    load_pos(wave, pos_next);
    for (int gl = wave; gl < ngroups; gl += 4) {
      const int g = group_of(gl);
      int pos_cur[SPL];
#pragma unroll
      for (int j = 0; j < SPL; ++j) pos_cur[j] = pos_next[j];
      load_pos(gl + 4, pos_next);
      if (g < d.ref_begin || g >= d.ref_begin + d.ref_count) continue;
      const int grel = g - d.ref_begin;

      // ---- gather ----
      // nf stays 0 unless a gathered pixel or an estimate is not finite
      // (0 * inf and 0 * NaN are NaN)
      float nf = 0.f;
      int nkeep = 0;   // kept coefficients of the group (weighted aggregation)
      // Lane (kl, a) takes row a of each of its slots' patches as row
      // projections (d.rowp: the row after the channel DFT, times V_F):
      // X[j][q] = q-th part (c = 3: f = 0, Re f = 1, Im f = 1) of P^ V_F.
      float X[SPL][C][8];
      int py[SPL], px[SPL];
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        // positions come from the caller's idx: clamp to valid patch corners
        split_pos(pos_cur[j], d.W, rW, py[j], px[j]);
        py[j] = min(max(py[j], 0), d.Hp - 1);
        px[j] = min(max(px[j], 0), d.Wp - 1);
        const float4* src =
            (const float4*)(d.rowp + ((size_t)(py[j] + a) * d.Wp + px[j]) * (8 * C));
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float4 v = src[2 * ch + h];
            X[j][ch][4 * h + 0] = active ? v.x : 0.f;
            X[j][ch][4 * h + 1] = active ? v.y : 0.f;
            X[j][ch][4 * h + 2] = active ? v.z : 0.f;
            X[j][ch][4 * h + 3] = active ? v.w : 0.f;
          }
      }

      // ---- t-SVD projection U^T * P * V per slot (Eq. 18, patch level) ----
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        if (C == 1) {
          // y = row a of P V (a non-finite pixel makes it non-finite)
          float y[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            y[b] = X[j][0][b];
            nf = fmaf(y[b], 0.f, nf);
          }
          transpose_rc(T, kl, a, y);
          float z[8];
          mv<false>(y, fb, FB_U0T, 1.f, z);   // z[i] = sum_r y[r] U[r][i]
#pragma unroll
          for (int i = 0; i < 8; ++i) X[j][0][i] = z[i];
        } else {
          // Y = P^ V_F, row a: f = 0 real, f = 1 complex
          float y0[8], y1r[8], y1i[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            y0[b] = X[j][0][b];
            y1r[b] = X[j][1][b];
            y1i[b] = X[j][2][b];
            nf = fmaf(y0[b], 0.f, nf);
          }
          transpose_rc(T, kl, a, y0);
          transpose_rc(T, kl, a, y1r);
          transpose_rc(T, kl, a, y1i);
          // Z = U_F^H Y: z[i] = sum_r conj(U[r][i]) y[r]
          float z0[8], z1r[8], z1i[8];
          mv<false>(y0, fb, FB_U0T, 1.f, z0);
          // z1 = conj(U_F(1))^T y1: (U1R - i U1I)^T (y1r + i y1i)
          cmv(y1r, y1i, fb, FB_U1RT, FB_U1IT, -1.f, FB_U1MT, z1r, z1i);
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const float sr = z1r[i], si = z1i[i];
            if (ft) {   // keep the Fourier coefficients: (F_0, Re F_1, Im F_1) / 3
              X[j][0][i] = z0[i];
              X[j][1][i] = sr;
              X[j][2][i] = si;
            } else {    // inverse DFT along the channel mode (its 1/3 is in the U slices)
              X[j][0][i] = fmaf(2.f, sr, z0[i]);
              X[j][1][i] = fmaf(-SQRT3, si, z0[i] - sr);
              X[j][2][i] = fmaf(SQRT3, si, z0[i] - sr);
            }
          }
        }
      }

      // ---- Haar along the group mode (Eq. 17-18), in-lane levels ----
#pragma unroll
      for (int st = 1; st < SPL; st <<= 1)
#pragma unroll
        for (int j = 0; j < SPL; j += 2 * st)
#pragma unroll
          for (int ch = 0; ch < C; ++ch)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const float u = X[j][ch][i], v = X[j + st][ch][i];
              X[j][ch][i] = u + v;
              X[j + st][ch][i] = u - v;
            }
      // cross-lane levels on the running sums (slot lanes kl ^ m)
#pragma unroll
      for (int m = 1; m < NL; m <<= 1) {
        const bool part = (kl & (m - 1)) == 0;
        const float sg = (kl & m) ? -1.f : 1.f;   // upper lane: o - x, lower: x + o
        // lanes outside the level keep their coefficients (exec mask, not a
        // select); partners of active lanes are active
        if (part) {
#pragma unroll
          for (int ch = 0; ch < C; ++ch)
#pragma unroll
            for (int i = 0; i < 8; ++i) X[0][ch][i] = haar_xlane(X[0][ch][i], m, sg);
        }
      }

      // ---- channel-Fourier threshold (FT): f = 0 alone, f = 1 with its conjugate ----
      if (ft) {
#pragma unroll
        for (int j = 0; j < SPL; ++j) {
          const int row = haar_row(kl * SPL + j, K);
          unsigned char mb0 = 0, mb1 = 0;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const float x0 = X[j][0][i], x1 = X[j][1][i], x2 = X[j][2][i];
            const bool k0 = x0 * x0 >= tq0[j];
            const bool k1 = fmaf(x1, x1, x2 * x2) >= tq1[j];
            X[j][0][i] = k0 ? x0 * wj[j] : 0.f;
            X[j][1][i] = k1 ? x1 * wj[j] : 0.f;
            X[j][2][i] = k1 ? x2 * wj[j] : 0.f;
            if (wtd) nkeep += __popcll(__ballot(k0 && active)) + 2 * __popcll(__ballot(k1 && active));
            if (MASKS && d.masks) {
              const unsigned long long b0 = __ballot(k0), b1 = __ballot(k1);
              if (i == a) {
                mb0 = (unsigned char)((b0 >> (8 * kl)) & 0xFFu);
                mb1 = (unsigned char)((b1 >> (8 * kl)) & 0xFFu);
              }
            }
          }
          if (MASKS && d.masks && active) {   // frequency f in mask channel f (f = 2 mirrors f = 1)
            unsigned char* mk = (unsigned char*)d.masks + ((size_t)grel * K + row) * C * 8 + a;
            mk[0] = mb0;
            mk[8] = mb1;
            mk[16] = mb1;
          }
        }
      }

      // ---- hard threshold (Eq. 19) or frozen mask; optional mask export ----
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        if (ft) break;
        const int k = kl * SPL + j;
        const int row = haar_row(k, K);
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          const size_t word = ((size_t)grel * K + row) * C + ch;   // 64-bit word index
          if (ADJ) {
            unsigned long long bits = 0;
            if (active) {
              const uint32_t* w = d.masks_in + 2 * word;
              bits = (unsigned long long)w[0] | ((unsigned long long)w[1] << 32);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
              X[j][ch][i] = ((bits >> (i * 8 + a)) & 1ull) ? X[j][ch][i] * wj[j] : 0.f;
          } else {
            unsigned char mybyte = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const bool keep = fabsf(X[j][ch][i]) >= tauj[j];
              X[j][ch][i] = keep ? X[j][ch][i] * wj[j] : 0.f;
              if (wtd) nkeep += __popcll(__ballot(keep && active));
              if (MASKS && d.masks) {
                const unsigned long long bal = __ballot(keep);
                const unsigned char byte = (unsigned char)((bal >> (8 * kl)) & 0xFFu);
                if (i == a) mybyte = byte;
              }
            }
            if (MASKS && d.masks && active) ((unsigned char*)d.masks)[word * 8 + a] = mybyte;
          }
        }
      }

      // ---- inverse Haar: cross-lane levels (coarse first), then in-lane ----
#pragma unroll
      for (int m = NL >> 1; m >= 1; m >>= 1) {
        const bool part = (kl & (m - 1)) == 0;
        const float sg = (kl & m) ? -1.f : 1.f;
        // lanes outside the level keep their coefficients (exec mask, not a
        // select); partners of active lanes are active
        if (part) {
#pragma unroll
          for (int ch = 0; ch < C; ++ch)
#pragma unroll
            for (int i = 0; i < 8; ++i) X[0][ch][i] = haar_xlane(X[0][ch][i], m, sg);
        }
      }
#pragma unroll
      for (int st = SPL >> 1; st >= 1; st >>= 1)
#pragma unroll
        for (int j = 0; j < SPL; j += 2 * st)
#pragma unroll
          for (int ch = 0; ch < C; ++ch)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const float u = X[j][ch][i], v = X[j + st][ch][i];
              X[j][ch][i] = u + v;
              X[j + st][ch][i] = u - v;
            }

      // group weight (1 when uniform): scales the estimates, and is added to
      // the weight plane for every pixel of the group's patches
      const float wg = wtd ? 1.f / (float)max(nkeep, 1) : 1.f;
      const unsigned long long fxw = wtd ? fx_from_float(wg * WEIGHT_SCALE) : 0ull;
      const float rge = rfxs / wg;

      // ---- inverse t-SVD projection U * S * V^T (Eq. 20) and write-back ----
      // The V slices of the last product carry the output scale (the
      // fixed-point scale, times 1/3 for c = 3), so for c = 3 the row comes
      // out as the fixed-point channel-DFT triple (F0, Re F1, Im F1) / 3 of
      // the estimate (fx_fourier): the inverse channel DFT moves to the
      // write-back.
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        float out[C][8];
        if (C == 1) {
          float y[8];
          mv<false>(X[j][0], fb, FB_U0, 1.f, y);   // y[r] = sum_i U[r][i] s[i]
          transpose_cr(T, kl, a, y);
          mv<false>(y, fb, FB_V0S, 1.f, out[0]);   // out[b] = sum_c y[c] V[b][c] (scaled)
          if (wtd)
#pragma unroll
            for (int b = 0; b < 8; ++b) out[0][b] *= wg;
        } else {
          float s0[8], s1r[8], s1i[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const float q0 = X[j][0][i], q1 = X[j][1][i], q2 = X[j][2][i];
            if (ft) {   // already in the Fourier domain (F / 3)
              s0[i] = q0;
              s1r[i] = q1;
              s1i[i] = q2;
            } else {
              s0[i] = q0 + q1 + q2;
              s1r[i] = q0 - 0.5f * (q1 + q2);
              s1i[i] = HALF_SQRT3 * (q2 - q1);
            }
          }
          // Y = U_F S^: y[r] = sum_i U[r][i] s[i]
          float y0[8], y1r[8], y1i[8];
          mv<false>(s0, fb, FB_U0, 1.f, y0);
          // y1 = U_F(1) s1: (U1R + i U1I)(s1r + i s1i)
          cmv(s1r, s1i, fb, FB_U1R, FB_U1I, 1.f, FB_U1P, y1r, y1i);
          transpose_cr(T, kl, a, y0);
          transpose_cr(T, kl, a, y1r);
          transpose_cr(T, kl, a, y1i);
          // P^ = Y V_F^H: p[b] = sum_c y[c] conj(V[b][c]) (scaled slices)
          mv<false>(y0, fb, FB_V0S, 1.f, out[0]);
          // p1 = conj(V_F(1)) y1 per row: (V1R - i V1I)(y1r + i y1i)
          cmv(y1r, y1i, fb, FB_V1RS, FB_V1IS, -1.f, FB_V1MS, out[1], out[2]);
          if (wtd)
#pragma unroll
            for (int b = 0; b < 8; ++b) {
              out[0][b] *= wg;
              out[1][b] *= wg;
              out[2][b] *= wg;
            }
        }
        const int ly = py[j] + a - AY0, lx = px[j] - AX0;
        // a patch outside the tile's reach (an idx entry that is not from
        // its reference's search window) goes straight to the image
        const bool inside = ly >= a && ly + PS - a <= AH && lx >= 0 && lx + PS <= AW;
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
#pragma unroll
          for (int b = 0; b < 8; ++b) nf = fmaf(out[ch][b], 0.f, nf);
        if (glob) {
          // row a of the slot's estimate into its export record
          if (active) {
            float4* ge = (float4*)(d.group_est + (((size_t)grel * K + kl * SPL + j) * C) * PS2 + a * 8);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
              ge[ch * (PS2 / 4)] = make_float4(out[ch][0], out[ch][1], out[ch][2], out[ch][3]);
              ge[ch * (PS2 / 4) + 1] = make_float4(out[ch][4], out[ch][5], out[ch][6], out[ch][7]);
            }
          }
        } else if (active) {
          const int k = kl * SPL + j;
          if (inside) {
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
              unsigned long long* rowp = acc + (ch * RA + ly) * CA + lx;
#pragma unroll
              for (int b = 0; b < 8; ++b) atomicAdd(rowp + b, fx_from<units>(out[ch][b]));
            }
            if (wtd) {
              unsigned long long* wrow = acc + (C * RA + ly) * CA + lx;
#pragma unroll
              for (int b = 0; b < 8; ++b) atomicAdd(wrow + b, fxw);
            }
          } else if constexpr (!BATCH || ADJ) {
            // (the batched forward filters the groups of its own match, which
            // always lie inside the tile: no cold path, no register cost; the
            // batched adjoint takes the caller's indices and keeps it)
            const int pix = (py[j] + a) * d.W + px[j];
            for (int b = 0; b < 8; ++b) {
              const float v3[3] = {out[0][b], out[C > 1 ? 1 : 0][b], out[C > 1 ? 2 : 0][b]};
              add_pixel_global<units>(d, C, pix + b, v3, fxs);
            }
            if (wtd)
              for (int b = 0; b < 8; ++b) add_weight_global(d, pix + b, fxw);
          }
          if (d.group_est) {   // image units, unweighted (c = 3: channel DFT inverted)
            float* ge = d.group_est + (((size_t)grel * K + k) * C) * PS2 + a * 8;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
              if (C == 3) {
                const float a0 = out[0][b], a1 = out[C > 1 ? 1 : 0][b], a2 = out[C > 1 ? 2 : 0][b];
                ge[b] = fmaf(2.f, a1, a0) * rge;
                ge[PS2 + b] = fmaf(-SQRT3, a2, a0 - a1) * rge;
                ge[2 * PS2 + b] = fmaf(SQRT3, a2, a0 - a1) * rge;
              } else {
                ge[b] = out[0][b] * rge;
              }
            }
          }
        }
      }
      if (__ballot(nf != 0.f)) poison_group(d, d.idx + (size_t)g * K, grel, K, C, rW, lane);
    }
    if (!glob) {
      __syncthreads();
      flush_tile(d, acc, C, RA, CA, AY0, AX0, AH, AW, units, fxs, wtd);
    }
  });
}

}  // namespace hts
