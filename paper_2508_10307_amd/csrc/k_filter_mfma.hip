// Collaborative filtering and aggregation for RGB groups on FP32 MFMA
// (Sec. III.B.2, Eq. 17-20; Eq. 2; Alg. 1 Step 2(2)-(4) and Step 3).
//
// The t-product projection U^T * P * V works per frequency f of the DFT
// along the channel mode (Eq. 5-6): P^(f) -> U_F(f)^H P^(f) V_F(f).  For
// c = 3, f = 1 is complex (f = 2 is its conjugate) and f = 0 is real.  Every
// product is written as a 16x16 real GEMM on v_mfma_f32_16x16x4f32:
//
//  * a "complex unit" (CU) is a 16-row operand: rows = 2 slots x 8 patch
//    rows, columns = (real/imag) x 8;
//  * f = 1 of each block of two slots is one CU, multiplied by the real
//    form [[Re, Im], [-Im, Re]] of the 8x8 basis slice;
//  * f = 0 of two blocks is packed as the real and imaginary halves of a
//    third CU and multiplied by diag(U_F(0), U_F(0)), so the real frequency
//    uses the same layout at the same cost as zero padding would;
//  * the basis operands live in VGPRs (32 per lane, loaded once per tile),
//    the data in registers; between the products only one xor-40 lane swap
//    (forward), one LDS transpose (inverse) and one DPP xor-8 exchange
//    move data.
//
// Lane l = 16 q + n (q = l / 16, n = l % 16, s = n / 8).  The Haar transform
// along the group mode pairs slots 2b, 2b+1 across lanes (xor 8) and the
// coarser levels inside each lane's registers; thresholding, mask export,
// the inverse Haar and the inverse projection follow; estimates accumulate in
// a fixed-point LDS tile exactly as in the vector-ALU filter (coverage counts
// come from the match indices alone and are computed by a separate
// histogram pass).
#include "hts_device.h"

namespace hts {

namespace {

typedef __attribute__((ext_vector_type(4))) float f4;

constexpr float SQ3 = 1.73205080756887729353f;
constexpr float HSQ3 = 0.86602540378443864676f;
// Transpose scratch: element (ro, s, r, b) at (s*8 + b)*TPB + r*2 + ro, so a
// lane writes its four values (r in {2q, 2q+1}, ro in {0, 1}) as one 16-byte
// store and reads its operands as two 8-byte loads; TPB = 20 keeps the
// 16-byte alignment and spreads the banks.
constexpr int TPB = 20;
constexpr int TSZ = 2 * 8 * TPB;                 // floats per wavefront

__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lane l <- lane l ^ 8 (rotation by 8 inside each 16-lane row)
__device__ inline float xor8(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, true));
}

// lane l <- lane l ^ 32 (v_permlane32_swap exchanges the upper half of its
// first operand with the lower half of its second)
__device__ inline float xor32(float v, bool upper) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(upper ? r[0] : r[1]);
}

__device__ inline int haar_row_m(int k, int K) {
  if (k == 0) return 0;
  const int L = __builtin_ctz(k) + 1;
  return (K >> L) + (k >> L);
}

// Unnormalised butterflies ((u + v, u - v)): the forward transform is D H
// (D = diag 2^(l/2), l = ctz(k) + 1 for slot k, log2 K for slot 0), so a
// coefficient is compared with tau 2^(l/2); the unscaled inverse applies
// H^T D, and scaling each kept coefficient by 2^-l first makes it exact.
__device__ inline int haar_level_m(int k, int K) {
  return k == 0 ? __builtin_ctz(K) : __builtin_ctz(k) + 1;
}
__device__ inline float haar_scale_m(int k, int K) {
  const int l = haar_level_m(k, K);
  const float p = (float)(1 << (l >> 1));
  return (l & 1) ? p * 1.41421356237309504880f : p;
}

}  // namespace

// K = 32 keeps 96 coefficients, 32 basis operands and the four products'
// operands per lane: it is built for one wavefront per SIMD (512 registers,
// AGPRs included) rather than spill to scratch.
// MASKS = 1 exports the keep-masks (when d.masks is set); the variant
// without the export keeps the ballots out of the register budget.
template <int K, int ADJ, int MASKS, int BATCH>
__global__ __launch_bounds__(256, K >= 32 ? 1 : 2) void k_filter_mfma(Launch L) {
  constexpr int C = 3;
  constexpr int NB = K / 2;            // blocks of two slots
  constexpr int NCU = NB + NB / 2;     // f=1 units + packed f=0 units
  extern __shared__ __align__(16) float fsm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, n = lane & 15, s = n >> 3, n8 = n & 7;
  const int r = (L.window - 1) / 2;
  const int st = L.stride;
  const int TY = L.fty, TX = L.ftx;
  const int RA = (TY - 1) * st + 2 * r + PS, CA = (TX - 1) * st + 2 * r + PS;
  constexpr int NP = C;
  unsigned long long* acc = (unsigned long long*)fsm;          // [NP][RA][CA] fixed point
  float* T = fsm + (2 * NP * RA * CA + 3) / 4 * 4 + wave * TSZ;   // transpose scratch (16 B aligned)
  const bool swap40 = ((lane >> 5) & 1) != ((lane >> 3) & 1);
  const bool upper32 = lane >= 32;

  for_each_item_t<W_FILT, BATCH>(L, [&](const auto& d, int item) __attribute__((always_inline)) {
    const int ntx = (d.nrx + TX - 1) / TX;
    const int iy0 = (item / ntx) * TY, ix0 = (item % ntx) * TX;
    const int iy1 = min(d.nry, iy0 + TY) - 1, ix1 = min(d.nrx, ix0 + TX) - 1;
    const int AY0 = max(0, ref_coord(iy0, st, d.Hp) - r);
    const int AY1 = min(d.Hp - 1, ref_coord(iy1, st, d.Hp) + r) + PS - 1;
    const int AX0 = max(0, ref_coord(ix0, st, d.Wp) - r);
    const int AX1 = min(d.Wp - 1, ref_coord(ix1, st, d.Wp) + r) + PS - 1;
    const int AW = AX1 - AX0 + 1, AH = AY1 - AY0 + 1;
    const int HW = d.H * d.W;
    // adjusted noise level (A-Haar-tSVD) when the descriptor carries one
    const float tau = d.sigma_dev ? L.tau_mult * *d.sigma_dev : d.tau;
    const float rW = 1.0f / (float)d.W;
    constexpr bool units = !ADJ;                   // integer units (fx_int_units)
    const float fxs = fx_scale(d, units);          // fixed-point scale
    const float rfxs = 1.f / fxs;
    const float sgl = s ? -1.f : 1.f;              // level-1 butterfly: odd slot o - v, even v + o
    const float* fb = d.fbasis;

    // ---- basis operands for the four products (see the header comment) ----
    // Every lane loads all three slices and combines them with 0 / +-1 weights
    // (no lane-dependent choice of which value to load, so the compiler
    // cannot turn the selection into predicated loads).
    float Bf1[4], Bf0[4], Af1[4], Af0[4], Ai1[4], Ai0[4], Bi1[4], Bi0[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      {  // forward right: k = (ri = ks/2, t = 2q + ks%2), column n = (ro = s, b = n8)
        const int ri = ks >> 1, t = 2 * q + (ks & 1), ro = s, b = n8;
        const float vr = fb[FB_V1R + t * 8 + b], vi = fb[FB_V1I + t * 8 + b], v0 = fb[FB_V0 + t * 8 + b];
        const float wd = ri == ro ? 1.f : 0.f, wo = ri == ro ? 0.f : (ri == 0 ? 1.f : -1.f);
        Bf1[ks] = wd * vr + wo * vi;
        Bf0[ks] = wd * v0;
      }
      {  // forward left: row n = (ro = (n%4)/2, i = 2(n/4) + n%2), k = (ri = q/2, r = 4(q%2) + ks)
        const int ro = (n & 3) >> 1, i = 2 * (n >> 2) + (n & 1), ri = q >> 1, rr = 4 * (q & 1) + ks;
        const float ur = fb[FB_U1R + rr * 8 + i], ui = fb[FB_U1I + rr * 8 + i], u0 = fb[FB_U0 + rr * 8 + i];
        const float wd = ri == ro ? 1.f : 0.f, wo = ri == ro ? 0.f : (ro == 0 ? 1.f : -1.f);
        Af1[ks] = wd * ur + wo * ui;
        Af0[ks] = wd * u0;
      }
      {  // inverse left: row n = (ro = (n%4)/2, r = 2(n/4) + n%2), k = (ri = ks/2, i = 2q + ks%2)
        const int ro = (n & 3) >> 1, rr = 2 * (n >> 2) + (n & 1), ri = ks >> 1, i = 2 * q + (ks & 1);
        const float ur = fb[FB_U1R + rr * 8 + i], ui = fb[FB_U1I + rr * 8 + i], u0 = fb[FB_U0 + rr * 8 + i];
        const float wd = ri == ro ? 1.f : 0.f, wo = ri == ro ? 0.f : (ro == 0 ? -1.f : 1.f);
        Ai1[ks] = wd * ur + wo * ui;
        Ai0[ks] = wd * u0;
      }
      {  // inverse right: k = (ri = ks/2, b = 2q + ks%2), column n = (ro = s, t = n8);
         // the slices carry the output scale (the fixed-point scale / 3)
        const int ri = ks >> 1, b = 2 * q + (ks & 1), ro = s, t = n8;
        const float vr = fb[FB_V1RS + t * 8 + b], vi = fb[FB_V1IS + t * 8 + b], v0 = fb[FB_V0S + t * 8 + b];
        const float wd = ri == ro ? 1.f : 0.f, wo = ri == ro ? 0.f : (ri == 0 ? -1.f : 1.f);
        Bi1[ks] = wd * vr + wo * vi;
        Bi0[ks] = wd * v0;
      }
    }

    __syncthreads();
    for (int e = tid; e < NP * RA * CA; e += 256) acc[e] = 0ull;
    __syncthreads();

    const int gw = ix1 - ix0 + 1;
    const int ngroups = (iy1 - iy0 + 1) * gw;
    for (int gl = wave; gl < ngroups; gl += 4) {
      const int g = (iy0 + gl / gw) * d.nrx + ix0 + gl % gw;
      if (g < d.ref_begin || g >= d.ref_begin + d.ref_count) continue;
      const int grel = g - d.ref_begin;
      const int* gidx = d.idx + (size_t)g * K;

      // ---- gather rows (slot 2b+s, patch row n8, columns 2q, 2q+1) + channel DFT ----
      // nf stays 0 unless a gathered pixel or an estimate is not finite
      // (0 * inf and 0 * NaN are NaN); the packed f = 0 products multiply
      // by zero blocks, which would turn an infinite pixel into NaN
      // coefficients that the threshold then drops, so inputs are checked too.
      float nf = 0.f;
      float X[NCU][4];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int pos = gidx[2 * b + s];
        int py, px;
        split_pos(pos, d.W, rW, py, px);
        py = min(max(py, 0), d.Hp - 1);
        px = min(max(px, 0), d.Wp - 1);
        const float* src = d.img + (py + n8) * d.W + px + 2 * q;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float p0 = src[e], p1 = src[HW + e], p2 = src[2 * HW + e];
          X[b][e] = p0 - 0.5f * (p1 + p2);             // Re P^(1)
          X[b][2 + e] = HSQ3 * (p2 - p1);              // Im P^(1)
          X[NB + b / 2][2 * (b & 1) + e] = p0 + p1 + p2;  // P^(0), packed
          nf = fmaf(p0 + p1 + p2, 0.f, nf);
        }
      }

      __builtin_amdgcn_sched_barrier(0);
      // ---- forward right product Y = P^ V_F, then the xor-40 lane swap ----
#pragma unroll
      for (int cu = 0; cu < NCU; ++cu) {
        __builtin_amdgcn_sched_barrier(0);  // one unit's accumulator live at a time
        f4 a4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) a4 = mma(X[cu][ks], cu < NB ? Bf1[ks] : Bf0[ks], a4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float o = xor32(xor8(a4[j]), upper32);   // lane l ^ 40, on the VALU
          X[cu][j] = swap40 ? o : a4[j];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // ---- forward left product Z = U_F^H Y ----
#pragma unroll
      for (int cu = 0; cu < NCU; ++cu) {
        __builtin_amdgcn_sched_barrier(0);  // one unit's accumulator live at a time
        f4 a4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) a4 = mma(cu < NB ? Af1[ks] : Af0[ks], X[cu][ks], a4);
#pragma unroll
        for (int j = 0; j < 4; ++j) X[cu][j] = a4[j];
      }
      __builtin_amdgcn_sched_barrier(0);
      // ---- inverse channel DFT -> coefficients S[b][ch][e] at (i = 2q + e, column n8) ----
      float S[NB][3][2];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float z0 = X[NB + b / 2][2 * (b & 1) + e], zr = X[b][e], zi = X[b][2 + e];
          S[b][0][e] = (z0 + 2.f * zr) * (1.f / 3.f);
          S[b][1][e] = (z0 - zr - SQ3 * zi) * (1.f / 3.f);
          S[b][2][e] = (z0 - zr + SQ3 * zi) * (1.f / 3.f);
        }

      __builtin_amdgcn_sched_barrier(0);
      // ---- Haar along the group (Eq. 9): slots 2b, 2b+1 across lanes, then blocks ----
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const float v = S[b][c][e], o = xor8(v);
            S[b][c][e] = fmaf(sgl, v, o);
          }
#pragma unroll
      for (int w = 1; w < NB; w <<= 1)
#pragma unroll
        for (int b = 0; b < NB; b += 2 * w)
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const float u = S[b][c][e], v = S[b + w][c][e];
              S[b][c][e] = s ? u : u + v;
              S[b + w][c][e] = s ? v : u - v;
            }

      __builtin_amdgcn_sched_barrier(0);
      // ---- hard threshold (Eq. 19) or frozen mask; mask export ----
      // Mask words (one 64-bit word per slot and channel, uniform values) go
      // to the wavefront's scratch from lane 0 and are stored once per group.
      unsigned long long* Tm = (unsigned long long*)T;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          __builtin_amdgcn_sched_barrier(0);
          if (ADJ) {
            const int row_s = haar_row_m(2 * b + s, K);
            const uint32_t* w = d.masks_in + 2 * (((size_t)grel * K + row_s) * C + c);
            const unsigned long long bits = (unsigned long long)w[0] | ((unsigned long long)w[1] << 32);
            const float wgt = 1.f / (float)(1 << haar_level_m(2 * b + s, K));
#pragma unroll
            for (int e = 0; e < 2; ++e)
              S[b][c][e] = ((bits >> ((2 * q + e) * 8 + n8)) & 1ull) ? S[b][c][e] * wgt : 0.f;
          } else {
            unsigned long long bal[2];
            const float thr = tau * (s ? 1.41421356237309504880f : haar_scale_m(2 * b, K));
            const float wgt = s ? 0.5f : 1.f / (float)(1 << haar_level_m(2 * b, K));
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const bool keep = fabsf(S[b][c][e]) >= thr;
              S[b][c][e] = keep ? S[b][c][e] * wgt : 0.f;
              bal[e] = __ballot(keep);
            }
            if (MASKS && d.masks) {
              // word of slot 2b+ss: byte 2q'+e <- ballot bits [16q' + 8ss, +8)
#pragma unroll
              for (int ss = 0; ss < 2; ++ss) {
                unsigned long long wrd = 0ull;
#pragma unroll
                for (int qq = 0; qq < 4; ++qq)
#pragma unroll
                  for (int e = 0; e < 2; ++e)
                    wrd |= ((bal[e] >> (16 * qq + 8 * ss)) & 0xFFull) << (8 * (2 * qq + e));
                if (lane == 0) Tm[(2 * b + ss) * 3 + c] = wrd;
              }
            }
          }
        }
      if (!ADJ && MASKS && d.masks) {
        wsync();
        unsigned long long* mw = (unsigned long long*)d.masks;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int w = h * 64 + lane;
          if (w < 6 * NB) {
            const int k = w / 3, c = w - 3 * k;
            mw[((size_t)grel * K + haar_row_m(k, K)) * C + c] = Tm[w];
          }
        }
        wsync();
      }


      __builtin_amdgcn_sched_barrier(0);
      // ---- inverse Haar: blocks (coarse first), then slot pairs across lanes ----
#pragma unroll
      for (int w = NB >> 1; w >= 1; w >>= 1)
#pragma unroll
        for (int b = 0; b < NB; b += 2 * w)
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const float u = S[b][c][e], v = S[b + w][c][e];
              S[b][c][e] = s ? u : u + v;
              S[b + w][c][e] = s ? v : u - v;
            }
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const float v = S[b][c][e], o = xor8(v);
            S[b][c][e] = fmaf(sgl, v, o);
          }

      __builtin_amdgcn_sched_barrier(0);
      // ---- channel DFT of the coefficients -> operands of the inverse left product ----
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float c0 = S[b][0][e], c1 = S[b][1][e], c2 = S[b][2][e];
          X[b][e] = c0 - 0.5f * (c1 + c2);
          X[b][2 + e] = HSQ3 * (c2 - c1);
          X[NB + b / 2][2 * (b & 1) + e] = c0 + c1 + c2;
        }
      __builtin_amdgcn_sched_barrier(0);
      // ---- inverse left product Y = U_F S^, transpose (r <-> column) through LDS ----
#pragma unroll
      for (int cu = 0; cu < NCU; ++cu) {
        __builtin_amdgcn_sched_barrier(0);  // one unit's accumulator live at a time
        f4 a4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) a4 = mma(cu < NB ? Ai1[ks] : Ai0[ks], X[cu][ks], a4);
        // lane (q, s, n8) holds (ro = j/2, r = 2q + j%2, column n8): order (r, ro)
        {
          f4 w4 = {a4[0], a4[2], a4[1], a4[3]};     // (r=2q,ro=0) (2q,1) (2q+1,0) (2q+1,1)
          *(f4*)(T + (s * 8 + n8) * TPB + 4 * q) = w4;
        }
        wsync();
        // A operand of the inverse right product: row (s, r' = n8), k = (ri = ks/2, b = 2q + ks%2)
        {
          typedef __attribute__((ext_vector_type(2))) float f2;
          const f2 u0 = *(const f2*)(T + (s * 8 + 2 * q) * TPB + 2 * n8);      // b = 2q: (ro 0, 1)
          const f2 u1 = *(const f2*)(T + (s * 8 + 2 * q + 1) * TPB + 2 * n8);  // b = 2q+1
          X[cu][0] = u0[0];   // ri 0, b 2q
          X[cu][1] = u1[0];   // ri 0, b 2q+1
          X[cu][2] = u0[1];   // ri 1, b 2q
          X[cu][3] = u1[1];   // ri 1, b 2q+1
        }
        wsync();
      }
      __builtin_amdgcn_sched_barrier(0);
      // ---- inverse right product P^ = Y V_F^H ----
#pragma unroll
      for (int cu = 0; cu < NCU; ++cu) {
        __builtin_amdgcn_sched_barrier(0);  // one unit's accumulator live at a time
        f4 a4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) a4 = mma(X[cu][ks], cu < NB ? Bi1[ks] : Bi0[ks], a4);
#pragma unroll
        for (int j = 0; j < 4; ++j) X[cu][j] = a4[j];
      }

      __builtin_amdgcn_sched_barrier(0);
      // ---- pair exchange and write-back of the fixed-point channel-DFT
      // triple (F0, Re F1, Im F1) / 3 (the write-back of the image inverts
      // the channel DFT) ----
      // lane (q, n): rows (s' = q/2, r = 4(q%2) + j), column t = n8; lanes with n < 8
      // finish block 2p, lanes with n >= 8 block 2p+1.
      const int hb = s;
#pragma unroll
      for (int p = 0; p < NB / 2; ++p) {
        const int bb = 2 * p + hb;
        const int k = 2 * bb + (q >> 1);
        const int pos = gidx[k];
        int py, px;
        split_pos(pos, d.W, rW, py, px);
        py = min(max(py, 0), d.Hp - 1);
        px = min(max(px, 0), d.Wp - 1);
        const int ly0 = py + 4 * (q & 1) - AY0, lx = px + n8 - AX0;
        const bool inside = py - AY0 >= 0 && py - AY0 + PS <= AH && px - AX0 >= 0 && px - AX0 + PS <= AW;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float send = hb ? X[2 * p][j] : X[2 * p + 1][j];
          const float recv = xor8(send);
          const float p0 = X[NB + p][j];
          const float pr = hb ? recv : X[2 * p][j];
          const float pi = hb ? X[2 * p + 1][j] : recv;
          const float o0 = p0, o1 = pr, o2 = pi;
          nf = fmaf(o0, 0.f, nf);
          nf = fmaf(o1, 0.f, nf);
          nf = fmaf(o2, 0.f, nf);
          if (inside) {
            unsigned long long* a0 = acc + (ly0 + j) * CA + lx;
            atomicAdd(a0, fx_from<units>(o0));
            atomicAdd(a0 + RA * CA, fx_from<units>(o1));
            atomicAdd(a0 + 2 * RA * CA, fx_from<units>(o2));
          } else if constexpr (!BATCH || ADJ) {   // outside the tile's reach: straight to the image
            const int pix = (py + 4 * (q & 1) + j) * d.W + px + n8;
            const float v3[3] = {o0, o1, o2};
            add_pixel_global<units>(d, C, pix, v3, fxs);
          }
          if (d.group_est) {   // image units: the channel DFT inverted
            float* ge = d.group_est + (((size_t)grel * K + k) * C) * PS2 + (4 * (q & 1) + j) * 8 + n8;
            ge[0] = fmaf(2.f, o1, o0) * rfxs;
            ge[PS2] = fmaf(-SQ3, o2, o0 - o1) * rfxs;
            ge[2 * PS2] = fmaf(SQ3, o2, o0 - o1) * rfxs;
          }
        }
      }
      if (__ballot(nf != 0.f)) poison_group(d, gidx, grel, K, C, rW, lane);
    }
    __syncthreads();
    flush_tile(d, acc, C, RA, CA, AY0, AX0, AH, AW, units, fxs);
  });
}

size_t filter_mfma_lds_bytes(int stride, int window, int ty, int tx) {
  const int r = (window - 1) / 2;
  const size_t RA = (size_t)(ty - 1) * stride + 2 * r + PS;
  const size_t CA = (size_t)(tx - 1) * stride + 2 * r + PS;
  return ((2 * 3 * RA * CA + 3) / 4 * 4 + 4 * TSZ) * sizeof(float);
}

bool filter_mfma_supported(int C, int K) { return C == 3 && (K == 4 || K == 8 || K == 16 || K == 32); }

hipError_t launch_filter_mfma(const Launch& L, int ty, int tx, int adjoint, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  const int g = xcd_grid(grid > 0 && grid < L.total ? grid : L.total);
  const size_t lds = filter_mfma_lds_bytes(L.stride, L.window, ty, tx);
  // batched launches (descriptor table) export masks when L.batch_masks is
  // set and run the adjoint when asked
  const bool batch = L.table != nullptr;
  const bool masks = batch ? L.batch_masks != 0 : L.one.masks != nullptr;
#define HTS_FM(KK)                                                                             \
  case KK:                                                                                     \
    if (adjoint) {                                                                             \
      if (batch) hipLaunchKernelGGL((k_filter_mfma<KK, 1, 0, 1>), dim3(g), dim3(256), lds, s, L); \
      else hipLaunchKernelGGL((k_filter_mfma<KK, 1, 0, 0>), dim3(g), dim3(256), lds, s, L);  \
    } else if (batch) {                                                                        \
      if (masks) hipLaunchKernelGGL((k_filter_mfma<KK, 0, 1, 1>), dim3(g), dim3(256), lds, s, L); \
      else hipLaunchKernelGGL((k_filter_mfma<KK, 0, 0, 1>), dim3(g), dim3(256), lds, s, L);  \
    } else if (masks) hipLaunchKernelGGL((k_filter_mfma<KK, 0, 1, 0>), dim3(g), dim3(256), lds, s, L); \
    else hipLaunchKernelGGL((k_filter_mfma<KK, 0, 0, 0>), dim3(g), dim3(256), lds, s, L);      \
    break;
  switch (L.K) {
    HTS_FM(4)
    HTS_FM(8)
    HTS_FM(16)
    HTS_FM(32)
    default: return hipErrorInvalidValue;
  }
#undef HTS_FM
  return hipGetLastError();
}

}  // namespace hts
