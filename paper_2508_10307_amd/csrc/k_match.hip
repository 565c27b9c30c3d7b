// Block matching (Sec. III.A, Eq. 10; Alg. 1 Step 1).
//
// One work group per 4x4 tile of references.  For each guide plane the tile
// uses, the pixel region covering the union of the 16 search windows is
// staged in LDS (integer guide, centred by an integer offset, which leaves
// every distance unchanged), then:
//
//  1. distance tiles of 16 references x 16 candidates, either as
//     |a|^2 + |b|^2 - 2 a.b with a.b on BF16 MFMA (FP32 accumulation; the
//     operands split into bf16 hi + lo parts when TERMS == 3) or as a plain
//     FP32 sum of squared differences on the vector ALUs;
//  2. every approximate distance d~ comes with a rigorous error bound E
//     (|d~ - d| <= E), so [d~ - E, d~ + E] brackets the exact distance;
//  3. pass 1 keeps, per lane and reference, the two smallest upper bounds;
//     T = the (K-1)-th smallest of those is an upper bound of the exact
//     (K-1)-th smallest distance;
//  4. pass 2 recomputes the tiles and shortlists every candidate with
//     d~ - E <= T: a superset of the exact top K-1, ties included;
//  5. the shortlist is re-ranked with exact integer distances (computed in
//     FP64, exact below 2^53) and sorted by (distance, index) on one
//     wavefront; slot 0 is the reference itself.
//
// A reference whose shortlist exceeds SHORT_CAP goes to a list handled by
// k_match_fallback (exact scan of the whole window).
#include "hts_device.h"

namespace hts {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;
typedef __attribute__((ext_vector_type(4))) unsigned uintx4;

// Error-bound coefficients: E = C1 sqrt(|a|^2 |b|^2) + C2 (|a|^2 + |b|^2) + 2
// for the norm+dot form.  With u = 2^-8 (bf16, round to nearest) the split
// a = hi + lo + r has |r| <= 1.01 u^2 |a|; dropping lo*lo and the residuals
// costs <= 3.1 u^2 sum|a_i b_i|; plain bf16 costs <= (2u + u^2) sum|a_i b_i|.
// FP32 accumulation of <= 192 exact products (any order, rounding to
// nearest or toward zero) adds <= 200 * 2^-23 sum|products|.  Cauchy-Schwarz
// bounds sum|a_i b_i| by |a| |b|.  The factor 2 of 2 a.b and a 1.25 margin
// give C1; C2 covers rounding the exact int64 norms to float and the final
// additions.  For the FP32 SSD form, |d~ - d| <= 64 * 2^-24 d~ / (1 - 2^-18),
// bounded by 2^-17 d~ + 2.
template <int TERMS> struct DotBound;
template <> struct DotBound<3> { static constexpr float C1 = 1.8e-4f; };
template <> struct DotBound<1> { static constexpr float C1 = 1.97e-2f; };
constexpr float BOUND_C2 = 9.5367431640625e-07f;  // 2^-20
constexpr float SSD_REL = 7.62939453125e-06f;     // 2^-17
constexpr float BOUND_ABS = 2.0f;

__device__ inline unsigned bf16_bits(__bf16 h) { return __builtin_bit_cast(unsigned short, h); }

// (hi | lo << 16) with hi = bf16(v), lo = bf16(v - hi); v is an integer
// below 2^23 in magnitude, so v - hi is exact in FP32.
__device__ inline unsigned split_pack(float v) {
  __bf16 h = (__bf16)v;
  __bf16 l = (__bf16)(v - (float)h);
  return bf16_bits(h) | (bf16_bits(l) << 16);
}

// The value of lane l ^ 32 (v_permlane32_swap exchanges the upper half of
// its first operand with the lower half of its second); hi: lane >= 32.
__device__ inline unsigned xor32_u32(unsigned v, bool hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return hi ? r[0] : r[1];
}
// Orders one wavefront's LDS writes before its later reads of other lanes'
// slots (the hardware keeps a wavefront's LDS accesses in order; this keeps
// the compiler from moving them).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline unsigned long long xor32_u64(unsigned long long v, bool hi) {
  const unsigned lo = xor32_u32((unsigned)v, hi), up = xor32_u32((unsigned)(v >> 32), hi);
  return ((unsigned long long)up << 32) | lo;
}

// Blocks per wavefront whose lower bounds stay in registers between the
// two passes (CACHE = 1): 36 covers windows up to 39 at stride 2 or 3.
constexpr int MAXBW = 36;

// NPL = 2 stages both guide planes of an RGB tile at once, so a tile whose
// references use both planes runs the distance passes once (every reference
// against its own plane: the A operand of a reference is zero in the
// products of the other plane); NPL = 1 runs the planes one after the other
// (windows too large for two plane slots in LDS).  SBS = 0 keeps no |b|
// array and takes the square root of |b|^2 where the bound needs it: the
// smaller footprint that lets two plane slots fit for larger windows.
template <int MODE, int TERMS, int CACHE, int NPL, int SBS>
__global__ __launch_bounds__(256, 2) void k_match(Launch L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const MatchGeom G = match_geom(L.stride, L.window, NPL, SBS);
  // plane slot q: staged guide (int), its bf16 split or float form, |b|^2, |b|
  auto GI = [&](int q) __attribute__((always_inline)) { return (int*)(smem + q * G.plane_bytes); };
  auto GB = [&](int q) __attribute__((always_inline)) {
    return (unsigned*)(smem + q * G.plane_bytes + G.rgn);
  };
  auto NB = [&](int q) __attribute__((always_inline)) {
    return (float*)(smem + q * G.plane_bytes + 2 * G.rgn);
  };
  auto SB = [&](int q) __attribute__((always_inline)) {
    return (float*)(smem + q * G.plane_bytes + 2 * G.rgn + G.nbsz);
  };
  float* tl = (float*)(smem + G.off_tl);
  unsigned* sl = (unsigned*)(smem + G.off_tl);     // reuses tl once T is known
  int* rinfo = (int*)(smem + G.off_misc);          // [16][8]
  float* rnorm = (float*)(rinfo + 128);            // [16][2] |a|^2, |a|
  float* Tp = rnorm + 32;                          // [16]
  int* scount = (int*)(Tp + 16);                   // [16]
  unsigned long long* keyb = (unsigned long long*)(smem + G.off_misc + 768);   // [4][64]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, n = lane & 15;
  const int r = (L.window - 1) / 2;
  const int s = L.stride;
  const int K = L.K;
  // diagnostics: shortlist sizes, counted per work group past the regular
  // LDS (allocated only when asked for), added to L.sl_hist at the end
  int* shist = (int*)(smem + G.bytes);
  if (L.sl_hist)
    for (int i = tid; i < SL_BINS; i += 256) shist[i] = 0;

  for_each_item_cd<W_MATCH>(L, [&](const auto& d, int item) __attribute__((always_inline)) {
    const int ntx = (d.nrx + MATCH_TX - 1) / MATCH_TX;
    const int iy0 = (item / ntx) * MATCH_TY, ix0 = (item % ntx) * MATCH_TX;
    const int iy1 = min(d.nry, iy0 + MATCH_TY) - 1, ix1 = min(d.nrx, ix0 + MATCH_TX) - 1;
    const int Y0 = max(0, ref_coord(iy0, s, d.Hp) - r);
    const int Y1 = min(d.Hp - 1, ref_coord(iy1, s, d.Hp) + r);
    const int X0 = max(0, ref_coord(ix0, s, d.Wp) - r);
    const int X1 = min(d.Wp - 1, ref_coord(ix1, s, d.Wp) + r);
    const int RYc = Y1 - Y0 + 1, RXc = X1 - X0 + 1;
    // candidate blocks of 2 rows x 8 columns (one MFMA column each)
    const int NYB = (RYc + 1) >> 1, NXB = (RXc + 7) >> 3, RXP = NXB * 8;
    const int rows = RYc + PS - 1, cols = RXP + PS - 1;
    const int pitch = G.pitch;

    __syncthreads();
    if (tid < 16) {
      const int iy = iy0 + (tid >> 2), ix = ix0 + (tid & 3);
      const bool valid = iy < d.nry && ix < d.nrx;
      const int ref = iy * d.nrx + ix;
      const int ry = valid ? ref_coord(iy, s, d.Hp) : Y0;
      const int rx = valid ? ref_coord(ix, s, d.Wp) : X0;
      const int plane = (L.C == 1 || !valid) ? 0 : (d.green[ref] ? 0 : 1);
      int* ri = rinfo + tid * 8;
      ri[0] = valid ? (1 << plane) : 0;
      ri[1] = ry - Y0;
      ri[2] = rx - X0;
      ri[3] = max(0, ry - r) - Y0;
      ri[4] = min(d.Hp - 1, ry + r) - Y0;
      ri[5] = max(0, rx - r) - X0;
      ri[6] = min(d.Wp - 1, rx + r) - X0;
      ri[7] = ref;
    }
    __syncthreads();
    int pmask = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) pmask |= rinfo[t * 8];

    for (int p = 0; p < 2; p += NPL) {
      // planes of this pass (bit q: guide plane q) and the slot of plane q
      const int pm = __builtin_amdgcn_readfirstlane(pmask & (NPL == 2 ? 3 : 1 << p));
      if (!pm) continue;
      auto slot = [&](int q) __attribute__((always_inline)) { return NPL == 2 ? q : 0; };
      __syncthreads();  // the previous plane's re-rank still reads the LDS region

      // ---- stage the region, centred by an integer offset per plane ----
      // Any integer offset leaves every distance unchanged; the floor of the
      // mean of a 16 x 16 sample of the region keeps the centred values (and
      // with them the error bounds) small.  Columns past the image read as 0.
      int moff[2] = {0, 0};
      {
        const int sy = (tid >> 4) * rows / 16;
        const int sx = min((tid & 15) * cols / 16, d.W - 1 - X0);
        int* part = (int*)Tp;   // free until the threshold step
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (!((pm >> q) & 1)) continue;
          // |v| < 3 * 2^20: the sum fits int32
          int v = d.gplanes[(size_t)q * d.H * d.W + (Y0 + sy) * d.W + X0 + sx];
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
          if (lane == 0) part[4 * q + wave] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q)
          moff[q] = (part[4 * q] + part[4 * q + 1] + part[4 * q + 2] + part[4 * q + 3]) >> 8;
      }
      // Each wavefront loads SROWS rows of both planes before it waits for
      // any of them (addresses clamped into the image, values masked after).
      constexpr int SROWS = 4;
      for (int x0 = 0; x0 < cols; x0 += 64) {
        const int x = x0 + lane;
        const int xc = min(X0 + x, d.W - 1);
        const bool in_img = X0 + x < d.W;
        for (int y0 = wave; y0 < rows; y0 += 4 * SROWS) {
          // (a plane this pass does not use reads plane 0 in its place: no
          // branch between the loads)
          int v[2][SROWS];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int* src = d.gplanes + (size_t)((pm >> q) & 1 ? q : 0) * d.H * d.W + xc;
#pragma unroll
            for (int u = 0; u < SROWS; ++u)
              v[q][u] = src[(size_t)(Y0 + min(y0 + 4 * u, rows - 1)) * d.W];
          }
          if (x >= cols) continue;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            if (!((pm >> q) & 1)) continue;
            int* gi = GI(slot(q));
            unsigned* gb = GB(slot(q));
#pragma unroll
            for (int u = 0; u < SROWS; ++u) {
              const int y = y0 + 4 * u;
              if (y < rows) {
                const int c = in_img ? v[q][u] - moff[q] : 0;
                gi[y * pitch + x] = c;
                gb[y * pitch + x] = MODE == 0 ? split_pack((float)c) : __float_as_uint((float)c);
              }
            }
          }
        }
      }
      // the row below the region, read by the last block row when RYc is
      // odd (then it lies inside the allocation, which has rows for an even
      // number of candidate rows)
      if (RYc & 1) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (!((pm >> q) & 1)) continue;
          for (int x = tid; x < cols; x += 256) {
            GI(slot(q))[rows * pitch + x] = 0;
            GB(slot(q))[rows * pitch + x] = 0u;
          }
        }
      }
      __syncthreads();

      // ---- exact candidate norms |b|^2 (norm+dot form only) ----
      // One task per (plane, column pair, 8 rows): per row the squares of
      // the 9 values under the pair's two windows, their two sums of 8 (the
      // second by sliding the first), then sliding sums down the rows; all
      // in FP64 (exact: |v| < 2^22, sums < 2^50, so the order of additions
      // does not matter).  Rows past the region repeat its last row: their
      // sums only reach the norms of candidate rows >= RYc, which are not
      // stored.
      if (MODE == 0) {
        const int nseg = (RYc + 7) >> 3;
        const int ncp = RXP >> 1;
        const int per_plane = ncp * nseg;
        const int q0 = (pm & 1) ? 0 : 1;
        const int ntask = per_plane * __builtin_popcount(pm);
        for (int task = tid; task < ntask; task += 256) {
          const int second = task >= per_plane;
          const int q = second ? 1 : q0;
          const int rem = task - (second ? per_plane : 0);
          const int cx = 2 * (rem % ncp), c0 = (rem / ncp) * 8;
          const int* gi = GI(slot(q));
          float* nbf = NB(slot(q));
          float* sbf = SB(slot(q));
          double ra[15], rb[15];
#pragma unroll
          for (int jj = 0; jj < 15; ++jj) {
            const int* row = gi + min(c0 + jj, rows - 1) * pitch + cx;
            double sq[PS + 1];
#pragma unroll
            for (int b = 0; b <= PS; ++b) {
              const double v = (double)row[b];
              sq[b] = v * v;
            }
            double a = 0.0;
#pragma unroll
            for (int b = 0; b < PS; ++b) a += sq[b];
            ra[jj] = a;
            rb[jj] = a + (sq[PS] - sq[0]);
          }
          double na = 0.0, nb = 0.0;
#pragma unroll
          for (int jj = 0; jj < 8; ++jj) {
            na += ra[jj];
            nb += rb[jj];
          }
#pragma unroll
          for (int jj = 0; jj < 8; ++jj) {
            const int cy = c0 + jj;
            if (cy < RYc) {
              const float fa = (float)na, fb = (float)nb;
              nbf[cy * RXP + cx] = fa;
              nbf[cy * RXP + cx + 1] = fb;
              if (SBS) {
                sbf[cy * RXP + cx] = sqrtf(fa);
                sbf[cy * RXP + cx + 1] = sqrtf(fb);
              }
            }
            if (jj < 7) {
              na += ra[jj + 8] - ra[jj];
              nb += rb[jj + 8] - rb[jj];
            }
          }
        }
        __syncthreads();
      }
      // reference norms: the reference is the candidate at its own position
      if (tid < 16) {
        const int* ri = rinfo + tid * 8;
        float na = 0.f;
        if (MODE == 0 && (ri[0] & pm)) na = NB(slot((ri[0] >> 1) & 1))[ri[1] * RXP + ri[2]];
        rnorm[2 * tid] = na;
        rnorm[2 * tid + 1] = sqrtf(na);
      }
      __syncthreads();

      // ---- per-lane reference state: references 4*kq + i, candidate column n ----
      // Reference 4*kq + i sits in tile row kq, so its window rows depend on
      // kq only; its window columns, as [wx0, wx0 + wxl) (wxl = 0 when the
      // reference uses neither plane of this pass); rq = the slot of its plane.
      int rpx[4], wx0[4], rq[4];
      unsigned wxl[4];
      float na[4], sa[4];
      const int rpy = rinfo[(4 * kq) * 8 + 1];
      const int wy0 = rinfo[(4 * kq) * 8 + 3];
      const unsigned wyl = (unsigned)(rinfo[(4 * kq) * 8 + 4] - wy0 + 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int* ri = rinfo + (4 * kq + i) * 8;
        rpx[i] = ri[2];
        wx0[i] = ri[5];
        wxl[i] = (ri[0] & pm) ? (unsigned)(ri[6] - ri[5] + 1) : 0u;
        rq[i] = slot((ri[0] >> 1) & 1);
        na[i] = rnorm[2 * (4 * kq + i)];
        sa[i] = rnorm[2 * (4 * kq + i) + 1];
      }
      // A operand per plane slot: reference n, patch rows 2kq + h (MFMA
      // 16x16x32 layout: k = 8 kq + column); zero in the slot of the plane it
      // does not use.  Rows 2kq + h put the four kq lane groups 2 * pitch
      // apart, which with pitch = 8 (mod 16) spreads their 16-word reads over
      // disjoint LDS banks.
      bf16x8 Ahi[NPL][2], Alo[NPL][2];
      if (MODE == 0) {
        const int* ri = rinfo + n * 8;
#pragma unroll
        for (int sq = 0; sq < NPL; ++sq) {
          const bool ok = (ri[0] & pm) && slot((ri[0] >> 1) & 1) == sq;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const unsigned* src = GB(sq) + (ri[1] + 2 * kq + h) * pitch + ri[2];
            unsigned w[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) w[b] = ok ? src[b] : 0u;
            uintx4 hi, lo;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              hi[b] = __builtin_amdgcn_perm(w[2 * b + 1], w[2 * b], 0x05040100u);
              lo[b] = __builtin_amdgcn_perm(w[2 * b + 1], w[2 * b], 0x07060302u);
            }
            Ahi[sq][h] = __builtin_bit_cast(bf16x8, hi);
            Alo[sq][h] = __builtin_bit_cast(bf16x8, lo);
          }
        }
      }

      // Distances of references 4*kq + i to candidate (cy, cx), their error
      // bounds, and whether the candidate is in the reference's window (and
      // is not the reference itself).  cy is the same on every lane.
      auto tile_dist = [&](int cy, int cx, float (&dt)[4], float (&E)[4], bool (&ok)[4])
          __attribute__((always_inline)) {
        if (MODE == 0) {
          // every reference against its own plane: the slots' products add
          floatx4 acc = {0.f, 0.f, 0.f, 0.f};
          float nbq[NPL], sbq[NPL];
#pragma unroll
          for (int sq = 0; sq < NPL; ++sq) {
            nbq[sq] = sbq[sq] = 0.f;
            if (NPL == 2 && !((pm >> sq) & 1)) continue;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const unsigned* src = GB(sq) + (cy + 2 * kq + h) * pitch + cx;
              unsigned w[8];
#pragma unroll
              for (int b = 0; b < 8; ++b) w[b] = src[b];
              uintx4 hi, lo;
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                hi[b] = __builtin_amdgcn_perm(w[2 * b + 1], w[2 * b], 0x05040100u);
                lo[b] = __builtin_amdgcn_perm(w[2 * b + 1], w[2 * b], 0x07060302u);
              }
              const bf16x8 Bhi = __builtin_bit_cast(bf16x8, hi);
              acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi[sq][h], Bhi, acc, 0, 0, 0);
              if (TERMS == 3) {
                const bf16x8 Blo = __builtin_bit_cast(bf16x8, lo);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi[sq][h], Blo, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Alo[sq][h], Bhi, acc, 0, 0, 0);
              }
            }
            nbq[sq] = NB(sq)[cy * RXP + cx];
            sbq[sq] = SBS ? SB(sq)[cy * RXP + cx] : sqrtf(nbq[sq]);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float nb = NPL == 2 && rq[i] ? nbq[NPL - 1] : nbq[0];
            const float sb = NPL == 2 && rq[i] ? sbq[NPL - 1] : sbq[0];
            dt[i] = (na[i] + nb) - 2.0f * acc[i];
            E[i] = DotBound<TERMS>::C1 * sa[i] * sb + BOUND_C2 * (na[i] + nb) + BOUND_ABS;
          }
        } else {
          float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
          for (int py = 0; py < PS; ++py) {
#pragma unroll
            for (int px = 0; px < PS; ++px) {
              float bq[NPL];
#pragma unroll
              for (int sq = 0; sq < NPL; ++sq)
                bq[sq] = __uint_as_float(GB(sq)[(cy + py) * pitch + cx + px]);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const float bv = NPL == 2 && rq[i] ? bq[NPL - 1] : bq[0];
                const float av = __uint_as_float(GB(rq[i])[(rpy + py) * pitch + rpx[i] + px]);
                const float df = av - bv;
                acc[i] = fmaf(df, df, acc[i]);
              }
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            dt[i] = acc[i];
            E[i] = SSD_REL * acc[i] + BOUND_ABS;
          }
        }
        const bool cy_ok = (unsigned)(cy - wy0) < wyl;
        const bool cy_self = cy == rpy;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          ok[i] = cy_ok & ((unsigned)(cx - wx0[i]) < wxl[i]) & !(cy_self & (cx == rpx[i]));
      };

      // Blocks (candidate rows 2yb, 2yb + 1 x columns 8xb .. 8xb + 7; lane n
      // takes row 2yb + n / 8, column 8xb + n % 8) are dealt round-robin to
      // the wavefronts; (yb, xb) advance by 4 blocks without a division.
      // Blocks of 8 columns pad the candidate columns to a multiple of 8
      // (40 at w = 31, s = 3) instead of 16.
      const int wv = __builtin_amdgcn_readfirstlane(wave);
      const int nblocks = NYB * NXB;
      const int nbw = nblocks > wv ? (nblocks - wv + 3) >> 2 : 0;
      const int yb0 = wv / NXB, xb0 = wv - yb0 * NXB;
      auto step = [&](int& yb, int& xb) __attribute__((always_inline)) {
        xb += 4;
        while (xb >= NXB) { xb -= NXB; ++yb; }
      };
      const int cyn = n >> 3, cxn = n & 7;   // this lane's candidate within a block
      constexpr unsigned INFB = 0x7f800000u;   // +inf

      // ---- pass 1: two smallest upper bounds per (lane, reference) ----
      // Upper bounds d~ + E are at least the exact distance, so never
      // negative (rounding is monotone).  With CACHE the lower bounds d~ - E
      // stay in registers for pass 2 as the upper 16 bits of their float
      // patterns, shifted arithmetically: a negative bound stays negative,
      // and truncation only lowers a non-negative one, so pass 2 still
      // shortlists a superset; two per register; 0x7FFF (above every
      // threshold's 16 bits, at most 0x7F80) marks a non-candidate.
      float m0[4], m1[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) m0[i] = m1[i] = __uint_as_float(INFB);
      unsigned lbc[CACHE ? MAXBW : 1][2];
      auto pass1 = [&](int yb, int xb, unsigned (&lbw)[2]) __attribute__((always_inline)) {
        float dt[4], E[4];
        bool ok[4];
        tile_dist(2 * yb + cyn, 8 * xb + cxn, dt, E, ok);
        unsigned lh[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float hv = ok[i] ? dt[i] + E[i] : __uint_as_float(INFB);
          m1[i] = __builtin_amdgcn_fmed3f(m0[i], m1[i], hv);   // m0 <= m1: min(m1, max(m0, hv))
          m0[i] = fminf(m0[i], hv);
          lh[i] = ok[i] ? (unsigned)(__float_as_int(dt[i] - E[i]) >> 16) & 0xFFFFu : 0x7FFFu;
        }
        lbw[0] = lh[0] | (lh[1] << 16);
        lbw[1] = lh[2] | (lh[3] << 16);
      };
      {
        int yb = yb0, xb = xb0;
        if constexpr (CACHE) {
#pragma unroll
          for (int j = 0; j < MAXBW; ++j) {
            if (j < nbw) pass1(yb, xb, lbc[j]);
            step(yb, xb);
          }
        } else {
          for (int j = 0; j < nbw; ++j) {
            unsigned lbw[2];
            pass1(yb, xb, lbw);
            step(yb, xb);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float* dst = tl + ((4 * kq + i) * 64 + wave * 16 + n) * 2;
        dst[0] = m0[i];
        dst[1] = m1[i];
      }
      __syncthreads();

      // ---- threshold T per reference: (K-1)-th smallest of its 128 list values ----
      // The values are non-negative floats (or +inf), ordered as their bit
      // patterns, which lie below 2^31.  T is the largest pattern t with
      // #{values < t} <= K-2, i.e. the (K-1)-th smallest value; it is built
      // bit by bit from the top, counting with ballots.  Each step only sets
      // lower bits, so the first 15 steps fix bits 30..16 of T for good; with
      // the cached bounds pass 2 compares those 16 bits alone, and the
      // search stops there.
      constexpr int T_LOW_BIT = CACHE ? 16 : 0;
      for (int t = wv; t < 16; t += 4) {
        if (!(rinfo[t * 8] & pm)) continue;
        const unsigned v0 = __float_as_uint(tl[t * 128 + lane]);
        const unsigned v1 = __float_as_uint(tl[t * 128 + 64 + lane]);
        const int g = K - 2;
        unsigned pre = 0;
        for (int bit = 30; bit >= T_LOW_BIT; --bit) {
          const unsigned cand = pre | (1u << bit);
          const int c = __popcll(__ballot(v0 < cand)) + __popcll(__ballot(v1 < cand));
          pre = c <= g ? cand : pre;
        }
        if (lane == 0) {
          Tp[t] = __uint_as_float(pre);
          scount[t] = 0;
        }
      }
      __syncthreads();

      // ---- pass 2: shortlist every candidate with d~ - E <= T ----
      // Shortlist entries are packed (cy << 8) | cx.
      // Tp is only set for references on this plane: the others get Th = 0,
      // which no non-candidate marker (0x7FFF) passes.
      float Ti[4];
      int Th[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        Ti[i] = Tp[4 * kq + i];
        Th[i] = wxl[i] ? (int)(__float_as_uint(Ti[i]) >> 16) : 0;
      }
      auto pass2 = [&](int yb, int xb, const bool (&h)[4]) __attribute__((always_inline)) {
        const int cy = 2 * yb + cyn, cx = 8 * xb + cxn;
        if (h[0] | h[1] | h[2] | h[3]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (h[i]) {
              const int t = 4 * kq + i;
              const int pos = atomicAdd(&scount[t], 1);
              if (pos < SHORT_CAP) sl[t * SHORT_CAP + pos] = ((unsigned)cy << 8) | (unsigned)cx;
            }
          }
        }
      };
      {
        int yb = yb0, xb = xb0;
        if constexpr (CACHE) {
#pragma unroll
          for (int j = 0; j < MAXBW; ++j) {
            if (j < nbw) {
              bool h[4];
#pragma unroll
              for (int i = 0; i < 4; ++i)   // the 16-bit bound, sign-extended
                h[i] = ((int)(lbc[j][i >> 1] << (16 - 16 * (i & 1))) >> 16) <= Th[i];
              pass2(yb, xb, h);
            }
            step(yb, xb);
          }
        } else {
          for (int j = 0; j < nbw; ++j) {
            float dt[4], E[4];
            bool ok[4], h[4];
            tile_dist(2 * yb + cyn, 8 * xb + cxn, dt, E, ok);
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = ok[i] && dt[i] - E[i] <= Ti[i];
            pass2(yb, xb, h);
            step(yb, xb);
          }
        }
      }
      __syncthreads();

      // ---- exact re-rank on one wavefront per reference ----
      // Exact squared distances in FP64: |differences| < 2^22, so every
      // product and partial sum (< 2^50) is an exact integer.
      for (int t = wv; t < 16; t += 4) {
        const int* ri = rinfo + t * 8;
        if (!(ri[0] & pm)) continue;
        const int ref = ri[7];
        const int* gi = GI(slot((ri[0] >> 1) & 1));   // the reference's guide plane
        const int nsl = __builtin_amdgcn_readfirstlane(scount[t]);
        if (L.sl_hist && lane == 0) atomicAdd(&shist[min(nsl, SHORT_CAP + 1)], 1);
        if (nsl > SHORT_CAP || nsl < K - 1) {
          if (lane == 0) d.fb_list[atomicAdd(d.fb_count, 1)] = ref;
          continue;
        }
        const int py0 = ri[1], px0 = ri[2], ty0 = ri[3], tx0 = ri[5];
        // exact squared distance of shortlist entry pk over the patch rows
        // [pb, pb + nr), in two FP64 accumulators (every partial sum is an
        // exact integer, so the grouping leaves the result unchanged)
        auto dist_rows = [&](unsigned pk, int pb, int nr) __attribute__((always_inline)) {
          const int cy = (int)(pk >> 8), cx = (int)(pk & 255u);
          double a0 = 0.0, a1 = 0.0;
#pragma unroll 2
          for (int r = 0; r < nr; ++r) {
            const int* rr = gi + (py0 + pb + r) * pitch + px0;   // the reference's row
            const int* cr = gi + (cy + pb + r) * pitch + cx;
#pragma unroll
            for (int px = 0; px < PS; px += 2) {
              const double u = (double)(rr[px] - cr[px]);
              const double v = (double)(rr[px + 1] - cr[px + 1]);
              a0 = fma(u, u, a0);
              a1 = fma(v, v, a1);
            }
          }
          return a0 + a1;
        };
        // key = distance << 12 | window index: distinct keys, so the rank of
        // a key among the nsl keys is its slot (minus one)
        auto make_key = [&](unsigned pk, double dd) __attribute__((always_inline)) {
          const int cy = (int)(pk >> 8), cx = (int)(pk & 255u);
          return ((unsigned long long)dd << 12) | (unsigned)((cy - ty0) * 64 + (cx - tx0));
        };
        auto emit = [&](int g, unsigned long long key) __attribute__((always_inline)) {
          const unsigned loc = (unsigned)(key & 0xFFFu);
          const int cy = Y0 + ty0 + (int)(loc >> 6), cx = X0 + tx0 + (int)(loc & 63u);
          d.idx[(size_t)ref * K + 1 + g] = cy * d.W + cx;
          if (L.count_hist) atomicAdd(d.hist + cy * d.W + cx, 1);
          if (d.dist) d.dist[(size_t)ref * K + 1 + g] = (long long)(key >> 12);
        };
        // ranks are counted against every key: read back from this
        // wavefront's LDS slots (one wavefront's LDS accesses complete in
        // order), or broadcast lane by lane past 64 entries
        unsigned long long* kb = keyb + wave * 64;
        if (nsl <= 32) {
          // lanes l and l + 32 share entry l % 32, each summing four patch
          // rows and counting against half of the keys
          const int e = lane & 31;
          const bool hi = lane >= 32;
          const unsigned pk = sl[t * SHORT_CAP + (e < nsl ? e : 0)];
          double dd = dist_rows(pk, hi ? 4 : 0, 4);
          dd += __longlong_as_double((long long)xor32_u64(
              (unsigned long long)__double_as_longlong(dd), hi));
          const unsigned long long key = e < nsl ? make_key(pk, dd) : ~0ull;
          if (!hi) kb[e] = key;
          wave_lds_sync();
          int rank = 0;
#pragma unroll
          for (int o = 0; o < 16; ++o) rank += kb[(hi ? 16 : 0) + o] < key ? 1 : 0;
          rank += (int)xor32_u32((unsigned)rank, hi);
          if (!hi && e < nsl && rank < K - 1) emit(rank, key);
        } else if (nsl <= 64) {
          const unsigned pk = sl[t * SHORT_CAP + (lane < nsl ? lane : 0)];
          const unsigned long long key = lane < nsl ? make_key(pk, dist_rows(pk, 0, PS)) : ~0ull;
          kb[lane] = key;
          wave_lds_sync();
          int rank = 0;
          for (int o0 = 0; o0 < nsl; o0 += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) rank += kb[o0 + u] < key ? 1 : 0;
          }
          if (lane < nsl && rank < K - 1) emit(rank, key);
        } else {
          unsigned long long key[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int j = 64 * h + lane;
            const unsigned pk = sl[t * SHORT_CAP + (j < nsl ? j : 0)];
            key[h] = j < nsl ? make_key(pk, dist_rows(pk, 0, PS)) : ~0ull;
          }
          auto bcast = [&](unsigned long long v, int src) __attribute__((always_inline)) {
            const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, src);
            const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), src);
            return ((unsigned long long)hi << 32) | lo;
          };
          int rank0 = 0, rank1 = 0;
          for (int o = 0; o < nsl; ++o) {
            const unsigned long long ko = bcast(o < 64 ? key[0] : key[1], o & 63);
            rank0 += ko < key[0] ? 1 : 0;
            rank1 += ko < key[1] ? 1 : 0;
          }
          if (rank0 < K - 1) emit(rank0, key[0]);
          if (64 + lane < nsl && rank1 < K - 1) emit(rank1, key[1]);
        }
        if (lane == 0) {
          d.idx[(size_t)ref * K] = (Y0 + py0) * d.W + X0 + px0;
          if (L.count_hist) atomicAdd(d.hist + (Y0 + py0) * d.W + X0 + px0, 1);
          if (d.dist) d.dist[(size_t)ref * K] = 0;
        }
      }
    }
  });
  if (L.sl_hist) {
    __syncthreads();
    for (int i = tid; i < SL_BINS; i += 256)
      if (shist[i]) atomicAdd(L.sl_hist + i, shist[i]);
  }
}

// Exact scan of the whole window for references whose certified shortlist
// overflowed: the window's guide pixels are staged in LDS, integer distances
// are computed for every candidate, and (distance, window index) keys are
// sorted bitonically in LDS (padded to the next power of two of the window's
// candidates); the first K-1 after the reference are kept.
// The (image, entry) pairs of all images are dealt round-robin to the work
// groups.
__global__ __launch_bounds__(256) void k_match_fallback(Launch L) {
  constexpr int WMAX = MAX_WINDOW + PS - 1;
  __shared__ unsigned long long keys[4096];
  __shared__ int win[WMAX * WMAX];
  const int tid = threadIdx.x;
  const int r = (L.window - 1) / 2;
  const int K = L.K;
  const int G = gridDim.x;
  const int nimg = L.table ? L.n_img : 1;
  __shared__ int counts[256];
  long long base = 0;   // global number of the image's first entry
  for (int i0 = 0; i0 < nimg; i0 += 256) {
    // the images' list lengths, 256 at a time (most are 0: no descriptor read)
    __syncthreads();
    if (i0 + tid < nimg) counts[tid] = *(L.table ? L.table[i0 + tid] : L.one).fb_count;
    __syncthreads();
    for (int im = i0; im < min(nimg, i0 + 256); ++im) {
      const int count = counts[im - i0];
      if (count == 0) continue;
      const ImgDesc d = L.table ? L.table[im] : L.one;
      const int j0 = (int)(((long long)blockIdx.x - base % G + G) % G);
      base += count;
      for (int j = j0; j < count; j += G) {
        const int ref = d.fb_list[j];
        const int ry = ref_coord(ref / d.nrx, L.stride, d.Hp);
        const int rx = ref_coord(ref % d.nrx, L.stride, d.Wp);
        const int y0 = max(0, ry - r), y1 = min(d.Hp - 1, ry + r);
        const int x0 = max(0, rx - r), x1 = min(d.Wp - 1, rx + r);
        const int wx = x1 - x0 + 1, nc = (y1 - y0 + 1) * wx;
        const int pw = wx + PS - 1, ph = y1 - y0 + PS;   // staged pixel region
        const int plane = (L.C == 1 || d.green[ref]) ? 0 : 1;
        const int* g = d.gplanes + (size_t)plane * d.H * d.W;
        __syncthreads();
        for (int e = tid; e < ph * pw; e += 256) {
          const int yy = e / pw, xx = e - yy * pw;
          win[yy * WMAX + xx] = g[(y0 + yy) * d.W + x0 + xx];
        }
        __syncthreads();
        const int* rp = win + (ry - y0) * WMAX + (rx - x0);
        int n2 = 256;   // keys sorted: the window's candidates, padded to a power of two
        while (n2 < nc) n2 <<= 1;
        for (int c = tid; c < n2; c += 256) {
          unsigned long long key = ~0ull;
          if (c < nc) {
            const int cy = c / wx, cx = c - cy * wx;
            if (cy + y0 != ry || cx + x0 != rx) {
              const int* cp = win + cy * WMAX + cx;
              long long dd = 0;
              for (int a = 0; a < PS; ++a)
#pragma unroll
                for (int b = 0; b < PS; ++b) {
                  const int df = rp[a * WMAX + b] - cp[a * WMAX + b];
                  dd += (long long)df * df;
                }
              key = ((unsigned long long)dd << 12) | (unsigned)(cy * 64 + cx);
            }
          }
          keys[c] = key;
        }
        __syncthreads();
        for (int k = 2; k <= n2; k <<= 1)
          for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = tid; i < n2; i += 256) {
              const int q = i ^ jj;
              if (q > i) {
                const unsigned long long a = keys[i], b = keys[q];
                const bool asc = (i & k) == 0;
                if (asc ? (a > b) : (a < b)) { keys[i] = b; keys[q] = a; }
              }
            }
            __syncthreads();
          }
        for (int i = tid; i < K - 1; i += 256) {
          const unsigned loc = (unsigned)(keys[i] & 0xFFFu);
          const int pos = (y0 + (int)(loc >> 6)) * d.W + x0 + (int)(loc & 63u);
          d.idx[(size_t)ref * K + 1 + i] = pos;
          if (L.count_hist) atomicAdd(d.hist + pos, 1);
          if (d.dist) d.dist[(size_t)ref * K + 1 + i] = (long long)(keys[i] >> 12);
        }
        if (tid == 0) {
          d.idx[(size_t)ref * K] = ry * d.W + rx;
          if (L.count_hist) atomicAdd(d.hist + ry * d.W + rx, 1);
          if (d.dist) d.dist[(size_t)ref * K] = 0;
        }
      }
    }
  }
}

size_t match_lds_bytes(int stride, int window) { return (size_t)match_geom(stride, window, 1).bytes; }

// Two plane slots when the image has two guide planes and they fit beside
// a second work group on the CU (160 KB of LDS), with the |b| arrays when
// those fit too; else one plane slot.  *sbs: keep the |b| arrays.
static int match_planes(int C, int stride, int window, int* sbs) {
  *sbs = 1;
  if (C != 3) return 1;
  if (match_geom(stride, window, 2, 1).bytes <= 80 * 1024) return 2;
  if (match_geom(stride, window, 2, 0).bytes <= 80 * 1024) {
    *sbs = 0;
    return 2;
  }
  return 1;
}

hipError_t launch_match(const Launch& L, int mode, int terms, int grid, hipStream_t s) {
  if (L.total <= 0) return hipSuccess;
  const int g = xcd_grid(grid > 0 && grid < L.total ? grid : L.total);
  int sbs = 1;
  const int npl = match_planes(L.C, L.stride, L.window, &sbs);
  const MatchGeom G = match_geom(L.stride, L.window, npl, sbs);
  const size_t lds = (size_t)G.bytes + (L.sl_hist ? SL_BINS * sizeof(int) : 0);
  const bool cache = ((G.ryc + 1) / 2 * (G.rxp / 8) + 3) / 4 <= MAXBW;
#define HTS_KM(M, T)                                                                          \
  if (npl == 2 && !sbs) {                                                                     \
    if (cache) hipLaunchKernelGGL((k_match<M, T, 1, 2, 0>), dim3(g), dim3(256), lds, s, L);   \
    else hipLaunchKernelGGL((k_match<M, T, 0, 2, 0>), dim3(g), dim3(256), lds, s, L);         \
  } else if (npl == 2) {                                                                      \
    if (cache) hipLaunchKernelGGL((k_match<M, T, 1, 2, 1>), dim3(g), dim3(256), lds, s, L);   \
    else hipLaunchKernelGGL((k_match<M, T, 0, 2, 1>), dim3(g), dim3(256), lds, s, L);         \
  } else {                                                                                    \
    if (cache) hipLaunchKernelGGL((k_match<M, T, 1, 1, 1>), dim3(g), dim3(256), lds, s, L);   \
    else hipLaunchKernelGGL((k_match<M, T, 0, 1, 1>), dim3(g), dim3(256), lds, s, L);         \
  }
  if (mode == HTS_MATCH_FP32) {
    HTS_KM(1, 1)
  } else if (terms == 1) {
    HTS_KM(0, 1)
  } else {
    HTS_KM(0, 3)
  }
#undef HTS_KM
  return hipGetLastError();
}

hipError_t launch_match_fallback(const Launch& L, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_match_fallback, dim3(grid > 0 ? grid : 256), dim3(256), 0, s, L);
  return hipGetLastError();
}

}  // namespace hts
