// Internal declarations shared by the host ABI (hts_api.cpp) and the HIP
// kernels.  Not part of the public interface (include/hts.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hts.h"

namespace hts {

constexpr int PS = 8;                  // patch size (only 8 is built)
constexpr int PS2 = PS * PS;
constexpr int QMAX = (1 << 20) - 1;    // clamp of the quantised guide
constexpr int MAX_WINDOW = 63;         // window-relative candidate index fits 12 bits
constexpr int MATCH_TY = 4;            // match tile: 4 x 4 references
constexpr int MATCH_TX = 4;
constexpr int SHORT_CAP = 128;         // certified shortlist capacity per reference
constexpr int SL_BINS = SHORT_CAP + 2;  // shortlist sizes 0..SHORT_CAP, then overflows
constexpr int PIX_CHUNK = 2048;        // pixels per work item of the element-wise stages
// General band counts (c other than 1 and 3: the spectral tubes of HSI)
constexpr int GEN_CMAX = 256;          // bands
constexpr int GEN_KMAX = 32;           // group size
constexpr int GEN_FC = 8;              // frequencies per covariance work item
constexpr int GEN_EIG_M = 16;          // eigenproblems per work group
constexpr int GEN_GRID = 32768;        // filter work groups (each with its own scratch)
__host__ __device__ inline bool general_c(int C) { return C != 1 && C != 3; }
__host__ __device__ inline int n_freq(int C) { return C / 2 + 1; }

// Work kinds: each image contributes a number of work items of each kind;
// batched launches walk a global list of (image, item) pairs.
enum WorkKind { W_PIX = 0, W_REF = 1, W_MATCH = 2, W_COV = 3, W_FILT = 4, W_BOX = 5, W_NKIND = 6 };
constexpr int BOX_TY = 16, BOX_TX = 64;  // output tile of the coverage box sum

// Filter tile shapes (references per tile); index = hts_params.tune & 7
// (0 = pick by LDS budget).
struct FiltShape { int ty, tx; };

// Per-image descriptor.  Passed by value for single-image calls, read from a
// device table for batched calls.
struct ImgDesc {
  const float* img;        // [C][H][W]
  float* out;              // [C][H][W] (nullable)
  int32_t* gplanes;        // [np][H][W] quantised guide planes
  uint8_t* green;          // [n_ref] GCP branch per reference
  int32_t* idx;            // [n_ref][K]
  long long* dist;         // [n_ref][K] (nullable)
  int32_t* fb_list;        // [n_ref] references whose shortlist overflowed
  int32_t* fb_count;       // [1]
  double* cov_part;        // [n_cov][cov_elems]
  double* basis64;         // U64[C][8][8], V64[C][8][8], eig[2][C/2+1][8]
  float* basis;            // U[C][8][8], V[C][8][8] (real tensors)
  float* fbasis;           // Fourier slices for the filter, see FB_* offsets
  float* num;              // [C][H][W] float accumulator (caller's, or adjoint input)
  unsigned long long* num64; // [C][H][W] fixed-point accumulator, nullable (encoding:
                             // fx_int_units, fx_fourier in hts_device.h)
  uint8_t* poison;         // [H][W] 1 where a non-finite estimate landed (with num64)
  uint32_t* fxmax;         // [1] bits of max |input| (sets the fixed-point scale)
  float* cnt;              // [H][W]
  int32_t* hist;           // [H][W] slot-position histogram (coverage counts)
  uint32_t* masks;         // keep-masks (nullable)
  const uint32_t* masks_in;// frozen masks for the adjoint (nullable)
  float* group_est;        // [ref_count][K][C][8][8] (nullable)
  int32_t H, W, Hp, Wp, nry, nrx, n_ref;
  int32_t ref_begin, ref_count;   // filter range
  float sigma, tau;
  int32_t n_cov;           // covariance partial blocks
  // noise-level adjustment (A-Haar-tSVD); n_samples = 0 when unused
  const int32_t* samples;  // [n_samples] sampled reference indices
  int32_t n_samples, gamma;
  float beta;
  int32_t* ranks;          // [n_samples] rank of each sampled group (nullable)
  float* sigma_dev;        // [1] adjusted sigma; when set, the filter's tau is tau_mult * *sigma_dev
  unsigned long long* wsum64; // [H][W] weight sums (fixed point, 2^-48 units) of the weighted
                              // aggregation; nullable (then weights go to cnt, or are uniform)
  float* rowp;             // c = 1, 3: row projections [H][Wp][8 C] (see launch_rowproj)
  float* U_ext;            // [C][8][8] caller's basis copy (batched state export / import)
  float* V_ext;
  double* ufg;             // general c: [2 * (C/2+1)][re/im][64] Fourier-domain eigenvectors
  float* gscratch;         // general c: filter scratch, [work group][K][C][64]
  int32_t num_enc;         // NUM_FINE | NUM_PIXELS bits: how num64 encodes the sums
                           // beyond what C and the flags say (fx_int_units, fx_fourier)
  int32_t woff[W_NKIND];   // first global work item of each kind (batched)
  int32_t wcnt[W_NKIND];   // work items of each kind
};

// Fourier-domain basis layout (float32), consumed by the filter:
//   c = 1: U0[8][8], V0[8][8]
//   c = 3: U0, V0 (f = 0, real), U1r, U1i, V1r, V1i (f = 1, complex)
constexpr int FB_U0 = 0, FB_V0 = 64, FB_U1R = 128, FB_U1I = 192, FB_V1R = 256, FB_V1I = 320;
// Row-major slices for the vector-ALU filter, whose products all read
// matrix rows: transposes (suffix T) for the forward products, and the sums
// or differences that the three-multiplication complex products use
// (P: real + imaginary part, M: real - imaginary part).  For c = 3 the
// transposed U slices are scaled by 1/3 (the inverse DFT that follows them).
constexpr int FB_V0T = 384, FB_V1RT = 448, FB_V1IT = 512, FB_V1PT = 576;
constexpr int FB_U0T = 640, FB_U1RT = 704, FB_U1IT = 768, FB_U1MT = 832;
constexpr int FB_U1P = 896, FB_V1M = 960;
// The slices of the inverse right product (V0, V1R, V1I, V1M) scaled by the
// output scale of the c = 1, 3 filters' estimates: the fixed-point scale
// times 1/3 for c = 3 (the inverse channel DFT's factor; 1 with the
// channel-Fourier threshold, whose coefficients already carry it).
constexpr int FB_V0S = 1024, FB_V1RS = 1088, FB_V1IS = 1152, FB_V1MS = 1216;
constexpr int FB_SIZE = 1280;

// Encoding of the fixed-point numerator num64 (see hts_device.h): integer
// units for the forward c = 1, 3 filters with uniform weights, else 2^-32
// units (NUM_FINE: the frozen adjoints, whose dot-product identity wants
// more than FP32-level rounding of each estimate); channel-DFT triples for
// c = 3 unless the band-count filter produced the sums (NUM_PIXELS).
constexpr int NUM_FINE = 1, NUM_PIXELS = 2;
__host__ __device__ inline bool fx_int_units(int C, int flags, int enc) {
  return (C == 1 || C == 3) && !(flags & HTS_FLAG_WEIGHTED) && !(enc & NUM_FINE);
}
__host__ __device__ inline bool fx_fourier(int C, int enc) { return C == 3 && !(enc & NUM_PIXELS); }

struct Launch {
  ImgDesc one;             // used when table == nullptr
  const ImgDesc* table;    // device table of n_img descriptors (batched)
  int32_t n_img;
  int32_t total;           // total work items of the launched kind
  int32_t C, K, stride, window;
  float tau_mult;
  int32_t gcp_num, gcp_den;
  int32_t flags;
  int32_t fty, ftx;        // filter tile shape (references)
  int32_t* sl_hist;        // diagnostics: shortlist-size histogram [SL_BINS] of the
                           // match (nullable; then no extra LDS)
  int32_t count_hist;      // 1: k_quant clears hist and the match adds every group's
                           // slot corners to it (the coverage histogram)
  int32_t batch_masks;     // batched filter launch: export the keep-masks (d.masks)
  int32_t adjoint;         // batched adjoint: k_adjoint_prep reads d.num and writes
                           // d.out; k_zero_accum keeps cnt; k_finalize divides by 1
};

// Match-kernel LDS geometry for a 4x4 reference tile at stride s and window
// w: candidate rows/cols of the union window (padded to whole 16-wide MFMA
// blocks) and the pixel region they read.
struct MatchGeom {
  int ryc, rxp, pitch, rows;   // max candidate rows, padded candidate cols, LDS pitch, pixel rows
  int rgn, nbsz, plane_bytes;  // bytes of one staged region, of one norm array, of one plane slot
  int off_tl, off_misc, bytes;
};
// LDS of the match: npl plane slots of [gi][gb][|b|^2][|b|] (sbs = 0: no
// |b| array, its square root is taken where it is used), then the list
// values of pass 1, which the shortlist of pass 2 reuses (the lists are dead
// once T is known), then per-reference data.
__host__ __device__ inline MatchGeom match_geom(int s, int w, int npl, int sbs = 1) {
  MatchGeom g;
  int r = (w - 1) / 2;
  g.ryc = (MATCH_TY - 1) * s + 2 * r + 1;
  int rxc = (MATCH_TX - 1) * s + 2 * r + 1;
  g.rxp = (rxc + 7) / 8 * 8;           // candidate columns in blocks of 8
  const int ry2 = (g.ryc + 1) / 2 * 2;  // candidate rows in blocks of 2
  // pitch = 8 (mod 16), at least the staged columns: see the A/B operand
  // rows of the match
  g.pitch = g.rxp + PS - 1;
  g.pitch += ((8 - g.pitch) % 16 + 16) % 16;
  g.rows = ry2 + PS - 1;
  g.rgn = g.rows * g.pitch * 4;
  g.nbsz = ry2 * g.rxp * 4;
  g.plane_bytes = 2 * g.rgn + (sbs ? 2 : 1) * g.nbsz;
  g.off_tl = npl * g.plane_bytes;
  const int lists = 16 * 64 * 2 * 4, shortlist = 16 * SHORT_CAP * 4;
  g.off_misc = g.off_tl + (lists > shortlist ? lists : shortlist);
  // rinfo [16][8], rnorm [16][2], Tp [16], scount [16], then the re-rank
  // keys [4][64] (8 bytes each)
  g.bytes = g.off_misc + 768 + 4 * 64 * 8;
  return g;
}

// Grid size for for_each_item: rounded up to a multiple of the 8 XCDs.
inline int xcd_grid(int g) { return g >= 8 ? (g + 7) / 8 * 8 : g; }

// Number of references along one axis for n_valid positions and stride s.
inline int ref_count_axis(int n_valid, int s) {
  int n = (n_valid - 1) / s + 1;
  if ((n - 1) * s != n_valid - 1) ++n;
  return n;
}

// FP64 entries of one covariance partial: c = 1 two real 8x8 matrices;
// c = 3 two real (f = 0) and two complex (f = 1); other c two complex per
// frequency f <= c/2, [U: f, then V: f][re/im][64].
__host__ __device__ inline int cov_elems(int C) {
  return C == 1 ? 2 * 64 : C == 3 ? 2 * 64 + 2 * 128 : 2 * n_freq(C) * 128;
}
// Covariance partial blocks: tiles of cov_tile x cov_tile references, whose
// pixel region (at most cov_region pixels square) is staged in LDS.
__host__ __device__ inline int cov_tile(int s) { return s <= 4 ? 16 : 8; }
__host__ __device__ inline int cov_region(int s) { return (cov_tile(s) - 1) * s + PS; }

// Kernel launchers (defined in the .hip files).  Each returns hipSuccess or
// the launch error.  `grid` = 0 means one work group per work item.
hipError_t launch_quant(const Launch& L, int grid, hipStream_t s);
hipError_t launch_gcp(const Launch& L, int grid, hipStream_t s);
hipError_t launch_match(const Launch& L, int mode, int terms, int grid, hipStream_t s);
hipError_t launch_match_fallback(const Launch& L, int grid, hipStream_t s);
hipError_t launch_reset_counters(const Launch& L, hipStream_t s);
hipError_t launch_cov(const Launch& L, int grid, hipStream_t s);
hipError_t launch_eig(const Launch& L, hipStream_t s);
hipError_t launch_vote(const Launch& L, hipStream_t s);
// surrogate threshold derivative: partial[n_ref] (scratch), out[0] = dL/dlambda
hipError_t launch_taugrad(const Launch& L, const float* g, double* partial, float kappa, float* out,
                          int grid, hipStream_t s);
hipError_t launch_fbasis(const Launch& L, const float* U, const float* V, hipStream_t s);
// Basis copies between the workspace (d.basis, U then V) and the caller's
// d.U_ext / d.V_ext of every image that has them: to_ext = 1 exports,
// 0 imports.
hipError_t launch_copy_basis(const Launch& L, int to_ext, hipStream_t s);
hipError_t launch_gbasis(const Launch& L, const float* g, const double* U64, const double* V64,
                         const double* eig, double* partial, int grid, double* M, float* grad,
                         hipStream_t s);
hipError_t launch_zero_accum(const Launch& L, int grid, hipStream_t s);
hipError_t launch_filter(const Launch& L, int shape_ty, int shape_tx, int adjoint, int grid,
                         hipStream_t s);
// Row projections for the vector-ALU filter (c = 1, 3): for every image row
// y and valid column start x, the 8-pixel row of the patch at (y, x) after
// the channel DFT, times the Fourier slices of V (the first product of the
// t-SVD projection, P^ V_F, which depends only on the row and the column
// start): d.rowp[(y * Wp + x) * 8C + 8q + b], q = 0 (f = 0; c = 1: the row
// itself), 1, 2 (real and imaginary part of f = 1).  Work items W_PIX.
hipError_t launch_rowproj(const Launch& L, int grid, hipStream_t s);
__host__ __device__ inline int rowp_floats(int C) { return 8 * C; }
hipError_t launch_finalize(const Launch& L, int grid, hipStream_t s);
hipError_t launch_scatter_est(const Launch& L, hipStream_t s);
hipError_t launch_adjoint_prep(const Launch& L, int grid, hipStream_t s);
hipError_t launch_absmax(const Launch& L, int grid, hipStream_t s);
hipError_t launch_synth(float* img, int C, int H, int W, hipStream_t s);
hipError_t launch_zero_hist(const Launch& L, int grid, hipStream_t s);
hipError_t launch_fill(float* p, int n, float v, hipStream_t s);   // fill kernel (graph-safe)
hipError_t launch_count_hist(const Launch& L, int grid, hipStream_t s);
hipError_t launch_count_box(const Launch& L, int grid, hipStream_t s);

// FP32-MFMA filter for RGB groups (K in {4, 8, 16, 32}).
bool filter_mfma_supported(int C, int K);
size_t filter_mfma_lds_bytes(int stride, int window, int ty, int tx);
hipError_t launch_filter_mfma(const Launch& L, int ty, int tx, int adjoint, int grid, hipStream_t s);

// Filter LDS bytes for a tile shape.
size_t filter_lds_bytes(int C, int K, int stride, int window, int ty, int tx, bool weighted = false);
// channel-Fourier threshold variant of the vector-ALU filter (c = 3)
hipError_t launch_filter_ft(const Launch& L, int g, size_t lds, bool batch, bool masks, bool wt,
                            hipStream_t s);
size_t match_lds_bytes(int stride, int window);   // one plane slot: the minimum

// General band counts (csrc/k_general.hip): covariances per (reference tile,
// frequency chunk), eigen-solves, real tensors, Fourier slices, filter.
hipError_t launch_basis_gen(const Launch& L, hipStream_t s);
hipError_t launch_fbasis_gen(const Launch& L, hipStream_t s);
hipError_t launch_filter_gen(const Launch& L, int grid, hipStream_t s);
size_t filter_gen_lds_bytes(int C);
size_t cov_gen_lds_bytes(int C);

}  // namespace hts
