/*
 * hts.h - C ABI of the MI355X (gfx950) Haar-tSVD denoiser hot path.
 *
 * Haar-tSVD (arXiv 2508.10307): for every reference patch of a noisy image,
 * find its K most similar patches in a local window (Sec. III.A, Eq. 10),
 * project the stacked group on a global t-SVD patch basis learned from all
 * reference patches (Sec. III.B.1, Eq. 11-12) combined with a Haar transform
 * along the group mode (Eq. 17-18), hard-threshold the coefficients (Eq. 19),
 * invert both transforms (Eq. 20) and average every estimate back into the
 * image (Eq. 2, Alg. 1 Step 3).  The paper states the problem as: noisy image
 * Y, patch size ps, group size K, window W and noise level sigma in, the
 * estimated clean image out (Alg. 1).
 *
 * Conventions shared by every entry point
 *  - Images are planar float32 [C][H][W], contiguous, in device memory.
 *    C is 1 (grey), 3 (RGB) or, for the spectral tubes of HSI (Sec. IV: a
 *    ps x ps x N_bands patch, other parameters unchanged), 2 and 4..256 with
 *    K <= 32 and no flags; ps must be 8.  The band counts other than 1 and 3
 *    run through hts_denoise, hts_match, hts_basis, hts_filter,
 *    hts_denoise_backward and hts_denoise_video (the other entry points
 *    return HTS_ERR_UNSUPPORTED for them).
 *  - Reference grid: top-left corners 0, s, 2s, ... along each axis plus the
 *    last valid position H-ps (resp. W-ps); references are numbered
 *    row-major over that grid (n_ref = n_ref_y * n_ref_x).
 *  - Match indices are int32 [n_ref][K]; entry = y*W + x of a patch's
 *    top-left corner.  Slot 0 is the reference itself, slots 1..K-1 the K-1
 *    closest other candidates of the truncated window ordered by
 *    (distance, index).  Distances are exact integers on the guide
 *    q = round_half_even(256*y) clamped to |q| <= 2^20-1; for C = 3 the guide
 *    of a reference is its green channel when
 *    gcp_num^2*|qG|^2 >= gcp_den^2*max(|qR|^2,|qB|^2) (Eq. 10 with
 *    gamma = gcp_num/gcp_den) and R+G+B otherwise; for other C it is the band
 *    mean on the same grid, round_half_even(sum_j q_j / C), exact integers.
 *  - Basis tensors U, V are float32 [C][ps][ps] (frontal slice j = U(:,:,j)).
 *  - Threshold masks are bit-packed: bit ((g*K + k)*C + ch)*64 + i*8 + j of a
 *    little-endian uint32 stream is 1 when Haar-t-SVD coefficient (k, ch, i, j)
 *    of group g survived the hard threshold (k = row of the K x K Haar matrix
 *    of Eq. 9, i/j = row/column of the projected patch).
 *  - Ownership: the caller owns every buffer, including the workspace sized
 *    by hts_workspace_size(); the library never allocates device memory.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  A returned status covers argument validation and launch
 *    errors; on any error nothing is launched.  Device faults surface at the
 *    caller's next synchronisation.  No C++ exception crosses this ABI.
 *  - Aggregation (Eq. 2) sums the estimates as 64-bit integers, scaled by a
 *    power of two set from the image's largest input magnitude M.  The
 *    forward filters of C = 1, 3 with uniform weights (hts_denoise, the
 *    batches, hts_filter, the video) round every estimate to a multiple of
 *    at most 2^-23 M (estimates are at most sqrt(64 K C) M <= 79 M, which
 *    that encoding holds without saturation); the weighted aggregation, the
 *    frozen adjoints and the other band counts keep 32 fractional bits
 *    below 2^11..2^12 = M (multiples of 2^-43 M; into hts_filter's float
 *    num: 32 fractional bits of the image values).  Integer sums do not
 *    depend on the order of the additions.
 *  - Reproducibility: match indices, distances, threshold masks and the
 *    outputs of hts_denoise, hts_denoise_batch and hts_denoise_backward are
 *    bit-for-bit the same from run to run, for any launch schedule of the
 *    same filter implementation and between the batched and single-image
 *    calls.  hts_filter and hts_aggregate add into caller-owned float32
 *    buffers with float atomics, whose last bits depend on the order of the
 *    additions.
 *  - Non-finite inputs: NaN quantises to 0 and +-inf to the clamp for
 *    matching.  A group that gathers a non-finite pixel, or whose estimates
 *    are not finite, makes every pixel of its K patches NaN in the output
 *    (or in num for hts_filter).  hts_denoise learns the basis from the
 *    image itself, so there one non-finite pixel makes the basis, and with
 *    it the whole output, NaN.
 */
#ifndef HTS_H
#define HTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HTS_OK = 0,
  HTS_ERR_INVALID = 1,      /* bad argument (null pointer, sizes, K, window...) */
  HTS_ERR_UNSUPPORTED = 2,  /* valid per the paper but not built (ps != 8, C > 256, ...) */
  HTS_ERR_WORKSPACE = 3,    /* workspace too small */
  HTS_ERR_HIP = 4           /* a HIP runtime call or launch failed */
} hts_status;

typedef enum {
  HTS_MATCH_BF16 = 0,       /* norm+dot distance tiles on BF16 MFMA (FP32 accumulate) */
  HTS_MATCH_FP32 = 1        /* plain FP32 SSD tiles on the vector ALUs (no MFMA) */
} hts_match_mode;

/* hts_params.flags: Eq. 2 with group weights w_g = 1 / max(1, number of
 * coefficients of group g kept by the hard threshold) instead of uniform
 * ones (the paper leaves the weights open; this is the BM3D-style choice):
 * x = sum_g w_g * estimates / sum_g w_g per pixel.  Honoured by hts_denoise,
 * hts_denoise_batch(_adaptive) and hts_filter (which then adds the weight
 * sums into cnt instead of coverage counts; estimates into num are
 * weighted); the vector-ALU filter runs.  hts_aggregate and
 * hts_denoise_backward return HTS_ERR_UNSUPPORTED with it. */
#define HTS_FLAG_WEIGHTED 1
/* hts_params.flags: threshold in the channel-Fourier domain (c = 3) instead
 * of Eq. 19 on the real core tensor: in the Haar domain of each group, the
 * f = 0 coefficient F_0 (DFT along the channel mode) is kept iff
 * |F_0| / sqrt(3) >= tau and the conjugate pair f = 1, 2 iff
 * sqrt(2/3) |F_1| >= tau (their orthonormal magnitudes), so whole pairs are
 * kept or dropped.  Exported masks then hold the decision of frequency f in
 * channel f.  No effect for c = 1.  Honoured by hts_denoise,
 * hts_denoise_batch(_adaptive) and hts_filter (vector-ALU filter);
 * hts_denoise_backward returns HTS_ERR_UNSUPPORTED with it. */
#define HTS_FLAG_FOURIER_THRESHOLD 2

typedef struct {
  int32_t ps;          /* patch size; must be 8                                  */
  int32_t stride;      /* reference stride s, 1 <= s <= ps                        */
  int32_t window;      /* odd full search-window width w, 3 <= w <= 63            */
  int32_t K;           /* group size, power of two, 2 <= K <= 64 (32 for C = 3)   */
  float tau_mult;      /* lambda: hard threshold tau = lambda * sigma (Eq. 19)    */
  int32_t gcp_num;     /* gamma = gcp_num / gcp_den (Eq. 10; 6/5 = 1.2), 1..64    */
  int32_t gcp_den;
  int32_t match_mode;  /* hts_match_mode                                          */
  int32_t flags;       /* 0 or HTS_FLAG_WEIGHTED | HTS_FLAG_FOURIER_THRESHOLD       */
  int32_t tune;        /* 0 = autotuned/default launch schedule, else a schedule id */
} hts_params;

/* Fill *p with the defaults: ps 8, stride 3, window 21, K 16, lambda 2.7,
 * gamma 6/5, BF16 matching, flags 0, tune 0. */
void hts_default_params(hts_params* p);

/* Number of references along each axis (reference grid, see above). */
hts_status hts_ref_grid(int32_t H, int32_t W, const hts_params* p,
                        int32_t* n_ref_y, int32_t* n_ref_x);

/* Workspace bytes needed by hts_match / hts_basis / hts_filter / hts_denoise
 * for one C x H x W image. */
hts_status hts_workspace_size(const hts_params* p, int32_t C, int32_t H, int32_t W,
                              size_t* bytes);

/* Alg. 1 Step 1 (Sec. III.A, Eq. 10): block matching of every reference.
 * idx   out, int32 [n_ref][K] (device).
 * dist  out, nullable, int64 [n_ref][K]: exact guide distances (slot 0 = 0).
 * green out, nullable, uint8 [n_ref]: 1 when the reference used the green guide.
 * Distance tiles run in p->match_mode; the shortlist they produce is
 * certified by an error bound and re-ranked exactly, so idx does not depend
 * on the mode. */
hts_status hts_match(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                     int32_t W, int32_t* idx, int64_t* dist, uint8_t* green,
                     void* ws, size_t ws_bytes, void* stream);

/* Alg. 1 Step 2(1) (Sec. III.B.1, Eq. 11-12): global basis from all
 * reference patches.  Covariances are accumulated and eigen-decomposed in
 * FP64 on the device, per frequency of the channel-mode DFT (descending
 * eigenvalues; each eigenvector scaled by a unit-modulus factor so that its
 * largest-modulus entry is real positive).
 * U, V    out, float32 [C][ps][ps] (device).
 * U64,V64 out, nullable, float64 [C][ps][ps].
 * eig     out, nullable, float64 [2][C/2+1][ps]: eigenvalues of the row (U)
 *         and column (V) covariances per frequency, descending. */
hts_status hts_basis(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                     int32_t W, float* U, float* V, double* U64, double* V64, double* eig,
                     void* ws, size_t ws_bytes, void* stream);

/* Alg. 1 Step 2(2)-(4) (Eq. 18-20) for references [ref_begin, ref_begin+ref_count):
 * gather each group, project with U^T * . * V (t-product) and H_K along the
 * group, keep coefficients with |s| >= tau_mult*sigma, invert.
 * idx        in, int32 [n_ref][K] (all references of the image).  Any
 *            grouping is accepted, not only hts_match's: a patch outside the
 *            accumulation tile of its work group (an entry beyond its
 *            reference's search window) is added straight into the image;
 *            an entry that is not a valid patch corner (0 <= y <= H-ps,
 *            0 <= x <= W-ps) is taken at the nearest valid corner, in the
 *            estimates and in cnt alike.
 * U, V       in, float32 [C][ps][ps].
 * num, cnt   in/out, nullable together: estimates are ADDED into
 *            num float32 [C][H][W] and coverage counts into cnt float32 [H][W]
 *            (Eq. 2 numerator and denominator); the caller zeroes them first.
 * group_est  out, nullable, float32 [ref_count][K][C][ps][ps].
 * masks      out, nullable, bit-packed keep-masks of the ref_count groups
 *            (ceil(ref_count*K*C*64/32) uint32 words; group index relative
 *            to ref_begin). */
hts_status hts_filter(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                      int32_t W, float sigma, const int32_t* idx, const float* U,
                      const float* V, int32_t ref_begin, int32_t ref_count, float* num,
                      float* cnt, float* group_est, uint32_t* masks, void* ws,
                      size_t ws_bytes, void* stream);

/* Alg. 1 Step 3 / Eq. 2 with uniform weights (estimates averaged).
 * group_est nullable: when given, the estimates of references
 *           [ref_begin, ref_begin+ref_count) are added into num / cnt at the
 *           positions idx gives.
 * out       nullable: when given, out = num / cnt (every pixel has cnt >= 1). */
hts_status hts_aggregate(const hts_params* p, const float* group_est, const int32_t* idx,
                         int32_t ref_begin, int32_t ref_count, int32_t C, int32_t H,
                         int32_t W, float* num, float* cnt, float* out, void* stream);

/* Algorithm 1 end to end: noisy image and sigma in, denoised image out.
 * idx_out, masks_out, U_out, V_out, cnt_out: nullable copies of the state a
 * backward pass needs (idx [n_ref][K], masks as in hts_filter for all n_ref
 * groups, U/V [C][ps][ps], cnt [H][W]). */
hts_status hts_denoise(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                       int32_t W, float sigma, float* out, int32_t* idx_out,
                       uint32_t* masks_out, float* U_out, float* V_out, float* cnt_out,
                       void* ws, size_t ws_bytes, void* stream);

typedef struct {
  const float* noisy;  /* device [C][H][W]                */
  float* out;          /* device [C][H][W]                */
  int32_t C, H, W;
  float sigma;
} hts_image;

/* Surrogate derivative of a loss with respect to tau_mult (an adjoint
 * extension: the hard threshold of Eq. 19 has a zero derivative almost
 * everywhere, so hts_denoise_backward returns 0 for it).  The keep-mask is
 * relaxed to m(s) = logistic((|s| - tau) / eps), eps = kappa * sigma, and with
 * idx, U, V and cnt (as hts_denoise saves them) frozen:
 *   grad_tau_mult[0] = sigma * sum over groups and coefficients of
 *                      r * s * (-logistic'(u) / eps),  u = (|s| - tau) / eps,
 * where s and r are the orthonormal Haar / t-SVD coefficients (Eq. 18) of
 * the groups of noisy and of grad_out / cnt (device [C][H][W]).  FP64 sums,
 * added in a fixed order (the same bits on every run); device float out.
 * sigma = 0 gives 0.  Errors: HTS_ERR_INVALID for null pointers, sigma < 0,
 * kappa <= 0 or non-finite; HTS_ERR_UNSUPPORTED with flags set; the
 * parameter and workspace checks of hts_denoise. */
hts_status hts_denoise_grad_tau(const hts_params* p, const float* noisy, const float* grad_out,
                                const int32_t* idx, const float* U, const float* V,
                                const float* cnt, int32_t C, int32_t H, int32_t W, float sigma,
                                float kappa, float* grad_tau_mult, void* ws, size_t ws_bytes,
                                void* stream);

/* Derivative through the learned basis (adjoint extension).  Alg. 1
 * Step 2(1) learns U, V from the noisy image itself (Eq. 11-12: the
 * eigenvectors of the per-frequency patch second moments C_U(f), C_V(f),
 * phase-normalised), so with idx, masks and cnt frozen dL/dnoisy has, beside
 * hts_denoise_backward's frozen-basis term, a term through U(noisy),
 * V(noisy).  This call ADDS that term into grad_in (device [C][H][W],
 * in/out):
 *   A_U(f) = sum over group slots of R^ V_F T'^^H + P^ V_F D^^H,
 *   A_V(f) = sum of R^^H U_F T'^ + P^^H U_F D^  (P / R: the slot's patch of
 *   noisy / of grad_out / cnt; T', D: their projections (Eq. 18) through the
 *   frozen mask and back; ^: DFT along the channel mode),
 * then per eigenproblem the first-order eigenvector perturbation (distinct
 * eigenvalues) with the phase convention's gauge term, and
 * dL/dP^_i = 2 Cbar_U P^_i + 2 P^_i Cbar_V added back at every reference
 * patch i.  noisy, grad_out: device [C][H][W]; idx, masks, cnt as
 * hts_denoise saves them; U64, V64 [C][ps][ps] and eig [2][C/2+1][ps]: the
 * FP64 basis and eigenvalues of hts_basis for noisy.  FP64 sums in a fixed
 * order (the same bits on every run).  Near-equal eigenvalues make the term
 * large (1 / (l_k - l_j)), as the eigenvectors themselves are then
 * ill-conditioned.  Errors: HTS_ERR_INVALID for null pointers;
 * HTS_ERR_UNSUPPORTED with flags set; the parameter and workspace checks of
 * hts_denoise. */
hts_status hts_denoise_backward_basis(const hts_params* p, const float* noisy,
                                      const float* grad_out, const int32_t* idx,
                                      const uint32_t* masks, const double* U64, const double* V64,
                                      const double* eig, const float* cnt, int32_t C, int32_t H,
                                      int32_t W, float* grad_in, void* ws, size_t ws_bytes,
                                      void* stream);

/* Video denoising with spatio-temporal patch search (Sec. IV: the search
 * runs over the spatial and the temporal dimension).  frames: device
 * float32 [T][C][H][W] (C = 1, 3, or 2..256 bands), out the same.  Each
 * frame has the reference grid of hts_match; a reference of frame t takes
 * candidates from frames t-dt..t+dt (truncated at the ends of the sequence)
 * inside its truncated spatial window, ranked by the exact guide distance of
 * hts_match (GCP branch from the reference patch for C = 3, band mean for
 * other C), ties to the lower stacked index; positions are numbered in the
 * frames stacked one above the other, idx = (t' H + y) W + x.  One basis for
 * the sequence (Eq. 11-12 over the reference patches of every frame); the
 * groups are filtered (Eq. 18-20) and averaged (Eq. 2) over the stacked
 * frames.  idx_out (nullable, int32 [T n_ref][K], references frame by
 * frame), masks_out (nullable, as hts_filter for the T n_ref groups),
 * U_out / V_out (nullable, float32 [C][ps][ps]), cnt_out (nullable, float32
 * [T H][W]).  Requires K <= 32, no flags and (2 min(dt, T-1) + 1) window^2
 * <= 4096 (HTS_ERR_UNSUPPORTED otherwise); HTS_ERR_INVALID for T < 1,
 * dt < 0, null frames / out / ws, sigma < 0 or non-finite. */
hts_status hts_video_workspace_size(const hts_params* p, int32_t T, int32_t C, int32_t H,
                                    int32_t W, int32_t dt, size_t* bytes);
hts_status hts_denoise_video(const hts_params* p, const float* frames, int32_t T, int32_t C,
                             int32_t H, int32_t W, int32_t dt, float sigma, float* out,
                             int32_t* idx_out, uint32_t* masks_out, float* U_out, float* V_out,
                             float* cnt_out, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of hts_denoise_video with the grouping, masks, basis and counts
 * of the forward pass frozen (the video counterpart of
 * hts_denoise_backward): grad_in = Place Q^T M Q Gather (grad_out / cnt) over
 * the stacked frames, Q = Haar along the group o t-SVD projection, M the
 * frozen keep-mask.  grad_out, grad_in: device float32 [T][C][H][W]; idx,
 * masks, U, V, cnt ([T H][W]) as hts_denoise_video returns them; the same
 * dt, parameters and workspace size as the forward call.  Errors as
 * hts_denoise_video, and HTS_ERR_INVALID for null pointers. */
hts_status hts_denoise_video_backward(const hts_params* p, const float* grad_out, int32_t T,
                                      int32_t C, int32_t H, int32_t W, int32_t dt,
                                      const int32_t* idx, const uint32_t* masks, const float* U,
                                      const float* V, const float* cnt, float* grad_in, void* ws,
                                      size_t ws_bytes, void* stream);

/* Diagnostics of the certified shortlist of hts_match (Alg. 1 Step 1):
 * the number of references whose shortlist overflowed (or held fewer than
 * K-1 entries) in the last hts_match / hts_denoise call on this workspace;
 * those references were matched by an exact scan of their whole window
 * instead, so their indices are the same either way.  count: device int32[1],
 * written asynchronously on `stream`.  The parameters and image shape must be
 * those of that call.  Errors: HTS_ERR_INVALID for null pointers, the
 * parameter and workspace checks of hts_match. */
hts_status hts_match_fallback_count(const hts_params* p, int32_t C, int32_t H, int32_t W,
                                   const void* ws, size_t ws_bytes, int32_t* count, void* stream);

/* The same for every image of the last hts_denoise_batch(_adaptive) call on
 * this workspace with these images: counts, device int32[n]. */
hts_status hts_batch_fallback_counts(const hts_params* p, const hts_image* imgs, int32_t n,
                                     const void* ws, size_t ws_bytes, int32_t* counts,
                                     void* stream);

/* Diagnostics of the certified match (Alg. 1 Step 1): the sizes of the
 * shortlists it re-ranks.  Runs the batched quantisation, Eq. 10 and the
 * match of hts_denoise_batch on these images (imgs[i].out and sigma are not
 * used; the workspace is that of hts_denoise_batch, whose idx it
 * overwrites) and writes counts (device int32[HTS_SHORTLIST_BINS]):
 * counts[s], s <= 128, = references whose shortlist held s candidates;
 * counts[129] = references whose shortlist overflowed (they take the exact
 * window scan).  Synchronises `stream` once (descriptor upload).
 * Errors: as hts_denoise_batch, HTS_ERR_INVALID for null counts. */
#define HTS_SHORTLIST_BINS 130
hts_status hts_batch_shortlist_histogram(const hts_params* p, const hts_image* imgs, int32_t n,
                                         void* ws, size_t ws_bytes, int32_t* counts,
                                         void* stream);

/* Workspace bytes for hts_denoise_batch over these n images (host array). */
hts_status hts_batch_workspace_size(const hts_params* p, const hts_image* imgs, int32_t n,
                                    size_t* bytes);

/* Algorithm 1 for n independent images of any sizes and noise levels (each
 * with its own reference grid, basis and sigma).  All images share C and
 * the method parameters.  The stages run as persistent kernels over a
 * device work list of (image, tile) items, captured once per parameter set
 * into a HIP graph and replayed; imgs is a host array. */
hts_status hts_denoise_batch(const hts_params* p, const hts_image* imgs, int32_t n,
                             void* ws, size_t ws_bytes, void* stream);

/* hts_denoise_batch with its stages launched one by one on `stream` (no
 * graph, no second stream), recording caller-created HIP events
 * (hipEvent_t, created with timing enabled) at the stage boundaries, so that
 * each stage's kernels can be timed with hipEventElapsedTime:
 *   events[0] start, [1] after quantisation and the Eq. 10 branch,
 *   [2] after the block matching (Alg. 1 Step 1), [3] after the covariances,
 *   [4] after the shortlist fallback, coverage counts, eigen-solves and
 *   Fourier slices (Step 2(1)), [5] after the fused filter and aggregation
 *   (Step 2(2)-(4) and Step 3, one launch), [6] after the write-back.
 * The same kernels, schedule and results as hts_denoise_batch.  Synchronises
 * `stream` once, before the first launch (descriptor upload).
 * Errors: HTS_ERR_INVALID unless n_events == HTS_BATCH_STAGE_EVENTS and
 * every event is non-null; otherwise as hts_denoise_batch. */
#define HTS_BATCH_STAGE_EVENTS 7
hts_status hts_denoise_batch_staged(const hts_params* p, const hts_image* imgs, int32_t n,
                                    void* ws, size_t ws_bytes, void* stream, void* const* events,
                                    int32_t n_events);

/* A-Haar-tSVD noise-level adjustment (Sec. III.D, Eq. 21-22; Algorithm
 * A-Haar-tSVD Step 1) for a caller-supplied sigma_est (the paper's CNN
 * estimator is not part of this library).  For each sampled group (the
 * reference indices samples[0..n_samples), device int32, drawn by the
 * caller; out-of-range entries are clamped to the reference grid), with the
 * K patches of its row of idx (device [n_ref][K], slot order as hts_match
 * writes it): lambda_m = sum over the group's C*64 values of
 * |DFT_K along the group mode|^2, m = 0..K-1, the eigenvalues of
 * circ(G) circ(G)^T; a = 1 + #{m : lambda_m < lambda_{K/2}} (the rank of
 * Eq. 21's alternating eigenvalue, ascending).  sigma_out (device float[1])
 * receives sigma_est / beta when more than half of the sampled groups have
 * a <= gamma (Eq. 22; paper values beta = 1.2, gamma = 13), else sigma_est.
 * ranks (device int32[n_samples], nullable) receives each a.  FP64
 * arithmetic; asynchronous on `stream`; no workspace.
 * Errors: HTS_ERR_INVALID for null pointers, n_samples outside
 * [1, 2^20], beta not positive and finite, sigma_est negative or not
 * finite, and the parameter checks of hts_match. */
hts_status hts_adapt_sigma(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                           int32_t W, const int32_t* idx, const int32_t* samples,
                           int32_t n_samples, float sigma_est, float beta, int32_t gamma,
                           int32_t* ranks, float* sigma_out, void* stream);

/* A-Haar-tSVD over a batch (Algorithm A-Haar-tSVD): hts_denoise_batch where
 * imgs[i].sigma is sigma_est of image i, and after the match of each image
 * the adjustment of hts_adapt_sigma runs on its sampled groups
 * (samples + i * n_samples); the filter then thresholds image i with
 * tau = tau_mult * sigma_out[i], read on the device (no host round trip).
 * Sub-images of one picture are passed as separate images.  ranks (nullable)
 * and sigma_out are device arrays [n][n_samples] and [n].  Workspace as for
 * hts_denoise_batch.  Errors as hts_denoise_batch and hts_adapt_sigma. */
hts_status hts_denoise_batch_adaptive(const hts_params* p, const hts_image* imgs, int32_t n,
                                      const int32_t* samples, int32_t n_samples, float beta,
                                      int32_t gamma, int32_t* ranks, float* sigma_out,
                                      void* ws, size_t ws_bytes, void* stream);

/* Adjoint of hts_denoise with the match indices, threshold masks, basis and
 * coverage count held fixed (the map noisy -> denoised is then linear;
 * derived from Eq. 18-20 and Eq. 2):
 *   grad_in = sum_g Gather_g^T Q^T M_g Q Gather_g (grad_out / cnt).
 * idx is taken as in hts_filter (any grouping; invalid corners at the
 * nearest valid one).
 * grad_tau_mult (nullable, device float) receives 0: the threshold enters
 * only through the frozen masks. */
hts_status hts_denoise_backward(const hts_params* p, const float* grad_out,
                                const int32_t* idx, const uint32_t* masks, const float* U,
                                const float* V, const float* cnt, int32_t C, int32_t H,
                                int32_t W, float* grad_in, float* grad_tau_mult, void* ws,
                                size_t ws_bytes, void* stream);

/* The state one image's backward pass needs (as hts_denoise exports it):
 * device buffers owned by the caller, all non-null.
 *   idx   [n_ref][K] int32;  masks  bit-packed as in hts_filter for all
 *   n_ref groups (n_ref K C 2 words);  U, V  [C][ps][ps];  cnt  [H][W]. */
typedef struct {
  int32_t* idx;
  uint32_t* masks;
  float* U;
  float* V;
  float* cnt;
} hts_state;

/* hts_denoise_batch that also writes every image's backward state into
 * states[i] (host array of n): the values hts_denoise writes through its
 * idx_out, masks_out, U_out, V_out and cnt_out for that image alone, bit for
 * bit.  Uniform aggregation with the real-domain threshold only (the masks
 * of Eq. 19).  Captured into its own HIP graph per parameter set, like
 * hts_denoise_batch; the state pointers may change between calls.  Same
 * workspace as hts_denoise_batch.  Errors: HTS_ERR_UNSUPPORTED with
 * HTS_FLAG_WEIGHTED or HTS_FLAG_FOURIER_THRESHOLD; HTS_ERR_INVALID for a
 * null states or a null state pointer; otherwise as hts_denoise_batch. */
hts_status hts_denoise_batch_save(const hts_params* p, const hts_image* imgs,
                                  const hts_state* states, int32_t n, void* ws, size_t ws_bytes,
                                  void* stream);

/* hts_denoise_backward for n images at once: imgs[i].noisy is grad_out of
 * image i and imgs[i].out receives its grad_in (the two may be the same
 * buffer); imgs[i].sigma is ignored; states[i] is the frozen state of that
 * image (from hts_denoise_batch_save or hts_denoise).  The same values as n
 * hts_denoise_backward calls, bit for bit; the stages run as persistent
 * launches over all images, captured into a HIP graph per parameter set.
 * Same workspace as hts_denoise_batch over these images.  Errors as
 * hts_denoise_batch_save. */
hts_status hts_denoise_batch_backward(const hts_params* p, const hts_image* imgs,
                                      const hts_state* states, int32_t n, void* ws,
                                      size_t ws_bytes, void* stream);

/* hts_denoise for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same stages and kernels, with the workspace taken from a fixed scratch
 * array of HTS_NOALLOC_SCRATCH_BYTES in the library's device code object
 * (one per GPU, held from the load of the library until the process ends)
 * instead of a caller buffer.  noisy / out as in hts_denoise; no state is
 * exported.  No device memory is allocated or freed by this call.
 * Images whose hts_workspace_size exceeds the scratch (e.g. RGB above about
 * 1024 x 1024 at K = 32, stride 3) return HTS_ERR_WORKSPACE and launch
 * nothing.  Every call on a GPU uses that GPU's one scratch array, which
 * keeps the last call's contents (each call clears what it reads first):
 * calls that overlap on one GPU, from any stream or thread, race. */
#define HTS_NOALLOC_SCRATCH_BYTES ((size_t)192 << 20)
hts_status hts_denoise_noalloc(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                               int32_t W, float sigma, float* out, void* stream);

/* Autotuner: time the launch schedules of the match and filter stages on
 * the current device for this parameter set and image shape, remember the
 * fastest (in memory, and in the cache file `cache_path` when non-null),
 * and return it in *tune_out (pass it as hts_params.tune).  Uses ws for
 * scratch; synchronises `stream`. */
hts_status hts_autotune(const hts_params* p, int32_t C, int32_t H, int32_t W,
                        const char* cache_path, int32_t* tune_out, void* ws,
                        size_t ws_bytes, void* stream);

/* Short static description of a status code. */
const char* hts_status_string(hts_status s);

/* Library version string. */
const char* hts_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HTS_H */
