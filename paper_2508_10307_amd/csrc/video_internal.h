// Internal declarations of the video path (spatio-temporal search over the
// frames stacked one above the other), of the split band-count basis
// launchers it uses, and of the band-count adjoint filter.
#pragma once
#include "hts_internal.h"

namespace hts {

// Geometry of one frame of the sequence and the temporal reach.
struct VideoGeo {
  int32_t T, H, Hp, Wp, nry, nrx, n_ref_frame, dt;
};

constexpr int VIDEO_CAND_MAX = 4096;   // candidates per reference (12-bit ordinal in the key)

hipError_t launch_stack(const float* frames, float* stacked, int T, int C, int H, int W,
                        bool inverse, hipStream_t s);
hipError_t launch_match_video(const Launch& L, const VideoGeo& v, hipStream_t s);
hipError_t launch_cov_gen(const Launch& L, hipStream_t s);
hipError_t launch_eig_gen(const Launch& L, hipStream_t s);
hipError_t launch_filter_gen_adj(const Launch& L, int grid, hipStream_t s);
// The vector-ALU filter of c = 1 and c = 3 for one image descriptor whose
// groups may gather patches anywhere in the image: L.total tiles of
// L.fty x L.ftx references over d.nry x d.nrx, every slot's estimate
// (fixed-point scaled) exported to d.group_est for launch_gather.
hipError_t launch_filter_stacked(const Launch& L, hipStream_t s);
constexpr int VIDEO_FTY = 4, VIDEO_FTX = 8;   // reference tile of one work group
// Aggregation of exported slot estimates est[n_ref K][C][8][8] (fixed-point
// scaled) into L.one.num64 over the whole image, from the corner histogram
// L.one.hist: bucket the slots by corner, then gather per output tile.
// scratch: gather_scratch_ints(H W) ints; list: n_ref K ints.
size_t gather_scratch_ints(long long n_pix);
bool gather_supported(long long n_pix);
hipError_t launch_gather(const Launch& L, const float* est, int* scratch, int* list,
                         hipStream_t s);

}  // namespace hts
