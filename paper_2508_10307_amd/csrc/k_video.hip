// Video path: spatio-temporal patch search (Sec. IV, colour video: the
// search runs over the spatial and the temporal dimension).  The T frames
// are stacked one above the other into one [C][T*H][W] image, so a group
// may gather patches of several frames and the band-count filter (which
// aggregates with fixed-point atomics, not through a window tile) and the
// coverage count work on the stacked image unchanged.
//
// k_match_video: one wavefront per reference (references frame by frame,
// row-major within a frame); candidates are every valid position of frames
// t - dt .. t + dt (truncated at the ends) inside the truncated spatial
// window, enumerated frame-major then row-major, which is the order of their
// stacked indices.  Lane l takes candidates l, l + 64, ...: the exact integer
// distance on the guide plane of the reference's kind (GCP test on the
// reference patch for c = 3), key = (distance << 12) | ordinal.  Keys below
// the running (K-1)-th smallest are compacted into a 64-entry LDS buffer of
// the wavefront; when the next 64 candidates could overflow it, one bitonic
// sort of 128 keys (running best 64 and the buffer) keeps the 64 smallest in
// order and lowers the threshold.  A key at or above the threshold already
// has K-1 smaller keys kept, so it can never enter the result.
#include "hts_device.h"
#include "video_internal.h"

namespace hts {

// [T][C][H][W] <-> [C][T*H][W] (inverse: stacked to frames).
__global__ void k_stack(const float* src, float* dst, int T, int C, int H, int W, int inverse) {
  const long long n = (long long)T * C * H * W;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    // e indexes the frame layout: ((t * C + c) * H + y) * W + x
    const long long x = e % W, y = (e / W) % H, c = (e / ((long long)W * H)) % C,
                    t = e / ((long long)W * H * C);
    const long long st = (c * T * H + t * H + y) * W + x;
    if (inverse) dst[e] = src[st];
    else dst[st] = src[e];
  }
}

hipError_t launch_stack(const float* frames, float* stacked, int T, int C, int H, int W,
                        bool inverse, hipStream_t s) {
  const long long n = (long long)T * C * H * W;
  const int grid = (int)std::min<long long>((n + 255) / 256, 65536);
  if (inverse) hipLaunchKernelGGL(k_stack, dim3(grid), dim3(256), 0, s, stacked, (float*)frames, T, C, H, W, 1);
  else hipLaunchKernelGGL(k_stack, dim3(grid), dim3(256), 0, s, frames, stacked, T, C, H, W, 0);
  return hipGetLastError();
}

// Lane l's 64-bit value, read by every lane (l wavefront-uniform).
__device__ inline unsigned long long lane_u64(unsigned long long v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// L.one: the stacked image (img, gplanes of the stacked image, idx / dist
// rows for T * n_ref_frame references).  Four wavefronts per work group.
__global__ __launch_bounds__(256) void k_match_video(Launch L, VideoGeo v) {
  __shared__ int refp[4][64];
  __shared__ unsigned long long kbuf[4][64];   // keys waiting for the next merge
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int a = lane >> 3, b = lane & 7;
  const ImgDesc& d = L.one;
  const int W = d.W;
  const long long plane_px = (long long)d.H * W;      // stacked plane
  const int r = (L.window - 1) / 2, K = L.K;
  const int n_all = v.T * v.n_ref_frame;
  for (int ref = blockIdx.x * 4 + wv; ref < n_all; ref += gridDim.x * 4) {
    const int t = ref / v.n_ref_frame, n = ref - t * v.n_ref_frame;
    const int ry = ref_coord(n / v.nrx, L.stride, v.Hp), rx = ref_coord(n % v.nrx, L.stride, v.Wp);
    const int prow = t * v.H + ry;                     // stacked row of the reference
    // guide plane of the reference's kind
    int plane = 0;
    if (L.C == 3) {
      long long nr = 0, ng = 0, nb = 0;
      const long long o = (long long)(prow + a) * W + rx + b;
      const long long qr = quantize(d.img[o]), qg = quantize(d.img[plane_px + o]),
                      qb = quantize(d.img[2 * plane_px + o]);
      nr = qr * qr;
      ng = qg * qg;
      nb = qb * qb;
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) {
        nr += __shfl_xor(nr, m, 64);
        ng += __shfl_xor(ng, m, 64);
        nb += __shfl_xor(nb, m, 64);
      }
      const long long lhs = (long long)L.gcp_num * L.gcp_num * ng;
      const long long rhs = (long long)L.gcp_den * L.gcp_den * (nr > nb ? nr : nb);
      plane = lhs >= rhs ? 0 : 1;
    }
    const int* g = d.gplanes + (size_t)plane * plane_px;
    refp[wv][lane] = g[(size_t)(prow + a) * W + rx + b];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    int rv[64];
#pragma unroll
    for (int q = 0; q < 64; ++q) rv[q] = refp[wv][q];
    const int t0 = max(0, t - v.dt), t1 = min(v.T - 1, t + v.dt);
    const int y0 = max(0, ry - r), y1 = min(v.Hp - 1, ry + r);
    const int x0 = max(0, rx - r), x1 = min(v.Wp - 1, rx + r);
    const int wx = x1 - x0 + 1, ncf = (y1 - y0 + 1) * wx, nc = (t1 - t0 + 1) * ncf;
    unsigned long long best = ~0ull;   // the 64 smallest merged keys, ascending over the lanes
    unsigned long long thr = ~0ull;    // the (K-1)-th smallest merged key
    int nbuf = 0;                      // keys in kbuf[wv] (wavefront-uniform)
    // merge the buffer into best and lower the threshold
    auto merge = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      unsigned long long key[2] = {best, lane < nbuf ? kbuf[wv][lane] : ~0ull};
      wave_sort_u64<2>(key);
      best = key[0];
      thr = lane_u64(best, K - 2);
      nbuf = 0;
      __builtin_amdgcn_wave_barrier();   // the buffer is rewritten after the reads
    };
    for (int c0 = 0; c0 < nc; c0 += 64) {
      const int c = c0 + lane;
      unsigned long long kk = ~0ull;
      if (c < nc) {
        const int tf = c / ncf, rem = c - tf * ncf;
        const int t2 = t0 + tf, cy = y0 + rem / wx, cx = x0 + rem % wx;
        if (!(t2 == t && cy == ry && cx == rx)) {
          const int* cp = g + (size_t)(t2 * v.H + cy) * W + cx;
          long long dd = 0;
#pragma unroll
          for (int aa = 0; aa < PS; ++aa)
#pragma unroll
            for (int bb = 0; bb < PS; ++bb) {
              const int df = cp[aa * W + bb] - rv[aa * 8 + bb];
              dd += (long long)df * df;
            }
          kk = ((unsigned long long)dd << 12) | (unsigned)c;
        }
      }
      unsigned long long m = __ballot(kk < thr);
      if (nbuf + __popcll(m) > 64) {
        merge();
        m = __ballot(kk < thr);
      }
      if (kk < thr) {
        const int slot = nbuf + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        kbuf[wv][slot] = kk;
      }
      nbuf += __popcll(m);
    }
    if (nbuf > 0) merge();
    // best on lane i: the i-th smallest (distance, ordinal)
    int* row = d.idx + (size_t)ref * K;
    if (lane == 0) {
      row[0] = prow * W + rx;
      if (d.dist) d.dist[(size_t)ref * K] = 0;
    }
    if (lane < K - 1) {
      const int c = (int)(best & 0xFFFull);
      const int tf = c / ncf, rem = c - tf * ncf;
      const int t2 = t0 + tf, cy = y0 + rem / wx, cx = x0 + rem % wx;
      row[1 + lane] = (t2 * v.H + cy) * W + cx;
      if (d.dist) d.dist[(size_t)ref * K + 1 + lane] = (long long)(best >> 12);
    }
    __builtin_amdgcn_wave_barrier();   // refp[wv] is rewritten by the next reference
  }
}

hipError_t launch_match_video(const Launch& L, const VideoGeo& v, hipStream_t s) {
  const int n_all = v.T * v.n_ref_frame;
  const int grid = std::max(1, std::min((n_all + 3) / 4, 8192));
  hipLaunchKernelGGL(k_match_video, dim3(grid), dim3(256), 0, s, L, v);
  return hipGetLastError();
}

}  // namespace hts
