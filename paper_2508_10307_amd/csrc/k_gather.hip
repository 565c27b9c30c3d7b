// Aggregation (Eq. 2; Alg. 1 Step 3) of exported slot estimates, for groups
// whose patches may lie anywhere in the image (the stacked frames of a
// video, where a group takes patches from several frames and no window tile
// covers them).  The filter writes every slot's estimate to its record
// est[s][ch][8][8] (s = g K + k, in the integer-unit encoding of the
// numerator: scaled, and for c = 3 the channel-DFT triples); then
//  1. the slots are bucketed by their patch corner: an exclusive scan of
//     the corner histogram (hist, the same counts the coverage uses) gives
//     each corner's first entry, and one pass writes every slot id into its
//     corner's bucket (the order inside a bucket is arbitrary);
//  2. one work group per output tile sums, in LDS and 64-bit fixed point,
//     the estimates of every slot whose corner lies up to 7 pixels above or
//     left of the tile.  Those slots are, per corner row, one contiguous run
//     of buckets.  The tile then stores its sums into the numerator.
// Integer sums do not depend on the order of the additions, so the result
// is the same, bit for bit, as adding every estimate with atomics.
#include "hts_device.h"
#include "video_internal.h"

namespace hts {

constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_BLOCK = 256 * SCAN_PER_THREAD;   // entries per scan work group

// Exclusive scan of one value per thread over a work group of 256 threads;
// *total receives the sum (every thread).
__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();   // sh may still be read by a previous call
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  int wbase = 0, t = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    wbase += w < wave ? sh[w] : 0;
    t += sh[w];
  }
  *total = t;
  return wbase + x - v;
}

// offs[i] = sum of cnt[0..i) within each block of SCAN_BLOCK entries;
// bsum[block] = the block's total.
__global__ __launch_bounds__(256) void k_scan_block(const int* cnt, int* offs, int* bsum, int n) {
  __shared__ int sh[8];
  const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  int v[SCAN_PER_THREAD];
  int t = 0;
#pragma unroll
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    v[i] = base + i < n ? cnt[base + i] : 0;
    t += v[i];
  }
  int total;
  int run = block_exclusive_scan(t, sh, &total);
#pragma unroll
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    if (base + i < n) offs[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the nb block totals in one work group (nb <= 256 * 64).
__global__ __launch_bounds__(256) void k_scan_sums(int* bsum, int nb) {
  __shared__ int sh[8];
  constexpr int PER = 64;
  const int base = threadIdx.x * PER;
  int t = 0;
  for (int i = 0; i < PER; ++i) t += base + i < nb ? bsum[base + i] : 0;
  int total;
  int run = block_exclusive_scan(t, sh, &total);
  for (int i = 0; i < PER; ++i) {
    if (base + i < nb) {
      const int v = bsum[base + i];
      bsum[base + i] = run;
      run += v;
    }
  }
}

__global__ __launch_bounds__(256) void k_scan_add(int* offs, const int* bsum, int n) {
  const int base = blockIdx.x * SCAN_BLOCK;
  const int add = bsum[blockIdx.x];
  for (int i = threadIdx.x; i < SCAN_BLOCK; i += 256)
    if (base + i < n) offs[base + i] += add;
}

// list[offs[corner] + arrival] = s for every slot s of the n_slots slots;
// cursor[] counts the arrivals per corner (zeroed by the caller).
__global__ __launch_bounds__(256) void k_fill_buckets(const int* idx, int n_slots, int W, int Hp,
                                                      int Wp, const int* offs, int* cursor,
                                                      int* list) {
  const float rW = 1.0f / (float)W;
  for (int s = blockIdx.x * 256 + threadIdx.x; s < n_slots; s += gridDim.x * 256) {
    int py, px;
    split_pos(idx[s], W, rW, py, px);
    py = min(max(py, 0), Hp - 1);
    px = min(max(px, 0), Wp - 1);
    const int pos = py * W + px;
    list[offs[pos] + atomicAdd(cursor + pos, 1)] = s;
  }
}

constexpr int GT_Y = 32, GT_X = 64, GT_XP = GT_X + 8;   // output tile (LDS pitch padded)
constexpr int GT_WAVES = 8;                            // 512 threads
constexpr int GT_SLOTS = 4;                            // slots per wavefront and pass

// One work group per GT_Y x GT_X tile of the image: lane = pixel (r, c) of a
// patch; each wavefront takes GT_SLOTS slots at a time (loads first, then
// the LDS additions), so that enough estimate loads are in flight.
template <int C>
__global__ __launch_bounds__(512) void k_gather_tiles(Launch L, const float* est, const int* offs,
                                                      const int* list) {
  __shared__ unsigned long long acc[C][GT_Y][GT_XP];
  const ImgDesc& d = L.one;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane >> 3, c = lane & 7;
  const int ntx = (d.W + GT_X - 1) / GT_X;
  const int y0 = (blockIdx.x / ntx) * GT_Y, x0 = (blockIdx.x % ntx) * GT_X;
  for (int e = threadIdx.x; e < C * GT_Y * GT_XP; e += 512) (&acc[0][0][0])[e] = 0ull;
  __syncthreads();
  const int cy0 = max(0, y0 - (PS - 1)), cy1 = min(d.Hp - 1, y0 + GT_Y - 1);
  const int xa = max(0, x0 - (PS - 1)), xb = min(d.Wp - 1, x0 + GT_X - 1);
  const size_t HW = (size_t)d.H * d.W;
  const float rW = 1.0f / (float)d.W;
  for (int cy = cy0; cy <= cy1 && xa <= xb; ++cy) {
    const int pa = cy * d.W + xa, pb = cy * d.W + xb;
    const int s0 = offs[pa], s1 = offs[pb] + d.hist[pb];
    for (int s = s0 + wave * GT_SLOTS; s < s1; s += GT_WAVES * GT_SLOTS) {
      float v[GT_SLOTS][C];
      int ly[GT_SLOTS], lx[GT_SLOTS];
      bool in[GT_SLOTS];
#pragma unroll
      for (int u = 0; u < GT_SLOTS; ++u) {
        const bool ok = s + u < s1;
        const int slot = list[ok ? s + u : s0];
        int qy, qx;                          // the corner (clamped as in the bucketing): row cy
        split_pos(d.idx[slot], d.W, rW, qy, qx);
        qx = min(max(qx, 0), d.Wp - 1);
        ly[u] = cy + r - y0;
        lx[u] = qx + c - x0;
        in[u] = ok && ly[u] >= 0 && ly[u] < GT_Y && lx[u] >= 0 && lx[u] < GT_X;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) v[u][ch] = est[((size_t)slot * C + ch) * PS2 + lane];
      }
#pragma unroll
      for (int u = 0; u < GT_SLOTS; ++u)
        if (in[u])
#pragma unroll
          for (int ch = 0; ch < C; ++ch) atomicAdd(&acc[ch][ly[u]][lx[u]], fx_from_units(v[u][ch]));
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < C * GT_Y * GT_X; e += 512) {
    const int ch = e / (GT_Y * GT_X), rem = e - ch * (GT_Y * GT_X);
    const int yy = rem / GT_X, xx = rem - yy * GT_X;
    if (y0 + yy < d.H && x0 + xx < d.W)
      d.num64[ch * HW + (size_t)(y0 + yy) * d.W + x0 + xx] = acc[ch][yy][xx];
  }
}

size_t gather_scratch_ints(long long n_pix) {
  const long long nb = (n_pix + SCAN_BLOCK - 1) / SCAN_BLOCK;
  return (size_t)(2 * n_pix + nb);   // offsets, cursor, block sums
}

bool gather_supported(long long n_pix) {
  return (n_pix + SCAN_BLOCK - 1) / SCAN_BLOCK <= 256 * 64;
}

hipError_t launch_gather(const Launch& L, const float* est, int* scratch, int* list,
                         hipStream_t s) {
  const ImgDesc& d = L.one;
  const int n = d.H * d.W;
  const int nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
  if (nb > 256 * 64 || (L.C != 1 && L.C != 3)) return hipErrorInvalidValue;
  int* offs = scratch;
  int* cursor = scratch + n;
  int* bsum = scratch + 2 * (size_t)n;
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(256), 0, s, d.hist, offs, bsum, n);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, s, offs, bsum, n);
  const hipError_t e = launch_fill((float*)cursor, n, 0.f, s);   // zero bits
  if (e != hipSuccess) return e;
  const int n_slots = d.n_ref * L.K;
  const int g = std::min((n_slots + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill_buckets, dim3(g), dim3(256), 0, s, d.idx, n_slots, d.W, d.Hp, d.Wp,
                     offs, cursor, list);
  const int tiles = ((d.H + GT_Y - 1) / GT_Y) * ((d.W + GT_X - 1) / GT_X);
  if (L.C == 1) hipLaunchKernelGGL(k_gather_tiles<1>, dim3(tiles), dim3(512), 0, s, L, est, offs, list);
  else hipLaunchKernelGGL(k_gather_tiles<3>, dim3(tiles), dim3(512), 0, s, L, est, offs, list);
  return hipGetLastError();
}

}  // namespace hts
