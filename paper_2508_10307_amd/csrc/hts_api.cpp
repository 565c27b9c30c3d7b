// Host side of the C ABI (include/hts.h): argument validation, workspace
// carving, launch sequences, batched persistent launches captured into HIP
// graphs, and the launch-schedule autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hts_internal.h"
#include "video_internal.h"

using namespace hts;

namespace {

constexpr size_t ALIGN = 256;
inline size_t al(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Filter tile shapes the schedule may pick (references per tile).
constexpr FiltShape kShapes[] = {{8, 8}, {8, 4}, {4, 8}, {4, 4}, {4, 2}, {2, 4}, {2, 2}, {2, 1}, {1, 1}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
constexpr size_t kFilterLdsBudget = 80 * 1024;   // two work groups per CU
constexpr size_t kLdsMax = 160 * 1024;

struct Geo {
  int C, H, W, Hp, Wp, nry, nrx, n_ref, n_cov, np;
  int K;
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Work groups of the band-count filter for n groups (one wavefront each):
// each holds its own scratch (K * C * 64 floats), kept within about 1 GB;
// at least one work group per CU and at most GEN_GRID, enough to fill every
// SIMD's wavefront slots, which hides the latency of the kernel's LDS and
// scratch round trips.
int gen_filter_grid(int n, int K, int C) {
  const size_t per = (size_t)K * C * 64 * 4;
  const int cap = (int)std::max<size_t>(256, std::min<size_t>(GEN_GRID, ((size_t)1 << 30) / per));
  return std::max(1, std::min(n, cap));
}

bool weighted(const hts_params* p) { return (p->flags & HTS_FLAG_WEIGHTED) != 0; }
bool fourier(const hts_params* p, int C) { return C == 3 && (p->flags & HTS_FLAG_FOURIER_THRESHOLD) != 0; }

hts_status check_params(const hts_params* p, int C) {
  if (!p) return HTS_ERR_INVALID;
  if (p->ps != PS) return HTS_ERR_UNSUPPORTED;
  if (C < 1 || C > GEN_CMAX) return HTS_ERR_UNSUPPORTED;
  if (!is_pow2(p->K) || p->K < 2 || p->K > 64) return HTS_ERR_INVALID;
  if (C == 3 && p->K > 32) return HTS_ERR_UNSUPPORTED;
  if (p->stride < 1 || p->stride > PS) return HTS_ERR_INVALID;
  if (p->window < 3 || p->window > MAX_WINDOW || (p->window & 1) == 0) return HTS_ERR_INVALID;
  if (!(p->tau_mult >= 0.f) || !std::isfinite(p->tau_mult)) return HTS_ERR_INVALID;
  if (p->gcp_num < 1 || p->gcp_num > 64 || p->gcp_den < 1 || p->gcp_den > 64) return HTS_ERR_INVALID;
  if (p->match_mode != HTS_MATCH_BF16 && p->match_mode != HTS_MATCH_FP32) return HTS_ERR_INVALID;
  if ((p->flags & ~(HTS_FLAG_WEIGHTED | HTS_FLAG_FOURIER_THRESHOLD)) != 0) return HTS_ERR_INVALID;
  if ((size_t)match_lds_bytes(p->stride, p->window) > kLdsMax) return HTS_ERR_UNSUPPORTED;
  if (general_c(C)) {   // spectral tubes: uniform Eq. 2 and Eq. 19 only
    if (p->K > GEN_KMAX || p->flags) return HTS_ERR_UNSUPPORTED;
    if (filter_gen_lds_bytes(C) > kLdsMax || cov_gen_lds_bytes(C) > kLdsMax) return HTS_ERR_UNSUPPORTED;
    return HTS_OK;
  }
  if (filter_lds_bytes(C, p->K, p->stride, p->window, 1, 1, weighted(p)) > kLdsMax)
    return HTS_ERR_UNSUPPORTED;
  return HTS_OK;
}

hts_status make_geo(const hts_params* p, int C, int H, int W, Geo& g) {
  hts_status st = check_params(p, C);
  if (st != HTS_OK) return st;
  if (H < PS || W < PS) return HTS_ERR_INVALID;
  if ((long long)C * H * W >= (1LL << 31)) return HTS_ERR_UNSUPPORTED;
  g.C = C; g.H = H; g.W = W; g.K = p->K;
  g.Hp = H - PS + 1; g.Wp = W - PS + 1;
  g.nry = ref_count_axis(g.Hp, p->stride);
  g.nrx = ref_count_axis(g.Wp, p->stride);
  g.n_ref = g.nry * g.nrx;
  {
    const int tr = cov_tile(p->stride);
    g.n_cov = ((g.nry + tr - 1) / tr) * ((g.nrx + tr - 1) / tr);
  }
  g.np = C == 3 ? 2 : 1;
  const int r = (p->window - 1) / 2;
  // every reference must have at least K candidates (the corner ones have fewest)
  if ((long long)std::min(g.Hp, r + 1) * std::min(g.Wp, r + 1) < p->K) return HTS_ERR_INVALID;
  if ((long long)g.n_ref * p->K >= (1LL << 31)) return HTS_ERR_UNSUPPORTED;
  return HTS_OK;
}

// Workspace carve-up for one image.
struct Carve {
  size_t gplanes, green, idx, fb_list, fb_count, cov, basis64, basis, fbasis, num, num64, cnt, hist,
      poison, fxmax, wsum64, gbasis, rowp, ufg, gscratch, total;
};

Carve carve(const Geo& g) {
  Carve c;
  size_t o = 0;
  c.gplanes = o; o += al((size_t)g.np * g.H * g.W * 4);
  c.green = o; o += al((size_t)g.n_ref);
  c.idx = o; o += al((size_t)g.n_ref * g.K * 4);
  c.fb_list = o; o += al((size_t)g.n_ref * 4);
  c.fb_count = o; o += al(4);
  c.cov = o; o += al((size_t)g.n_cov * cov_elems(g.C) * 8);
  c.basis64 = o; o += al((size_t)(2 * g.C * 64 + 2 * (g.C / 2 + 1) * 8) * 8);
  c.basis = o; o += al((size_t)2 * g.C * 64 * 4);
  c.fbasis = o; o += al((size_t)std::max(FB_SIZE, 2 * n_freq(g.C) * 128) * 4);
  c.num = o; o += al((size_t)g.C * g.H * g.W * 4);
  c.cnt = o; o += al((size_t)g.H * g.W * 4);
  c.hist = o; o += al((size_t)g.H * g.W * 4);
  c.num64 = o; o += al((size_t)g.C * g.H * g.W * 8);
  c.poison = o; o += al((size_t)g.H * g.W);
  c.fxmax = o; o += al(4);
  c.wsum64 = o; o += al((size_t)g.H * g.W * 8);
  c.gbasis = o; o += al((size_t)4 * 128 * 8);   // covariance cotangents of the basis derivative
  const bool gen = general_c(g.C);
  c.rowp = o; o += gen ? 0 : al((size_t)g.H * g.Wp * rowp_floats(g.C) * 4);
  c.ufg = o; o += gen ? al((size_t)2 * n_freq(g.C) * 128 * 8) : 0;
  c.gscratch = o;
  o += gen ? al((size_t)gen_filter_grid(g.n_ref, g.K, g.C) * g.K * g.C * 64 * 4) : 0;
  c.total = o;
  return c;
}

void fill_counts(const Geo& g, const hts_params* p, int fty, int ftx, ImgDesc& d) {
  d.wcnt[W_PIX] = (g.H * g.W + PIX_CHUNK - 1) / PIX_CHUNK;
  d.wcnt[W_REF] = (g.n_ref + 255) / 256;
  d.wcnt[W_MATCH] = ((g.nry + MATCH_TY - 1) / MATCH_TY) * ((g.nrx + MATCH_TX - 1) / MATCH_TX);
  d.wcnt[W_COV] = g.n_cov;
  d.wcnt[W_FILT] = ((g.nry + fty - 1) / fty) * ((g.nrx + ftx - 1) / ftx);
  d.wcnt[W_BOX] = ((g.H + BOX_TY - 1) / BOX_TY) * ((g.W + BOX_TX - 1) / BOX_TX);
  for (int k = 0; k < W_NKIND; ++k) d.woff[k] = 0;
  (void)p;
}

ImgDesc make_desc(const Geo& g, const hts_params* p, char* ws, const Carve& c, const float* img,
                  float sigma, int fty, int ftx) {
  ImgDesc d;
  std::memset(&d, 0, sizeof(d));
  d.img = img;
  d.gplanes = (int32_t*)(ws + c.gplanes);
  d.green = (uint8_t*)(ws + c.green);
  d.idx = (int32_t*)(ws + c.idx);
  d.fb_list = (int32_t*)(ws + c.fb_list);
  d.fb_count = (int32_t*)(ws + c.fb_count);
  d.cov_part = (double*)(ws + c.cov);
  d.basis64 = (double*)(ws + c.basis64);
  d.basis = (float*)(ws + c.basis);
  d.fbasis = (float*)(ws + c.fbasis);
  d.num = (float*)(ws + c.num);
  d.cnt = (float*)(ws + c.cnt);
  d.hist = (int32_t*)(ws + c.hist);
  d.num64 = (unsigned long long*)(ws + c.num64);
  d.poison = (uint8_t*)(ws + c.poison);
  d.fxmax = (uint32_t*)(ws + c.fxmax);
  d.wsum64 = weighted(p) ? (unsigned long long*)(ws + c.wsum64) : nullptr;
  d.ufg = general_c(g.C) ? (double*)(ws + c.ufg) : nullptr;
  d.gscratch = general_c(g.C) ? (float*)(ws + c.gscratch) : nullptr;
  d.rowp = general_c(g.C) ? nullptr : (float*)(ws + c.rowp);
  d.H = g.H; d.W = g.W; d.Hp = g.Hp; d.Wp = g.Wp;
  d.nry = g.nry; d.nrx = g.nrx; d.n_ref = g.n_ref;
  d.ref_begin = 0; d.ref_count = g.n_ref;
  d.sigma = sigma;
  d.tau = p->tau_mult * sigma;
  d.n_cov = g.n_cov;
  fill_counts(g, p, fty, ftx, d);
  return d;
}

Launch make_launch(const hts_params* p, int C, const ImgDesc& d, int kind, int fty, int ftx) {
  Launch L;
  std::memset(&L, 0, sizeof(L));
  L.one = d;
  L.table = nullptr;
  L.n_img = 1;
  L.total = kind >= 0 ? d.wcnt[kind] : 1;
  L.C = C; L.K = p->K; L.stride = p->stride; L.window = p->window;
  L.tau_mult = p->tau_mult;
  L.gcp_num = p->gcp_num; L.gcp_den = p->gcp_den;
  L.flags = p->flags;
  L.fty = fty; L.ftx = ftx;
  return L;
}

// ---- launch schedule (tune word) ----
// bits 0-3: filter tile shape index + 1 (0 = largest shape within the LDS budget)
// bits 4-5: BF16 match terms (0 = default 3, 1 = one product, 2 = hi/lo split)
// bits 6-7: filter implementation (0 = FP32 MFMA where built, 1 = vector ALU)
struct Schedule { int fty, ftx, terms, valu; };

int tuned_word(const hts_params* p, int C);

// LDS bytes of the filter implementation for a tile shape, and the LDS a
// work group may take: the MFMA filter at K = 32 runs one work group per CU
// (register bound), every other variant two.
size_t filter_impl_lds(const hts_params* p, int C, bool valu, int ty, int tx) {
  return valu ? filter_lds_bytes(C, p->K, p->stride, p->window, ty, tx, weighted(p))
              : filter_mfma_lds_bytes(p->stride, p->window, ty, tx);
}
size_t filter_impl_budget(const hts_params* p, bool valu) {
  return !valu && p->K >= 32 ? kLdsMax : kFilterLdsBudget;
}

Schedule schedule_for(const hts_params* p, int C) {
  Schedule s;
  const int tune = p->tune ? p->tune : tuned_word(p, C);
  // the weighted aggregation and the Fourier threshold are built into the
  // vector-ALU filter only
  s.valu = ((tune >> 6) & 3) == 1 || !filter_mfma_supported(C, p->K) || weighted(p) ||
           fourier(p, C);
  int si = (tune & 15) - 1;
  // a tune word chosen without the weight plane may no longer fit beside a
  // second work group: then the largest shape that does
  if (si < 0 || si >= kNumShapes ||
      filter_impl_lds(p, C, s.valu, kShapes[si].ty, kShapes[si].tx) > kLdsMax ||
      (weighted(p) &&
       filter_impl_lds(p, C, s.valu, kShapes[si].ty, kShapes[si].tx) > filter_impl_budget(p, s.valu))) {
    si = kNumShapes - 1;
    for (int i = 0; i < kNumShapes; ++i)
      if (filter_impl_lds(p, C, s.valu, kShapes[i].ty, kShapes[i].tx) <= filter_impl_budget(p, s.valu)) { si = i; break; }
  }
  s.fty = kShapes[si].ty;
  s.ftx = kShapes[si].tx;
  const int t = (tune >> 4) & 3;
  s.terms = t == 1 ? 1 : 3;
  return s;
}

#define HIPCHK(x) do { if ((x) != hipSuccess) return HTS_ERR_HIP; } while (0)

// count_hist: the match also builds the coverage histogram (d.hist) of the
// groups it forms.
hts_status run_match(const hts_params* p, int C, const Schedule& sc, ImgDesc d, hipStream_t s,
                     bool count_hist = false) {
  auto LM = [&](int kind) {
    Launch L = make_launch(p, C, d, kind, sc.fty, sc.ftx);
    L.count_hist = count_hist ? 1 : 0;
    return L;
  };
  HIPCHK(launch_reset_counters(LM(-1), s));
  HIPCHK(launch_quant(LM(W_PIX), 0, s));
  HIPCHK(launch_gcp(LM(W_REF), 0, s));
  HIPCHK(launch_match(LM(W_MATCH), p->match_mode, sc.terms, 0, s));
  HIPCHK(launch_match_fallback(LM(-1), 256, s));
  return HTS_OK;
}

hts_status run_basis(const hts_params* p, int C, const Schedule& sc, ImgDesc d, hipStream_t s) {
  if (general_c(C)) {
    HIPCHK(launch_basis_gen(make_launch(p, C, d, -1, sc.fty, sc.ftx), s));
    return HTS_OK;
  }
  HIPCHK(launch_cov(make_launch(p, C, d, W_COV, sc.fty, sc.ftx), 0, s));
  HIPCHK(launch_eig(make_launch(p, C, d, -1, sc.fty, sc.ftx), s));
  return HTS_OK;
}

// Coverage counts of references [ref_begin, ref_begin+ref_count) added into
// d.cnt: histogram of the groups' patch corners (unless the match already
// built it), then its 8x8 box sum.
hts_status run_count(const hts_params* p, int C, const Schedule& sc, const ImgDesc& d,
                     bool hist_ready, hipStream_t s) {
  if (!hist_ready) {
    HIPCHK(launch_zero_hist(make_launch(p, C, d, W_PIX, sc.fty, sc.ftx), 0, s));
    HIPCHK(launch_count_hist(make_launch(p, C, d, W_REF, sc.fty, sc.ftx), 0, s));
  }
  HIPCHK(launch_count_box(make_launch(p, C, d, W_BOX, sc.fty, sc.ftx), 0, s));
  return HTS_OK;
}

// U, V (nullable): a caller's basis to use instead of the workspace copy.
// hist_ready: d.hist already holds the coverage histogram of these groups.
hts_status run_filter(const hts_params* p, int C, const Schedule& sc, ImgDesc d, int adjoint,
                      hipStream_t s, const float* U = nullptr, const float* V = nullptr,
                      bool hist_ready = false) {
  if (general_c(C)) {   // the spectral-tube filter
    const size_t nb = (size_t)C * PS2 * sizeof(float);
    if (U) HIPCHK(hipMemcpyAsync(d.basis, U, nb, hipMemcpyDeviceToDevice, s));
    if (V) HIPCHK(hipMemcpyAsync(d.basis + C * PS2, V, nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_fbasis_gen(make_launch(p, C, d, -1, sc.fty, sc.ftx), s));
    const Launch Lf = make_launch(p, C, d, W_FILT, sc.fty, sc.ftx);
    const int gg = gen_filter_grid(d.ref_count, p->K, C);
    if (adjoint) HIPCHK(launch_filter_gen_adj(Lf, gg, s));
    else HIPCHK(launch_filter_gen(Lf, gg, s));
    if (d.cnt) return run_count(p, C, sc, d, hist_ready, s);
    return HTS_OK;
  }
  HIPCHK(launch_fbasis(make_launch(p, C, d, -1, sc.fty, sc.ftx), U, V, s));
  if (sc.valu) HIPCHK(launch_rowproj(make_launch(p, C, d, W_PIX, sc.fty, sc.ftx), 0, s));
  const Launch L = make_launch(p, C, d, W_FILT, sc.fty, sc.ftx);
  if (sc.valu) HIPCHK(launch_filter(L, sc.fty, sc.ftx, adjoint, 0, s));
  else HIPCHK(launch_filter_mfma(L, sc.fty, sc.ftx, adjoint, 0, s));
  // weighted without a fixed-point weight plane: the filter adds the weight
  // sums into cnt itself
  if (!adjoint && d.cnt && !(weighted(p) && !d.wsum64)) return run_count(p, C, sc, d, hist_ready, s);
  return HTS_OK;
}

// ---------------------------------------------------------------- devices
int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cus[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

// ---------------------------------------------------------------- autotune cache
// key: device arch + the parameters a schedule depends on; value: tune word.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "gfx?";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string tune_key(const hts_params* p, int C) {
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s C=%d s=%d w=%d K=%d mode=%d flags=%d", arch_name().c_str(), C,
                p->stride, p->window, p->K, p->match_mode, p->flags);
  return buf;
}

int tuned_word(const hts_params* p, int C) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune.empty()) return 0;
  auto it = g_tune.find(tune_key(p, C));
  return it == g_tune.end() ? 0 : it->second;
}

void load_cache_file(const char* path) {
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    char* bar = std::strrchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    const int w = std::atoi(bar + 1);
    if (w > 0) g_tune[line] = w;     // corrupt or zero entries are ignored
  }
  std::fclose(f);
}

// ---------------------------------------------------------------- batches
struct BatchPlan {
  std::vector<ImgDesc> descs;   // n entries
  int totals[W_NKIND];
  size_t table_off, bytes;
  Schedule sc;
};

hts_status plan_batch(const hts_params* p, const hts_image* imgs, int n, char* base, bool check_ptrs,
                      BatchPlan& plan) {
  if (!p || !imgs || n < 1) return HTS_ERR_INVALID;
  const int C = imgs[0].C;
  hts_status st = check_params(p, C);
  if (st != HTS_OK) return st;
  if (general_c(C)) return HTS_ERR_UNSUPPORTED;   // spectral tubes: single-image calls only
  plan.sc = schedule_for(p, C);
  plan.descs.assign(n, ImgDesc());
  for (int k = 0; k < W_NKIND; ++k) plan.totals[k] = 0;
  size_t off = 0;
  plan.table_off = off;
  off += al((size_t)n * sizeof(ImgDesc));
  for (int i = 0; i < n; ++i) {
    const hts_image& im = imgs[i];
    if (im.C != C) return HTS_ERR_INVALID;
    if (!(im.sigma >= 0.f) || !std::isfinite(im.sigma)) return HTS_ERR_INVALID;
    if (check_ptrs && (!im.noisy || !im.out)) return HTS_ERR_INVALID;
    Geo g;
    st = make_geo(p, C, im.H, im.W, g);
    if (st != HTS_OK) return st;
    const Carve c = carve(g);
    ImgDesc d = make_desc(g, p, base ? base + off : nullptr, c, im.noisy, im.sigma, plan.sc.fty,
                          plan.sc.ftx);
    d.out = im.out;
    for (int k = 0; k < W_NKIND; ++k) {
      d.woff[k] = plan.totals[k];
      if ((long long)plan.totals[k] + d.wcnt[k] >= (1LL << 31)) return HTS_ERR_UNSUPPORTED;
      plan.totals[k] += d.wcnt[k];
    }
    plan.descs[i] = d;
    off += c.total;
  }
  plan.bytes = off;
  return HTS_OK;
}

Launch batch_launch(const hts_params* p, int C, const ImgDesc* table, int n, int total, const Schedule& sc) {
  Launch L;
  std::memset(&L, 0, sizeof(L));
  L.table = table;
  L.n_img = n;
  L.total = total;
  L.C = C; L.K = p->K; L.stride = p->stride; L.window = p->window;
  L.tau_mult = p->tau_mult;
  L.gcp_num = p->gcp_num; L.gcp_den = p->gcp_den;
  L.flags = p->flags;
  L.fty = sc.fty; L.ftx = sc.ftx;
  return L;
}

// Second stream and fork/join events of the batch pipeline, per device,
// created on first use (default priority); side == nullptr if creation
// failed, and the pipeline then runs on one stream.  Callers hold
// g_graph_mu.
struct Branch {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
Branch branch_for_device() {
  static Branch br[64];
  static bool tried[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return Branch();
  if (!tried[dev]) {
    tried[dev] = true;
    Branch b;
    if (hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&b.join, hipEventDisableTiming) == hipSuccess) {
      br[dev] = b;
    } else {
      (void)hipGetLastError();
    }
  }
  return br[dev];
}

// All stages of Algorithm 1 over the batch, as persistent launches sized to
// the device (work groups loop over the global (image, item) list).
// ev (nullable, HTS_BATCH_STAGE_EVENTS hipEvent_t): recorded at the stage
// boundaries; then every stage runs on s (no side stream), in the order of
// the graph.
// save: the filter also writes every image's keep-masks (d.masks) and the
// basis is copied out to d.U_ext / d.V_ext.
hts_status enqueue_batch(const hts_params* p, int C, const BatchPlan& plan, const ImgDesc* table,
                         hipStream_t s, hipEvent_t const* ev = nullptr, bool save = false) {
  const int n = (int)plan.descs.size();
  const int cus = device_cus();
  const Schedule& sc = plan.sc;
  auto LK = [&](int kind) { return batch_launch(p, C, table, n, kind >= 0 ? plan.totals[kind] : 0, sc); };
  auto LC = [&](int kind) {   // stages that also build the coverage histogram
    Launch L = LK(kind);
    L.count_hist = 1;
    return L;
  };
  auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
  HIPCHK(mark(0));
  HIPCHK(launch_reset_counters(LK(-1), s));
  HIPCHK(launch_quant(LC(W_PIX), cus * 8, s));
  HIPCHK(launch_gcp(LK(W_REF), cus * 8, s));
  HIPCHK(mark(1));
  // The covariances depend on the images only: they run on a second stream
  // beside the match (a branch of the captured graph) and join after it.
  // Forked before quantisation instead, so that they also ran beside it and
  // GCP, they made the match 1.8x slower on MI355X (16 -> 29 ms on the
  // 64-image batch; measured, with the same results).  The eigen-solves (one
  // work group per image, a barrier-bound Jacobi) run after the join on
  // their own, so they hold none of the match's compute-unit slots.
  const Branch br = ev ? Branch() : branch_for_device();
  hipStream_t bs = s;
  if (br.side) {
    HIPCHK(hipEventRecord(br.fork, s));
    HIPCHK(hipStreamWaitEvent(br.side, br.fork, 0));
    bs = br.side;
  }
  HIPCHK(launch_match(LC(W_MATCH), p->match_mode, sc.terms, cus * 2, s));
  HIPCHK(mark(2));
  HIPCHK(launch_cov(LK(W_COV), cus * 4, bs));
  HIPCHK(mark(3));
  if (br.side) HIPCHK(hipEventRecord(br.join, bs));
  HIPCHK(launch_match_fallback(LC(-1), cus, s));
  if (plan.descs[0].n_samples > 0) HIPCHK(launch_vote(LK(-1), s));   // A-Haar-tSVD sigma
  HIPCHK(launch_zero_accum(LK(W_PIX), cus * 8, s));
  HIPCHK(launch_count_box(LK(W_BOX), cus * 8, s));
  if (br.side) HIPCHK(hipStreamWaitEvent(s, br.join, 0));
  HIPCHK(launch_eig(LK(-1), s));
  HIPCHK(launch_fbasis(LK(-1), nullptr, nullptr, s));
  if (save) HIPCHK(launch_copy_basis(LK(-1), 1, s));
  if (sc.valu) HIPCHK(launch_rowproj(LK(W_PIX), cus * 8, s));
  HIPCHK(mark(4));
  Launch Lf = LK(W_FILT);
  Lf.batch_masks = save ? 1 : 0;
  if (sc.valu) HIPCHK(launch_filter(Lf, sc.fty, sc.ftx, 0, cus * 2, s));
  else HIPCHK(launch_filter_mfma(Lf, sc.fty, sc.ftx, 0, cus * 2, s));
  HIPCHK(mark(5));
  HIPCHK(launch_finalize(LK(W_PIX), cus * 8, s));
  HIPCHK(mark(6));
  return HTS_OK;
}

// The frozen-map adjoint of every image of the batch (descriptors as
// hts_denoise_batch_backward builds them: img = the workspace buffer that
// receives r, num = grad_out, out = grad_in, idx / masks_in / cnt / U_ext /
// V_ext = the caller's state), in the order of hts_denoise_backward.
hts_status enqueue_batch_backward(const hts_params* p, int C, const BatchPlan& plan,
                                  const ImgDesc* table, hipStream_t s) {
  const int n = (int)plan.descs.size();
  const int cus = device_cus();
  const Schedule& sc = plan.sc;
  auto LK = [&](int kind) {
    Launch L = batch_launch(p, C, table, n, kind >= 0 ? plan.totals[kind] : 0, sc);
    L.adjoint = 1;
    return L;
  };
  HIPCHK(launch_reset_counters(LK(-1), s));          // fxmax = 0
  HIPCHK(launch_adjoint_prep(LK(W_PIX), cus * 8, s));  // r = g / cnt, max |r|
  HIPCHK(launch_zero_accum(LK(W_PIX), cus * 8, s));    // keeps the caller's cnt
  HIPCHK(launch_copy_basis(LK(-1), 0, s));
  HIPCHK(launch_fbasis(LK(-1), nullptr, nullptr, s));
  if (sc.valu) HIPCHK(launch_rowproj(LK(W_PIX), cus * 8, s));
  if (sc.valu) HIPCHK(launch_filter(LK(W_FILT), sc.fty, sc.ftx, 1, cus * 2, s));
  else HIPCHK(launch_filter_mfma(LK(W_FILT), sc.fty, sc.ftx, 1, cus * 2, s));
  HIPCHK(launch_finalize(LK(W_PIX), cus * 8, s));      // grad_in = numerator
  return HTS_OK;
}

// One captured graph per shape-set (parameters, image shapes, workspace);
// images' pointers and noise levels live in the device table and may change
// between replays.
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  hipEvent_t copied = nullptr;
  bool used = false;
  std::vector<ImgDesc> host;     // staging for the table upload
};
std::mutex g_graph_mu;
std::map<std::string, GraphEntry> g_graphs;
hipStream_t g_capture_stream[64] = {nullptr};

// The key holds the schedule the parameters resolve to (tile shape, filter
// implementation, distance-tile terms), not only the tune word: with
// tune = 0 the schedule comes from the autotune table, which hts_autotune
// (or a cache file) may change between calls, and a graph captured for the
// old schedule would launch the filter over the old tile grid.
std::string graph_key(const hts_params* p, const Schedule& sc, const hts_image* imgs, int n,
                      const void* ws, const char* tag) {
  std::string k = tag;
  k += "|";
  char buf[160];
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::snprintf(buf, sizeof(buf), "%d|%d %d %d %d %a %d %d %d %d|%d %d %d %d|%p|", dev, p->ps,
                p->stride, p->window, p->K, (double)p->tau_mult, p->gcp_num, p->gcp_den,
                p->match_mode, p->flags, sc.fty, sc.ftx, sc.valu, sc.terms, ws);
  k += buf;
  for (int i = 0; i < n; ++i) {
    std::snprintf(buf, sizeof(buf), "%dx%dx%d;", imgs[i].C, imgs[i].H, imgs[i].W);
    k += buf;
  }
  return k;
}

}  // namespace

extern "C" {

void hts_default_params(hts_params* p) {
  // flags is reserved (0)
  if (!p) return;
  p->ps = 8; p->stride = 3; p->window = 21; p->K = 16; p->tau_mult = 2.7f;
  p->gcp_num = 6; p->gcp_den = 5; p->match_mode = HTS_MATCH_BF16; p->flags = 0; p->tune = 0;
}

const char* hts_status_string(hts_status s) {
  switch (s) {
    case HTS_OK: return "ok";
    case HTS_ERR_INVALID: return "invalid argument";
    case HTS_ERR_UNSUPPORTED: return "unsupported configuration";
    case HTS_ERR_WORKSPACE: return "workspace too small";
    case HTS_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* hts_version(void) { return "hts 0.1 (gfx950)"; }

hts_status hts_ref_grid(int32_t H, int32_t W, const hts_params* p, int32_t* ny, int32_t* nx) {
  if (!p || !ny || !nx) return HTS_ERR_INVALID;
  if (p->stride < 1 || p->stride > PS || p->ps != PS) return p && p->ps != PS ? HTS_ERR_UNSUPPORTED : HTS_ERR_INVALID;
  if (H < PS || W < PS) return HTS_ERR_INVALID;
  *ny = ref_count_axis(H - PS + 1, p->stride);
  *nx = ref_count_axis(W - PS + 1, p->stride);
  return HTS_OK;
}

hts_status hts_workspace_size(const hts_params* p, int32_t C, int32_t H, int32_t W, size_t* bytes) {
  if (!bytes) return HTS_ERR_INVALID;
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  *bytes = carve(g).total;
  return HTS_OK;
}

hts_status hts_match(const hts_params* p, const float* noisy, int32_t C, int32_t H, int32_t W,
                     int32_t* idx, int64_t* dist, uint8_t* green, void* ws, size_t ws_bytes,
                     void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (!noisy || !idx || !ws) return HTS_ERR_INVALID;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  const Schedule sc = schedule_for(p, C);
  ImgDesc d = make_desc(g, p, (char*)ws, c, noisy, 0.f, sc.fty, sc.ftx);
  d.idx = idx;
  d.dist = (long long*)dist;
  if (green) d.green = green;
  return run_match(p, C, sc, d, (hipStream_t)stream);
}

hts_status hts_basis(const hts_params* p, const float* noisy, int32_t C, int32_t H, int32_t W,
                     float* U, float* V, double* U64, double* V64, double* eig, void* ws,
                     size_t ws_bytes, void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (!noisy || !U || !V || !ws) return HTS_ERR_INVALID;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  const Schedule sc = schedule_for(p, C);
  hipStream_t s = (hipStream_t)stream;
  ImgDesc d = make_desc(g, p, (char*)ws, c, noisy, 0.f, sc.fty, sc.ftx);
  st = run_basis(p, C, sc, d, s);
  if (st != HTS_OK) return st;
  const size_t nb = (size_t)C * 64;
  HIPCHK(hipMemcpyAsync(U, d.basis, nb * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(V, d.basis + nb, nb * 4, hipMemcpyDeviceToDevice, s));
  if (U64) HIPCHK(hipMemcpyAsync(U64, d.basis64, nb * 8, hipMemcpyDeviceToDevice, s));
  if (V64) HIPCHK(hipMemcpyAsync(V64, d.basis64 + nb, nb * 8, hipMemcpyDeviceToDevice, s));
  if (eig) HIPCHK(hipMemcpyAsync(eig, d.basis64 + 2 * nb, (size_t)2 * (C / 2 + 1) * 8 * 8, hipMemcpyDeviceToDevice, s));
  return HTS_OK;
}

hts_status hts_filter(const hts_params* p, const float* noisy, int32_t C, int32_t H, int32_t W,
                      float sigma, const int32_t* idx, const float* U, const float* V,
                      int32_t ref_begin, int32_t ref_count, float* num, float* cnt,
                      float* group_est, uint32_t* masks, void* ws, size_t ws_bytes, void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (!noisy || !idx || !U || !V || !ws) return HTS_ERR_INVALID;
  if ((num == nullptr) != (cnt == nullptr)) return HTS_ERR_INVALID;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return HTS_ERR_INVALID;
  if (ref_begin < 0 || ref_count < 0 || (long long)ref_begin + ref_count > g.n_ref) return HTS_ERR_INVALID;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  if (ref_count == 0) return HTS_OK;
  const Schedule sc = schedule_for(p, C);
  hipStream_t s = (hipStream_t)stream;
  ImgDesc d = make_desc(g, p, (char*)ws, c, noisy, sigma, sc.fty, sc.ftx);
  d.idx = const_cast<int32_t*>(idx);
  d.ref_begin = ref_begin;
  d.ref_count = ref_count;
  d.group_est = group_est;
  d.masks = masks;
  d.num64 = nullptr;      // estimates go to a float numerator (the caller's or scratch)
  d.poison = nullptr;
  d.wsum64 = nullptr;     // weighted: the weight sums go to cnt
  if (num) {
    d.num = num;
    d.cnt = cnt;
  } else {
    d.cnt = nullptr;      // no numerator asked for: no coverage counts either
  }
  if (fx_int_units(C, p->flags, 0)) {   // the scale of the filter's integer-unit tiles
    HIPCHK(launch_fill((float*)d.fxmax, 1, 0.f, s));
    HIPCHK(launch_absmax(make_launch(p, C, d, W_PIX, sc.fty, sc.ftx), 0, s));
  }
  return run_filter(p, C, sc, d, 0, s, U, V);
}

hts_status hts_aggregate(const hts_params* p, const float* group_est, const int32_t* idx,
                         int32_t ref_begin, int32_t ref_count, int32_t C, int32_t H, int32_t W,
                         float* num, float* cnt, float* out, void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (general_c(C)) return HTS_ERR_UNSUPPORTED;   // spectral tubes: hts_denoise, hts_match, hts_basis
  if (weighted(p)) return HTS_ERR_UNSUPPORTED;   // estimates carry no group weights
  if (!num || !cnt) return HTS_ERR_INVALID;
  if (group_est && !idx) return HTS_ERR_INVALID;
  if (ref_begin < 0 || ref_count < 0 || (long long)ref_begin + ref_count > g.n_ref) return HTS_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const Schedule sc = schedule_for(p, C);
  ImgDesc d;
  std::memset(&d, 0, sizeof(d));
  d.H = g.H; d.W = g.W; d.Hp = g.Hp; d.Wp = g.Wp; d.nry = g.nry; d.nrx = g.nrx; d.n_ref = g.n_ref;
  d.idx = const_cast<int32_t*>(idx);
  d.num = num; d.cnt = cnt; d.out = out;
  d.ref_begin = ref_begin; d.ref_count = ref_count;
  d.group_est = const_cast<float*>(group_est);
  fill_counts(g, p, sc.fty, sc.ftx, d);
  if (group_est && ref_count > 0) HIPCHK(launch_scatter_est(make_launch(p, C, d, -1, sc.fty, sc.ftx), s));
  if (out) HIPCHK(launch_finalize(make_launch(p, C, d, W_PIX, sc.fty, sc.ftx), 0, s));
  return HTS_OK;
}

hts_status hts_denoise(const hts_params* p, const float* noisy, int32_t C, int32_t H, int32_t W,
                       float sigma, float* out, int32_t* idx_out, uint32_t* masks_out,
                       float* U_out, float* V_out, float* cnt_out, void* ws, size_t ws_bytes,
                       void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (!noisy || !out || !ws) return HTS_ERR_INVALID;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return HTS_ERR_INVALID;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  const Schedule sc = schedule_for(p, C);
  hipStream_t s = (hipStream_t)stream;
  ImgDesc d = make_desc(g, p, (char*)ws, c, noisy, sigma, sc.fty, sc.ftx);
  if (idx_out) d.idx = idx_out;
  if (cnt_out) d.cnt = cnt_out;
  d.masks = masks_out;
  d.out = out;
  st = run_match(p, C, sc, d, s, true);
  if (st != HTS_OK) return st;
  st = run_basis(p, C, sc, d, s);
  if (st != HTS_OK) return st;
  HIPCHK(launch_zero_accum(make_launch(p, C, d, W_PIX, sc.fty, sc.ftx), 0, s));
  st = run_filter(p, C, sc, d, 0, s, nullptr, nullptr, true);
  if (st != HTS_OK) return st;
  HIPCHK(launch_finalize(make_launch(p, C, d, W_PIX, sc.fty, sc.ftx), 0, s));
  const size_t nb = (size_t)C * 64;
  if (U_out) HIPCHK(hipMemcpyAsync(U_out, d.basis, nb * 4, hipMemcpyDeviceToDevice, s));
  if (V_out) HIPCHK(hipMemcpyAsync(V_out, d.basis + nb, nb * 4, hipMemcpyDeviceToDevice, s));
  return HTS_OK;
}

static bool adapt_args_ok(int32_t n_samples, float beta) {
  return n_samples >= 1 && n_samples <= (1 << 20) && beta > 0.f && std::isfinite(beta);
}

hts_status hts_adapt_sigma(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                           int32_t W, const int32_t* idx, const int32_t* samples,
                           int32_t n_samples, float sigma_est, float beta, int32_t gamma,
                           int32_t* ranks, float* sigma_out, void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (general_c(C)) return HTS_ERR_UNSUPPORTED;   // spectral tubes: hts_denoise, hts_match, hts_basis
  if (!noisy || !idx || !samples || !sigma_out || !adapt_args_ok(n_samples, beta)) return HTS_ERR_INVALID;
  if (!(sigma_est >= 0.f) || !std::isfinite(sigma_est)) return HTS_ERR_INVALID;
  ImgDesc d;
  std::memset(&d, 0, sizeof(d));
  d.img = noisy;
  d.idx = const_cast<int32_t*>(idx);
  d.H = g.H; d.W = g.W; d.Hp = g.Hp; d.Wp = g.Wp;
  d.nry = g.nry; d.nrx = g.nrx; d.n_ref = g.n_ref;
  d.sigma = sigma_est;
  d.samples = samples;
  d.n_samples = n_samples;
  d.beta = beta;
  d.gamma = gamma;
  d.ranks = ranks;
  d.sigma_dev = sigma_out;
  Launch L;
  std::memset(&L, 0, sizeof(L));
  L.one = d;
  L.C = C; L.K = p->K; L.stride = p->stride; L.window = p->window;
  L.tau_mult = p->tau_mult;
  HIPCHK(launch_vote(L, (hipStream_t)stream));
  return HTS_OK;
}

hts_status hts_denoise_backward(const hts_params* p, const float* grad_out, const int32_t* idx,
                                const uint32_t* masks, const float* U, const float* V,
                                const float* cnt, int32_t C, int32_t H, int32_t W, float* grad_in,
                                float* grad_tau_mult, void* ws, size_t ws_bytes, void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (weighted(p)) return HTS_ERR_UNSUPPORTED;   // adjoint of the uniform average only
  if (fourier(p, C)) return HTS_ERR_UNSUPPORTED;  // masks of the real-domain threshold only
  if (!grad_out || !idx || !masks || !U || !V || !cnt || !grad_in || !ws) return HTS_ERR_INVALID;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  const Schedule sc = schedule_for(p, C);
  hipStream_t s = (hipStream_t)stream;
  ImgDesc d = make_desc(g, p, (char*)ws, c, grad_out, 0.f, sc.fty, sc.ftx);
  d.cnt = const_cast<float*>(cnt);
  // r = grad_out / cnt into the workspace image buffer (and max |r|)
  HIPCHK(launch_fill((float*)d.fxmax, 1, 0.f, s));
  HIPCHK(launch_adjoint_prep(make_launch(p, C, d, W_PIX, sc.fty, sc.ftx), 0, s));
  ImgDesc a = d;
  a.img = d.num;               // r
  a.num = nullptr;             // the adjoint accumulates in the fixed-point numerator
  a.cnt = nullptr;
  a.idx = const_cast<int32_t*>(idx);
  a.masks_in = masks;
  a.num_enc = NUM_FINE;        // the adjoint's numerator in 2^-32 units
  HIPCHK(launch_zero_accum(make_launch(p, C, a, W_PIX, sc.fty, sc.ftx), 0, s));
  st = run_filter(p, C, sc, a, 1, s, U, V);
  if (st != HTS_OK) return st;
  a.out = grad_in;             // grad_in = numerator (no division)
  HIPCHK(launch_finalize(make_launch(p, C, a, W_PIX, sc.fty, sc.ftx), 0, s));
  if (grad_tau_mult) HIPCHK(launch_fill(grad_tau_mult, 1, 0.f, s));
  return HTS_OK;
}

hts_status hts_denoise_grad_tau(const hts_params* p, const float* noisy, const float* grad_out,
                                const int32_t* idx, const float* U, const float* V,
                                const float* cnt, int32_t C, int32_t H, int32_t W, float sigma,
                                float kappa, float* grad_tau_mult, void* ws, size_t ws_bytes,
                                void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (general_c(C)) return HTS_ERR_UNSUPPORTED;   // spectral tubes: hts_denoise, hts_match, hts_basis
  if (!noisy || !grad_out || !idx || !U || !V || !cnt || !grad_tau_mult || !ws) return HTS_ERR_INVALID;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return HTS_ERR_INVALID;
  if (!(kappa > 0.f) || !std::isfinite(kappa)) return HTS_ERR_INVALID;
  if (weighted(p) || fourier(p, C)) return HTS_ERR_UNSUPPORTED;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  const Schedule sc = schedule_for(p, C);
  hipStream_t s = (hipStream_t)stream;
  if (sigma == 0.f) {   // tau = 0 and a zero-width relaxation: no defined surrogate slope
    HIPCHK(launch_fill(grad_tau_mult, 1, 0.f, s));
    return HTS_OK;
  }
  ImgDesc d = make_desc(g, p, (char*)ws, c, noisy, sigma, sc.fty, sc.ftx);
  d.idx = const_cast<int32_t*>(idx);
  d.cnt = const_cast<float*>(cnt);
  HIPCHK(launch_fbasis(make_launch(p, C, d, -1, sc.fty, sc.ftx), U, V, s));
  // the fixed-point numerator plane (>= 8 * n_ref bytes) holds the per-group partials
  HIPCHK(launch_taugrad(make_launch(p, C, d, -1, sc.fty, sc.ftx), grad_out, (double*)d.num64, kappa,
                        grad_tau_mult, device_cus() * 8, s));
  return HTS_OK;
}

hts_status hts_denoise_backward_basis(const hts_params* p, const float* noisy,
                                      const float* grad_out, const int32_t* idx,
                                      const uint32_t* masks, const double* U64, const double* V64,
                                      const double* eig, const float* cnt, int32_t C, int32_t H,
                                      int32_t W, float* grad_in, void* ws, size_t ws_bytes,
                                      void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (general_c(C)) return HTS_ERR_UNSUPPORTED;   // spectral tubes: hts_denoise, hts_match, hts_basis
  if (!noisy || !grad_out || !idx || !masks || !U64 || !V64 || !eig || !cnt || !grad_in || !ws)
    return HTS_ERR_INVALID;
  if (weighted(p) || fourier(p, C)) return HTS_ERR_UNSUPPORTED;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  const Schedule sc = schedule_for(p, C);
  hipStream_t s = (hipStream_t)stream;
  ImgDesc d = make_desc(g, p, (char*)ws, c, noisy, 0.f, sc.fty, sc.ftx);
  d.idx = const_cast<int32_t*>(idx);
  d.cnt = const_cast<float*>(cnt);
  d.masks_in = masks;
  // one FP64 partial (2 x (C/2+1) complex 8x8) per work group, in the
  // fixed-point numerator plane
  const int nm = 2 * (C / 2 + 1);
  const size_t per = (size_t)nm * 128 * sizeof(double);
  const int grid = (int)std::max<size_t>(
      1, std::min<size_t>({(size_t)device_cus() * 8, (size_t)g.n_ref, (size_t)C * H * W * 8 / per}));
  HIPCHK(launch_gbasis(make_launch(p, C, d, -1, sc.fty, sc.ftx), grad_out, U64, V64, eig,
                       (double*)d.num64, grid, (double*)((char*)ws + c.gbasis), grad_in, s));
  return HTS_OK;
}

hts_status hts_match_fallback_count(const hts_params* p, int32_t C, int32_t H, int32_t W,
                                   const void* ws, size_t ws_bytes, int32_t* count, void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (!ws || !count) return HTS_ERR_INVALID;
  const Carve c = carve(g);
  if (ws_bytes < c.total) return HTS_ERR_WORKSPACE;
  HIPCHK(hipMemcpyAsync(count, (const char*)ws + c.fb_count, sizeof(int32_t),
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return HTS_OK;
}

hts_status hts_batch_fallback_counts(const hts_params* p, const hts_image* imgs, int32_t n,
                                     const void* ws, size_t ws_bytes, int32_t* counts,
                                     void* stream) {
  if (!ws || !counts) return HTS_ERR_INVALID;
  BatchPlan plan;
  hts_status st = plan_batch(p, imgs, n, (char*)ws, false, plan);
  if (st != HTS_OK) return st;
  if (ws_bytes < plan.bytes) return HTS_ERR_WORKSPACE;
  for (int i = 0; i < n; ++i)
    HIPCHK(hipMemcpyAsync(counts + i, plan.descs[i].fb_count, sizeof(int32_t),
                          hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return HTS_OK;
}

hts_status hts_batch_shortlist_histogram(const hts_params* p, const hts_image* imgs, int32_t n,
                                         void* ws, size_t ws_bytes, int32_t* counts,
                                         void* stream) {
  static_assert(HTS_SHORTLIST_BINS == SL_BINS, "shortlist bins");
  if (!ws || !counts || !imgs || n < 1) return HTS_ERR_INVALID;
  for (int i = 0; i < n; ++i)
    if (!imgs[i].noisy) return HTS_ERR_INVALID;
  std::vector<hts_image> im(imgs, imgs + n);   // out and sigma play no part
  for (auto& m : im) {
    m.out = nullptr;
    m.sigma = 0.f;
  }
  BatchPlan plan;
  hts_status st = plan_batch(p, im.data(), n, (char*)ws, false, plan);
  if (st != HTS_OK) return st;
  if (ws_bytes < plan.bytes) return HTS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int C = imgs[0].C;
  ImgDesc* table = (ImgDesc*)((char*)ws + plan.table_off);
  HIPCHK(hipMemcpyAsync(table, plan.descs.data(), plan.descs.size() * sizeof(ImgDesc),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));   // the upload reads pageable host memory
  const int cus = device_cus();
  auto LK = [&](int kind) {
    return batch_launch(p, C, table, n, kind >= 0 ? plan.totals[kind] : 0, plan.sc);
  };
  HIPCHK(launch_fill((float*)counts, SL_BINS, 0.f, s));   // zero bits
  HIPCHK(launch_reset_counters(LK(-1), s));
  HIPCHK(launch_quant(LK(W_PIX), cus * 8, s));
  HIPCHK(launch_gcp(LK(W_REF), cus * 8, s));
  Launch Lm = LK(W_MATCH);
  Lm.sl_hist = counts;
  HIPCHK(launch_match(Lm, p->match_mode, plan.sc.terms, cus * 2, s));
  return HTS_OK;
}

hts_status hts_batch_workspace_size(const hts_params* p, const hts_image* imgs, int32_t n,
                                    size_t* bytes) {
  if (!bytes) return HTS_ERR_INVALID;
  BatchPlan plan;
  hts_status st = plan_batch(p, imgs, n, nullptr, false, plan);
  if (st != HTS_OK) return st;
  *bytes = plan.bytes;
  return HTS_OK;
}

// Sampled groups and adjusted sigma of every image for the adaptive variant.
struct AdaptArgs {
  const int32_t* samples;   // device [n][n_samples]
  int32_t n_samples, gamma;
  float beta;
  int32_t* ranks;           // device [n][n_samples], nullable
  float* sigma_out;         // device [n]
};

}  // extern "C"

namespace {

// Uploads the descriptor table of `plan` and replays the graph of `key`,
// capturing it first (enq(stream) enqueues the stages); eager launches on
// the caller's stream if capture or instantiation fails.
template <class Enq>
hts_status replay_batch(const std::string& key, const BatchPlan& plan, ImgDesc* table,
                               hipStream_t s, Enq&& enq) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  if (g_graphs.size() >= 64 && !g_graphs.count(key)) {
    // bounded cache: drop every entry (after the device is idle) and start over
    HIPCHK(hipDeviceSynchronize());
    for (auto& kv : g_graphs) {
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      if (kv.second.copied) (void)hipEventDestroy(kv.second.copied);
    }
    g_graphs.clear();
  }
  GraphEntry& e = g_graphs[key];
  if (!e.copied) HIPCHK(hipEventCreateWithFlags(&e.copied, hipEventDisableTiming));
  if (e.used) HIPCHK(hipEventSynchronize(e.copied));   // previous upload has read the staging
  e.host = plan.descs;
  e.used = true;
  HIPCHK(hipMemcpyAsync(table, e.host.data(), e.host.size() * sizeof(ImgDesc), hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(e.copied, s));
  if (!e.exec) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return HTS_ERR_UNSUPPORTED;
    if (!g_capture_stream[dev]) HIPCHK(hipStreamCreateWithFlags(&g_capture_stream[dev], hipStreamNonBlocking));
    hipStream_t cs = g_capture_stream[dev];
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hts_status est = enq(cs);
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (est != HTS_OK || ce != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return enq(s);   // eager launches on the caller's stream
    }
    const hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      e.exec = nullptr;
      (void)hipGetLastError();
      return enq(s);
    }
  }
  HIPCHK(hipGraphLaunch(e.exec, s));
  return HTS_OK;
}

}  // namespace

extern "C" {

static hts_status denoise_batch_impl(const hts_params* p, const hts_image* imgs, int32_t n,
                                     void* ws, size_t ws_bytes, void* stream,
                                     const AdaptArgs* ad, const hts_state* states = nullptr) {
  if (!ws) return HTS_ERR_INVALID;
  BatchPlan plan;
  hts_status st = plan_batch(p, imgs, n, (char*)ws, true, plan);
  if (st != HTS_OK) return st;
  if (ws_bytes < plan.bytes) return HTS_ERR_WORKSPACE;
  for (int i = 0; i < n; ++i) {
    ImgDesc& d = plan.descs[i];
    if (ad) {
      d.samples = ad->samples + (size_t)i * ad->n_samples;
      d.n_samples = ad->n_samples;
      d.gamma = ad->gamma;
      d.beta = ad->beta;
      d.ranks = ad->ranks ? ad->ranks + (size_t)i * ad->n_samples : nullptr;
      d.sigma_dev = ad->sigma_out + i;
    }
    if (states) {   // the match, the coverage counts and the filter write the caller's state
      d.idx = states[i].idx;
      d.masks = states[i].masks;
      d.cnt = states[i].cnt;
      d.U_ext = states[i].U;
      d.V_ext = states[i].V;
    }
  }
  const int C = imgs[0].C;
  ImgDesc* table = (ImgDesc*)((char*)ws + plan.table_off);
  const std::string key = graph_key(p, plan.sc, imgs, n, ws, ad ? "A" : states ? "S" : "");
  return replay_batch(key, plan, table, (hipStream_t)stream, [&](hipStream_t cs) {
    return enqueue_batch(p, C, plan, table, cs, nullptr, states != nullptr);
  });
}

static bool states_ok(const hts_state* states, int32_t n) {
  if (!states || n < 1) return false;
  for (int i = 0; i < n; ++i) {
    const hts_state& t = states[i];
    if (!t.idx || !t.masks || !t.U || !t.V || !t.cnt) return false;
  }
  return true;
}

hts_status hts_denoise_batch(const hts_params* p, const hts_image* imgs, int32_t n, void* ws,
                             size_t ws_bytes, void* stream) {
  return denoise_batch_impl(p, imgs, n, ws, ws_bytes, stream, nullptr);
}

hts_status hts_denoise_batch_save(const hts_params* p, const hts_image* imgs,
                                  const hts_state* states, int32_t n, void* ws, size_t ws_bytes,
                                  void* stream) {
  if (!p || !imgs || n < 1) return HTS_ERR_INVALID;
  if (weighted(p) || fourier(p, imgs[0].C)) return HTS_ERR_UNSUPPORTED;   // masks of Eq. 19 only
  if (!states_ok(states, n)) return HTS_ERR_INVALID;
  return denoise_batch_impl(p, imgs, n, ws, ws_bytes, stream, nullptr, states);
}

hts_status hts_denoise_batch_backward(const hts_params* p, const hts_image* imgs,
                                      const hts_state* states, int32_t n, void* ws,
                                      size_t ws_bytes, void* stream) {
  if (!p || !imgs || n < 1 || !ws) return HTS_ERR_INVALID;
  if (weighted(p) || fourier(p, imgs[0].C)) return HTS_ERR_UNSUPPORTED;   // adjoint of Eq. 19-20, 2
  if (!states_ok(states, n)) return HTS_ERR_INVALID;
  std::vector<hts_image> gi(imgs, imgs + n);   // sigma plays no part in the adjoint
  for (auto& im : gi) im.sigma = 0.f;
  BatchPlan plan;
  hts_status st = plan_batch(p, gi.data(), n, (char*)ws, true, plan);
  if (st != HTS_OK) return st;
  if (ws_bytes < plan.bytes) return HTS_ERR_WORKSPACE;
  for (int i = 0; i < n; ++i) {
    ImgDesc& d = plan.descs[i];
    d.fb_count = nullptr;   // the forward's fallback counts stay readable
    d.img = d.num;   // r = grad_out / cnt (workspace)
    d.num = const_cast<float*>(imgs[i].noisy);
    d.out = imgs[i].out;
    d.sigma = 0.f;
    d.tau = 0.f;
    d.idx = states[i].idx;
    d.masks_in = states[i].masks;
    d.num_enc = NUM_FINE;   // the adjoint's numerator in 2^-32 units
    d.masks = nullptr;
    d.cnt = states[i].cnt;
    d.U_ext = states[i].U;
    d.V_ext = states[i].V;
  }
  const int C = imgs[0].C;
  ImgDesc* table = (ImgDesc*)((char*)ws + plan.table_off);
  const std::string key = graph_key(p, plan.sc, gi.data(), n, ws, "B");
  return replay_batch(key, plan, table, (hipStream_t)stream, [&](hipStream_t cs) {
    return enqueue_batch_backward(p, C, plan, table, cs);
  });
}

hts_status hts_denoise_batch_adaptive(const hts_params* p, const hts_image* imgs, int32_t n,
                                      const int32_t* samples, int32_t n_samples, float beta,
                                      int32_t gamma, int32_t* ranks, float* sigma_out,
                                      void* ws, size_t ws_bytes, void* stream) {
  if (!samples || !sigma_out || !adapt_args_ok(n_samples, beta)) return HTS_ERR_INVALID;
  const AdaptArgs ad{samples, n_samples, gamma, beta, ranks, sigma_out};
  return denoise_batch_impl(p, imgs, n, ws, ws_bytes, stream, &ad);
}

hts_status hts_denoise_batch_staged(const hts_params* p, const hts_image* imgs, int32_t n,
                                    void* ws, size_t ws_bytes, void* stream, void* const* events,
                                    int32_t n_events) {
  if (!ws || !events || n_events != HTS_BATCH_STAGE_EVENTS) return HTS_ERR_INVALID;
  for (int i = 0; i < n_events; ++i)
    if (!events[i]) return HTS_ERR_INVALID;
  BatchPlan plan;
  hts_status st = plan_batch(p, imgs, n, (char*)ws, true, plan);
  if (st != HTS_OK) return st;
  if (ws_bytes < plan.bytes) return HTS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  ImgDesc* table = (ImgDesc*)((char*)ws + plan.table_off);
  // the table upload reads pageable host memory: wait for it before the
  // staging vector goes away
  HIPCHK(hipMemcpyAsync(table, plan.descs.data(), plan.descs.size() * sizeof(ImgDesc),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return enqueue_batch(p, imgs[0].C, plan, table, s, (hipEvent_t const*)events);
}

hts_status hts_autotune(const hts_params* p, int32_t C, int32_t H, int32_t W,
                        const char* cache_path, int32_t* tune_out, void* ws, size_t ws_bytes,
                        void* stream) {
  Geo g;
  hts_status st = make_geo(p, C, H, W, g);
  if (st != HTS_OK) return st;
  if (general_c(C)) return HTS_ERR_UNSUPPORTED;   // spectral tubes: hts_denoise, hts_match, hts_basis
  if (!tune_out || !ws) return HTS_ERR_INVALID;
  const std::string key = tune_key(p, C);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_file(cache_path);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) { *tune_out = it->second; return HTS_OK; }
  }
  const Carve c = carve(g);
  const size_t img_b = al((size_t)C * H * W * 4), idx_b = al((size_t)g.n_ref * g.K * 4);
  if (ws_bytes < c.total + 2 * img_b + idx_b) return HTS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  float* img = (float*)(base + c.total);
  float* out = (float*)(base + c.total + img_b);
  int32_t* idx = (int32_t*)(base + c.total + 2 * img_b);
  HIPCHK(launch_synth(img, C, H, W, s));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto time_it = [&](auto&& fn) -> float {
    float best = 1e30f;
    for (int rep = 0; rep < 5; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess) return 1e30f;
      if (fn() != HTS_OK) return 1e30f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1e30f;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best = std::min(best, ms);
    }
    return best;
  };
  hts_params q = *p;
  q.tune = 0;
  Schedule base_sc = schedule_for(&q, C);
  ImgDesc d = make_desc(g, &q, base, c, img, 25.f, base_sc.fty, base_sc.ftx);
  d.idx = idx;
  d.out = out;
  // Candidates are timed in a fixed order, and the first one within
  // kTieMargin of the fastest wins: measurements a few per cent apart are
  // noise, and the order puts the preferred variant first (the hi/lo split,
  // whose tighter bounds give shorter shortlists; larger filter tiles, which
  // flush fewer tile borders and gather with more reuse).
  constexpr float kTieMargin = 1.02f;
  auto pick = [&](const std::vector<float>& t) {
    float best = 1e30f;
    for (float v : t) best = std::min(best, v);
    for (size_t i = 0; i < t.size(); ++i)
      if (t[i] <= best * kTieMargin) return (int)i;
    return 0;
  };
  // distance-tile variant (BF16 only: one product or hi/lo split)
  int best_terms = 3;
  if (p->match_mode == HTS_MATCH_BF16) {
    const int cand[2] = {3, 1};
    std::vector<float> times;
    for (int terms : cand) {
      Schedule sc = base_sc;
      sc.terms = terms;
      times.push_back(time_it([&] { return run_match(&q, C, sc, d, s); }));
    }
    best_terms = cand[pick(times)];
  }
  {
    Schedule sc = base_sc;
    sc.terms = best_terms;
    st = run_match(&q, C, sc, d, s);
    if (st == HTS_OK) st = run_basis(&q, C, sc, d, s);
    if (st != HTS_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return st; }
  }
  // filter implementation and tile shape
  std::vector<float> ftimes;
  std::vector<std::pair<int, int>> fcand;   // (valu, shape)
  for (int valu = filter_mfma_supported(C, p->K) && !weighted(p) && !fourier(p, C) ? 0 : 1;
       valu <= 1; ++valu) {
    for (int i = 0; i < kNumShapes; ++i) {
      if (filter_impl_lds(p, C, valu, kShapes[i].ty, kShapes[i].tx) > kLdsMax) continue;
      Schedule sc = base_sc;
      sc.valu = valu;
      sc.fty = kShapes[i].ty;
      sc.ftx = kShapes[i].tx;
      ImgDesc di = d;
      fill_counts(g, &q, sc.fty, sc.ftx, di);
      ftimes.push_back(time_it([&] {
        if (launch_zero_accum(make_launch(&q, C, di, W_PIX, sc.fty, sc.ftx), 0, s) != hipSuccess) return HTS_ERR_HIP;
        return run_filter(&q, C, sc, di, 0, s);
      }));
      fcand.push_back({valu, i});
    }
  }
  const int fi = fcand.empty() ? -1 : pick(ftimes);
  const int best_valu = fi < 0 ? 1 : fcand[fi].first, best_shape = fi < 0 ? 0 : fcand[fi].second;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int word = (best_shape + 1) | ((best_terms == 1 ? 1 : 2) << 4) | (best_valu << 6);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = word;
    if (cache_path) {
      FILE* f = std::fopen(cache_path, "a");
      if (f) { std::fprintf(f, "%s|%d\n", key.c_str(), word); std::fclose(f); }
    }
  }
  *tune_out = word;
  return HTS_OK;
}

// ---- video: spatio-temporal search over the stacked frames ----

namespace {

struct VideoPlan {
  Geo f;                 // one frame
  VideoGeo v;
  int n_ref, np, NF, grid;
  size_t stacked, sout, gplanes, idx, cov, basis64, basis, fbasis, ufg, num64, cnt, hist, poison,
      fxmax, fb_count, gscratch, rowp, est, gscr, list, total;
};

hts_status plan_video(const hts_params* p, int T, int C, int H, int W, int dt, VideoPlan& vp) {
  hts_status st = make_geo(p, C, H, W, vp.f);
  if (st != HTS_OK) return st;
  if (T < 1 || dt < 0) return HTS_ERR_INVALID;
  if (p->flags || p->K > GEN_KMAX) return HTS_ERR_UNSUPPORTED;   // uniform Eq. 2 and Eq. 19
  if ((long long)(2 * std::min(dt, T - 1) + 1) * p->window * p->window > VIDEO_CAND_MAX)
    return HTS_ERR_UNSUPPORTED;
  const long long px = (long long)T * H * W;
  if (px * C >= (1LL << 31) || (long long)T * vp.f.n_ref * p->K >= (1LL << 31)) return HTS_ERR_UNSUPPORTED;
  if (!general_c(C) && !gather_supported(px)) return HTS_ERR_UNSUPPORTED;
  vp.n_ref = T * vp.f.n_ref;
  vp.np = C == 3 ? 2 : 1;
  vp.NF = n_freq(C);
  vp.grid = gen_filter_grid(vp.n_ref, p->K, C);
  vp.v = VideoGeo{T, H, vp.f.Hp, vp.f.Wp, vp.f.nry, vp.f.nrx, vp.f.n_ref, dt};
  size_t o = 0;
  vp.stacked = o; o += al((size_t)px * C * 4);
  vp.sout = o; o += al((size_t)px * C * 4);
  vp.gplanes = o; o += al((size_t)px * vp.np * 4);
  vp.idx = o; o += al((size_t)vp.n_ref * p->K * 4);
  vp.cov = o; o += al((size_t)T * vp.f.n_cov * cov_elems(C) * 8);
  vp.basis64 = o; o += al((size_t)(2 * C * 64 + 2 * vp.NF * 8) * 8);
  vp.basis = o; o += al((size_t)2 * C * 64 * 4);
  vp.fbasis = o; o += al((size_t)std::max(FB_SIZE, 2 * vp.NF * 128) * 4);
  vp.ufg = o; o += al((size_t)2 * vp.NF * 128 * 8);
  vp.num64 = o; o += al((size_t)px * C * 8);
  vp.cnt = o; o += al((size_t)px * 4);
  vp.hist = o; o += al((size_t)px * 4);
  vp.poison = o; o += al((size_t)px);
  vp.fxmax = o; o += al(4);
  vp.fb_count = o; o += al(4);
  vp.gscratch = o; o += al((size_t)vp.grid * p->K * C * 64 * 4);
  vp.rowp = o; o += general_c(C) ? 0 : al((size_t)T * H * vp.f.Wp * rowp_floats(C) * 4);
  // c = 1, 3: every slot's estimate, then the corner buckets of the gather
  const size_t slots = general_c(C) ? 0 : (size_t)vp.n_ref * p->K;
  vp.est = o; o += al(slots * C * 64 * 4);
  vp.gscr = o; o += general_c(C) ? 0 : al(gather_scratch_ints(px) * 4);
  vp.list = o; o += al(slots * 4);
  vp.total = o;
  return HTS_OK;
}

}  // namespace

hts_status hts_video_workspace_size(const hts_params* p, int32_t T, int32_t C, int32_t H,
                                    int32_t W, int32_t dt, size_t* bytes) {
  if (!bytes) return HTS_ERR_INVALID;
  VideoPlan vp;
  const hts_status st = plan_video(p, T, C, H, W, dt, vp);
  if (st != HTS_OK) return st;
  *bytes = vp.total;
  return HTS_OK;
}

hts_status hts_denoise_video(const hts_params* p, const float* frames, int32_t T, int32_t C,
                             int32_t H, int32_t W, int32_t dt, float sigma, float* out,
                             int32_t* idx_out, uint32_t* masks_out, float* U_out, float* V_out,
                             float* cnt_out, void* ws, size_t ws_bytes, void* stream) {
  VideoPlan vp;
  hts_status st = plan_video(p, T, C, H, W, dt, vp);
  if (st != HTS_OK) return st;
  if (!frames || !out || !ws) return HTS_ERR_INVALID;
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return HTS_ERR_INVALID;
  if (ws_bytes < vp.total) return HTS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* b = (char*)ws;
  const int TH = T * H;
  // descriptor of the stacked image [C][T*H][W]
  ImgDesc d;
  std::memset(&d, 0, sizeof(d));
  d.img = (const float*)(b + vp.stacked);
  d.out = (float*)(b + vp.sout);
  d.gplanes = (int32_t*)(b + vp.gplanes);
  d.idx = idx_out ? idx_out : (int32_t*)(b + vp.idx);
  d.fb_count = (int32_t*)(b + vp.fb_count);
  d.cov_part = (double*)(b + vp.cov);
  d.basis64 = (double*)(b + vp.basis64);
  d.basis = (float*)(b + vp.basis);
  d.fbasis = (float*)(b + vp.fbasis);
  d.ufg = (double*)(b + vp.ufg);
  d.num64 = (unsigned long long*)(b + vp.num64);
  d.cnt = cnt_out ? cnt_out : (float*)(b + vp.cnt);
  d.hist = (int32_t*)(b + vp.hist);
  d.poison = (uint8_t*)(b + vp.poison);
  d.fxmax = (uint32_t*)(b + vp.fxmax);
  d.gscratch = (float*)(b + vp.gscratch);
  d.rowp = general_c(C) ? nullptr : (float*)(b + vp.rowp);
  d.masks = masks_out;
  d.H = TH; d.W = W; d.Hp = TH - PS + 1; d.Wp = W - PS + 1;
  d.nry = vp.f.nry; d.nrx = vp.f.nrx; d.n_ref = vp.n_ref;
  d.ref_begin = 0; d.ref_count = vp.n_ref;
  d.sigma = sigma;
  d.tau = p->tau_mult * sigma;
  d.n_cov = T * vp.f.n_cov;
  d.wcnt[W_PIX] = (int)(((long long)TH * W + PIX_CHUNK - 1) / PIX_CHUNK);
  d.wcnt[W_REF] = (vp.n_ref + 255) / 256;
  d.wcnt[W_BOX] = ((TH + BOX_TY - 1) / BOX_TY) * ((W + BOX_TX - 1) / BOX_TX);
  auto LS = [&](const ImgDesc& dd, int kind) {
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.one = dd;
    L.n_img = 1;
    L.total = kind >= 0 ? dd.wcnt[kind] : 1;
    L.C = C; L.K = p->K; L.stride = p->stride; L.window = p->window;
    L.tau_mult = p->tau_mult;
    L.gcp_num = p->gcp_num; L.gcp_den = p->gcp_den;
    return L;
  };
  HIPCHK(launch_stack(frames, (float*)d.img, T, C, H, W, false, s));
  // guide planes (and the magnitude that sets the fixed-point scale)
  HIPCHK(launch_reset_counters(LS(d, -1), s));
  HIPCHK(launch_quant(LS(d, W_PIX), 0, s));
  HIPCHK(launch_match_video(LS(d, -1), vp.v, s));
  // one basis for the sequence: every frame's covariance partials, in
  // frame order, then the eigen-solves over all of them
  for (int t = 0; t < T; ++t) {
    ImgDesc df;
    std::memset(&df, 0, sizeof(df));
    df.img = frames + (size_t)t * C * H * W;
    df.cov_part = d.cov_part + (size_t)t * vp.f.n_cov * cov_elems(C);
    df.H = H; df.W = W; df.Hp = vp.f.Hp; df.Wp = vp.f.Wp;
    df.nry = vp.f.nry; df.nrx = vp.f.nrx; df.n_ref = vp.f.n_ref;
    df.n_cov = vp.f.n_cov;
    df.wcnt[W_COV] = vp.f.n_cov;
    if (general_c(C)) HIPCHK(launch_cov_gen(LS(df, -1), s));
    else HIPCHK(launch_cov(LS(df, W_COV), 0, s));
  }
  if (general_c(C)) HIPCHK(launch_eig_gen(LS(d, -1), s));
  else HIPCHK(launch_eig(LS(d, -1), s));
  // filter and average over the stacked image
  HIPCHK(launch_zero_accum(LS(d, W_PIX), 0, s));
  if (general_c(C)) {
    HIPCHK(launch_fbasis_gen(LS(d, -1), s));
    HIPCHK(launch_filter_gen(LS(d, -1), vp.grid, s));
  } else {
    // c = 1, 3: the vector-ALU filter over tiles of the stacked reference
    // grid (T * nry rows), with global aggregation
    HIPCHK(launch_fbasis(LS(d, -1), nullptr, nullptr, s));
    HIPCHK(launch_rowproj(LS(d, W_PIX), 0, s));
    ImgDesc dv = d;
    dv.nry = T * vp.f.nry;
    dv.group_est = (float*)(b + vp.est);   // every slot's estimate, exported
    Launch Lv = LS(dv, -1);
    Lv.fty = VIDEO_FTY;
    Lv.ftx = VIDEO_FTX;
    Lv.total = ((dv.nry + VIDEO_FTY - 1) / VIDEO_FTY) * ((dv.nrx + VIDEO_FTX - 1) / VIDEO_FTX);
    HIPCHK(launch_filter_stacked(Lv, s));
  }
  HIPCHK(launch_zero_hist(LS(d, W_PIX), 0, s));
  HIPCHK(launch_count_hist(LS(d, W_REF), 0, s));
  if (!general_c(C))   // the estimates, bucketed by corner, gathered per output tile
    HIPCHK(launch_gather(LS(d, -1), (const float*)(b + vp.est), (int*)(b + vp.gscr),
                         (int*)(b + vp.list), s));
  HIPCHK(launch_count_box(LS(d, W_BOX), 0, s));
  HIPCHK(launch_finalize(LS(d, W_PIX), 0, s));
  HIPCHK(launch_stack(out, d.out, T, C, H, W, true, s));
  const size_t nb = (size_t)C * 64;
  if (U_out) HIPCHK(hipMemcpyAsync(U_out, d.basis, nb * 4, hipMemcpyDeviceToDevice, s));
  if (V_out) HIPCHK(hipMemcpyAsync(V_out, d.basis + nb, nb * 4, hipMemcpyDeviceToDevice, s));
  return HTS_OK;
}

hts_status hts_denoise_video_backward(const hts_params* p, const float* grad_out, int32_t T,
                                      int32_t C, int32_t H, int32_t W, int32_t dt,
                                      const int32_t* idx, const uint32_t* masks, const float* U,
                                      const float* V, const float* cnt, float* grad_in, void* ws,
                                      size_t ws_bytes, void* stream) {
  VideoPlan vp;
  hts_status st = plan_video(p, T, C, H, W, dt, vp);
  if (st != HTS_OK) return st;
  if (!grad_out || !idx || !masks || !U || !V || !cnt || !grad_in || !ws) return HTS_ERR_INVALID;
  if (ws_bytes < vp.total) return HTS_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* b = (char*)ws;
  const int TH = T * H;
  ImgDesc d;
  std::memset(&d, 0, sizeof(d));
  d.img = (const float*)(b + vp.stacked);        // grad_out, stacked
  d.num = (float*)(b + vp.sout);                 // r = grad_out / cnt, stacked
  d.cnt = const_cast<float*>(cnt);
  d.fb_count = (int32_t*)(b + vp.fb_count);
  d.fxmax = (uint32_t*)(b + vp.fxmax);
  d.H = TH; d.W = W; d.Hp = TH - PS + 1; d.Wp = W - PS + 1;
  d.nry = vp.f.nry; d.nrx = vp.f.nrx; d.n_ref = vp.n_ref;
  d.ref_begin = 0; d.ref_count = vp.n_ref;
  d.wcnt[W_PIX] = (int)(((long long)TH * W + PIX_CHUNK - 1) / PIX_CHUNK);
  auto LS = [&](const ImgDesc& dd, int kind) {
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.one = dd;
    L.n_img = 1;
    L.total = kind >= 0 ? dd.wcnt[kind] : 1;
    L.C = C; L.K = p->K; L.stride = p->stride; L.window = p->window;
    L.tau_mult = p->tau_mult;
    return L;
  };
  HIPCHK(launch_stack(grad_out, (float*)d.img, T, C, H, W, false, s));
  HIPCHK(launch_reset_counters(LS(d, -1), s));
  HIPCHK(launch_adjoint_prep(LS(d, W_PIX), 0, s));
  // the transpose of the frozen-mask map on r, summed in fixed point
  ImgDesc a = d;
  a.img = d.num;
  a.num = nullptr;
  a.cnt = nullptr;
  a.idx = const_cast<int32_t*>(idx);
  a.masks_in = masks;
  a.num64 = (unsigned long long*)(b + vp.num64);
  a.poison = (uint8_t*)(b + vp.poison);
  a.basis = (float*)(b + vp.basis);
  a.fbasis = (float*)(b + vp.fbasis);
  a.gscratch = (float*)(b + vp.gscratch);
  a.out = (float*)(b + vp.stacked);              // grad_out is no longer needed
  a.num_enc = NUM_FINE | NUM_PIXELS;             // k_filter_gen's pixel sums
  const size_t nb = (size_t)C * PS2 * sizeof(float);
  HIPCHK(hipMemcpyAsync(a.basis, U, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(a.basis + C * PS2, V, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_fbasis_gen(LS(a, -1), s));
  HIPCHK(launch_zero_accum(LS(a, W_PIX), 0, s));
  HIPCHK(launch_filter_gen_adj(LS(a, -1), vp.grid, s));
  HIPCHK(launch_finalize(LS(a, W_PIX), 0, s));   // no cnt: the numerator itself
  HIPCHK(launch_stack(grad_in, a.out, T, C, H, W, true, s));
  return HTS_OK;
}

}  // extern "C"
