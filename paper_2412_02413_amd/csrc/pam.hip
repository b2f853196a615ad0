// Host side of the AS-TAX library: plan (the paper's pre-run, Section II-E),
// validation, workspace layout and kernel launches behind the C-ABI of pam.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/pam.h"
#include "kernels.hpp"
#include "k3_fields.hpp"
#include "k3_fields16.hpp"
#include "k3_factored.hpp"
#include "k2_fft.hpp"
#include "k3_fft.hpp"
#include "k3_tea.hpp"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMinSamples = 32;
constexpr int kMaxSamples = 16384;
constexpr int kMaxNx = 512;

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (ok && hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

// One bin subset per record length n_samples / 2^j.
struct Level {
  int n_t = 0;
  int stride = 1;        // 2^j
  int n_sel = 0;
  int32_t* d_ksel = nullptr;  // bin k on the level's own grid
  double* d_kz = nullptr;     // [n_sel][kz_row(N)] signed kz / (2 pi) of the selected bins
  double* d_kzff = nullptr;   // [n_sel][N2][N1] the same values at q = N2 q1 + q2 (factored kernels)
  int32_t* d_ev = nullptr;    // [n_sel] 1 if any lateral wavenumber of the bin is evanescent
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// round-to-nearest-even FP32 -> BF16 / FP16 bit patterns, and back
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float from_bf16(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t to_fp16(float f) {
  const _Float16 h = (_Float16)f;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}
float from_fp16(uint16_t u) {
  _Float16 h;
  std::memcpy(&h, &u, 2);
  return (float)h;
}
bool is_split(int prec) { return prec != PAM_PREC_FP32; }
bool is_fp16(int prec) { return prec == PAM_PREC_SPLIT_FP16 || prec == PAM_PREC_FP16; }

}  // namespace

struct pam_plan_s {
  int device = 0;
  int L = 0, n_t = 0, N = 0, n_z = 0, n_sub = 0, n_bins = 0;
  double eps = 1e-3;
  int precision = 0, zero_evanescent = 0;
  int coherence = 0;          // adjacent-pixel cross-spectra with the n_sub = 1 sums
  std::vector<int32_t> bins;  // k on the plan grid
  std::vector<Level> levels;
  // device tables
  double* d_z = nullptr;       // [n_z]
  float2* d_tw = nullptr;      // [n_t/2] time-FFT twiddles
  float2* d_twx = nullptr;     // [N] lateral DFT twiddles
  float* d_masks = nullptr;    // [n_sub][L]
  int32_t col0 = 0, col_step = 1;  // grid column of element l: col0 + col_step * l
  float* d_basis = nullptr;    // [N][N] slot-major cos/sin basis (FP32 kernel)
  uint16_t* d_bhi = nullptr;   // [N/8][N][8] basis (slot groups, x, slots), 16-bit hi (split kernels)
  uint16_t* d_blo = nullptr;   // same layout, 16-bit lo
  bool ff = false;             // inverse lateral transform factored into two 16-point stages (N = 256, 512)
  float* d_ff_w32 = nullptr;   // [64][16] 16-point DFT matrix in FP32 operand order
  uint16_t* d_ff_w16 = nullptr;  // [64][2][16] the same in 16-bit operand order, hi then lo per k-step
  float2* d_ff_tw = nullptr;   // [64][8] twiddles / 16 in stage-1 output order
  float2* d_ff_tw2 = nullptr;  // [64][8] N = 512 combination twiddles in stage-3 output order
  float2* d_ff_tw_vec = nullptr;  // [16][16] stage twiddles of the vector FFT kernel
  float2* d_ff_tw2_vec = nullptr;  // [16][16] N = 512 combination twiddles of the vector FFT kernel
  // frequency-domain delay-and-sum (pam_fd_tea_tax)
  double fs = 0, c = 0;        // sampling rate, sound speed
  double dx = 0, x_first = 0;  // lateral grid spacing and coordinate of column 0
  double xl_first = 0, pitch = 0;  // coordinate of element 0 and element pitch
  int32_t* d_subs = nullptr;   // [L] bit i set if sub-aperture i holds element l
  int k3_slots = 512;          // K3 workgroups resident on the device at once
  int n_cus = 256;             // compute units of the plan's device
  std::vector<void*> allocs;
};

namespace {

// allocation-failure injection for tests (pam_debug_fail_allocation) and the count of
// device allocations the library's plans hold (pam_debug_live_allocations)
std::atomic<int> g_fail_alloc{-1};
std::atomic<long long> g_live_allocs{0};

void free_plan(pam_plan_s* p) {
  if (!p) return;
  for (void* q : p->allocs) {
    (void)hipFree(q);
    --g_live_allocs;
  }
  delete p;
}

template <typename T>
pam_status_t upload(pam_plan_s* p, T** dst, const T* src, size_t n) {
  void* ptr = nullptr;
  const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  int armed = g_fail_alloc.load();
  while (armed >= 0 && !g_fail_alloc.compare_exchange_weak(armed, armed - 1)) {
  }
  if (armed == 0) return PAM_ERR_OOM;  // injected failure (the counter is now disarmed)
  if (hipMalloc(&ptr, bytes) != hipSuccess) return PAM_ERR_OOM;
  p->allocs.push_back(ptr);
  ++g_live_allocs;
  if (n && hipMemcpy(ptr, src, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return PAM_ERR_DEVICE;
  *dst = static_cast<T*>(ptr);
  return PAM_OK;
}

pam_status_t validate(const pam_geometry_t* g) {
  if (!g) return PAM_ERR_INVALID_ARG;
  if (g->n_elements < 1 || !finite_pos(g->pitch_m) || !finite_pos(g->fs_hz) || !finite_pos(g->c_mps))
    return PAM_ERR_INVALID_ARG;
  if (g->n_samples < 2) return PAM_ERR_INVALID_ARG;
  if (!is_pow2(g->n_samples) || g->n_samples < kMinSamples || g->n_samples > kMaxSamples)
    return PAM_ERR_UNSUPPORTED;
  if (g->n_bands < 1 || !g->band_lo_hz || !g->band_hi_hz) return PAM_ERR_INVALID_ARG;
  for (int b = 0; b < g->n_bands; ++b) {
    const double lo = g->band_lo_hz[b], hi = g->band_hi_hz[b];
    if (!std::isfinite(lo) || !std::isfinite(hi) || lo < 0.0 || hi < lo) return PAM_ERR_INVALID_ARG;
  }
  if (g->n_depths < 1 || !g->depths_m) return PAM_ERR_INVALID_ARG;
  for (int d = 0; d < g->n_depths; ++d)
    if (!std::isfinite(g->depths_m[d]) || g->depths_m[d] < 0.0) return PAM_ERR_INVALID_ARG;
  if (g->n_x < g->n_elements || g->n_x < 2) return PAM_ERR_INVALID_ARG;
  if (g->n_x % 32 != 0 || g->n_x > kMaxNx) return PAM_ERR_UNSUPPORTED;
  if (g->lateral != PAM_LATERAL_PAD && g->lateral != PAM_LATERAL_STUFF) return PAM_ERR_INVALID_ARG;
  if (g->lateral == PAM_LATERAL_STUFF && g->n_x % g->n_elements != 0) return PAM_ERR_INVALID_ARG;
  if (g->n_sub < 1 || g->n_sub > 3) return PAM_ERR_INVALID_ARG;
  if (g->apod) {
    for (int i = 0; i < g->n_sub * g->n_elements; ++i)
      if (g->apod[i] > 1) return PAM_ERR_INVALID_ARG;
  } else if (g->pattern_m < 0) {
    return PAM_ERR_INVALID_ARG;
  }
  if (!(g->eps >= 0.0 && g->eps < 1.0)) return PAM_ERR_INVALID_ARG;
  if (g->precision < PAM_PREC_FP32 || g->precision > PAM_PREC_FP16) return PAM_ERR_INVALID_ARG;
  if (g->evanescent != PAM_EVAN_DECAY && g->evanescent != PAM_EVAN_ZERO) return PAM_ERR_INVALID_ARG;
  if (g->coherence != 0 && g->coherence != 1) return PAM_ERR_INVALID_ARG;
  if (g->coherence && (g->n_sub != 1 || g->n_x != 256 || (g->n_depths & 1))) return PAM_ERR_UNSUPPORTED;
  return PAM_OK;
}

// bins 0 < k < n_t/2 whose frequency k*fs/n_t lies in a closed band
std::vector<int32_t> select_bins(const pam_geometry_t* g) {
  std::vector<int32_t> ks;
  for (int k = 1; k < (g->n_samples + 1) / 2; ++k) {
    const double f = ((double)k * g->fs_hz) / (double)g->n_samples;
    for (int b = 0; b < g->n_bands; ++b) {
      if (g->band_lo_hz[b] <= f && f <= g->band_hi_hz[b]) {
        ks.push_back(k);
        break;
      }
    }
  }
  return ks;
}

struct LaunchShape {
  int n_dt, nw, xt, n_xg, n_split, bins_per_split;
  int ct;   // > 0: 16-depth kernels with ct 16-column tiles per consumer wave
  int fw;   // < 0: the factored two-stage kernel (N = 256, 512)
};

// Workgroup tiling of one frame: depth tiles x column groups, before any bin split.
LaunchShape k3_tiles(const pam_plan_s* p) {
  LaunchShape s;
  s.xt = 1;
  s.ct = 0;
  s.fw = 0;
  if (p->ff) {
    // all columns per workgroup, ft_depths (vector FFT) depths per workgroup
    s.fw = -1;
    s.nw = pam::kFfWaves;
    const int dpw = p->N == 512 ? pam::ft_depths<512>() : (p->N == 256 ? pam::ft_depths<256>() : pam::ft_depths<128>());
    s.n_dt = (p->n_z + dpw - 1) / dpw;
    s.n_xg = 1;
  } else if (p->N % 64 == 0) {
    // 16 depths x 64 ct columns per workgroup (4 consumer + 4 producer waves)
    s.ct = p->N % 256 == 0 ? 4 : (p->N % 128 == 0 ? 2 : 1);
    s.nw = 4;
    s.n_dt = (p->n_z + 15) / 16;
    s.n_xg = p->N / (64 * s.ct);
  } else {
    // 32 depths x 32 nw columns per workgroup (nw consumer + nw producer waves)
    s.n_dt = (p->n_z + 31) / 32;
    const int tiles = p->N / 32;
    s.nw = (tiles % 4 == 0) ? 4 : (tiles % 2 == 0 ? 2 : 1);
    s.n_xg = p->N / (32 * s.nw * s.xt);
  }
  s.n_split = 1;
  s.bins_per_split = 0;
  return s;
}

int n_acc(int n_sub, int coherence = 0) { return n_sub == 3 ? 6 : (n_sub == 2 ? 3 : (coherence ? 5 : 1)); }

// Partial-sum planes a group's workspace holds beyond one per frame: room for two rounds of
// extra workgroups.  A group of F frames splits its bins at most 1 + spare / F ways, so its
// accumulator region (F + spare planes) and with it the workspace size never shrink as F
// grows: a workspace sized for F frames serves every call of fewer frames.
int64_t k3_spare_planes(const pam_plan_s* p) {
  const LaunchShape t = k3_tiles(p);
  const int64_t tiles = (int64_t)t.n_dt * t.n_xg;
  return (2 * (int64_t)std::max(1, p->k3_slots) + tiles - 1) / tiles;
}

// The bin split of a K3 launch over n groups of frames (F[g] frames of n_sel[g] bins).
// A frame is tiles = n_dt n_xg workgroups; splitting its bins s ways makes s workgroups of
// ceil(n_sel / s) bins each, whose partial sums K4 adds.  The device holds p->k3_slots
// workgroups at once, so near-equal workgroups run in rounds: n workgroups of at most b bins
// take about ceil(n / slots) (b + c) bin-times, c (two bins) standing for a workgroup's
// start and its partial-sum write, and every split beyond the first costs K4 one more
// partial-sum plane per frame (n_acc pix floats, read at about 4 TB/s against about 5 us
// per bin).  Returns the bins-per-workgroup cap b (every group splits into ceil(n_sel / b)
// parts) that minimises the estimate, the largest such b on ties, at least 8 bins (or the
// widest band when narrower), among the caps whose splits fit the spare planes.
int k3_bin_cap(const pam_plan_s* p, const int64_t* F, const int* n_sel, int n, double* cost_out = nullptr) {
  const LaunchShape t = k3_tiles(p);
  const int64_t tiles = (int64_t)t.n_dt * t.n_xg;
  const int64_t spare = k3_spare_planes(p);
  int max_n = 0;
  for (int g = 0; g < n; ++g) max_n = std::max(max_n, n_sel[g]);
  if (max_n == 0) {
    if (cost_out) *cost_out = 0;
    return 1;
  }
  const double slots = std::max(1, p->k3_slots);
  const double plane_cost = (double)n_acc(p->n_sub, p->coherence) * p->n_z * p->N * 4.0 / 4e12 / 5e-6;
  // The estimate is constant between the caps where some group's split count changes, so it is evaluated at the
  // top of each such piece: for every group g and split count s, the largest cap that splits g s ways
  // (n_g for s = 1, ceil(n_g / (s - 1)) - 1 after), in decreasing order (a merge over the groups' sequences,
  // no storage).  This equals trying every cap.
  const int min_b = std::min(8, max_n);
  auto top = [&](int g, int s) { return s == 1 ? n_sel[g] : (n_sel[g] + s - 2) / (s - 1) - 1; };
  int next_s[pam::kMaxGroups];
  int live = 0;
  for (int g = 0; g < n; ++g) {
    next_s[g] = 1;
    live += F[g] > 0 && n_sel[g] > 0;
  }
  double best = 0;
  int best_b = max_n;
  for (bool first = true;; first = false) {
    int b = -1;
    for (int g = 0; g < n; ++g)
      if (F[g] > 0 && n_sel[g] > 0) b = std::max(b, top(g, next_s[g]));
    if (first) b = max_n;
    if (b < min_b) break;
    for (int g = 0; g < n; ++g)      // step every group past this cap
      if (F[g] > 0 && n_sel[g] > 0)
        while (top(g, next_s[g]) >= b) ++next_s[g];
    int64_t n_wg = 0;
    int job = 0;
    double k4 = 0, work = 0;
    bool fits = true;
    for (int g = 0; g < n; ++g) {
      if (F[g] == 0 || n_sel[g] == 0) continue;
      const int split = (n_sel[g] + b - 1) / b;
      const int bins = (n_sel[g] + split - 1) / split;
      fits = fits && (int64_t)(split - 1) * F[g] <= spare;
      n_wg += F[g] * tiles * split;
      work += (double)F[g] * tiles * split * (bins + 2.0);
      job = std::max(job, bins);
      k4 += plane_cost * (double)F[g] * (split - 1);
    }
    if (!fits) break;                      // smaller caps split further still
    // equal workgroups (one group) run in rounds; unequal ones (several groups, longest first) take about
    // their total work over the slots plus one longest workgroup
    const double cost = live > 1 ? work / slots + (job + 2.0) + k4 : std::ceil((double)n_wg / slots) * (job + 2.0) + k4;
    if (b == max_n || cost < best - 1e-9) {
      best = cost;
      best_b = b;
    }
  }
  if (cost_out) *cost_out = best;
  return best_b;
}

// The launch shape of one group: its tiling, and its bins split under the cap b.
LaunchShape k3_shape(const pam_plan_s* p, int n_sel, int b) {
  LaunchShape s = k3_tiles(p);
  if (n_sel == 0) {
    s.n_split = 1;
    s.bins_per_split = 0;
    return s;
  }
  const int split = (n_sel + b - 1) / b;
  s.bins_per_split = (n_sel + split - 1) / split;
  s.n_split = (n_sel + s.bins_per_split - 1) / s.bins_per_split;
  return s;
}

const Level* level_for(const pam_plan_s* p, int n_t) {
  for (const Level& lv : p->levels)
    if (lv.n_t == n_t) return &lv;
  return nullptr;
}

// bin_cap: the bins-per-workgroup cap of the launch this group is part of (-1: the group alone)
pam_status_t layout(const pam_plan_s* p, int64_t F, int n_t, pam_workspace_layout_t* out, int bin_cap = -1) {
  const Level* lv = level_for(p, n_t);
  if (!lv) return PAM_ERR_INVALID_ARG;
  if (bin_cap < 0) bin_cap = k3_bin_cap(p, &F, &lv->n_sel, 1);
  const LaunchShape s = k3_shape(p, lv->n_sel, bin_cap);
  const size_t pix = (size_t)p->n_z * p->N;
  const size_t n_blk = (pix + 255) / 256;
  pam_workspace_layout_t L{};
  size_t o = 0;
  L.spectra = o;  o = align256(o + (size_t)F * lv->n_sel * p->L * sizeof(float2));
  L.coeffs = o;   o = align256(o + (size_t)F * lv->n_sel * p->n_sub * p->N * sizeof(float2));
  L.scales = o;   o = align256(o + (size_t)F * lv->n_sel * sizeof(float));
  const size_t planes = F > 0 ? (size_t)F + (size_t)k3_spare_planes(p) : 0;   // >= n_split F
  L.accum = o;    o = align256(o + planes * n_acc(p->n_sub, p->coherence) * pix * sizeof(float));
  L.energy = o;   o = align256(o + (size_t)F * pix * sizeof(float));
  L.weight = o;   o = align256(o + (size_t)F * pix * sizeof(float));
  L.blockmax = o; o = align256(o + (size_t)F * n_blk * sizeof(float));
  L.total = std::max<size_t>(o, 256);
  L.n_sel = lv->n_sel;
  L.n_split = s.n_split;
  L.n_acc = n_acc(p->n_sub, p->coherence);
  *out = L;
  return PAM_OK;
}

// Where a K3 dispatch goes: a launch on stream st, or, with occ set, no launch but the
// number of the kernel's workgroups one CU holds (written to *occ).
struct Target {
  hipStream_t st;
  int* occ;
};

// K3 kernels: NC consumer + NC producer waves, NC*32 columns per workgroup.
// LDS above 64 KiB needs the per-kernel attribute.
// (Every kernel shares one signature, so the attribute is set per launch rather
// than cached in a per-instantiation static.)
template <typename K>
hipError_t launch_with_lds(K kernel, int nc, size_t lds, const pam::K3Args& a, int blocks, Target st) {
  const hipError_t attr =
      hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  if (st.occ)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(st.occ, reinterpret_cast<const void*>(kernel), nc * 128, lds);
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(nc * 128), lds, st.st, a);
  return hipGetLastError();
}

template <int NSUB, int NC>
hipError_t launch_prec(int precision, const pam::K3Args& a, int blocks, Target st) {
  switch (precision) {
    case PAM_PREC_SPLIT_BF16:
      return launch_with_lds(pam::k3_fields_split<__bf16, 3, NSUB, NC>, NC, pam::k3_split_lds<3, NSUB, NC>(), a, blocks, st);
    case PAM_PREC_SPLIT_FP16:
      return launch_with_lds(pam::k3_fields_split<_Float16, 3, NSUB, NC>, NC, pam::k3_split_lds<3, NSUB, NC>(), a, blocks, st);
    case PAM_PREC_BF16:
      return launch_with_lds(pam::k3_fields_split<__bf16, 1, NSUB, NC>, NC, pam::k3_split_lds<1, NSUB, NC>(), a, blocks, st);
    case PAM_PREC_FP16:
      return launch_with_lds(pam::k3_fields_split<_Float16, 1, NSUB, NC>, NC, pam::k3_split_lds<1, NSUB, NC>(), a, blocks, st);
    default:
      return launch_with_lds(pam::k3_fields_fp32<NSUB, NC>, NC, pam::k3_fp32_lds<NSUB, NC>(), a, blocks, st);
  }
}

template <int NSUB, int CT>
hipError_t launch_prec16(int precision, const pam::K3Args& a, int blocks, Target st) {
  switch (precision) {
    case PAM_PREC_SPLIT_BF16:
      return launch_with_lds(pam::k3f16_split<__bf16, 3, NSUB, CT>, 4, pam::k3f16_split_lds<3, NSUB, CT>(), a, blocks, st);
    case PAM_PREC_SPLIT_FP16:
      return launch_with_lds(pam::k3f16_split<_Float16, 3, NSUB, CT>, 4, pam::k3f16_split_lds<3, NSUB, CT>(), a, blocks, st);
    case PAM_PREC_BF16:
      return launch_with_lds(pam::k3f16_split<__bf16, 1, NSUB, CT>, 4, pam::k3f16_split_lds<1, NSUB, CT>(), a, blocks, st);
    case PAM_PREC_FP16:
      return launch_with_lds(pam::k3f16_split<_Float16, 1, NSUB, CT>, 4, pam::k3f16_split_lds<1, NSUB, CT>(), a, blocks, st);
    default:
      return launch_with_lds(pam::k3f16_fp32<NSUB, CT>, 4, pam::k3f16_fp32_lds<NSUB, CT>(), a, blocks, st);
  }
}

// Kernels with more than 64 KB of dynamic LDS: the attribute is set before each launch
// for the largest size the instantiation takes.
template <typename K>
hipError_t launch_big_lds(K kernel, int nw, size_t lds, size_t lds_max, const pam::K3Args& a,
                          const pam::K3Groups& grp, int blocks, Target st) {
  const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
  if (attr != hipSuccess) return attr;
  if (lds > lds_max) return hipErrorInvalidValue;
  if (st.occ)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(st.occ, reinterpret_cast<const void*>(kernel), nw * 64, lds);
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(nw * 64), lds, st.st, a, grp);
  return hipGetLastError();
}

template <int NSUB, int R>
hipError_t launch_ff_r(int precision, const pam::K3Args& a, const pam::K3Groups& grp, int blocks, Target st) {
  using namespace pam;
  const size_t lds = k3ff_lds<NSUB, R>();
  switch (precision) {
    case PAM_PREC_SPLIT_BF16: return launch_big_lds(k3ff<__bf16, 3, NSUB, false, R>, kFfWaves, lds, lds, a, grp, blocks, st);
    case PAM_PREC_SPLIT_FP16: return launch_big_lds(k3ff<_Float16, 3, NSUB, false, R>, kFfWaves, lds, lds, a, grp, blocks, st);
    case PAM_PREC_BF16: return launch_big_lds(k3ff<__bf16, 1, NSUB, false, R>, kFfWaves, lds, lds, a, grp, blocks, st);
    case PAM_PREC_FP16: return launch_big_lds(k3ff<_Float16, 1, NSUB, false, R>, kFfWaves, lds, lds, a, grp, blocks, st);
    default: return launch_big_lds(k3ff<float, 1, NSUB, false, R>, kFfWaves, lds, lds, a, grp, blocks, st);
  }
}

template <int NSUB>
hipError_t launch_ff(int precision, const pam::K3Args& a, const pam::K3Groups& grp, int blocks, Target st) {
  // FP32 operands: the vector FFT kernel (32, 16 or 8 depths per workgroup; 16 and 8 like k3ff)
  if (precision == PAM_PREC_FP32 && a.N == 256)
    return launch_big_lds(pam::k3fft<NSUB>, pam::kFtWaves, pam::k3fft_lds<NSUB>(), pam::k3fft_lds<NSUB>(), a, grp,
                          blocks, st);
  if (precision == PAM_PREC_FP32 && a.N == 512)
    return launch_big_lds(pam::k3fft<NSUB, false, 512>, pam::kFtWaves, pam::k3fft_lds<NSUB, 512>(),
                          pam::k3fft_lds<NSUB, 512>(), a, grp, blocks, st);
  if (precision == PAM_PREC_FP32 && a.N == 128)
    return launch_big_lds(pam::k3fft<NSUB, false, 128>, pam::kFtWaves, pam::k3fft_lds<NSUB, 128>(),
                          pam::k3fft_lds<NSUB, 128>(), a, grp, blocks, st);
  return a.N == 512 ? launch_ff_r<NSUB, 2>(precision, a, grp, blocks, st)
                    : launch_ff_r<NSUB, 1>(precision, a, grp, blocks, st);
}

template <int NSUB>
hipError_t launch_shape(int precision, const LaunchShape& s, const pam::K3Args& a, const pam::K3Groups& grp,
                        int blocks, Target st) {
  if (s.fw < 0) return launch_ff<NSUB>(precision, a, grp, blocks, st);
  if (grp.n > 0) return hipErrorInvalidValue;      // grouped work lists run on the factored kernels only
  if (s.ct == 4) return launch_prec16<NSUB, 4>(precision, a, blocks, st);
  if (s.ct == 2) return launch_prec16<NSUB, 2>(precision, a, blocks, st);
  if (s.ct == 1) return launch_prec16<NSUB, 1>(precision, a, blocks, st);
  if (s.nw == 4) return launch_prec<NSUB, 4>(precision, a, blocks, st);
  if (s.nw == 2) return launch_prec<NSUB, 2>(precision, a, blocks, st);
  return launch_prec<NSUB, 1>(precision, a, blocks, st);
}

hipError_t launch_k3(int precision, int n_sub, const LaunchShape& s, const pam::K3Args& a, const pam::K3Groups& grp,
                     int blocks, Target st, int coherence) {
  if (coherence) {
    using namespace pam;
    const size_t lds = k3ff_lds<1>();
    switch (precision) {
      case PAM_PREC_SPLIT_BF16: return launch_big_lds(k3ff<__bf16, 3, 1, true>, kFfWaves, lds, lds, a, grp, blocks, st);
      case PAM_PREC_SPLIT_FP16: return launch_big_lds(k3ff<_Float16, 3, 1, true>, kFfWaves, lds, lds, a, grp, blocks, st);
      case PAM_PREC_BF16: return launch_big_lds(k3ff<__bf16, 1, 1, true>, kFfWaves, lds, lds, a, grp, blocks, st);
      case PAM_PREC_FP16: return launch_big_lds(k3ff<_Float16, 1, 1, true>, kFfWaves, lds, lds, a, grp, blocks, st);
      default: return launch_big_lds(k3fft<1, true>, kFtWaves, k3fft_lds<1>(), k3fft_lds<1>(), a, grp, blocks, st);
    }
  }
  switch (n_sub) {
    case 3: return launch_shape<3>(precision, s, a, grp, blocks, st);
    case 2: return launch_shape<2>(precision, s, a, grp, blocks, st);
    default: return launch_shape<1>(precision, s, a, grp, blocks, st);
  }
}

}  // namespace

extern "C" {

const char* pam_status_string(pam_status_t s) {
  switch (s) {
    case PAM_OK: return "ok";
    case PAM_ERR_INVALID_ARG: return "invalid argument";
    case PAM_ERR_OOM: return "out of memory";
    case PAM_ERR_DEVICE: return "device error";
    case PAM_ERR_UNSUPPORTED: return "unsupported size or mode";
    case PAM_ERR_WORKSPACE: return "workspace missing or too small";
  }
  return "unknown status";
}

pam_status_t pam_plan(const pam_geometry_t* g, int device, pam_plan_t* out) {
  if (!out) return PAM_ERR_INVALID_ARG;
  *out = nullptr;
  pam_status_t st = validate(g);
  if (st != PAM_OK) return st;
  std::vector<int32_t> ks = select_bins(g);
  if (ks.empty()) return PAM_ERR_INVALID_ARG;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return PAM_ERR_DEVICE;
  DeviceGuard guard(device);
  if (!guard.ok) return PAM_ERR_DEVICE;

  pam_plan_s* p = new (std::nothrow) pam_plan_s();
  if (!p) return PAM_ERR_OOM;
  p->device = device;
  p->L = g->n_elements;
  p->n_t = g->n_samples;
  p->N = g->n_x;
  p->n_z = g->n_depths;
  p->n_sub = g->n_sub;
  p->n_bins = (int)ks.size();
  p->eps = g->eps > 0.0 ? g->eps : 1e-3;
  p->precision = g->precision;
  p->zero_evanescent = g->evanescent == PAM_EVAN_ZERO;
  p->coherence = g->coherence;
  p->bins = ks;
  const int L = p->L, N = p->N, HQ = N / 2 + 1;

  // lateral placement: grid column of each element and grid spacing
  double dx;
  if (g->lateral == PAM_LATERAL_PAD) {
    p->col0 = (N - L) / 2;
    p->col_step = 1;
    dx = g->pitch_m;
  } else {
    p->col0 = 0;
    p->col_step = N / L;
    dx = g->pitch_m / p->col_step;
  }
  // element and pixel coordinates (array centre at x = 0)
  {
    const double centre = p->col0 + p->col_step * (L - 1) / 2.0;
    p->fs = g->fs_hz;
    p->c = g->c_mps;
    p->dx = dx;
    p->x_first = -centre * dx;
    p->xl_first = (p->col0 - centre) * dx;
    p->pitch = p->col_step * dx;
  }
  // apodization masks: explicit or Pattern-m (a_i[l] = 1 iff floor(l/m) mod n == i)
  std::vector<float> masks((size_t)p->n_sub * L, 0.f);
  const int m = g->pattern_m > 0 ? g->pattern_m : 16;
  for (int i = 0; i < p->n_sub; ++i)
    for (int l = 0; l < L; ++l)
      masks[(size_t)i * L + l] = g->apod ? (float)g->apod[(size_t)i * L + l] : (((l / m) % p->n_sub) == i ? 1.f : 0.f);
  // kz / (2 pi) in cycles per metre for the folded half grid q = 0..N/2:
  // k / (2 pi) = f / c and kx_q / (2 pi) = q / (N dx); negative values mark
  // evanescent components (decay rate / (2 pi)).
  std::vector<double> kz((size_t)p->n_bins * HQ);
  for (int b = 0; b < p->n_bins; ++b) {
    const double f = ((double)ks[b] * g->fs_hz) / (double)g->n_samples;
    const double kc = f / g->c_mps;
    for (int q = 0; q < HQ; ++q) {
      const double kxc = (double)q / ((double)N * dx);
      const double d = kc * kc - kxc * kxc;
      kz[(size_t)b * HQ + q] = d >= 0.0 ? std::sqrt(d) : -std::sqrt(-d);
    }
  }
  std::vector<double> z(g->depths_m, g->depths_m + p->n_z);
  // transform tables from exact integer angles
  std::vector<float2> tw(p->n_t / 2), twx(N);
  for (int i = 0; i < p->n_t / 2; ++i) {
    const double a = 2.0 * kPi * (double)i / (double)p->n_t;
    tw[i] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  for (int i = 0; i < N; ++i) {
    const double a = 2.0 * kPi * (double)i / (double)N;
    twx[i] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  // Factored transform for N = 256 and 512 (k3_factored.hpp, and the vector FFT of k3_fft.hpp
  // in FP32), and N = 128 in FP32 (k3_fft.hpp); the other cases take the folded DFT basis
  // (k3_fields*.hpp), built only for them.
  p->ff = (N == 256 || N == 512 || (N == 128 && p->precision == PAM_PREC_FP32));
  std::vector<float> basis(p->ff ? 0 : (size_t)N * N);
  for (int s = 0; s < (p->ff ? 0 : N); ++s) {
    const int q = s >> 1;
    for (int x = 0; x < N; ++x) {
      double v;
      if ((s & 1) == 0) {
        v = std::cos(2.0 * kPi * (double)(((long long)q * x) % N) / (double)N);
      } else if (q == 0) {
        v = (x & 1) ? -1.0 : 1.0;  // cos(pi x)
      } else {
        v = std::sin(2.0 * kPi * (double)(((long long)q * x) % N) / (double)N);
      }
      basis[(size_t)s * N + x] = (float)v;
    }
  }

  std::vector<uint16_t> bhi, blo;
  if (is_split(p->precision) && !p->ff) {
    bhi.resize((size_t)N * N);
    blo.resize((size_t)N * N);
    const bool h16 = is_fp16(p->precision);
    for (int s = 0; s < N; ++s)
      for (int x = 0; x < N; ++x) {
        const float v = basis[(size_t)s * N + x];
        const uint16_t hi = h16 ? to_fp16(v) : to_bf16(v);
        const float r = v - (h16 ? from_fp16(hi) : from_bf16(hi));
        // groups of 8 slots, then x, then the 8 slots: one 16-byte piece per (group, x)
        const size_t o = ((size_t)(s / 8) * N + x) * 8 + s % 8;
        bhi[o] = hi;
        blo[o] = h16 ? to_fp16(r) : to_bf16(r);
      }
  }

  // Factored transform (N = 256 = 16 x 16; N = 512 as two such transforms over even and
  // odd q): the 16-point DFT matrix W(x, m) = e^{2 pi i m x / 16} in real form, rows
  // (x, re/im) = x + 16 ro, the stage twiddles and (N = 512) the combination twiddles, all
  // in lane order of the matrix-core operands.  Lane l: column c = l % 32, half h = l / 32.
  std::vector<float> ff_w32;
  std::vector<uint16_t> ff_w16;
  std::vector<float2> ff_tw, ff_tw2, ff_tw_vec, ff_tw2_vec;
  if (p->ff) {
    auto wval = [](int row, int m, int ri) {
      const int x = row % 16, ro = row / 16;
      const double th = 2.0 * kPi * (double)((m * x) % 16) / 16.0;
      const double c = std::cos(th), sn = std::sin(th);
      return ro == 0 ? (ri == 0 ? c : -sn) : (ri == 0 ? sn : c);
    };
    ff_w32.resize(64 * 16);
    ff_w16.resize(64 * 32);
    ff_tw.resize(64 * 8);
    const bool h16 = is_fp16(p->precision);
    for (int l = 0; l < 64; ++l) {
      const int c = l % 32, h = l / 32;
      // FP32 k-step t: k = 2t + h <-> input m = 8h + t/2, re/im t%2
      for (int t = 0; t < 16; ++t) ff_w32[l * 16 + t] = (float)wval(c, 8 * h + t / 2, t % 2);
      // 16-bit k-step s, element j: k = 16s + 8h + j <-> m = 8h + 4s + j/2, re/im j%2
      for (int s2 = 0; s2 < 2; ++s2)
        for (int j = 0; j < 8; ++j) {
          const float v = (float)wval(c, 8 * h + 4 * s2 + j / 2, j % 2);
          const uint16_t hi = h16 ? to_fp16(v) : to_bf16(v);
          const float r = v - (h16 ? from_fp16(hi) : from_bf16(hi));
          ff_w16[l * 32 + s2 * 16 + j] = hi;
          ff_w16[l * 32 + s2 * 16 + 8 + j] = h16 ? to_fp16(r) : to_bf16(r);
        }
      // stage-1 output v (0..7) of lane l is x1 = 8(v/4) + 4h + v%4 of column q2 = c % 16
      for (int v = 0; v < 8; ++v) {
        const int x1 = 8 * (v / 4) + 4 * h + v % 4, q2 = c % 16;
        const double th = 2.0 * kPi * (double)((q2 * x1) % 256) / 256.0;
        const double sc = h16 ? 1.0 / 16.0 : 1.0;   // FP16 operands keep stage-1 results in range
        ff_tw[l * 8 + v] = make_float2((float)(std::cos(th) * sc), (float)(std::sin(th) * sc));
      }
    }
    // vector FFT kernel: [x1][j] = e^{2 pi i q2 x1 / N} with q2 = j (N = 256, 512) or j % 8 (N = 128)
    ff_tw_vec.resize(256);
    const int NT = N == 128 ? 128 : 256;
    for (int x1 = 0; x1 < 16; ++x1)
      for (int jj = 0; jj < 16; ++jj) {
        const int q2 = N == 128 ? jj % 8 : jj;
        const double th = 2.0 * kPi * (double)((q2 * x1) % NT) / (double)NT;
        ff_tw_vec[x1 * 16 + jj] = make_float2((float)std::cos(th), (float)std::sin(th));
      }
    // vector FFT kernel, N = 512: [x2][j] = e^{2 pi i (j + 16 x2) / 512}
    ff_tw2_vec.assign(256, make_float2(0.f, 0.f));
    if (N == 512)
      for (int x2 = 0; x2 < 16; ++x2)
        for (int j = 0; j < 16; ++j) {
          const double th = 2.0 * kPi * (double)(j + 16 * x2) / 512.0;
          ff_tw2_vec[x2 * 16 + j] = make_float2((float)std::cos(th), (float)std::sin(th));
        }
    // stage-3 output v of lane l is x' = c % 16 + 16 (8(v/4) + 4h + v%4) of half c / 16
    ff_tw2.assign(64 * 8, make_float2(0.f, 0.f));
    if (N == 512)
      for (int l = 0; l < 64; ++l)
        for (int v = 0; v < 8; ++v) {
          const int c = l % 32, h = l / 32, xp = c % 16 + 16 * (8 * (v / 4) + 4 * h + v % 4);
          const double th = 2.0 * kPi * (double)xp / 512.0;
          ff_tw2[l * 8 + v] = make_float2((float)std::cos(th), (float)std::sin(th));
        }
  }

  do {
    if (is_split(p->precision) && !p->ff) {
      if ((st = upload(p, &p->d_bhi, bhi.data(), bhi.size())) != PAM_OK) break;
      if ((st = upload(p, &p->d_blo, blo.data(), blo.size())) != PAM_OK) break;
    }
    if (p->ff) {
      if ((st = upload(p, &p->d_ff_w32, ff_w32.data(), ff_w32.size())) != PAM_OK) break;
      if ((st = upload(p, &p->d_ff_w16, ff_w16.data(), ff_w16.size())) != PAM_OK) break;
      if ((st = upload(p, &p->d_ff_tw, ff_tw.data(), ff_tw.size())) != PAM_OK) break;
      if ((st = upload(p, &p->d_ff_tw2, ff_tw2.data(), ff_tw2.size())) != PAM_OK) break;
      if ((st = upload(p, &p->d_ff_tw_vec, ff_tw_vec.data(), ff_tw_vec.size())) != PAM_OK) break;
      if ((st = upload(p, &p->d_ff_tw2_vec, ff_tw2_vec.data(), ff_tw2_vec.size())) != PAM_OK) break;
    }
    if ((st = upload(p, &p->d_z, z.data(), z.size())) != PAM_OK) break;
    if ((st = upload(p, &p->d_tw, tw.data(), tw.size())) != PAM_OK) break;
    if ((st = upload(p, &p->d_twx, twx.data(), twx.size())) != PAM_OK) break;
    if ((st = upload(p, &p->d_masks, masks.data(), masks.size())) != PAM_OK) break;
    {
      std::vector<int32_t> subs(L, 0);
      for (int i = 0; i < p->n_sub; ++i)
        for (int l = 0; l < L; ++l)
          if (masks[(size_t)i * L + l] != 0.f) subs[l] |= 1 << i;
      if ((st = upload(p, &p->d_subs, subs.data(), subs.size())) != PAM_OK) break;
    }
    if (!p->ff && (st = upload(p, &p->d_basis, basis.data(), basis.size())) != PAM_OK) break;
    // bin subsets for records of n_t / 2^j samples
    for (int stride = 1; p->n_t / stride >= kMinSamples; stride <<= 1) {
      Level lv;
      lv.n_t = p->n_t / stride;
      lv.stride = stride;
      std::vector<int32_t> ksel;
      std::vector<double> kz_lv;
      for (int b = 0; b < p->n_bins; ++b)
        if (ks[b] % stride == 0) {
          ksel.push_back(ks[b] / stride);
          kz_lv.insert(kz_lv.end(), kz.begin() + (size_t)b * HQ, kz.begin() + (size_t)(b + 1) * HQ);
          kz_lv.resize(kz_lv.size() + (pam::kz_row(N) - HQ), 0.0);
        }
      lv.n_sel = (int)ksel.size();
      if ((st = upload(p, &lv.d_ksel, ksel.data(), ksel.size())) != PAM_OK) break;
      if ((st = upload(p, &lv.d_kz, kz_lv.data(), kz_lv.size())) != PAM_OK) break;
      if (p->ff) {
        // [n_sel][r][q1] at q = (N / 16) q1 + r; kz depends on q through min(q, N - q)
        std::vector<double> kzff((size_t)lv.n_sel * N);
        const int n2 = N / 16;
        for (int b = 0; b < lv.n_sel; ++b)
          for (int r = 0; r < n2; ++r)
            for (int q1 = 0; q1 < 16; ++q1) {
              const int q = n2 * q1 + r, qf = std::min(q, N - q);
              kzff[(size_t)b * N + r * 16 + q1] = kz_lv[(size_t)b * pam::kz_row(N) + qf];
            }
        if ((st = upload(p, &lv.d_kzff, kzff.data(), kzff.size())) != PAM_OK) break;
        std::vector<int32_t> ev(lv.n_sel, 0);
        for (int b = 0; b < lv.n_sel; ++b)
          for (int q = 0; q < N; ++q) ev[b] |= kzff[(size_t)b * N + q] < 0.0 ? 1 : 0;
        if ((st = upload(p, &lv.d_ev, ev.data(), ev.size())) != PAM_OK) break;
      }
      p->levels.push_back(lv);
    }
  } while (false);
  if (st != PAM_OK) {
    free_plan(p);
    return st;
  }
  // the K3 workgroups the device holds at once: the bin split plans its launches in rounds of these
  {
    pam::K3Args a{};
    a.N = p->N;
    const pam::K3Groups none{};
    int occ = 0, cus = 0;
    if (launch_k3(p->precision, p->n_sub, k3_tiles(p), a, none, 0, Target{nullptr, &occ}, p->coherence) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || occ < 1 ||
        cus < 1) {
      free_plan(p);
      return PAM_ERR_DEVICE;
    }
    p->k3_slots = occ * cus;
    p->n_cus = cus;
  }
  *out = p;
  return PAM_OK;
}

pam_status_t pam_plan_get_info(pam_plan_t p, pam_plan_info_t* info) {
  if (!p || !info) return PAM_ERR_INVALID_ARG;
  info->n_bins = p->n_bins;
  info->n_z = p->n_z;
  info->n_x = p->N;
  info->n_sub = p->n_sub;
  info->n_elements = p->L;
  info->n_samples = p->n_t;
  info->n_pairs = p->n_sub == 3 ? 3 : (p->n_sub == 2 ? 1 : 0);
  info->device = p->device;
  return PAM_OK;
}

pam_status_t pam_plan_get_bins(pam_plan_t p, int32_t* bins, int32_t capacity) {
  if (!p || !bins || capacity < p->n_bins) return PAM_ERR_INVALID_ARG;
  std::memcpy(bins, p->bins.data(), sizeof(int32_t) * p->n_bins);
  return PAM_OK;
}

pam_status_t pam_workspace_layout(pam_plan_t p, int64_t n_frames, int32_t n_t, pam_workspace_layout_t* out) {
  if (!p || !out || n_frames < 0) return PAM_ERR_INVALID_ARG;
  return layout(p, n_frames, n_t, out);
}

pam_status_t pam_workspace_size(pam_plan_t p, int64_t n_frames, int32_t n_t, size_t* bytes) {
  if (!bytes) return PAM_ERR_INVALID_ARG;
  pam_workspace_layout_t L;
  pam_status_t st = pam_workspace_layout(p, n_frames, n_t, &L);
  if (st == PAM_OK) *bytes = L.total;
  return st;
}

}  // extern "C"

namespace {

// method 0: angular spectrum (K1, K2, K3 fields, K4); method 1: frequency-domain
// delay-and-sum (K1, K3 TEA fields, K4; no lateral transform)
// Workspace of a grouped call: the groups' layouts back to back (each 256-byte aligned).
// *one_launch: the fields stage runs as one grouped launch over all groups (factored kernels, more than one
// group with frames, and the cost estimate of that launch below the sum of the groups' own launches); cap[g]:
// group g's bins-per-workgroup cap, the shared one for a grouped launch, else the group's own.
pam_status_t grouped_layout(const pam_plan_s* p, const pam_group_t* groups, int n_groups,
                            pam_workspace_layout_t* W, size_t* base, size_t* total,
                            int* cap, bool* one_launch) {
  if (n_groups < 1 || n_groups > pam::kMaxGroups || !groups) return PAM_ERR_INVALID_ARG;
  int64_t F_total = 0;
  int64_t F[pam::kMaxGroups];
  int n_sel[pam::kMaxGroups];
  int live = 0;
  for (int g = 0; g < n_groups; ++g) {
    if (groups[g].n_frames < 0) return PAM_ERR_INVALID_ARG;
    const Level* lv = level_for(p, groups[g].n_t);
    if (!lv) return PAM_ERR_INVALID_ARG;
    F[g] = groups[g].n_frames;
    n_sel[g] = lv->n_sel;
    F_total += groups[g].n_frames;
    live += groups[g].n_frames > 0;
  }
  if (F_total > 65535) return PAM_ERR_UNSUPPORTED;
  double separate = 0;
  for (int g = 0; g < n_groups; ++g) {
    double c = 0;
    cap[g] = k3_bin_cap(p, &F[g], &n_sel[g], 1, &c);
    separate += c;
  }
  *one_launch = false;
  if (p->ff && live > 1) {
    double together = 0;
    const int shared = k3_bin_cap(p, F, n_sel, n_groups, &together);
    if (together < separate) {
      *one_launch = true;
      for (int g = 0; g < n_groups; ++g) cap[g] = shared;
    }
  }
  size_t o = 0;
  for (int g = 0; g < n_groups; ++g) {
    const pam_status_t st = layout(p, groups[g].n_frames, groups[g].n_t, &W[g], cap[g]);
    if (st != PAM_OK) return st;
    base[g] = o;
    o = align256(o + W[g].total);
  }
  *total = std::max<size_t>(o, 256);
  return PAM_OK;
}

// One call over groups of frames, each group one record length, frames packed group after
// group in rf and in the outputs.  K1, K2 and K4 run per group; K3 runs as one grouped
// work list on the factored kernels (else per group).  events: stage marks (one group only).
pam_status_t run_groups(pam_plan_t p, const float* rf, const pam_group_t* groups, int n_groups, float* image,
                        float* nncc, float* rho_pairs, void* workspace, size_t ws_bytes, void* hip_stream,
                        void* const* events, int method) {
  if (!p) return PAM_ERR_INVALID_ARG;
  // per group, fixed arrays of at most kMaxGroups entries: the call allocates no host memory either
  pam_workspace_layout_t W[pam::kMaxGroups];
  size_t wbase[pam::kMaxGroups];
  size_t total = 0;
  int cap[pam::kMaxGroups];
  bool one_launch = false;
  pam_status_t st = grouped_layout(p, groups, n_groups, W, wbase, &total, cap, &one_launch);
  if (st != PAM_OK) return st;
  if (events && n_groups != 1) return PAM_ERR_INVALID_ARG;
  int64_t F_total = 0;
  for (int g = 0; g < n_groups; ++g) F_total += groups[g].n_frames;
  if (F_total == 0) return PAM_OK;
  if (!rf || !image) return PAM_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < total || (reinterpret_cast<uintptr_t>(workspace) & 255u)) return PAM_ERR_WORKSPACE;
  if (rho_pairs && p->n_sub == 1) return PAM_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok) return PAM_ERR_DEVICE;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  auto mark = [&](int i) -> bool {
    return !events || hipEventRecord(static_cast<hipEvent_t>(events[i]), stream) == hipSuccess;
  };
  if (!mark(0)) return PAM_ERR_DEVICE;
  const int pix = p->n_z * p->N;
  const int n_pairs = p->n_sub == 3 ? 3 : (p->n_sub == 2 ? 1 : 0);

  // per group: its record length level, frames, workspace and output pointers
  struct G {
    const Level* lv;
    int F, n_t;
    const float* rf;
    float *image, *nncc, *rho;
    float2 *spectra, *coeffs;
    float *scales, *accum, *energy, *weight, *blockmax;
    LaunchShape s;
  };
  G gs[pam::kMaxGroups] = {};
  {
    size_t rf_off = 0, out_off = 0;
    for (int g = 0; g < n_groups; ++g) {
      G& q = gs[g];
      q.lv = level_for(p, groups[g].n_t);
      q.F = (int)groups[g].n_frames;
      q.n_t = groups[g].n_t;
      q.rf = rf + rf_off;
      q.image = image + out_off * pix;
      q.nncc = nncc ? nncc + out_off * pix : nullptr;
      q.rho = rho_pairs ? rho_pairs + out_off * n_pairs * pix : nullptr;
      char* ws = static_cast<char*>(workspace) + wbase[g];
      q.spectra = reinterpret_cast<float2*>(ws + W[g].spectra);
      q.coeffs = reinterpret_cast<float2*>(ws + W[g].coeffs);
      q.scales = reinterpret_cast<float*>(ws + W[g].scales);
      q.accum = reinterpret_cast<float*>(ws + W[g].accum);
      q.energy = reinterpret_cast<float*>(ws + W[g].energy);
      q.weight = reinterpret_cast<float*>(ws + W[g].weight);
      q.blockmax = reinterpret_cast<float*>(ws + W[g].blockmax);
      q.s = k3_shape(p, q.lv->n_sel, cap[g]);
      rf_off += (size_t)q.F * p->L * q.n_t;
      out_off += (size_t)q.F;
    }
  }

  // The stages of one group.
  // K1: time FFT, one workgroup per (channel, frame)
  auto stage_k1 = [&](const G& q) -> pam_status_t {
    if (q.F == 0) return PAM_OK;
    pam::K1Args a{q.rf, q.spectra, p->d_tw, q.lv->d_ksel, p->L, q.n_t, ilog2(q.n_t / 2), q.lv->stride, q.lv->n_sel,
                  q.F};
    // two channels per workgroup where they divide L (up to 4096 samples), else one
    const int ch = (p->L % 2 == 0 && q.n_t <= 4096) ? 2 : 1;
    const size_t lds = (size_t)ch * (q.n_t / 2 + q.n_t / 16) * sizeof(float2);   // ch k1_lds_points
    const long long items = (long long)p->L / ch * q.F;
    auto k1 = [&](auto kernel) -> bool {
      // n_t = 16384 takes more than 64 KiB of LDS: the kernel needs the attribute
      if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return false;
      // From 2048 samples one workgroup per channel group (the groups of a frame are resident together, so
      // their partial bin lines meet in L2: 0.047 vs 0.050 ms for 64 x 128 channels of 4096 samples); shorter
      // records persistent, as many workgroups as the device holds, each walking its groups with the next
      // group's samples prefetched (0.011 vs 0.012 ms for 64 x 64 channels of 1024 samples).
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kernel), 256 * ch, lds) !=
              hipSuccess ||
          occ < 1)
        return false;
      const unsigned blocks =
          (unsigned)(q.n_t >= 2048 ? items : std::min<long long>(items, (long long)occ * p->n_cus));
      hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256 * ch), lds, stream, a);
      return true;
    };
    bool ok = false;
    switch (ilog2(q.n_t / 2) * 8 + ch) {   // n_t = 32 .. 16384
      case 4 * 8 + 1: ok = k1(pam::k1_time_fft<4>); break;
      case 5 * 8 + 1: ok = k1(pam::k1_time_fft<5>); break;
      case 6 * 8 + 1: ok = k1(pam::k1_time_fft<6>); break;
      case 7 * 8 + 1: ok = k1(pam::k1_time_fft<7>); break;
      case 8 * 8 + 1: ok = k1(pam::k1_time_fft<8>); break;
      case 9 * 8 + 1: ok = k1(pam::k1_time_fft<9>); break;
      case 10 * 8 + 1: ok = k1(pam::k1_time_fft<10>); break;
      case 11 * 8 + 1: ok = k1(pam::k1_time_fft<11>); break;
      case 12 * 8 + 1: ok = k1(pam::k1_time_fft<12>); break;
      case 13 * 8 + 1: ok = k1(pam::k1_time_fft<13>); break;
      case 4 * 8 + 2: ok = k1(pam::k1_time_fft<4, 2>); break;
      case 5 * 8 + 2: ok = k1(pam::k1_time_fft<5, 2>); break;
      case 6 * 8 + 2: ok = k1(pam::k1_time_fft<6, 2>); break;
      case 7 * 8 + 2: ok = k1(pam::k1_time_fft<7, 2>); break;
      case 8 * 8 + 2: ok = k1(pam::k1_time_fft<8, 2>); break;
      case 9 * 8 + 2: ok = k1(pam::k1_time_fft<9, 2>); break;
      case 10 * 8 + 2: ok = k1(pam::k1_time_fft<10, 2>); break;
      case 11 * 8 + 2: ok = k1(pam::k1_time_fft<11, 2>); break;
      default: return PAM_ERR_UNSUPPORTED;
    }
    if (!ok) return PAM_ERR_DEVICE;
    if (hipGetLastError() != hipSuccess) return PAM_ERR_DEVICE;
    return PAM_OK;
  };
  // K2: apodization + lateral transform, per (frame, bin)
  auto stage_k2 = [&](const G& q) -> pam_status_t {
    if (method != 0 || q.F == 0) return PAM_OK;
    const long long items = (long long)q.F * q.lv->n_sel;
    if (items > 0x7fffffffLL) return PAM_ERR_UNSUPPORTED;
    pam::K2Args a{q.spectra, q.coeffs, q.scales, p->d_twx, p->d_masks, p->L, p->N, p->n_sub, q.lv->n_sel,
                  p->col0, p->col_step, p->ff ? pam::kFfN1 : 0, is_fp16(p->precision) ? 1 : 0, (int32_t)items};
    if (p->ff) {
      // factored order: the lateral FFT, one wave per (frame, bin)
      const dim3 grid((unsigned)((items + 3) / 4));
      switch (p->N * 4 + p->n_sub) {
        case 128 * 4 + 1: hipLaunchKernelGGL((pam::k2_fft<1, 8>), grid, dim3(256), 0, stream, a); break;
        case 128 * 4 + 2: hipLaunchKernelGGL((pam::k2_fft<2, 8>), grid, dim3(256), 0, stream, a); break;
        case 128 * 4 + 3: hipLaunchKernelGGL((pam::k2_fft<3, 8>), grid, dim3(256), 0, stream, a); break;
        case 256 * 4 + 1: hipLaunchKernelGGL((pam::k2_fft<1, 16>), grid, dim3(256), 0, stream, a); break;
        case 256 * 4 + 2: hipLaunchKernelGGL((pam::k2_fft<2, 16>), grid, dim3(256), 0, stream, a); break;
        case 256 * 4 + 3: hipLaunchKernelGGL((pam::k2_fft<3, 16>), grid, dim3(256), 0, stream, a); break;
        case 512 * 4 + 1: hipLaunchKernelGGL((pam::k2_fft<1, 32>), grid, dim3(256), 0, stream, a); break;
        case 512 * 4 + 2: hipLaunchKernelGGL((pam::k2_fft<2, 32>), grid, dim3(256), 0, stream, a); break;
        case 512 * 4 + 3: hipLaunchKernelGGL((pam::k2_fft<3, 32>), grid, dim3(256), 0, stream, a); break;
        default: return PAM_ERR_UNSUPPORTED;
      }
    } else {
      const size_t lds = (size_t)(p->N + 3 * p->L + 2 * p->n_sub * p->N) * sizeof(float2);
      if (p->n_sub == 3)
        hipLaunchKernelGGL(pam::k2_lateral<3>, dim3(q.lv->n_sel, q.F), dim3(256), lds, stream, a);
      else if (p->n_sub == 2)
        hipLaunchKernelGGL(pam::k2_lateral<2>, dim3(q.lv->n_sel, q.F), dim3(256), lds, stream, a);
      else
        hipLaunchKernelGGL(pam::k2_lateral<1>, dim3(q.lv->n_sel, q.F), dim3(256), lds, stream, a);
    }
    if (hipGetLastError() != hipSuccess) return PAM_ERR_DEVICE;
    return PAM_OK;
  };
  auto args_for = [&](const G& q) {
    return pam::K3Args{q.coeffs, q.scales, q.lv->d_kz, p->d_z, p->d_basis, p->d_bhi, p->d_blo, q.accum,
                       p->N, p->n_z, q.lv->n_sel, q.F, q.s.n_dt, q.s.n_xg, q.s.n_split, q.s.bins_per_split,
                       p->zero_evanescent, q.lv->d_kzff, p->d_ff_w32, p->d_ff_w16, p->d_ff_tw, q.lv->d_ev,
                       p->d_ff_tw2, p->d_ff_tw_vec, p->d_ff_tw2_vec};
  };
  // K3: the fields and cross-spectra sums of one group (frequency-domain delay-and-sum for method 1,
  // else propagate / inverse lateral transform / cross-spectra)
  auto stage_k3 = [&](const G& q) -> pam_status_t {
    if (q.F == 0) return PAM_OK;
    if (method == 1) {
      pam::TeaArgs a{q.spectra, q.lv->d_ksel, p->d_subs, p->d_z, q.accum, p->x_first, p->dx, p->xl_first, p->pitch,
                     p->fs / ((double)q.n_t * p->c), p->L, p->N, p->n_z, q.lv->n_sel, q.F, q.s.n_split,
                     q.s.bins_per_split, (pix + pam::TEA_THREADS - 1) / pam::TEA_THREADS};
      const long long blocks = (long long)q.F * a.n_ptile * q.s.n_split;
      if (blocks > 0x7fffffffLL) return PAM_ERR_UNSUPPORTED;
      const size_t lds = (size_t)pam::TEA_BC * p->L * sizeof(float2);
      if (p->n_sub == 3)
        hipLaunchKernelGGL(pam::k3_tea<3>, dim3((unsigned)blocks), dim3(pam::TEA_THREADS), lds, stream, a);
      else if (p->n_sub == 2)
        hipLaunchKernelGGL(pam::k3_tea<2>, dim3((unsigned)blocks), dim3(pam::TEA_THREADS), lds, stream, a);
      else
        hipLaunchKernelGGL(pam::k3_tea<1>, dim3((unsigned)blocks), dim3(pam::TEA_THREADS), lds, stream, a);
      if (hipGetLastError() != hipSuccess) return PAM_ERR_DEVICE;
      return PAM_OK;
    }
    const pam::K3Groups none{};
    const long long blocks = (long long)q.F * q.s.n_dt * q.s.n_xg * q.s.n_split;
    if (blocks > 0x7fffffffLL) return PAM_ERR_UNSUPPORTED;
    if (launch_k3(p->precision, p->n_sub, q.s, args_for(q), none, (int)blocks, Target{stream, nullptr}, p->coherence) !=
        hipSuccess)
      return PAM_ERR_DEVICE;
    return PAM_OK;
  };
  // K4: NCC / weight / energy, then NNCC and image
  auto stage_k4 = [&](int g) -> pam_status_t {
    const G& q = gs[g];
    if (q.F == 0) return PAM_OK;
    const int n_blk = (pix + 255) / 256;
    pam::K4Args a{q.accum, q.energy, q.weight, q.blockmax, q.rho, q.image, q.nncc, pix, q.F, W[g].n_split,
                  p->n_sub, n_blk, W[g].n_acc, p->eps};
    hipLaunchKernelGGL(pam::k4_weight, dim3(n_blk, q.F), dim3(256), 0, stream, a);
    if (hipGetLastError() != hipSuccess) return PAM_ERR_DEVICE;
    hipLaunchKernelGGL(pam::k4_image, dim3(n_blk, q.F), dim3(256), 0, stream, a);
    if (hipGetLastError() != hipSuccess) return PAM_ERR_DEVICE;
    return PAM_OK;
  };

  if (!one_launch && n_groups > 1) {
    // group after group, each through all four stages: a group's fields launch reads the coefficients its
    // K2 has just written while they are still in the last-level cache (one group's worth; the stage-major
    // order made the fields launches of 4 + 4 + 4 frames of 256 elements 7-24 % slower)
    for (int g = 0; g < n_groups; ++g) {
      if ((st = stage_k1(gs[g])) != PAM_OK || (st = stage_k2(gs[g])) != PAM_OK ||
          (st = stage_k3(gs[g])) != PAM_OK || (st = stage_k4(g)) != PAM_OK)
        return st;
    }
    return PAM_OK;
  }
  // stage after stage (one group, with the stage marks, or one grouped fields launch)
  for (int g = 0; g < n_groups; ++g)
    if ((st = stage_k1(gs[g])) != PAM_OK) return st;
  if (!mark(1)) return PAM_ERR_DEVICE;
  for (int g = 0; g < n_groups; ++g)
    if ((st = stage_k2(gs[g])) != PAM_OK) return st;
  if (!mark(2)) return PAM_ERR_DEVICE;
  if (method == 0 && one_launch) {
    // one launch over every group: a grouped work list on the factored kernels
    pam::K3Groups grp{};
    long long blocks = 0;
    const G* first = nullptr;
    // the work list runs the groups with the longest workgroups first (a short tail)
    const G* order[pam::kMaxGroups];
    int n_order = 0;
    for (int g = 0; g < n_groups; ++g)
      if (gs[g].F > 0) order[n_order++] = &gs[g];
    for (int k = 1; k < n_order; ++k)      // stable insertion sort, longest workgroups first (no buffer)
      for (int m = k; m > 0 && order[m - 1]->s.bins_per_split < order[m]->s.bins_per_split; --m)
        std::swap(order[m - 1], order[m]);
    for (int k = 0; k < n_order; ++k) {
      const G* qp = order[k];
      const G& q = *qp;
      if (!first) first = &q;
      pam::K3Group& e = grp.g[grp.n++];
      e = pam::K3Group{q.coeffs, q.scales, q.lv->d_kzff, q.lv->d_ev, q.accum, (int32_t)blocks, q.F, q.lv->n_sel,
                       q.s.n_split, q.s.bins_per_split};
      blocks += (long long)q.F * q.s.n_dt * q.s.n_xg * q.s.n_split;
    }
    if (blocks > 0x7fffffffLL) return PAM_ERR_UNSUPPORTED;
    if (launch_k3(p->precision, p->n_sub, first->s, args_for(*first), grp, (int)blocks, Target{stream, nullptr}, p->coherence) !=
        hipSuccess)
      return PAM_ERR_DEVICE;
  } else {
    for (int g = 0; g < n_groups; ++g)
      if ((st = stage_k3(gs[g])) != PAM_OK) return st;
  }
  if (!mark(3)) return PAM_ERR_DEVICE;
  for (int g = 0; g < n_groups; ++g)
    if ((st = stage_k4(g)) != PAM_OK) return st;
  if (!mark(4)) return PAM_ERR_DEVICE;
  return PAM_OK;
}

pam_status_t run_as_tax(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t, float* image,
                        float* nncc, float* rho_pairs, void* workspace, size_t ws_bytes, void* hip_stream,
                        void* const* events, int method = 0) {
  if (!p || n_frames < 0) return PAM_ERR_INVALID_ARG;
  if (n_frames > 65535) return PAM_ERR_UNSUPPORTED;
  const pam_group_t one{n_t, n_frames};
  return run_groups(p, rf, &one, 1, image, nncc, rho_pairs, workspace, ws_bytes, hip_stream, events, method);
}

}  // namespace

extern "C" {

pam_status_t pam_as_tax(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t, float* image,
                        float* nncc, float* rho_pairs, void* workspace, size_t ws_bytes, void* hip_stream) {
  return run_as_tax(p, rf, n_frames, n_t, image, nncc, rho_pairs, workspace, ws_bytes, hip_stream, nullptr);
}

pam_status_t pam_as_tax_events(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t, float* image,
                               float* nncc, float* rho_pairs, void* workspace, size_t ws_bytes,
                               void* hip_stream, void* const* events) {
  if (!events) return PAM_ERR_INVALID_ARG;
  for (int i = 0; i < PAM_N_STAGE_EVENTS; ++i)
    if (!events[i]) return PAM_ERR_INVALID_ARG;
  return run_as_tax(p, rf, n_frames, n_t, image, nncc, rho_pairs, workspace, ws_bytes, hip_stream, events);
}

pam_status_t pam_fd_tea_tax(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t, float* image,
                            float* nncc, float* rho_pairs, void* workspace, size_t ws_bytes, void* hip_stream) {
  return run_as_tax(p, rf, n_frames, n_t, image, nncc, rho_pairs, workspace, ws_bytes, hip_stream, nullptr, 1);
}

void pam_destroy(pam_plan_t p) { free_plan(p); }

pam_status_t pam_workspace_size_grouped(pam_plan_t p, const pam_group_t* groups, int32_t n_groups, size_t* bytes) {
  if (!p || !bytes) return PAM_ERR_INVALID_ARG;
  pam_workspace_layout_t W[pam::kMaxGroups];
  size_t base[pam::kMaxGroups];
  int cap[pam::kMaxGroups];
  bool one_launch = false;
  return grouped_layout(p, groups, n_groups, W, base, bytes, cap, &one_launch);
}

pam_status_t pam_as_tax_grouped(pam_plan_t p, const float* rf, const pam_group_t* groups, int32_t n_groups,
                                float* image, float* nncc, float* rho_pairs, void* workspace, size_t ws_bytes,
                                void* hip_stream) {
  return run_groups(p, rf, groups, n_groups, image, nncc, rho_pairs, workspace, ws_bytes, hip_stream, nullptr, 0);
}

void pam_debug_fail_allocation(int32_t n) { g_fail_alloc.store(n < 0 ? -1 : n); }

int64_t pam_debug_live_allocations(void) { return g_live_allocs.load(); }

int32_t pam_debug_grouped_one_launch(pam_plan_t p, const pam_group_t* groups, int32_t n_groups) {
  if (!p) return PAM_ERR_INVALID_ARG;
  pam_workspace_layout_t W[pam::kMaxGroups];
  size_t base[pam::kMaxGroups];
  size_t total = 0;
  int cap[pam::kMaxGroups];
  bool one_launch = false;
  const pam_status_t st = grouped_layout(p, groups, n_groups, W, base, &total, cap, &one_launch);
  return st != PAM_OK ? (int32_t)st : (one_launch ? 1 : 0);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Entry point that allocates nothing: the workspace is a file-scope device array.
// In host code `scratch` names a host-side stand-in, not device memory; its device
// address on each GPU comes from hipGetSymbolAddress (taken once per device, with
// that device current) and only that address is ever handed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PAM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the caller has made it current).
pam_status_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return PAM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PAM_ERR_DEVICE;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return PAM_OK;
}

}  // namespace

extern "C" {

pam_status_t pam_as_tax_noalloc(pam_plan_t p, const float* rf, int64_t n_frames, int32_t n_t, float* image,
                                float* nncc, float* rho_pairs, void* hip_stream) {
  if (!p || n_frames < 0) return PAM_ERR_INVALID_ARG;
  pam_workspace_layout_t W;
  pam_status_t st = layout(p, n_frames, n_t, &W);
  if (st != PAM_OK) return st;
  if (W.total > (size_t)PAM_NOALLOC_SCRATCH_BYTES) return PAM_ERR_WORKSPACE;
  if (n_frames == 0) return PAM_OK;
  void* ws = nullptr;
  {
    DeviceGuard guard(p->device);
    if (!guard.ok) return PAM_ERR_DEVICE;
    if ((st = scratch_address(p->device, &ws)) != PAM_OK) return st;
  }
  return run_as_tax(p, rf, n_frames, n_t, image, nncc, rho_pairs, ws, (size_t)PAM_NOALLOC_SCRATCH_BYTES,
                    hip_stream, nullptr);
}

}  // extern "C"
