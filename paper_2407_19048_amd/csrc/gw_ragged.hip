// Uneven (ragged) batches: signals of several size classes (sample rate,
// window length, Welch stretch) generated together.  Each stage is one
// persistent launch over every class:
//   k_sample_params_ragged  ceil(B/256) / 256   prior draws with the class's
//                                              configuration per signal
//   k_welch_ragged          CUs*gw / 256        Welch PSDs; a group is one
//                                              L = 4096 item or two L = 2048
//                                              items (128-thread sub-blocks)
//   k_window_ragged         CUs*gv / 1024       fused window items; a group
//                                              holds 16384/NC items of one
//                                              class, one NC/16-thread
//                                              sub-block each
// Workgroups pull group indices from an atomic counter until the queue is
// empty.  Groups are ordered largest transform first, so the tail of the
// launch is made of the shortest items.  The two stages are separate
// launches because the persistent Welch kernel keeps ~240 VGPRs of twiddles
// and accumulators live (two waves per SIMD), while a 1024-thread window
// workgroup is limited to 128 VGPRs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gw_fft.hpp"
#include "gw_physics.hpp"
#include "gw_internal.hpp"
#include "gw_items.hpp"
#include "../../include/gwgen.h"

using namespace gw;

namespace {
constexpr int kMaxCls = GW_RAGGED_MAX_CLASSES;
constexpr int kWinThreads = 1024;    // window workgroup: one NC = 16384 item
constexpr int kWelchThreads = 256;   // Welch workgroup: one L = 4096 item
}  // namespace

struct gw_ragged {
  int n_cls = 0, n_det = 0, precision = 1;
  int64_t B = 0;
  gw_config cfg[kMaxCls];
  DevCfg dc[kMaxCls];
  double welch_norm[kMaxCls];
  std::vector<int64_t> out_off, psd_off;  // [B+1] float offsets
  int n_wgroups = 0, n_vgroups = 0;
  int wend[2] = {0, 0}, vend[4] = {0, 0, 0, 0};  // group index ends per size slot
  // device plan
  DevCfg* d_cfgs = nullptr;
  int32_t* d_cls = nullptr;
  int64_t* d_out_off = nullptr;
  int64_t* d_psd_off = nullptr;
  int4* d_wgroups = nullptr;   // {class, first item, count, L}
  int32_t* d_witems = nullptr;  // signal * n_det + det
  int4* d_vgroups = nullptr;   // {class, first item, count, N/2}
  int32_t* d_vitems = nullptr;
  double* kcbrt = nullptr;
  double* lnk3 = nullptr;
  void* tw[4] = {nullptr, nullptr, nullptr, nullptr};   // exp(-2 pi i n / M), M = 2048 << s
  void* twr[4] = {nullptr, nullptr, nullptr, nullptr};  // exp(-2 pi i k / 2M), k <= M/2
  int n_cu = 256;
  int ord_win = 0, ord_welch = 0, grid_win = 1, grid_welch = 2;
  int win_mode = 0;                      // 0: one persistent launch, 1: one launch per class
  int cls_first[kMaxCls], cls_items[kMaxCls];  // window item range of each class
  int wcls_first[kMaxCls], wcls_items[kMaxCls];  // Welch item range of each class
  int welch_mode = 1;  // Welch issue: 0 one persistent launch, 1 one launch per class
  std::string err;
};

namespace {

// ------------------------------------------------------------ device side

struct RSampleArgs {
  const DevCfg* cfgs;
  const int32_t* cls;
  uint64_t seed, first;
  const uint64_t* batch;  // device batch index (graph replays) or NULL
  int64_t B;
  int64_t span[kMaxCls];
  double* params;
  int64_t* offset;
  float* params_f32;
  uint32_t* status;
  WfScalars* wf;
  DetScalars* dsc;
};

__global__ __launch_bounds__(256) void k_sample_params_ragged(RSampleArgs a) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= a.B) return;
  const int c = a.cls[i];
  const uint64_t first = a.batch ? *a.batch * uint64_t(a.B) : a.first;
  int64_t span = a.span[0];
#pragma unroll
  for (int k = 1; k < kMaxCls; ++k)
    if (c == k) span = a.span[k];
  draw_sample(a.cfgs[c], a.seed, first + uint64_t(i), i, a.B, span, double(c), a.params, a.offset, a.params_f32,
              a.status, a.wf, a.dsc);
}

struct RWelchArgs {
  const DevCfg* cfgs;
  const int4* groups;
  const int32_t* items;
  int n_groups;
  const int64_t* offset;
  const int64_t* psd_off;
  float* psd;
  const float* bg[kMaxCls];
  int64_t L_bg[kMaxCls];
  double norm[kMaxCls];
  const void* tw2048;
  const void* tw4096;
  uint32_t* queue;
  int end[2];  // groups of L = 2048 << s end at end[s] (sizes in decreasing order)
};

template <class ACC, int L, int ORD>
__device__ __forceinline__ void welch_group(const RWelchArgs& a, int4 gr, int t, float* lds) {
  constexpr int NT = L / 16, LS = LdsSize<L>::value;
  const int j = t / NT;  // sub-block; NT >= 128, so uniform over a wavefront
  const int tl = t - j * NT;
  const bool active = j < gr.z;
  const int it = __builtin_amdgcn_readfirstlane(load_const(a.items + gr.y + min(j, gr.z - 1)));
  const DevCfg cf = load_const(a.cfgs + gr.x);
  const int D = cf.n_det;
  const int b = it / D, d = it - b * D;
  const float* x = a.bg[gr.x] + int64_t(d) * a.L_bg[gr.x] + load_const(a.offset + b);
  float* out = a.psd + load_const(a.psd_off + b) + int64_t(d) * cf.Fw;
  const cpx<float>* tw = opaque(reinterpret_cast<const cpx<float>*>(L == 4096 ? a.tw4096 : a.tw2048));
  welch_item<float, ACC, L, ORD>(cf.K, a.norm[gr.x], tl, x, out, tw, lds + j * 2 * LS, lds + j * 2 * LS + LS, active);
}

// Groups [g, end) of one transform size; returns the first group index this
// workgroup drew beyond them.  One loop per size keeps only that size's
// loop-invariant twiddles live.
template <class ACC, int L, int ORD>
__device__ __forceinline__ int welch_size_loop(const RWelchArgs& a, int g, int end, int t, float* lds, int* s_g) {
  while (g < end) {
    welch_group<ACC, L, ORD>(a, load_const(a.groups + g), t, lds);
    __syncthreads();
    if (t == 0) *s_g = int(atomicAdd(a.queue, 1u));
    __syncthreads();
    g = __builtin_amdgcn_readfirstlane(*s_g);
  }
  return g;
}

// One class per launch: block i takes the class's i-th Welch item, L/16
// threads, 3 waves per SIMD (no queue loop, so only one item's state is live).
template <class ACC, int L, int ORD>
__global__ __launch_bounds__(L / 16, 3) void k_welch_class(RWelchArgs a, int cls, int first) {
  constexpr int LS = LdsSize<L>::value;
  __shared__ float lds[2 * LS];
  const int it = load_const(a.items + first + int(blockIdx.x));
  const DevCfg cf = load_const(a.cfgs + cls);
  const int D = cf.n_det;
  const int b = it / D, d = it - b * D;
  const float* x = a.bg[cls] + int64_t(d) * a.L_bg[cls] + load_const(a.offset + b);
  float* out = a.psd + load_const(a.psd_off + b) + int64_t(d) * cf.Fw;
  const cpx<float>* tw = reinterpret_cast<const cpx<float>*>(L == 4096 ? a.tw4096 : a.tw2048);
  welch_item<float, ACC, L, ORD>(cf.K, a.norm[cls], threadIdx.x, x, out, tw, lds, lds + LS, true);
}

template <class ACC, int ORD>
__global__ __launch_bounds__(kWelchThreads, 2) void k_welch_ragged(RWelchArgs a) {
  __shared__ float lds[2 * LdsSize<4096>::value];
  __shared__ int s_g;
  const int t = threadIdx.x;
  if (t == 0) s_g = int(atomicAdd(a.queue, 1u));
  __syncthreads();
  int g = __builtin_amdgcn_readfirstlane(s_g);
  g = welch_size_loop<ACC, 4096, 0>(a, g, a.end[1], t, lds, &s_g);
  welch_size_loop<ACC, 2048, ORD>(a, g, a.end[0], t, lds, &s_g);
}

struct RWinArgs {
  WinArgs w;  // shared pointers: params, B, out, status, kcbrt, lnk3, wf, dsc, offset
  const DevCfg* cfgs;
  const int4* groups;
  const int32_t* items;
  int n_groups;
  const int64_t* out_off;
  const int64_t* psd_off;
  const float* psd;
  const float* bg[kMaxCls];
  int64_t L_bg[kMaxCls];
  const void* tw[4];
  const void* twr[4];
  uint32_t* queue;
  int end[4];  // groups of NC = 2048 << s end at end[s] (sizes in decreasing order)
};

template <int NC> struct Log2Sub2048 { static constexpr int value = NC == 2048 ? 0 : NC == 4096 ? 1 : NC == 8192 ? 2 : 3; };

template <class TP, int NC, int ORD>
__device__ __forceinline__ void window_group(const RWinArgs& a, int4 gr, int t, float* lds, uint32_t* sflag) {
  constexpr int NT = NC / 16, LS = LdsSize<NC>::value, S = Log2Sub2048<NC>::value;
  const int j = t / NT;  // sub-block; NT >= 128, so uniform over a wavefront
  const int tl = t - j * NT;
  const bool active = j < gr.z;
  const int it = __builtin_amdgcn_readfirstlane(load_const(a.items + gr.y + min(j, gr.z - 1)));
  const DevCfg cf = load_const(a.cfgs + gr.x);
  const int D = cf.n_det;
  const int b = it / D, d = it - b * D;
  const float* x = a.bg[gr.x] + int64_t(d) * a.L_bg[gr.x] + load_const(a.w.offset + b) + cf.P;
  const float* psd = a.psd + load_const(a.psd_off + b) + int64_t(d) * cf.Fw;
  float* o = a.w.out + load_const(a.out_off + b) + int64_t(d) * cf.N;
  WinArgs w = a.w;
  w.kcbrt = opaque(w.kcbrt);
  w.lnk3 = opaque(w.lnk3);
  window_item<float, TP, false, NC, 1, ORD>(cf, w, tl, b, d, x, nullptr, nullptr, psd, o,
                                            opaque(reinterpret_cast<const cpx<float>*>(a.tw[S])),
                                            opaque(reinterpret_cast<const cpx<float>*>(a.twr[S])), lds + j * 2 * LS,
                                            lds + j * 2 * LS + LS, active, sflag + j);
  __syncthreads();
  if (tl == 0 && active && sflag[j] && a.w.status) atomicOr(a.w.status + b, sflag[j]);
}

template <class TP, int NC, int ORD>
__device__ __forceinline__ int window_size_loop(const RWinArgs& a, int g, int end, int t, float* lds, int* s_g,
                                                uint32_t* sflag) {
  while (g < end) {
    window_group<TP, NC, ORD>(a, load_const(a.groups + g), t, lds, sflag);
    __syncthreads();
    if (t == 0) *s_g = int(atomicAdd(a.queue, 1u));
    if (t < 8) sflag[t] = 0u;
    __syncthreads();
    g = __builtin_amdgcn_readfirstlane(*s_g);
  }
  return g;
}

template <class TP, int ORD>
__global__ __launch_bounds__(kWinThreads) void k_window_ragged(RWinArgs a) {
  __shared__ float lds[2 * LdsSize<16384>::value];
  __shared__ int s_g;
  __shared__ uint32_t sflag[8];
  const int t = threadIdx.x;
  if (t == 0) s_g = int(atomicAdd(a.queue, 1u));
  if (t < 8) sflag[t] = 0u;
  __syncthreads();
  int g = __builtin_amdgcn_readfirstlane(s_g);
  g = window_size_loop<TP, 16384, ORD>(a, g, a.end[3], t, lds, &s_g, sflag);
  g = window_size_loop<TP, 8192, ORD>(a, g, a.end[2], t, lds, &s_g, sflag);
  g = window_size_loop<TP, 4096, 0>(a, g, a.end[1], t, lds, &s_g, sflag);
  window_size_loop<TP, 2048, ORD>(a, g, a.end[0], t, lds, &s_g, sflag);
}

// Window stage issued per class: one NC/16-thread workgroup per item of
// class `cls` (items first .. first + gridDim.x - 1), at the occupancy of the
// batch kernel of that size.
template <int NC> struct ClassOcc { static constexpr int value = NC >= 16384 ? 1 : NC >= 8192 ? 4 : 8; };

template <class TP, int NC, int ORD>
__global__ __launch_bounds__(NC / 16, ClassOcc<NC>::value) void k_window_class(RWinArgs a, int cls, int first) {
  constexpr int LS = LdsSize<NC>::value, S = Log2Sub2048<NC>::value;
  __shared__ float lds[2 * LS];
  __shared__ uint32_t sflag;
  const int t = threadIdx.x;
  if (t == 0) sflag = 0u;
  const int it = load_const(a.items + first + int(blockIdx.x));
  const DevCfg cf = load_const(a.cfgs + cls);
  const int D = cf.n_det;
  const int b = it / D, d = it - b * D;
  const float* x = a.bg[cls] + int64_t(d) * a.L_bg[cls] + load_const(a.w.offset + b) + cf.P;
  const float* psd = a.psd + load_const(a.psd_off + b) + int64_t(d) * cf.Fw;
  float* o = a.w.out + load_const(a.out_off + b) + int64_t(d) * cf.N;
  window_item<float, TP, false, NC, 1, ORD>(cf, a.w, t, b, d, x, nullptr, nullptr, psd, o,
                                            reinterpret_cast<const cpx<float>*>(a.tw[S]),
                                            reinterpret_cast<const cpx<float>*>(a.twr[S]), lds, lds + LS, true,
                                            &sflag);
  __syncthreads();
  if (t == 0 && sflag && a.w.status) atomicOr(a.w.status + b, sflag);
}

__global__ void k_fill_u32_r(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// -------------------------------------------------------------- host side
gw_status rfail(gw_ragged* r, gw_status s, const std::string& m) {
  if (r) r->err = m;
  return s;
}

gw_status rcheck(gw_ragged* r, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return rfail(r, GW_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return GW_OK;
}

int64_t align256(int64_t v) { return ((v + 255) / 256) * 256; }

struct RLayout {
  int64_t params, offset, wf, dsc, ctr, psd, total;
};

RLayout layout(const gw_ragged* r) {
  RLayout l;
  const int64_t B = r->B;
  l.params = 0;
  l.offset = l.params + align256(B * 12 * 8);
  l.wf = l.offset + align256(B * 8);
  l.dsc = l.wf + align256(B * int64_t(sizeof(WfScalars)));
  l.ctr = l.dsc + align256(B * r->n_det * int64_t(sizeof(DetScalars)));
  l.psd = l.ctr + 256;  // batch counter (u64) at +0, queue heads (u32) at +64
  l.total = l.psd + align256(r->psd_off[B] * 4);
  return l;
}

template <class T>
bool upload(void** dst, const std::vector<T>& h) {
  if (hipMalloc(dst, sizeof(T) * std::max<size_t>(h.size(), 1)) != hipSuccess) return false;
  if (!h.empty() && hipMemcpy(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice) != hipSuccess) return false;
  return true;
}

std::vector<cpx<float>> twiddles(int n, int denom) {
  std::vector<cpx<float>> h(n);
  for (int i = 0; i < n; ++i) {
    const double ang = -2.0 * M_PI * double(i) / double(denom);
    h[i] = {float(std::cos(ang)), float(std::sin(ang))};
  }
  return h;
}

int size_slot(int M) { return M == 2048 ? 0 : M == 4096 ? 1 : M == 8192 ? 2 : 3; }

bool same_shared_fields(const gw_config& a, const gw_config& b) {
  if (a.n_det != b.n_det || a.approximant != b.approximant || a.precision != b.precision) return false;
  for (int d = 0; d < a.n_det; ++d)
    if (a.det_id[d] != b.det_id[d]) return false;
  for (int i = 0; i < 2; ++i)
    if (a.mc[i] != b.mc[i] || a.q[i] != b.q[i] || a.chi[i] != b.chi[i] || a.dl[i] != b.dl[i] ||
        a.f0[i] != b.f0[i] || a.quality[i] != b.quality[i] || a.hrss[i] != b.hrss[i])
      return false;
  return true;
}

gw_status check_call(gw_ragged* r, const float* const* bg, const int64_t* L_bg, const float* out,
                     const float* params_f32, const uint32_t* status, const void* ws, int64_t ws_bytes,
                     int64_t* span) {
  if (!bg || !L_bg || !out || !ws) return rfail(r, GW_EINVAL, "NULL pointer");
  if (!((reinterpret_cast<uintptr_t>(out) & 15u) == 0) || !((reinterpret_cast<uintptr_t>(ws) & 15u) == 0) ||
      (params_f32 && (reinterpret_cast<uintptr_t>(params_f32) & 15u)) ||
      (status && (reinterpret_cast<uintptr_t>(status) & 3u)))
    return rfail(r, GW_EINVAL, "misaligned pointer");
  if (ws_bytes < layout(r).total) return rfail(r, GW_EINVAL, "workspace too small");
  for (int c = 0; c < kMaxCls; ++c) span[c] = 1;
  for (int c = 0; c < r->n_cls; ++c) {
    if (!bg[c]) return rfail(r, GW_EINVAL, "background pointer is NULL");
    if (reinterpret_cast<uintptr_t>(bg[c]) & 3u) return rfail(r, GW_EINVAL, "background not 4-byte aligned");
    span[c] = L_bg[c] - r->dc[c].P - r->dc[c].N + 1;
    if (span[c] <= 0) return rfail(r, GW_EINVAL, "L_bg < P + N for a class");
  }
  return GW_OK;
}

constexpr int kStageParams = 1, kStageWelch = 2, kStageWindow = 4, kStageAll = 7;

template <class ACC>
void launch_welch_ragged(const gw_ragged* r, const RWelchArgs& a, hipStream_t st) {
  if (r->welch_mode == 1) {
    // largest transforms first
    for (int pass = 0; pass < 2; ++pass)
      for (int c = 0; c < r->n_cls; ++c) {
        const int L = r->dc[c].L;
        if (r->wcls_items[c] == 0 || (pass == 0) != (L == 4096)) continue;
        const dim3 grid(unsigned(r->wcls_items[c]));
        if (L == 4096)
          hipLaunchKernelGGL((k_welch_class<ACC, 4096, 0>), grid, dim3(256), 0, st, a, c, r->wcls_first[c]);
        else if (r->ord_welch)
          hipLaunchKernelGGL((k_welch_class<ACC, 2048, 1>), grid, dim3(128), 0, st, a, c, r->wcls_first[c]);
        else
          hipLaunchKernelGGL((k_welch_class<ACC, 2048, 0>), grid, dim3(128), 0, st, a, c, r->wcls_first[c]);
      }
    return;
  }
  const dim3 grid = dim3(unsigned(r->n_cu * r->grid_welch));
  if (r->ord_welch) hipLaunchKernelGGL((k_welch_ragged<ACC, 1>), grid, dim3(kWelchThreads), 0, st, a);
  else hipLaunchKernelGGL((k_welch_ragged<ACC, 0>), grid, dim3(kWelchThreads), 0, st, a);
}

template <class TP, int ORD>
void launch_window_class(const gw_ragged* r, const RWinArgs& a, int c, hipStream_t st) {
  const dim3 grid = dim3(unsigned(r->cls_items[c]));
  const int first = r->cls_first[c];
  switch (r->dc[c].N / 2) {
    case 16384: hipLaunchKernelGGL((k_window_class<TP, 16384, ORD>), grid, dim3(1024), 0, st, a, c, first); break;
    case 8192: hipLaunchKernelGGL((k_window_class<TP, 8192, ORD>), grid, dim3(512), 0, st, a, c, first); break;
    case 4096: hipLaunchKernelGGL((k_window_class<TP, 4096, 0>), grid, dim3(256), 0, st, a, c, first); break;
    default: hipLaunchKernelGGL((k_window_class<TP, 2048, ORD>), grid, dim3(128), 0, st, a, c, first); break;
  }
}

template <class TP>
void launch_window_ragged(const gw_ragged* r, const RWinArgs& a, hipStream_t st) {
  if (r->win_mode == 1) {
    // largest transforms first, as in the persistent queue
    int order[kMaxCls];
    for (int c = 0; c < r->n_cls; ++c) order[c] = c;
    std::stable_sort(order, order + r->n_cls, [&](int x, int y) { return r->dc[x].N > r->dc[y].N; });
    for (int k = 0; k < r->n_cls; ++k) {
      const int c = order[k];
      if (r->cls_items[c] == 0) continue;
      if (r->ord_win) launch_window_class<TP, 1>(r, a, c, st);
      else launch_window_class<TP, 0>(r, a, c, st);
    }
    return;
  }
  const dim3 grid = dim3(unsigned(r->n_cu * r->grid_win));
  if (r->ord_win) hipLaunchKernelGGL((k_window_ragged<TP, 1>), grid, dim3(kWinThreads), 0, st, a);
  else hipLaunchKernelGGL((k_window_ragged<TP, 0>), grid, dim3(kWinThreads), 0, st, a);
}

gw_status enqueue_ragged(gw_ragged* r, uint64_t seed, uint64_t batch_index, bool use_counter,
                         const float* const* bg, const int64_t* L_bg, const int64_t* span, float* out,
                         float* params_f32, uint32_t* status, void* ws, int stages, hipStream_t st) {
  const RLayout l = layout(r);
  char* w = static_cast<char*>(ws);
  double* params = reinterpret_cast<double*>(w + l.params);
  int64_t* offset = reinterpret_cast<int64_t*>(w + l.offset);
  WfScalars* wf = reinterpret_cast<WfScalars*>(w + l.wf);
  DetScalars* dsc = reinterpret_cast<DetScalars*>(w + l.dsc);
  uint64_t* batch = reinterpret_cast<uint64_t*>(w + l.ctr);
  uint32_t* queue = reinterpret_cast<uint32_t*>(w + l.ctr + 64);
  float* psd = reinterpret_cast<float*>(w + l.psd);
  const int64_t B = r->B;
  gw_status s = GW_OK;
  if (stages & kStageParams) {
    RSampleArgs a;
    std::memset(&a, 0, sizeof(a));
    a.cfgs = r->d_cfgs;
    a.cls = r->d_cls;
    a.seed = seed;
    a.first = batch_index * uint64_t(B);
    a.batch = use_counter ? batch : nullptr;
    a.B = B;
    for (int c = 0; c < kMaxCls; ++c) a.span[c] = span[c];
    a.params = params;
    a.offset = offset;
    a.params_f32 = params_f32;
    a.status = status;
    a.wf = wf;
    a.dsc = dsc;
    hipLaunchKernelGGL(k_sample_params_ragged, dim3(unsigned((B + 255) / 256)), dim3(256), 0, st, a);
    if ((s = rcheck(r, "k_sample_params_ragged")) != GW_OK) return s;
  }
  if (stages & kStageWelch) {
    hipLaunchKernelGGL(k_fill_u32_r, dim3(1), dim3(256), 0, st, queue, int64_t(1), 0u);
    if ((s = rcheck(r, "k_fill_u32")) != GW_OK) return s;
    RWelchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.cfgs = r->d_cfgs;
    a.groups = r->d_wgroups;
    a.items = r->d_witems;
    a.n_groups = r->n_wgroups;
    a.offset = offset;
    a.psd_off = r->d_psd_off;
    a.psd = psd;
    for (int c = 0; c < r->n_cls; ++c) {
      a.bg[c] = bg[c];
      a.L_bg[c] = L_bg[c];
      a.norm[c] = r->welch_norm[c];
    }
    a.tw2048 = r->tw[0];
    a.tw4096 = r->tw[1];
    a.queue = queue;
    a.end[0] = r->wend[0];
    a.end[1] = r->wend[1];
    if (r->precision == 0) launch_welch_ragged<float>(r, a, st);
    else launch_welch_ragged<double>(r, a, st);
    if ((s = rcheck(r, "k_welch_ragged")) != GW_OK) return s;
  }
  if (stages & kStageWindow) {
    hipLaunchKernelGGL(k_fill_u32_r, dim3(1), dim3(256), 0, st, queue + 1, int64_t(1), 0u);
    if ((s = rcheck(r, "k_fill_u32")) != GW_OK) return s;
    RWinArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w.cf = r->dc[0];
    a.w.offset = offset;
    a.w.params = params;
    a.w.B = B;
    a.w.out = out;
    a.w.status = status;
    a.w.kcbrt = r->kcbrt;
    a.w.lnk3 = r->lnk3;
    a.w.wf = wf;
    a.w.dsc = dsc;
    a.cfgs = r->d_cfgs;
    a.groups = r->d_vgroups;
    a.items = r->d_vitems;
    a.n_groups = r->n_vgroups;
    a.out_off = r->d_out_off;
    a.psd_off = r->d_psd_off;
    a.psd = psd;
    for (int c = 0; c < r->n_cls; ++c) {
      a.bg[c] = bg[c];
      a.L_bg[c] = L_bg[c];
    }
    for (int k = 0; k < 4; ++k) {
      a.tw[k] = r->tw[k];
      a.twr[k] = r->twr[k];
    }
    a.queue = queue + 1;
    for (int k = 0; k < 4; ++k) a.end[k] = r->vend[k];
    if (r->precision == 0) launch_window_ragged<float>(r, a, st);
    else launch_window_ragged<double>(r, a, st);
    if ((s = rcheck(r, "k_window_ragged")) != GW_OK) return s;
  }
  return GW_OK;
}

}  // namespace

extern "C" {

gw_status gw_ragged_destroy(gw_ragged* r) {
  if (!r) return GW_OK;
  void* ptrs[] = {r->d_cfgs, r->d_cls, r->d_out_off, r->d_psd_off, r->d_wgroups, r->d_witems,
                  r->d_vgroups, r->d_vitems, r->kcbrt, r->lnk3};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < 4; ++k) {
    if (r->tw[k]) (void)hipFree(r->tw[k]);
    if (r->twr[k]) (void)hipFree(r->twr[k]);
  }
  delete r;
  return GW_OK;
}

const char* gw_ragged_last_error(const gw_ragged* r) { return r ? r->err.c_str() : "ragged handle is NULL"; }

gw_status gw_ragged_create(const gw_config* classes, int32_t n_classes, const int32_t* cls, int64_t B,
                           gw_ragged** out) {
  if (!out) return GW_EINVAL;
  *out = nullptr;
  if (!classes || !cls || n_classes < 1 || n_classes > kMaxCls || B < 1) return GW_EINVAL;
  gw_ragged* r = new gw_ragged();
  r->n_cls = n_classes;
  r->B = B;
  auto bail = [&](gw_status s) {
    gw_ragged_destroy(r);
    return s;
  };
  for (int c = 0; c < n_classes; ++c) {
    std::string why;
    if (validate_config(&classes[c], &r->dc[c], &why) != GW_OK) return bail(GW_EINVAL);
    r->cfg[c] = classes[c];
    const DevCfg& d = r->dc[c];
    if (d.precision == 2 || d.N > 32768) return bail(GW_EUNSUPPORTED);
    if (d.N < 2 * d.L) return bail(GW_EINVAL);
    if (!same_shared_fields(classes[0], classes[c])) return bail(GW_EINVAL);
    r->welch_norm[c] = 1.0 / (double(d.K) * d.fs * (3.0 * d.L / 8.0));
  }
  r->n_det = r->dc[0].n_det;
  r->precision = r->dc[0].precision;
  const int D = r->n_det;
  if (B * D >= (int64_t(1) << 31)) return bail(GW_EINVAL);
  std::vector<int32_t> hcls(cls, cls + B);
  for (int64_t i = 0; i < B; ++i)
    if (hcls[i] < 0 || hcls[i] >= n_classes) return bail(GW_EINVAL);
  r->out_off.assign(B + 1, 0);
  r->psd_off.assign(B + 1, 0);
  for (int64_t i = 0; i < B; ++i) {
    r->out_off[i + 1] = r->out_off[i] + int64_t(D) * r->dc[hcls[i]].N;
    r->psd_off[i + 1] = r->psd_off[i] + int64_t(D) * r->dc[hcls[i]].Fw;
  }
  // Work groups: classes by transform size, largest first; items of one
  // class in signal order, then detector.
  std::vector<int> order(n_classes);
  auto build = [&](bool welch, std::vector<int4>& groups, std::vector<int32_t>& items) {
    for (int c = 0; c < n_classes; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      const int sx = welch ? r->dc[x].L : r->dc[x].N / 2, sy = welch ? r->dc[y].L : r->dc[y].N / 2;
      return sx > sy;
    });
    for (int c : order) {
      const int M = welch ? r->dc[c].L : r->dc[c].N / 2;
      const int G = welch ? 4096 / M : 16384 / M;
      const int first = int(items.size());
      for (int64_t i = 0; i < B; ++i)
        if (hcls[i] == c)
          for (int d = 0; d < D; ++d) items.push_back(int32_t(i * D + d));
      const int n = int(items.size()) - first;
      for (int k = 0; k < n; k += G) groups.push_back(int4{c, first + k, std::min(G, n - k), M});
    }
  };
  std::vector<int4> wg, vg;
  std::vector<int32_t> wi, vi;
  build(true, wg, wi);
  build(false, vg, vi);
  for (int c = 0; c < kMaxCls; ++c) r->cls_first[c] = r->cls_items[c] = r->wcls_first[c] = r->wcls_items[c] = 0;
  for (const int4& g : vg) {
    if (r->cls_items[g.x] == 0) r->cls_first[g.x] = g.y;
    r->cls_items[g.x] += g.z;
  }
  for (const int4& g : wg) {
    if (r->wcls_items[g.x] == 0) r->wcls_first[g.x] = g.y;
    r->wcls_items[g.x] += g.z;
  }
  r->n_wgroups = int(wg.size());
  r->n_vgroups = int(vg.size());
  // sizes appear in decreasing order: the groups of size slot s end where
  // the first group of a smaller size starts (or at the end)
  for (int k = 0; k < 2; ++k) {
    int e = 0;
    for (int g = 0; g < r->n_wgroups; ++g)
      if (size_slot(wg[g].w) >= k) e = g + 1;
    r->wend[k] = e;
  }
  for (int k = 0; k < 4; ++k) {
    int e = 0;
    for (int g = 0; g < r->n_vgroups; ++g)
      if (size_slot(vg[g].w) >= k) e = g + 1;
    r->vend[k] = e;
  }
  // tables
  int Fmax = 0;
  bool need_tw[4] = {false, false, false, false}, need_twr[4] = {false, false, false, false};
  for (int c = 0; c < n_classes; ++c) {
    Fmax = std::max(Fmax, r->dc[c].F);
    need_tw[size_slot(r->dc[c].N / 2)] = need_twr[size_slot(r->dc[c].N / 2)] = true;
    need_tw[size_slot(r->dc[c].L)] = true;
  }
  std::vector<double> hc(Fmax), hl(Fmax);
  for (int k = 0; k < Fmax; ++k) {
    hc[k] = std::cbrt(double(k));
    hl[k] = k > 0 ? std::log(double(k)) / 3.0 : 0.0;
  }
  std::vector<DevCfg> hcfg(r->dc, r->dc + n_classes);
  std::vector<int64_t> hout(r->out_off.begin(), r->out_off.end() - 1), hpsd(r->psd_off.begin(), r->psd_off.end() - 1);
  bool ok = upload(reinterpret_cast<void**>(&r->d_cfgs), hcfg) && upload(reinterpret_cast<void**>(&r->d_cls), hcls) &&
            upload(reinterpret_cast<void**>(&r->d_out_off), hout) &&
            upload(reinterpret_cast<void**>(&r->d_psd_off), hpsd) &&
            upload(reinterpret_cast<void**>(&r->d_wgroups), wg) && upload(reinterpret_cast<void**>(&r->d_witems), wi) &&
            upload(reinterpret_cast<void**>(&r->d_vgroups), vg) && upload(reinterpret_cast<void**>(&r->d_vitems), vi) &&
            upload(reinterpret_cast<void**>(&r->kcbrt), hc) && upload(reinterpret_cast<void**>(&r->lnk3), hl);
  for (int k = 0; k < 4 && ok; ++k) {
    const int M = 2048 << k;
    if (need_tw[k]) ok = upload(&r->tw[k], twiddles(M, M));
    if (ok && need_twr[k]) ok = upload(&r->twr[k], twiddles(M / 2 + 1, 2 * M));
  }
  if (!ok) return bail(GW_ENOMEM);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    r->n_cu = ncu;
  *out = r;
  return GW_OK;
}

gw_status gw_ragged_query(const gw_ragged* r, int32_t key, int64_t* value) {
  if (!r || !value) return GW_EINVAL;
  switch (key) {
    case GW_RQ_B: *value = r->B; break;
    case GW_RQ_OUT_FLOATS: *value = r->out_off[r->B]; break;
    case GW_RQ_PSD_FLOATS: *value = r->psd_off[r->B]; break;
    case GW_RQ_WORKSPACE: *value = layout(r).total; break;
    case GW_RQ_PSD_OFFSET: *value = layout(r).psd; break;
    case GW_RQ_NCLASSES: *value = r->n_cls; break;
    default: return GW_EINVAL;
  }
  return GW_OK;
}

gw_status gw_ragged_offsets(const gw_ragged* r, int64_t* out_offset, int64_t* psd_offset) {
  if (!r) return GW_EINVAL;
  if (out_offset) std::copy(r->out_off.begin(), r->out_off.end(), out_offset);
  if (psd_offset) std::copy(r->psd_off.begin(), r->psd_off.end(), psd_offset);
  return GW_OK;
}

gw_status gw_generate_ragged(gw_ragged* r, uint64_t seed, uint64_t batch_index, const float* const* bg,
                             const int64_t* L_bg, float* out, float* params_f32, uint32_t* status, void* workspace,
                             int64_t workspace_bytes, hipStream_t stream) {
  if (!r) return GW_EINVAL;
  int64_t span[kMaxCls];
  gw_status s = check_call(r, bg, L_bg, out, params_f32, status, workspace, workspace_bytes, span);
  if (s != GW_OK) return s;
  if (batch_index > (UINT64_MAX - uint64_t(r->B)) / uint64_t(r->B))
    return rfail(r, GW_EINVAL, "batch_index overflows");
  return enqueue_ragged(r, seed, batch_index, false, bg, L_bg, span, out, params_f32, status, workspace, kStageAll,
                        stream);
}

gw_status gw_ragged_graph_create(gw_ragged* r, uint64_t seed, uint64_t first_batch, const float* const* bg,
                                 const int64_t* L_bg, float* out, float* params_f32, uint32_t* status,
                                 void* workspace, int64_t workspace_bytes, gw_graph** graph) {
  if (!r) return GW_EINVAL;
  if (!graph) return rfail(r, GW_EINVAL, "graph is NULL");
  *graph = nullptr;
  int64_t span[kMaxCls];
  gw_status s = check_call(r, bg, L_bg, out, params_f32, status, workspace, workspace_bytes, span);
  if (s != GW_OK) return s;
  uint64_t* batch = reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) + layout(r).ctr);
  std::string why;
  s = capture_graph(
      [&](hipStream_t st) {
        return enqueue_ragged(r, seed, 0, true, bg, L_bg, span, out, params_f32, status, workspace, kStageAll, st);
      },
      batch, first_batch, graph, &why);
  if (s != GW_OK) return rfail(r, s, why + (r->err.empty() ? "" : ": " + r->err));
  return GW_OK;
}

gw_status gw_ragged_set_tuning(gw_ragged* r, int32_t key, int64_t value) {
  if (!r) return GW_EINVAL;
  switch (key) {
    case GW_RTUNE_ORD_WINDOW:
    case GW_RTUNE_ORD_WELCH:
      if (value < 0 || value > 1) return rfail(r, GW_EINVAL, "radix order must be 0 or 1");
      (key == GW_RTUNE_ORD_WINDOW ? r->ord_win : r->ord_welch) = int(value);
      return GW_OK;
    case GW_RTUNE_GRID_WINDOW:
    case GW_RTUNE_GRID_WELCH:
      if (value < 1 || value > 8) return rfail(r, GW_EINVAL, "grid must be 1..8 workgroups per CU");
      (key == GW_RTUNE_GRID_WINDOW ? r->grid_win : r->grid_welch) = int(value);
      return GW_OK;
    case GW_RTUNE_WINDOW_MODE:
      if (value < 0 || value > 1) return rfail(r, GW_EINVAL, "window mode must be 0 or 1");
      r->win_mode = int(value);
      return GW_OK;
    case GW_RTUNE_WELCH_MODE:
      if (value < 0 || value > 1) return rfail(r, GW_EINVAL, "Welch mode must be 0 or 1");
      r->welch_mode = int(value);
      return GW_OK;
    default: return rfail(r, GW_EINVAL, "unknown tuning key");
  }
}

gw_status gw_ragged_get_tuning(const gw_ragged* r, int32_t key, int64_t* value) {
  if (!r || !value) return GW_EINVAL;
  switch (key) {
    case GW_RTUNE_ORD_WINDOW: *value = r->ord_win; break;
    case GW_RTUNE_ORD_WELCH: *value = r->ord_welch; break;
    case GW_RTUNE_GRID_WINDOW: *value = r->grid_win; break;
    case GW_RTUNE_GRID_WELCH: *value = r->grid_welch; break;
    case GW_RTUNE_WINDOW_MODE: *value = r->win_mode; break;
    case GW_RTUNE_WELCH_MODE: *value = r->welch_mode; break;
    default: return GW_EINVAL;
  }
  return GW_OK;
}

gw_status gw_ragged_autotune(gw_ragged* r, const float* const* bg, const int64_t* L_bg, float* out, void* workspace,
                             int64_t workspace_bytes, int32_t reps, double* report) {
  if (!r) return GW_EINVAL;
  if (reps < 1 || reps > 1000) return rfail(r, GW_EINVAL, "reps must be 1..1000");
  int64_t span[kMaxCls];
  gw_status s = check_call(r, bg, L_bg, out, nullptr, nullptr, workspace, workspace_bytes, span);
  if (s != GW_OK) return s;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return rfail(r, GW_EHIP, "hipStreamCreate");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int saved[6] = {r->ord_welch, r->grid_welch, r->ord_win, r->grid_win, r->win_mode, r->welch_mode};
  const int grids[3] = {1, 2, 4};
  double ms[12];
  std::fill(ms, ms + 12, 1e300);  // best of kTuneRounds interleaved rounds
  auto time_stage = [&](int stage, double* res) {
    s = enqueue_ragged(r, 1, 0, false, bg, L_bg, span, out, nullptr, nullptr, workspace, stage, st);  // warm-up
    if (s == GW_OK && hipEventRecord(e0, st) != hipSuccess) s = rfail(r, GW_EHIP, "hipEventRecord");
    for (int k = 0; k < reps && s == GW_OK; ++k)
      s = enqueue_ragged(r, 1, 0, false, bg, L_bg, span, out, nullptr, nullptr, workspace, stage, st);
    if (s == GW_OK && hipEventRecord(e1, st) != hipSuccess) s = rfail(r, GW_EHIP, "hipEventRecord");
    if (s == GW_OK && hipEventSynchronize(e1) != hipSuccess) s = rfail(r, GW_EHIP, "hipEventSynchronize");
    // a failed timing query fails the tuner rather than reading as 0 ms
    float t = 0.f;
    if (s == GW_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) s = rfail(r, GW_EHIP, "hipEventElapsedTime");
    if (s == GW_OK) *res = std::min(*res, double(t) / reps);
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    s = rfail(r, GW_EHIP, "hipEventCreate");
  } else {
    s = enqueue_ragged(r, 1, 0, false, bg, L_bg, span, out, nullptr, nullptr, workspace, kStageAll, st);
    for (int round = 0; round < kTuneRounds && s == GW_OK; ++round) {
      r->welch_mode = 0;
      for (int o = 0; o < 2 && s == GW_OK; ++o)
        for (int gi = 0; gi < 3 && s == GW_OK; ++gi) {
          r->ord_welch = o;
          r->grid_welch = grids[gi];
          time_stage(kStageWelch, &ms[o * 3 + gi]);
        }
      r->welch_mode = 1;
      for (int o = 0; o < 2 && s == GW_OK; ++o) {
        r->ord_welch = o;
        time_stage(kStageWelch, &ms[10 + o]);
      }
      for (int m = 0; m < 2 && s == GW_OK; ++m)
        for (int o = 0; o < 2 && s == GW_OK; ++o) {
          r->ord_win = o;
          r->win_mode = m;
          r->grid_win = saved[3];
          time_stage(kStageWindow, &ms[6 + 2 * m + o]);
        }
    }
  }
  if (s == GW_OK) {
    int best = 0;
    for (int k = 1; k < 6; ++k)
      if (ms[k] < ms[best]) best = k;
    const int bc = ms[11] < ms[10] ? 11 : 10;
    if (ms[bc] < ms[best]) {
      r->welch_mode = 1;
      r->ord_welch = bc - 10;
      r->grid_welch = saved[1];
    } else {
      r->welch_mode = 0;
      r->ord_welch = best / 3;
      r->grid_welch = grids[best % 3];
    }
    int bw = 6;
    for (int k = 7; k < 10; ++k)
      if (ms[k] < ms[bw]) bw = k;
    r->win_mode = (bw - 6) / 2;
    r->ord_win = (bw - 6) % 2;
    if (report) std::copy(ms, ms + 12, report);
  } else {
    r->ord_welch = saved[0];
    r->grid_welch = saved[1];
    r->ord_win = saved[2];
    r->grid_win = saved[3];
    r->win_mode = saved[4];
    r->welch_mode = saved[5];
  }
  if (hipStreamSynchronize(st) != hipSuccess && s == GW_OK) s = rfail(r, GW_EHIP, "hipStreamSynchronize");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  return s;
}

}  // extern "C"
