// libgwgen.so: HIP kernels for gfx950 and the C ABI declared in gwgen.h.
//
// Kernels (grid / block):
//   k_sample_params    ceil(B/256) / 256      prior draws, one thread per sample
//   k_gen_fd_waveform  (ceil(F/256), B) / 256 plus/cross on the window grid
//   k_project          (ceil(F/256), B) / 256 detector projection + time shift
//   k_inject           B*D / (N/32)           irfft of the projected signal + noise
//   k_welch            B*D / (L/16)           segmented Welch PSD, one block per
//                                             (sample, detector)
//   k_window<SRC>      B*D / (N/32)           rfft -> (+ signal) -> whiten -> irfft;
//                                             SRC 0 reads strain (whiten), SRC 1
//                                             reads the background and generates
//                                             the signal in registers (fused)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "gw_fft.hpp"
#include "gw_physics.hpp"
#include "gw_internal.hpp"
#include "gw_items.hpp"
#include "../../include/gwgen.h"

using namespace gw;

namespace {

// ------------------------------------------------------------ prior draws
struct SampleArgs {
  DevCfg cf;
  uint64_t seed, first;
  const uint64_t* batch;  // device batch index (graph replays): first = *batch * B, or NULL
  int64_t B, span;
  double* params;
  int64_t* offset;
  float* params_f32;
  uint32_t* status;
  WfScalars* wf;     // [B] waveform constants for the fused kernel, or NULL
  DetScalars* dsc;   // [B][D] antenna patterns and delays, or NULL
  uint32_t ext_k = 1;  // sky positions per intrinsic draw
};

__global__ __launch_bounds__(256) void k_sample_params(SampleArgs a) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= a.B) return;
  const uint64_t first = a.batch ? *a.batch * uint64_t(a.B) : a.first;
  draw_sample(a.cf, a.seed, first + uint64_t(i), i, a.B, a.span, 0.0, a.params, a.offset, a.params_f32, a.status,
              a.wf, a.dsc, a.ext_k);
}

// -------------------------------------------------------- plus / cross
struct WaveArgs {
  DevCfg cf;
  const double* params;
  int64_t B;
  const double* kcbrt;
  const double* lnk3;
  float* hp;
  float* hc;
};

template <class TP, bool FULL>
__global__ __launch_bounds__(256) void k_gen_fd_waveform(WaveArgs a) {
  __shared__ WfScalars w;
  const int64_t b = blockIdx.x;
  if (threadIdx.x == 0) wf_setup(a.params, a.B, b, a.cf, w);
  __syncthreads();
  const int F = a.cf.F;
  for (int k = threadIdx.x; k < F; k += 256) {
    float2 hp = {0.f, 0.f}, hc = {0.f, 0.f};
    if (k > 0 && k >= a.cf.kmin && k < w.kend && a.cf.approximant == 2) {
      // sine-Gaussian: h+ = ap [e^{i phi0} G(f - f0) + e^{-i phi0} G(f + f0)],
      // hx = ax [-i e^{i phi0} G(f - f0) + i e^{-i phi0} G(f + f0)]
      const double f = double(k) * a.cf.invT;
      const TP xm = TP(f - w.sg_f0), xp = TP(f + w.sg_f0);
      const TP gm = TP(w.sg_G0) * exp(-TP(w.sg_pt2) * xm * xm), gp = TP(w.sg_G0) * exp(-TP(w.sg_pt2) * xp * xp);
      TP sp, cp;
      sincos_rev(TP(w.sg_rphi), &sp, &cp);
      const TP emx = gm * cp, emy = gm * sp, epx = gp * cp, epy = -gp * sp;
      const TP ap = TP(0.5) * (TP(1) + TP(w.cosi) * TP(w.cosi)), ax = TP(w.cosi);
      hp = {float(ap * (emx + epx)), float(ap * (emy + epy))};
      hc = {float(ax * (emy - epy)), float(ax * (epx - emx))};
    } else if (k > 0 && k >= a.cf.kmin && k < w.kend) {
      const double kc = a.kcbrt[k], lk = a.lnk3[k];
      TP rev = wf_phase_rev<TP, FULL>(w, k, kc, lk, a.cf.invT) + TP(w.pconst);
      rev = frac1(rev);
      TP s, c;
      sincos_rev(rev, &s, &c);
      const TP A = wf_amplitude<TP>(w, k, kc, a.cf.invT);
      const TP cp = A * TP(0.5) * (TP(1) + TP(w.cosi) * TP(w.cosi));
      const TP cx = A * TP(w.cosi);
      // h+ = A cp e^{-i Psi};  hx = -i A cx e^{-i Psi}
      hp = {float(cp * c), float(-cp * s)};
      hc = {float(-cx * s), float(-cx * c)};
    }
    reinterpret_cast<float2*>(a.hp)[b * F + k] = hp;
    reinterpret_cast<float2*>(a.hc)[b * F + k] = hc;
  }
}

// ------------------------------------------------------------ projection
struct ProjArgs {
  DevCfg cf;
  const double* params;
  int64_t B;
  const float* hp;
  const float* hc;
  float* hdet;
};

template <class TP>
__global__ __launch_bounds__(256) void k_project(ProjArgs a) {
  __shared__ DetScalars ds[GW_MAX_DET];
  const int64_t b = blockIdx.y;
  const int D = a.cf.n_det;
  if (threadIdx.x < D) {
    const int64_t B = a.B;
    ds[threadIdx.x] = det_response(a.cf.det[threadIdx.x], a.params[6 * B + b], a.params[7 * B + b],
                                   a.params[8 * B + b], a.params[10 * B + b]);
  }
  __syncthreads();
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int F = a.cf.F;
  if (k >= F) return;
  const float2 hp = reinterpret_cast<const float2*>(a.hp)[b * F + k];
  const float2 hc = reinterpret_cast<const float2*>(a.hc)[b * F + k];
  for (int d = 0; d < D; ++d) {
    const TP rev = frac1(TP(k) * TP(ds[d].tau * a.cf.invT));
    float s, c;
    sincos_rev(float(rev), &s, &c);
    const float fp = float(ds[d].fp), fx = float(ds[d].fx), fs = float(a.cf.fs);
    const float2 h = {fs * (fp * hp.x + fx * hc.x), fs * (fp * hp.y + fx * hc.y)};
    // h * e^{-i phi}
    reinterpret_cast<float2*>(a.hdet)[(b * D + d) * F + k] = {h.x * c + h.y * s, h.y * c - h.x * s};
  }
}

// Second launch bound: minimum waves per SIMD (clamped to what LDS allows);
// 4 waves per SIMD gives a budget of 128 VGPRs.
template <int NC> struct WinOcc { static constexpr int value = NC >= 16384 ? 1 : NC >= 8192 ? 4 : NC >= 2048 ? 8 : 16; };

template <class T, class TP, bool FULL, int NC, int SRC, int ORD>
__global__ __launch_bounds__(NC / 16, WinOcc<NC>::value) void k_window(WinArgs a) {
  constexpr int LS = LdsSize<NC>::value;
  __shared__ T lds[2 * LS];
  __shared__ uint32_t sflag;
  __shared__ float snodes[SRC == 3 ? 2 * kSurrNodes : 1];
  const int t = threadIdx.x;
  const int64_t bd = blockIdx.x;
  const int D = a.cf.n_det;
  const int64_t b = bd / D;
  const int d = int(bd - b * D);
  const int N = 2 * NC;
  if (t == 0) sflag = 0;
  const float* x = nullptr;
  const float* hrow = nullptr;
  const float* nz = nullptr;
  if constexpr (SRC == 0) x = a.src + bd * N;
  else if constexpr (SRC == 2) {
    hrow = a.src + bd * 2 * (NC + 1);
    nz = a.bg + int64_t(d) * a.L_bg + a.offset[b] + a.cf.P;
  } else x = a.src + int64_t(d) * a.L_bg + a.offset[b] + a.cf.P;
  const float* psd = SRC == 4 ? a.psd + int64_t(d) * (NC + 1) : a.psd + bd * a.cf.Fw;
  float* o = a.out + bd * (SRC == 4 ? N - 2 * a.crop : N);
  float* o2 = SRC == 5 ? a.out2 + bd * N : nullptr;
  window_item<T, TP, FULL, NC, SRC, ORD>(a.cf, a, t, b, d, x, hrow, nz, psd, o,
                                         reinterpret_cast<const cpx<T>*>(a.tw), reinterpret_cast<const cpx<T>*>(a.twr),
                                         lds, lds + LS, true, &sflag, SRC == 3 ? snodes : nullptr, o2);
  __syncthreads();
  if (t == 0 && sflag && a.status) atomicOr(a.status + b, sflag);
}

// ------------------------------------------------------------------ Welch
struct WelchArgs {
  DevCfg cf;
  const float* bg;
  int64_t L_bg;
  const int64_t* offset;
  float* psd;
  const void* tw;  // cpx<T>[L], exp(-2 pi i n / L)
  double norm;     // 1 / (K fs sum w^2)
};

// OCC: waves per SIMD the register allocation must allow (2, or 3 with the
// loop-invariant twiddles partly spilled and reloaded per segment pair).
template <class T, class ACC, int NC, int ORD, int OCC>
__global__ __launch_bounds__(NC / 16, OCC) void k_welch(WelchArgs a) {
  constexpr int LS = LdsSize<NC>::value;
  __shared__ T lds[2 * LS];
  const int64_t bd = blockIdx.x;
  const int D = a.cf.n_det;
  const int64_t b = bd / D;
  const int d = int(bd - b * D);
  welch_item<T, ACC, NC, ORD>(a.cf.K, a.norm, threadIdx.x, a.bg + int64_t(d) * a.L_bg + a.offset[b],
                              a.psd + bd * a.cf.Fw, reinterpret_cast<const cpx<T>*>(a.tw), lds, lds + LS, true);
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// batch counter of graph replays (vector stores, one lane)
__global__ void k_set_u64(uint64_t* p, uint64_t v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_add_u64(uint64_t* p, uint64_t v) {
  if (threadIdx.x == 0) *p += v;
}

// ------------------------------------------------------- per-run PSD mode
// Chunk c of the run PSD covers segments [cK, (c+1)K): its stretch starts at c K S.
__global__ void k_chunk_offsets(int64_t* off, int64_t n, int64_t stride) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) off[i] = i * stride;
}

// out[d][k] = mean over chunks of part[c][d][k] (binary64 sum).
__global__ void k_mean_chunks(const float* part, int64_t n_chunks, int n_det, int Fw, float* out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_det * Fw) return;
  double sum = 0.0;
  for (int64_t c = 0; c < n_chunks; ++c) sum += double(part[c * int64_t(n_det) * Fw + i]);
  out[i] = float(sum / double(n_chunks));
}

// Truncated whitening filter of one detector, by one workgroup of NC/16
// threads: the whitening gain g on the window grid (from the PSD row), its
// impulse response by an inverse real transform, the cos^2 taper over
// circular lags |n| < M/2, and the magnitude of the forward real transform.
struct FiltArgs {
  DevCfg cf;
  const float* psd;  // [D][Fw]
  float* filt;       // [D][NC + 1]
  int M;
  const void* tw;    // cpx<T>[NC]
  const void* twr;   // cpx<T>[NC/2 + 1]
  uint32_t* status;  // [D] GW_STATUS_* bits of each detector's PSD, or NULL
};

template <class T, int NC>
__global__ __launch_bounds__(NC / 16) void k_filter(FiltArgs a) {
  constexpr int NT = NC / 16, LS = LdsSize<NC>::value;
  __shared__ T lds[2 * LS];
  T* sre = lds;
  T* sim = lds + LS;
  const int t = threadIdx.x;
  const int d = blockIdx.x;
  const DevCfg& cf = a.cf;
  const float* psd = a.psd + int64_t(d) * cf.Fw;
  const cpx<T>* twr = reinterpret_cast<const cpx<T>*>(a.twr);
  PowTwiddle<T, NC, 0> tw{reinterpret_cast<const cpx<T>*>(a.tw)};
  uint32_t flag = 0;
  __shared__ uint32_t dflag;  // the detector's status bits (visible after the first barrier)
  if (t == 0) dflag = 0u;
  // 1. g is real and even: pack it for the half-length inverse transform
  for (int i = 0; i <= 8; ++i) {
    const int k = t + NT * i;
    if (k > NC / 2) break;
    const int km = NC - k;
    const cpx<T> W = twr[k];
    const cpx<T> Yk = {whiten_gain<T>(cf, psd, k, NC, flag), T(0)};
    const cpx<T> Ym = km == k ? Yk : cpx<T>{whiten_gain<T>(cf, psd, km, NC, flag), T(0)};
    const cpx<T> p = cscale(cadd(Yk, cconj(Ym)), T(0.5));
    const cpx<T> q = twmul<+1>(cscale(csub(Yk, cconj(Ym)), T(0.5)), W);
    sre[lpad<T>(k)] = p.x - q.y;
    sim[lpad<T>(k)] = p.y + q.x;
    if (k != 0 && km != k) {
      sre[lpad<T>(km)] = p.x + q.y;
      sim[lpad<T>(km)] = -p.y + q.x;
    }
  }
  __syncthreads();
  cpx<T> v[16];
  block_fft<T, NC, +1, true, 0>(v, sre, sim, t, tw);
  // 2. v[e] holds samples 2n, 2n+1 of the response (times NC): scale and taper
  const int N = 2 * NC;
  const T sc = T(1) / T(NC);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int n = fft_out_index<NC, 0>(t, e);
    T h[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int m = 2 * n + j;
      const int lag = m <= NC ? m : m - N;
      T sn, cs;
      sincospi_t(T(lag) / T(a.M), &sn, &cs);
      h[j] = 2 * abs(lag) < a.M ? cs * cs : T(0);
    }
    v[e] = {v[e].x * sc * h[0], v[e].y * sc * h[1]};
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int i = lpad<T>(fft_out_index<NC, 0>(t, e));
    sre[i] = v[e].x;
    sim[i] = v[e].y;
  }
  __syncthreads();
  // 3. forward real transform of the tapered response
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = lpad<T>(t + NT * j);
    v[fft_in_slot<NC, 0>(j)] = {sre[i], sim[i]};
  }
  __syncthreads();
  block_fft<T, NC, -1, false, 0>(v, sre, sim, t, tw);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int i = lpad<T>(fft_out_index<NC, 0>(t, e));
    sre[i] = v[e].x;
    sim[i] = v[e].y;
  }
  __syncthreads();
  float* out = a.filt + int64_t(d) * (NC + 1);
  for (int i = 0; i <= 8; ++i) {
    const int k = t + NT * i;
    if (k > NC / 2) break;
    const int km = NC - k;
    const cpx<T> W = twr[k];
    const cpx<T> A = {sre[lpad<T>(k)], sim[lpad<T>(k)]};
    const cpx<T> Bm = {sre[lpad<T>(km & (NC - 1))], sim[lpad<T>(km & (NC - 1))]};
    const cpx<T> s = cadd(A, cconj(Bm));
    const cpx<T> u = cmul(W, csub(A, cconj(Bm)));
    out[k] = float(fabs(T(0.5) * (s.x + u.y)));
    if (km != k) out[km] = float(fabs(T(0.5) * (s.x - u.y)));
  }
  // bins with a non-finite or non-positive PSD were dropped from the gain
  if (flag) atomicOr(&dflag, flag);
  __syncthreads();
  if (t == 0 && a.status) a.status[d] = dflag;
}

}  // namespace

// ======================================================================= host

namespace {

const char* const kDetNames[3] = {"H1", "L1", "V1"};
// geodetic latitude [deg N], longitude [deg E], x-arm and y-arm azimuth [deg
// from North toward East]: public site survey values
const double kSites[3][4] = {
    {46.45514, -119.40766, 324.0000, 234.0000},
    {30.56289, -90.77424, 252.2835, 162.2835},
    {43.63141, 10.50450, 19.4326, 289.4326},
};

DetGeom make_detector(int id) {
  const double deg = M_PI / 180.0;
  const double lat = kSites[id][0] * deg, lon = kSites[id][1] * deg;
  const double a = 6378137.0, f = 1.0 / 298.257223563, e2 = f * (2.0 - f);
  const double nu = a / std::sqrt(1.0 - e2 * std::sin(lat) * std::sin(lat));
  DetGeom g;
  g.r[0] = nu * std::cos(lat) * std::cos(lon);
  g.r[1] = nu * std::cos(lat) * std::sin(lon);
  g.r[2] = nu * (1.0 - e2) * std::sin(lat);
  const double east[3] = {-std::sin(lon), std::cos(lon), 0.0};
  const double north[3] = {-std::sin(lat) * std::cos(lon), -std::sin(lat) * std::sin(lon), std::cos(lat)};
  double x[3], y[3];
  const double zx = kSites[id][2] * deg, zy = kSites[id][3] * deg;
  for (int i = 0; i < 3; ++i) {
    x[i] = std::cos(zx) * north[i] + std::sin(zx) * east[i];
    y[i] = std::cos(zy) * north[i] + std::sin(zy) * east[i];
  }
  const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  for (int m = 0; m < 6; ++m) {
    const int i = ij[m][0], j = ij[m][1];
    g.D[m] = 0.5 * (x[i] * x[j] - y[i] * y[j]);
  }
  return g;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

gw_status fail(gw_ctx* c, gw_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

gw_status check_launch(gw_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, GW_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return GW_OK;
}

}  // namespace

namespace gw {
gw_status ctx_fail(gw_ctx* c, gw_status s, const std::string& msg) { return fail(c, s, msg); }
gw_status ctx_check_launch(gw_ctx* c, const char* what) { return check_launch(c, what); }

// Capture `enqueue` plus a batch-index increment into a graph on a private
// stream; the device counter `batch` starts at `first`.
gw_status capture_graph(const std::function<gw_status(hipStream_t)>& enqueue, uint64_t* batch, uint64_t first,
                        gw_graph** out, std::string* why) {
  if (hipMemcpy(batch, &first, sizeof(first), hipMemcpyHostToDevice) != hipSuccess) {
    *why = "hipMemcpy batch counter";
    return GW_EHIP;
  }
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    *why = "hipStreamCreate";
    return GW_EHIP;
  }
  gw_graph* g = new gw_graph();
  g->batch = batch;
  gw_status s = GW_OK;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    *why = "hipStreamBeginCapture";
    s = GW_EHIP;
  } else {
    s = enqueue(st);
    if (s == GW_OK) {
      hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, st, batch, uint64_t(1));
      if (hipGetLastError() != hipSuccess) {
        *why = "k_add_u64";
        s = GW_EHIP;
      }
    } else {
      *why = "a launch failed during capture";
    }
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (s == GW_OK && e != hipSuccess) {
      *why = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
      s = GW_EHIP;
    }
    g->graph = graph;
    if (s == GW_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      *why = "hipGraphInstantiate";
      s = GW_EHIP;
    }
  }
  (void)hipStreamDestroy(st);
  if (s != GW_OK) {
    gw_graph_destroy(g);
    return s;
  }
  *out = g;
  return GW_OK;
}
}  // namespace gw

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

template <class T>
gw_status upload_twiddles(gw_ctx* c, void** dst, int n, int denom) {
  std::vector<cpx<T>> h(n);
  for (int i = 0; i < n; ++i) {
    const double ang = -2.0 * M_PI * double(i) / double(denom);
    h[i] = {T(std::cos(ang)), T(std::sin(ang))};
  }
  if (hipMalloc(dst, sizeof(cpx<T>) * n) != hipSuccess) return fail(c, GW_ENOMEM, "hipMalloc twiddles");
  if (hipMemcpy(*dst, h.data(), sizeof(cpx<T>) * n, hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, GW_EHIP, "hipMemcpy twiddles");
  return GW_OK;
}

// Per-bin tables of the long-window bins pass in the transposed layout of
// its spectrum (row k mod N2, column k / N2, rows of N1): one allocation
// of double[NC] k^(1/3), double[NC] ln(k)/3, cpx<float>[NC] exp(-2 pi i k/N).
// Also the column twiddles W_NC^(m1 k2) at [k2][m1] (c->tw_long), so that a
// wavefront's threads (consecutive m1) read consecutive entries.
gw_status upload_long_tables(gw_ctx* c, int NC) {
  const int N1 = long_row_length(NC), N2 = NC / N1;
  std::vector<double> kc(NC), lk(NC);
  std::vector<cpx<float>> tw(NC), twc(NC);
  for (int k = 0; k < NC; ++k) {
    const int p = (k % N2) * N1 + k / N2;
    kc[p] = std::cbrt(double(k));
    lk[p] = k > 0 ? std::log(double(k)) / 3.0 : 0.0;
    const double ang = -2.0 * M_PI * double(k) / double(2 * NC);
    tw[p] = {float(std::cos(ang)), float(std::sin(ang))};
  }
  for (int k2 = 0; k2 < N2; ++k2)
    for (int m1 = 0; m1 < N1; ++m1) {
      const int n = int((int64_t(m1) * k2) & (NC - 1));
      const double ang = -2.0 * M_PI * double(n) / double(NC);
      twc[size_t(k2) * N1 + m1] = {float(std::cos(ang)), float(std::sin(ang))};
    }
  if (hipMalloc(&c->tw_long, sizeof(cpx<float>) * size_t(NC)) != hipSuccess)
    return fail(c, GW_ENOMEM, "hipMalloc column twiddles");
  if (hipMemcpy(c->tw_long, twc.data(), sizeof(cpx<float>) * size_t(NC), hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, GW_EHIP, "hipMemcpy column twiddles");
  const size_t nd = sizeof(double) * size_t(NC), nt = sizeof(cpx<float>) * size_t(NC);
  if (hipMalloc(&c->long_tabs, 2 * nd + nt) != hipSuccess) return fail(c, GW_ENOMEM, "hipMalloc long tables");
  char* base = static_cast<char*>(c->long_tabs);
  if (hipMemcpy(base, kc.data(), nd, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + nd, lk.data(), nd, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + 2 * nd, tw.data(), nt, hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, GW_EHIP, "hipMemcpy long tables");
  return GW_OK;
}

gw_status validate_cfg(const gw_config* g, DevCfg* dc, std::string* why) {
  auto bad = [&](const char* m) { *why = m; return GW_EINVAL; };
  if (!g) return bad("config is NULL");
  if (g->n_det < 1 || g->n_det > GW_MAX_DET) return bad("n_det must be in 1..4");
  for (int d = 0; d < g->n_det; ++d)
    if (g->det_id[d] < 0 || g->det_id[d] > 2) return bad("det_id must be 0 (H1), 1 (L1) or 2 (V1)");
  if (!(g->fs > 0) || !(g->t_window > 0) || !(g->psd_length > 0) || !(g->fftlen > 0))
    return bad("fs, t_window, psd_length, fftlen must be positive");
  const double Nd = g->t_window * g->fs, Pd = g->psd_length * g->fs, Ld = g->fftlen * g->fs;
  const double Sd = (g->fftlen - g->overlap) * g->fs;
  auto integral = [](double v) { return std::fabs(v - std::round(v)) < 1e-9 && v < 1e12; };
  if (!integral(Nd) || !integral(Pd) || !integral(Ld) || !integral(Sd))
    return bad("t_window, psd_length, fftlen and overlap must be whole numbers of samples");
  const int64_t N = std::llround(Nd), P = std::llround(Pd), L = std::llround(Ld), S = std::llround(Sd);
  // the window transforms run NC = N/2 in {1024, ..., 16384} points in one
  // workgroup (four-step beyond): shorter windows have no kernel
  if (!is_pow2(N) || N < 2048 || N > (int64_t(1) << 20))
    return bad("N = t_window*fs must be a power of two in [2048, 2^20]");
  if (N > 32768 && g->precision == 2) return GW_EUNSUPPORTED;
  if (!is_pow2(L) || L < 2048 || L > 4096) return bad("L = fftlen*fs must be 2048 or 4096");
  if (S * 2 != L) return bad("overlap must be half of fftlen (stride L/2)");
  if (P < L || (P - L) % S) return bad("psd_length*fs - L must be a non-negative multiple of the stride");
  if (N % L) return bad("t_window must be a whole multiple of fftlen");
  if (!(g->f_min >= 0) || !(g->f_min < 0.5 * g->fs)) return bad("f_min must be in [0, fs/2)");
  if (g->approximant < 0 || g->approximant > 2) return bad("approximant must be 0, 1 or 2");
  if (g->approximant == 2) {
    if (!(g->f0[0] > 0) || !(g->f0[1] >= g->f0[0]) || !(g->f0[1] < 0.5 * g->fs)) return bad("bad f0 range");
    if (!(g->quality[0] > 0) || !(g->quality[1] >= g->quality[0])) return bad("bad quality range");
    if (!(g->hrss[0] > 0) || !(g->hrss[1] >= g->hrss[0])) return bad("bad hrss range");
  }
  if (g->precision < 0 || g->precision > 2) return bad("precision must be 0, 1 or 2");
  if (g->approximant != 2) {
    if (!(g->mc[0] > 0) || !(g->mc[1] >= g->mc[0])) return bad("bad chirp-mass range");
    if (!(g->q[0] > 0) || !(g->q[1] >= g->q[0]) || g->q[1] > 1) return bad("bad mass-ratio range (0 < q <= 1)");
    if (!(g->chi[0] > -1) || !(g->chi[1] < 1) || !(g->chi[1] >= g->chi[0])) return bad("bad spin range (|chi| < 1)");
    if (!(g->dl[0] > 0) || !(g->dl[1] >= g->dl[0])) return bad("bad distance range");
  }
  if (g->precision == 2 && N > 16384) return GW_EUNSUPPORTED;
  DevCfg c;
  std::memset(&c, 0, sizeof(c));
  c.n_det = g->n_det;
  c.N = int(N);
  c.F = int(N / 2 + 1);
  c.P = int(P);
  c.L = int(L);
  c.S = int(S);
  c.K = int((P - L) / S + 1);
  c.Fw = int(L / 2 + 1);
  c.ratio = int(N / L);
  c.log2_ratio = 0;
  while ((1 << c.log2_ratio) < c.ratio) ++c.log2_ratio;
  c.inv_ratio = 1.0 / double(c.ratio);
  c.approximant = g->approximant;
  c.precision = g->precision;
  c.fs = g->fs;
  c.T = g->t_window;
  c.invT = 1.0 / g->t_window;
  c.f_min = g->f_min;
  for (int i = 0; i < 2; ++i) {
    c.mc[i] = g->mc[i];
    c.q[i] = g->q[i];
    c.chi[i] = g->chi[i];
    c.dl[i] = g->dl[i];
    c.f0r[i] = g->f0[i];
    c.Qr[i] = g->quality[i];
    c.hrssr[i] = g->hrss[i];
  }
  // first bin with k/T >= f_min (k/T rounded as the binary64 grid is formed)
  int k = int(std::ceil(g->f_min * g->t_window));
  while (k > 0 && double(k - 1) / g->t_window >= g->f_min) --k;
  while (double(k) / g->t_window < g->f_min) ++k;
  c.kmin = k;
  // defaults before any autotuning: the variants measured fastest at the
  // paper-scale shape (binary32 transforms of L = 4096 fit 3 waves per SIMD
  // without spills; the 8192-point window prefers its radix-2 pass first)
  c.occ_welch = (c.L == 4096 && c.precision != 2) ? 3 : 2;
  // windows longer than 32768 samples: 1 selects the fused row-pair pass
  c.ord_win = ((c.N == 16384 || c.N > 32768) && c.precision != 2) ? 1 : 0;
  for (int d = 0; d < g->n_det; ++d) c.det[d] = make_detector(g->det_id[d]);
  *dc = c;
  return GW_OK;
}

}  // namespace

namespace gw {
gw_status validate_config(const gw_config* g, DevCfg* dc, std::string* why) { return validate_cfg(g, dc, why); }
}  // namespace gw

// Static scratch area of the allocation-free batch entry point: one copy per
// device, held until the process ends.  Its name is only a host-side stand-in
// in host code; the device address of each device's copy is resolved once,
// with that device current (resolve_scratch), and used from then on.
static __device__ __align__(256) unsigned char scratch[GW_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxScratchDevices = 256;
void* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of the current device's scratch area (resolved on first use).
gw_status resolve_scratch(int dev, void** addr, std::string* why) {
  if (dev < 0 || dev >= kMaxScratchDevices) {
    *why = "device index out of range for the scratch table";
    return GW_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return GW_EHIP;
    }
    g_scratch_addr[dev] = p;
  }
  *addr = g_scratch_addr[dev];
  return GW_OK;
}

static int64_t ws_params_bytes(int64_t B) { return ((B * 12 * 8 + 255) / 256) * 256; }
static int64_t ws_offset_bytes(int64_t B) { return ((B * 8 + 255) / 256) * 256; }
static int64_t ws_psd_bytes(const DevCfg& d, int64_t B) { return ((B * d.n_det * d.Fw * 4 + 255) / 256) * 256; }
static int64_t ws_wf_bytes(int64_t B) { return ((B * int64_t(sizeof(WfScalars)) + 255) / 256) * 256; }
static int64_t ws_det_bytes(const DevCfg& d, int64_t B) { return ((B * d.n_det * int64_t(sizeof(DetScalars)) + 255) / 256) * 256; }
// 256 bytes after the per-sample arrays hold the graph batch counter
static int64_t ws_counter_offset(const DevCfg& d, int64_t B) {
  return ws_params_bytes(B) + ws_offset_bytes(B) + ws_psd_bytes(d, B) + ws_wf_bytes(B) + ws_det_bytes(d, B);
}

// dispatch a k_window instantiation on the window FFT size and radix order
template <class T, class TP, bool FULL, int SRC, int ORD>
static void launch_window_ord(const DevCfg& d, int64_t blocks, const WinArgs& a, hipStream_t stream) {
  const int NC = d.N / 2;
  switch (NC) {
    case 1024: hipLaunchKernelGGL((k_window<T, TP, FULL, 1024, SRC, ORD>), dim3(unsigned(blocks)), dim3(64), 0, stream, a); break;
    case 2048: hipLaunchKernelGGL((k_window<T, TP, FULL, 2048, SRC, ORD>), dim3(unsigned(blocks)), dim3(128), 0, stream, a); break;
    case 4096: hipLaunchKernelGGL((k_window<T, TP, FULL, 4096, SRC, 0>), dim3(unsigned(blocks)), dim3(256), 0, stream, a); break;
    case 8192: hipLaunchKernelGGL((k_window<T, TP, FULL, 8192, SRC, ORD>), dim3(unsigned(blocks)), dim3(512), 0, stream, a); break;
    default:
      if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((k_window<T, TP, FULL, 16384, SRC, ORD>), dim3(unsigned(blocks)), dim3(1024), 0, stream, a);
      break;
  }
}

template <class T, class TP, bool FULL, int SRC>
static void launch_window(const DevCfg& d, int64_t blocks, const WinArgs& a, hipStream_t stream) {
  if constexpr (sizeof(T) == 4) {
    if (d.ord_win) launch_window_ord<T, TP, FULL, SRC, 1>(d, blocks, a, stream);
    else launch_window_ord<T, TP, FULL, SRC, 0>(d, blocks, a, stream);
  } else {
    launch_window_ord<T, TP, FULL, SRC, 0>(d, blocks, a, stream);
  }
}

template <int SRC>
void launch_window_prec(const DevCfg& d, int64_t blocks, const WinArgs& a, hipStream_t stream) {
  if (d.precision == 0) launch_window<float, float, false, SRC>(d, blocks, a, stream);
  else if (d.precision == 1) launch_window<float, double, false, SRC>(d, blocks, a, stream);
  else launch_window<double, double, true, SRC>(d, blocks, a, stream);
}

static WinArgs win_args(gw_ctx* c) {
  WinArgs a;
  std::memset(&a, 0, sizeof(a));
  a.cf = c->dc;
  a.kcbrt = c->kcbrt;
  a.lnk3 = c->lnk3;
  a.k53 = c->k53;
  a.tw = c->tw_win;
  a.twr = c->twr_win;
  return a;
}

template <class T, class ACC, int OCC>
static void launch_welch_occ(const DevCfg& d, int64_t blocks, const WelchArgs& a, hipStream_t stream) {
  if (d.L == 2048) {
    if (d.ord_welch)
      hipLaunchKernelGGL((k_welch<T, ACC, 2048, 1, OCC>), dim3(unsigned(blocks)), dim3(128), 0, stream, a);
    else
      hipLaunchKernelGGL((k_welch<T, ACC, 2048, 0, OCC>), dim3(unsigned(blocks)), dim3(128), 0, stream, a);
  } else {
    hipLaunchKernelGGL((k_welch<T, ACC, 4096, 0, OCC>), dim3(unsigned(blocks)), dim3(256), 0, stream, a);
  }
}

template <class T, class ACC>
static void launch_welch(const DevCfg& d, int64_t blocks, const WelchArgs& a, hipStream_t stream) {
  if constexpr (sizeof(T) == 4) {
    if (d.occ_welch == 3) launch_welch_occ<T, ACC, 3>(d, blocks, a, stream);
    else launch_welch_occ<T, ACC, 2>(d, blocks, a, stream);
  } else {
    // binary64: one radix order, occupancy as the registers allow
    if (d.L == 2048) hipLaunchKernelGGL((k_welch<T, ACC, 2048, 0, 1>), dim3(unsigned(blocks)), dim3(128), 0, stream, a);
    else hipLaunchKernelGGL((k_welch<T, ACC, 4096, 0, 1>), dim3(unsigned(blocks)), dim3(256), 0, stream, a);
  }
}

template <class T>
static void launch_filter(const DevCfg& d, const FiltArgs& a, hipStream_t stream) {
  const dim3 grid = dim3(unsigned(d.n_det));
  switch (d.N / 2) {
    case 1024: hipLaunchKernelGGL((k_filter<T, 1024>), grid, dim3(64), 0, stream, a); break;
    case 2048: hipLaunchKernelGGL((k_filter<T, 2048>), grid, dim3(128), 0, stream, a); break;
    case 4096: hipLaunchKernelGGL((k_filter<T, 4096>), grid, dim3(256), 0, stream, a); break;
    case 8192: hipLaunchKernelGGL((k_filter<T, 8192>), grid, dim3(512), 0, stream, a); break;
    default:
      if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_filter<T, 16384>), grid, dim3(1024), 0, stream, a);
      break;
  }
}

static gw_status welch_launch(gw_ctx* c, const float* bg, int64_t L_bg, const int64_t* offset, int64_t B,
                              float* psd, hipStream_t stream) {
  const DevCfg& d = c->dc;
  WelchArgs a{d, bg, L_bg, offset, psd, c->tw_welch, 1.0 / (double(d.K) * d.fs * (3.0 * d.L / 8.0))};
  const int64_t blocks = B * d.n_det;
  if (d.precision == 0) launch_welch<float, float>(d, blocks, a, stream);
  else if (d.precision == 1) launch_welch<float, double>(d, blocks, a, stream);
  else launch_welch<double, double>(d, blocks, a, stream);
  return check_launch(c, "k_welch");
}

constexpr int kStageParams = 1, kStageWelch = 2, kStageWindow = 4, kStageAll = 7;
constexpr int64_t kMaxBlocks = int64_t(1) << 31;

// Host checks shared by the batch entry points (nothing is launched).
static gw_status check_batch_args(gw_ctx* c, int64_t B, const float* bg, int64_t L_bg, const float* out,
                                  const float* params_f32, const uint32_t* status, const void* workspace,
                                  int64_t workspace_bytes) {
  if (B < 0 || B * c->dc.n_det >= kMaxBlocks) return fail(c, GW_EINVAL, "bad B");
  if (B == 0) return GW_OK;
  if (!bg || !out || !workspace) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned4(bg) || !aligned16(out) || !aligned16(workspace) || (params_f32 && !aligned16(params_f32)) ||
      (status && !aligned4(status)))
    return fail(c, GW_EINVAL, "misaligned pointer");
  int64_t need = 0;
  gw_workspace_size(c, B, &need);
  if (workspace_bytes < need) return fail(c, GW_EINVAL, "workspace too small");
  if (L_bg - c->dc.P - c->dc.N + 1 <= 0) return fail(c, GW_EINVAL, "L_bg < P + N");
  return GW_OK;
}

// Queue the fused batch (prior draws, Welch PSDs, fused window kernel), or
// the stages selected by `stages`.  `batch` (device, nullable) supplies the
// batch index at run time for graph replays.
static gw_status enqueue_batch(gw_ctx* c, uint64_t seed, uint64_t batch_index, const uint64_t* batch, int64_t B,
                               const float* bg, int64_t L_bg, float* out, float* params_f32, uint32_t* status,
                               void* workspace, int stages, hipStream_t stream, uint32_t ext_k = 1,
                               float* out_ref = nullptr) {
  const int64_t span = L_bg - c->dc.P - c->dc.N + 1;
  char* ws = static_cast<char*>(workspace);
  double* params = reinterpret_cast<double*>(ws);
  int64_t* offset = reinterpret_cast<int64_t*>(ws + ws_params_bytes(B));
  float* psd = reinterpret_cast<float*>(ws + ws_params_bytes(B) + ws_offset_bytes(B));
  WfScalars* wf = reinterpret_cast<WfScalars*>(ws + ws_params_bytes(B) + ws_offset_bytes(B) + ws_psd_bytes(c->dc, B));
  DetScalars* dsc = reinterpret_cast<DetScalars*>(reinterpret_cast<char*>(wf) + ws_wf_bytes(B));
  gw_status s = GW_OK;
  if (stages & kStageParams) {
    SampleArgs sa{c->dc, seed, batch_index * uint64_t(B), batch, B, span, params, offset, params_f32, status, wf, dsc,
                  ext_k};
    hipLaunchKernelGGL(k_sample_params, dim3(unsigned((B + 255) / 256)), dim3(256), 0, stream, sa);
    s = check_launch(c, "k_sample_params");
    if (s != GW_OK) return s;
  }
  if (stages & kStageWelch) {
    s = welch_launch(c, bg, L_bg, offset, B, psd, stream);
    if (s != GW_OK) return s;
  }
  if (stages & kStageWindow) {
    WinArgs a = win_args(c);
    a.src = bg;
    a.L_bg = L_bg;
    a.offset = offset;
    a.params = params;
    a.B = B;
    a.psd = psd;
    a.out = out;
    a.status = status;
    a.wf = wf;
    a.dsc = dsc;
    if (c->dc.N > 32768) {
      if (out_ref) return fail(c, GW_EUNSUPPORTED, "view pairs need N <= 32768");
      return long_window(c, 1, a, bg, nullptr, B * c->dc.n_det, stream);
    }
    if (out_ref) {
      // view pairs: one pass, the reference view (same windows, PSDs and
      // parameters, signal at t_ref) from the same noise spectrum
      a.out2 = out_ref;
      a.t_ref = c->dc.T - 1.5;
      launch_window_prec<5>(c->dc, B * c->dc.n_det, a, stream);
      s = check_launch(c, "k_window<view pair>");
    } else {
      launch_window_prec<1>(c->dc, B * c->dc.n_det, a, stream);
      s = check_launch(c, "k_window<fused>");
    }
  }
  return s;
}

}  // namespace

extern "C" {

const char* gw_strerror(gw_status s) {
  switch (s) {
    case GW_OK: return "ok";
    case GW_EINVAL: return "invalid argument";
    case GW_ENOMEM: return "device allocation failed";
    case GW_EHIP: return "HIP error";
    case GW_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* gw_last_error(const gw_ctx* ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

gw_status gw_destroy(gw_ctx* c) {
  if (!c) return GW_OK;
  (void)hipFree(c->kcbrt);
  (void)hipFree(c->lnk3);
  (void)hipFree(c->k53);
  (void)hipFree(c->tw_win);
  (void)hipFree(c->twr_win);
  (void)hipFree(c->tw_welch);
  (void)hipFree(c->tw_long);
  (void)hipFree(c->long_tabs);
  delete c;
  return GW_OK;
}

gw_status gw_create(const gw_config* cfg, gw_ctx** out) {
  if (!out) return GW_EINVAL;
  *out = nullptr;
  DevCfg dc;
  std::string why;
  gw_status s = validate_cfg(cfg, &dc, &why);
  if (s != GW_OK) return s;
  gw_ctx* c = new gw_ctx();
  c->cfg = *cfg;
  c->dc = dc;
  if (hipGetDevice(&c->device) != hipSuccess) {
    gw_destroy(c);
    return GW_EHIP;
  }
  s = resolve_scratch(c->device, &c->scratch, &c->err);
  if (s != GW_OK) {
    gw_destroy(c);
    return s;
  }
  std::vector<double> hc(dc.F), hl(dc.F), h53(dc.F);
  for (int k = 0; k < dc.F; ++k) {
    hc[k] = std::cbrt(double(k));
    hl[k] = k > 0 ? std::log(double(k)) / 3.0 : 0.0;
    h53[k] = k > 0 ? std::pow(double(k), -5.0 / 3.0) : 0.0;
  }
  if (hipMalloc(&c->kcbrt, sizeof(double) * dc.F) != hipSuccess ||
      hipMalloc(&c->lnk3, sizeof(double) * dc.F) != hipSuccess ||
      hipMalloc(&c->k53, sizeof(double) * dc.F) != hipSuccess) {
    gw_destroy(c);
    return GW_ENOMEM;
  }
  if (hipMemcpy(c->kcbrt, hc.data(), sizeof(double) * dc.F, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->lnk3, hl.data(), sizeof(double) * dc.F, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->k53, h53.data(), sizeof(double) * dc.F, hipMemcpyHostToDevice) != hipSuccess) {
    gw_destroy(c);
    return GW_EHIP;
  }
  const int NC = dc.N / 2;
  if (dc.precision == 2) {
    s = upload_twiddles<double>(c, &c->tw_win, NC, NC);
    if (s == GW_OK) s = upload_twiddles<double>(c, &c->twr_win, NC / 2 + 1, dc.N);
    if (s == GW_OK) s = upload_twiddles<double>(c, &c->tw_welch, dc.L, dc.L);
  } else {
    // windows longer than 32768 samples transform rows of N1 (four-step)
    const int NCt = NC > 16384 ? long_row_length(NC) : NC;
    s = upload_twiddles<float>(c, &c->tw_win, NCt, NCt);
    if (s == GW_OK) s = upload_twiddles<float>(c, &c->twr_win, NC / 2 + 1, dc.N);
    if (s == GW_OK) s = upload_twiddles<float>(c, &c->tw_welch, dc.L, dc.L);
    if (s == GW_OK && NC > 16384) s = upload_long_tables(c, NC);
  }
  if (s != GW_OK) {
    gw_destroy(c);
    return s;
  }
  *out = c;
  return GW_OK;
}

gw_status gw_query(const gw_ctx* c, int32_t key, int64_t* value) {
  if (!c || !value) return GW_EINVAL;
  const DevCfg& d = c->dc;
  switch (key) {
    case GW_Q_N: *value = d.N; break;
    case GW_Q_F: *value = d.F; break;
    case GW_Q_P: *value = d.P; break;
    case GW_Q_L: *value = d.L; break;
    case GW_Q_K: *value = d.K; break;
    case GW_Q_FW: *value = d.Fw; break;
    case GW_Q_NDET: *value = d.n_det; break;
    case GW_Q_NPARAMS: *value = GW_N_PARAMS; break;
    default: return GW_EINVAL;
  }
  return GW_OK;
}

gw_status gw_workspace_size(const gw_ctx* c, int64_t B, int64_t* bytes) {
  if (!c || !bytes || B < 0) return GW_EINVAL;
  *bytes = ws_counter_offset(c->dc, B) + 256;
  return GW_OK;
}

#define GW_CHECK_CTX(c) \
  if (!(c)) return GW_EINVAL;

gw_status sample_params(gw_ctx* c, uint64_t seed, uint64_t first_index, int64_t B, int64_t L_bg,
                        double* params, int64_t* offset, hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (B < 0) return fail(c, GW_EINVAL, "B < 0");
  if (B == 0) return GW_OK;
  if (!params || !offset) return fail(c, GW_EINVAL, "params/offset is NULL");
  if (!aligned16(params) || !aligned16(offset)) return fail(c, GW_EINVAL, "params/offset not 16-byte aligned");
  const int64_t span = L_bg - c->dc.P - c->dc.N + 1;
  if (span <= 0) return fail(c, GW_EINVAL, "L_bg < P + N");
  SampleArgs a{c->dc, seed, first_index, nullptr, B, span, params, offset, nullptr, nullptr, nullptr, nullptr};
  hipLaunchKernelGGL(k_sample_params, dim3(unsigned((B + 255) / 256)), dim3(256), 0, stream, a);
  return check_launch(c, "k_sample_params");
}

gw_status gen_fd_waveform(gw_ctx* c, const double* params, int64_t B, float* hp, float* hc, hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (B < 0 || B > 0x7fffffff) return fail(c, GW_EINVAL, "bad B");
  if (B == 0) return GW_OK;
  if (!params || !hp || !hc) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned16(params) || !aligned16(hp) || !aligned16(hc)) return fail(c, GW_EINVAL, "pointer not 16-byte aligned");
  WaveArgs a{c->dc, params, B, c->kcbrt, c->lnk3, hp, hc};
  const dim3 grid = dim3(unsigned(B));
  if (c->dc.precision == 0) hipLaunchKernelGGL((k_gen_fd_waveform<float, false>), grid, dim3(256), 0, stream, a);
  else if (c->dc.precision == 1) hipLaunchKernelGGL((k_gen_fd_waveform<double, false>), grid, dim3(256), 0, stream, a);
  else hipLaunchKernelGGL((k_gen_fd_waveform<double, true>), grid, dim3(256), 0, stream, a);
  return check_launch(c, "k_gen_fd_waveform");
}

gw_status project_detectors(gw_ctx* c, const double* params, const float* hp, const float* hc, int64_t B,
                            float* hdet, hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (B < 0 || B > 65535) return fail(c, GW_EINVAL, "B must be in [0, 65535]");
  if (B == 0) return GW_OK;
  if (!params || !hp || !hc || !hdet) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned16(params) || !aligned16(hp) || !aligned16(hc) || !aligned16(hdet))
    return fail(c, GW_EINVAL, "pointer not 16-byte aligned");
  ProjArgs a{c->dc, params, B, hp, hc, hdet};
  dim3 grid(unsigned((c->dc.F + 255) / 256), unsigned(B));
  if (c->dc.precision == 0) hipLaunchKernelGGL((k_project<float>), grid, dim3(256), 0, stream, a);
  else hipLaunchKernelGGL((k_project<double>), grid, dim3(256), 0, stream, a);
  return check_launch(c, "k_project");
}

gw_status inject(gw_ctx* c, const float* bg, int64_t L_bg, const int64_t* offset, const float* hdet, int64_t B,
                 float* strain, hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (B < 0 || B * c->dc.n_det >= kMaxBlocks) return fail(c, GW_EINVAL, "bad B");
  if (B == 0) return GW_OK;
  if (!bg || !offset || !hdet || !strain) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned4(bg) || !aligned16(offset) || !aligned16(hdet) || !aligned16(strain))
    return fail(c, GW_EINVAL, "misaligned pointer");
  if (L_bg < int64_t(c->dc.P) + c->dc.N) return fail(c, GW_EINVAL, "L_bg < P + N");
  WinArgs a = win_args(c);
  a.src = hdet;
  a.bg = bg;
  a.L_bg = L_bg;
  a.offset = offset;
  a.out = strain;
  if (c->dc.N > 32768) return long_window(c, 2, a, bg, hdet, B * c->dc.n_det, stream);
  launch_window_prec<2>(c->dc, B * c->dc.n_det, a, stream);
  return check_launch(c, "k_window<inject>");
}

gw_status welch_psd(gw_ctx* c, const float* bg, int64_t L_bg, const int64_t* offset, int64_t B, float* psd,
                    hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (B < 0 || B * c->dc.n_det >= kMaxBlocks) return fail(c, GW_EINVAL, "bad B");
  if (B == 0) return GW_OK;
  if (!bg || !offset || !psd) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned4(bg) || !aligned16(offset) || !aligned16(psd)) return fail(c, GW_EINVAL, "misaligned pointer");
  if (L_bg < int64_t(c->dc.P) + c->dc.N) return fail(c, GW_EINVAL, "L_bg < P + N");
  return welch_launch(c, bg, L_bg, offset, B, psd, stream);
}

gw_status whiten(gw_ctx* c, const float* strain, const float* psd, int64_t B, float* out, uint32_t* status,
                 hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (B < 0 || B * c->dc.n_det >= kMaxBlocks) return fail(c, GW_EINVAL, "bad B");
  if (B == 0) return GW_OK;
  if (!strain || !psd || !out) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned16(strain) || !aligned16(psd) || !aligned16(out) || (status && !aligned4(status)))
    return fail(c, GW_EINVAL, "misaligned pointer");
  if (status) {
    hipLaunchKernelGGL(k_fill_u32, dim3(unsigned((B + 255) / 256)), dim3(256), 0, stream, status, B, 0u);
    gw_status s = check_launch(c, "k_fill_u32");
    if (s != GW_OK) return s;
  }
  WinArgs a = win_args(c);
  a.src = strain;
  a.psd = psd;
  a.out = out;
  a.status = status;
  if (c->dc.N > 32768) return long_window(c, 0, a, strain, nullptr, B * c->dc.n_det, stream);
  launch_window_prec<0>(c->dc, B * c->dc.n_det, a, stream);
  return check_launch(c, "k_window<whiten>");
}

static int64_t ws_nodes_bytes(int64_t B) { return ((B * 2 * 1024 * 4 + 255) / 256) * 256; }
static int64_t ws_logmm_bytes(int64_t B) { return ((B * 4 + 255) / 256) * 256; }

gw_status gw_workspace_size_surrogate(const gw_ctx* c, int64_t B, int64_t* bytes) {
  gw_status s = gw_workspace_size(c, B, bytes);
  if (s != GW_OK) return s;
  *bytes += ws_nodes_bytes(B) + ws_logmm_bytes(B);
  return GW_OK;
}

gw_status gw_generate_batch_surrogate(gw_ctx* c, gw_surrogate* sg, uint64_t seed, uint64_t batch_index, int64_t B,
                                      const float* bg, int64_t L_bg, float* out, float* params_f32, uint32_t* status,
                                      float log10_mm_max, void* workspace, int64_t workspace_bytes, hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (!sg) return fail(c, GW_EINVAL, "surrogate is NULL");
  if (c->dc.approximant != 1) return fail(c, GW_EUNSUPPORTED, "the surrogate models approximant 1");
  if (c->dc.N > 32768) return fail(c, GW_EUNSUPPORTED, "the surrogate batch needs N <= 32768");
  if (B < 0 || B * c->dc.n_det >= kMaxBlocks) return fail(c, GW_EINVAL, "bad B");
  if (B == 0) return GW_OK;
  if (!bg || !out || !workspace) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned4(bg) || !aligned16(out) || !aligned16(workspace) || (params_f32 && !aligned16(params_f32)) ||
      (status && !aligned4(status)))
    return fail(c, GW_EINVAL, "misaligned pointer");
  int64_t need = 0;
  gw_workspace_size_surrogate(c, B, &need);
  if (workspace_bytes < need) return fail(c, GW_EINVAL, "workspace too small");
  const int64_t span = L_bg - c->dc.P - c->dc.N + 1;
  if (span <= 0) return fail(c, GW_EINVAL, "L_bg < P + N");
  if (batch_index > (UINT64_MAX - uint64_t(B)) / uint64_t(B)) return fail(c, GW_EINVAL, "batch_index overflows");
  char* ws = static_cast<char*>(workspace);
  double* params = reinterpret_cast<double*>(ws);
  int64_t* offset = reinterpret_cast<int64_t*>(ws + ws_params_bytes(B));
  float* psd = reinterpret_cast<float*>(ws + ws_params_bytes(B) + ws_offset_bytes(B));
  WfScalars* wf = reinterpret_cast<WfScalars*>(ws + ws_params_bytes(B) + ws_offset_bytes(B) + ws_psd_bytes(c->dc, B));
  DetScalars* dsc = reinterpret_cast<DetScalars*>(reinterpret_cast<char*>(wf) + ws_wf_bytes(B));
  float* nodes = reinterpret_cast<float*>(ws + ws_counter_offset(c->dc, B) + 256);
  float* logmm = reinterpret_cast<float*>(reinterpret_cast<char*>(nodes) + ws_nodes_bytes(B));
  SampleArgs sa{c->dc, seed, batch_index * uint64_t(B), nullptr, B, span, params, offset, params_f32, status, wf, dsc};
  hipLaunchKernelGGL(k_sample_params, dim3(unsigned((B + 255) / 256)), dim3(256), 0, stream, sa);
  gw_status s = check_launch(c, "k_sample_params");
  if (s != GW_OK) return s;
  s = gw_surrogate_nodes(sg, params, B, nodes, logmm, stream);
  if (s != GW_OK) return fail(c, s, std::string("surrogate: ") + gw_surrogate_last_error(sg));
  s = welch_launch(c, bg, L_bg, offset, B, psd, stream);
  if (s != GW_OK) return s;
  WinArgs a = win_args(c);
  a.src = bg;
  a.L_bg = L_bg;
  a.offset = offset;
  a.params = params;
  a.B = B;
  a.psd = psd;
  a.out = out;
  a.status = status;
  a.wf = wf;
  a.dsc = dsc;
  a.nodes = nodes;
  a.logmm = logmm;
  a.logmm_max = log10_mm_max;
  launch_window_prec<3>(c->dc, B * c->dc.n_det, a, stream);
  return check_launch(c, "k_window<surrogate>");
}

gw_status gw_generate_batch(gw_ctx* c, uint64_t seed, uint64_t batch_index, int64_t B, const float* bg,
                            int64_t L_bg, float* out, float* params_f32, uint32_t* status, void* workspace,
                            int64_t workspace_bytes, hipStream_t stream) {
  GW_CHECK_CTX(c);
  gw_status s = check_batch_args(c, B, bg, L_bg, out, params_f32, status, workspace, workspace_bytes);
  if (s != GW_OK || B == 0) return s;
  if (batch_index > (UINT64_MAX - uint64_t(B)) / uint64_t(B)) return fail(c, GW_EINVAL, "batch_index overflows");
  return enqueue_batch(c, seed, batch_index, nullptr, B, bg, L_bg, out, params_f32, status, workspace, kStageAll,
                       stream);
}

gw_status gw_generate_batch_noalloc(gw_ctx* c, uint64_t seed, uint64_t batch_index, int64_t B, const float* bg,
                                    int64_t L_bg, float* out, float* params_f32, uint32_t* status,
                                    hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (B < 0) return fail(c, GW_EINVAL, "bad B");
  int64_t need = 0;
  gw_workspace_size(c, B, &need);
  if (need > GW_SCRATCH_BYTES)
    return fail(c, GW_EINVAL, "batch too large for the static scratch area (needs " + std::to_string(need) +
                                  " bytes, the area holds " + std::to_string(int64_t(GW_SCRATCH_BYTES)) + ")");
  if (!c->scratch) return fail(c, GW_EHIP, "scratch area not resolved");
  // nothing in the area must start at zero: the prior kernel writes the
  // parameters, offsets, status and per-sample constants, Welch every PSD bin
  return gw_generate_batch(c, seed, batch_index, B, bg, L_bg, out, params_f32, status, c->scratch,
                           GW_SCRATCH_BYTES, stream);
}

gw_status gw_graph_create(gw_ctx* c, uint64_t seed, uint64_t first_batch, int64_t B, const float* bg, int64_t L_bg,
                          float* out, float* params_f32, uint32_t* status, void* workspace, int64_t workspace_bytes,
                          gw_graph** graph) {
  GW_CHECK_CTX(c);
  if (!graph) return fail(c, GW_EINVAL, "graph is NULL");
  *graph = nullptr;
  gw_status s = check_batch_args(c, B, bg, L_bg, out, params_f32, status, workspace, workspace_bytes);
  if (s != GW_OK) return s;
  if (B == 0) return fail(c, GW_EINVAL, "B must be positive");
  uint64_t* batch = reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) + ws_counter_offset(c->dc, B));
  std::string why;
  s = capture_graph(
      [&](hipStream_t st) {
        return enqueue_batch(c, seed, 0, batch, B, bg, L_bg, out, params_f32, status, workspace, kStageAll, st);
      },
      batch, first_batch, graph, &why);
  if (s != GW_OK) return fail(c, s, why);
  return GW_OK;
}

gw_status gw_graph_launch(gw_graph* g, hipStream_t stream) {
  if (!g) return GW_EINVAL;
  const hipError_t e = hipGraphLaunch(g->exec, stream);
  if (e != hipSuccess) {
    g->err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
    return GW_EHIP;
  }
  return GW_OK;
}

gw_status gw_graph_set_batch(gw_graph* g, uint64_t batch_index, hipStream_t stream) {
  if (!g) return GW_EINVAL;
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, stream, g->batch, batch_index);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g->err = std::string("k_set_u64: ") + hipGetErrorString(e);
    return GW_EHIP;
  }
  return GW_OK;
}

const char* gw_graph_last_error(const gw_graph* g) { return g ? g->err.c_str() : "graph is NULL"; }

gw_status gw_graph_destroy(gw_graph* g) {
  if (!g) return GW_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return GW_OK;
}

gw_status gw_set_tuning(gw_ctx* c, int32_t key, int64_t value) {
  GW_CHECK_CTX(c);
  switch (key) {
    case GW_TUNE_ORD_WINDOW:
    case GW_TUNE_ORD_WELCH:
      if (value < 0 || value > 1) return fail(c, GW_EINVAL, "radix order must be 0 or 1");
      if (c->dc.precision == 2 && value != 0) return fail(c, GW_EUNSUPPORTED, "binary64 kernels have one radix order");
      (key == GW_TUNE_ORD_WINDOW ? c->dc.ord_win : c->dc.ord_welch) = int(value);
      return GW_OK;
    case GW_TUNE_OCC_WELCH:
      if (value < 2 || value > 3) return fail(c, GW_EINVAL, "Welch occupancy must be 2 or 3");
      c->dc.occ_welch = int(value);
      return GW_OK;
    default: return fail(c, GW_EINVAL, "unknown tuning key");
  }
}

gw_status gw_get_tuning(const gw_ctx* c, int32_t key, int64_t* value) {
  if (!c || !value) return GW_EINVAL;
  switch (key) {
    case GW_TUNE_ORD_WINDOW: *value = c->dc.ord_win; break;
    case GW_TUNE_ORD_WELCH: *value = c->dc.ord_welch; break;
    case GW_TUNE_OCC_WELCH: *value = c->dc.occ_welch; break;
    default: return GW_EINVAL;
  }
  return GW_OK;
}

gw_status gw_autotune(gw_ctx* c, int64_t B, const float* bg, int64_t L_bg, float* out, void* workspace,
                      int64_t workspace_bytes, int32_t reps, double* report) {
  GW_CHECK_CTX(c);
  gw_status s = check_batch_args(c, B, bg, L_bg, out, nullptr, nullptr, workspace, workspace_bytes);
  if (s != GW_OK) return s;
  if (B == 0 || reps < 1 || reps > 1000) return fail(c, GW_EINVAL, "need B > 0 and 1 <= reps <= 1000");
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return fail(c, GW_EHIP, "hipStreamCreate");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // Welch variants: (order, occupancy) = (0,2), (1,2), (0,3), (1,3); window: order 0, 1
  // best of kTuneRounds interleaved rounds, so that clock ramps and other
  // drifts do not favour the variants timed last
  double ms[6];
  std::fill(ms, ms + 6, 1e300);
  const bool b64 = c->dc.precision == 2;
  const int saved[3] = {c->dc.ord_welch, c->dc.occ_welch, c->dc.ord_win};
  auto time_stage = [&](int mask, double* res) {
    s = enqueue_batch(c, 1, 0, nullptr, B, bg, L_bg, out, nullptr, nullptr, workspace, mask, st);  // warm-up
    if (s == GW_OK && hipEventRecord(e0, st) != hipSuccess) s = fail(c, GW_EHIP, "hipEventRecord");
    for (int r = 0; r < reps && s == GW_OK; ++r)
      s = enqueue_batch(c, 1, 0, nullptr, B, bg, L_bg, out, nullptr, nullptr, workspace, mask, st);
    if (s == GW_OK && hipEventRecord(e1, st) != hipSuccess) s = fail(c, GW_EHIP, "hipEventRecord");
    if (s == GW_OK && hipEventSynchronize(e1) != hipSuccess) s = fail(c, GW_EHIP, "hipEventSynchronize");
    // a failed timing query fails the tuner rather than reading as 0 ms
    float t = 0.f;
    if (s == GW_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) s = fail(c, GW_EHIP, "hipEventElapsedTime");
    if (s == GW_OK) *res = std::min(*res, double(t) / reps);
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    s = fail(c, GW_EHIP, "hipEventCreate");
  } else {
    s = enqueue_batch(c, 1, 0, nullptr, B, bg, L_bg, out, nullptr, nullptr, workspace, kStageAll, st);
    for (int round = 0; round < kTuneRounds && s == GW_OK; ++round) {
      for (int v = 0; v < 4 && s == GW_OK; ++v) {
        if (b64 && v > 0) { ms[v] = ms[0]; continue; }
        c->dc.ord_welch = v & 1;
        c->dc.occ_welch = 2 + (v >> 1);
        time_stage(kStageWelch, &ms[v]);
      }
      for (int o = 0; o < 2 && s == GW_OK; ++o) {
        if (b64 && o > 0) { ms[4 + o] = ms[4]; continue; }
        c->dc.ord_win = o;
        time_stage(kStageWindow, &ms[4 + o]);
      }
    }
  }
  if (s == GW_OK) {
    int best = 0;
    for (int v = 1; v < 4; ++v)
      if (ms[v] < ms[best]) best = v;
    c->dc.ord_welch = b64 ? 0 : (best & 1);
    c->dc.occ_welch = b64 ? 2 : 2 + (best >> 1);
    c->dc.ord_win = (!b64 && ms[5] < ms[4]) ? 1 : 0;
    if (report) std::copy(ms, ms + 6, report);
  } else {
    c->dc.ord_welch = saved[0];
    c->dc.occ_welch = saved[1];
    c->dc.ord_win = saved[2];
  }
  if (hipStreamSynchronize(st) != hipSuccess && s == GW_OK) s = fail(c, GW_EHIP, "hipStreamSynchronize");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  return s;
}

// ------------------------------------------------------- per-run PSD mode
static int64_t align256(int64_t v) { return ((v + 255) / 256) * 256; }

gw_status gw_run_psd_workspace_size(const gw_ctx* c, int64_t n_chunks, int64_t* bytes) {
  if (!c || !bytes || n_chunks < 1) return GW_EINVAL;
  *bytes = align256(n_chunks * 8) + align256(n_chunks * c->dc.n_det * int64_t(c->dc.Fw) * 4);
  return GW_OK;
}

gw_status gw_run_psd(gw_ctx* c, const float* bg, int64_t L_bg, int64_t n_chunks, float* psd, void* workspace,
                     int64_t workspace_bytes, hipStream_t stream) {
  GW_CHECK_CTX(c);
  const DevCfg& d = c->dc;
  if (n_chunks < 1 || n_chunks * d.n_det >= kMaxBlocks) return fail(c, GW_EINVAL, "bad n_chunks");
  if (!bg || !psd || !workspace) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned4(bg) || !aligned16(psd) || !aligned16(workspace)) return fail(c, GW_EINVAL, "misaligned pointer");
  const int64_t stride = int64_t(d.K) * d.S;
  if ((n_chunks - 1) * stride + d.P > L_bg) return fail(c, GW_EINVAL, "n_chunks stretches exceed the background");
  int64_t need = 0;
  gw_run_psd_workspace_size(c, n_chunks, &need);
  if (workspace_bytes < need) return fail(c, GW_EINVAL, "workspace too small");
  int64_t* off = static_cast<int64_t*>(workspace);
  float* part = reinterpret_cast<float*>(static_cast<char*>(workspace) + align256(n_chunks * 8));
  hipLaunchKernelGGL(k_chunk_offsets, dim3(unsigned((n_chunks + 255) / 256)), dim3(256), 0, stream, off, n_chunks,
                     stride);
  gw_status s = check_launch(c, "k_chunk_offsets");
  if (s != GW_OK) return s;
  s = welch_launch(c, bg, L_bg, off, n_chunks, part, stream);
  if (s != GW_OK) return s;
  const int n = d.n_det * d.Fw;
  hipLaunchKernelGGL(k_mean_chunks, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, part, n_chunks, d.n_det,
                     d.Fw, psd);
  return check_launch(c, "k_mean_chunks");
}

gw_status gw_whiten_filter(gw_ctx* c, const float* psd, int64_t M, float* filt, uint32_t* status,
                           hipStream_t stream) {
  GW_CHECK_CTX(c);
  const DevCfg& d = c->dc;
  if (!psd || !filt) return fail(c, GW_EINVAL, "NULL pointer");
  if (!aligned4(psd) || !aligned4(filt)) return fail(c, GW_EINVAL, "misaligned pointer");
  if (M < 2 || M >= d.N || (M & 1)) return fail(c, GW_EINVAL, "M must be even with 2 <= M < N");
  if (d.N > 32768) return fail(c, GW_EUNSUPPORTED, "the per-run filter needs N <= 32768");
  if (status && !aligned4(status)) return fail(c, GW_EINVAL, "misaligned pointer");
  FiltArgs a{d, psd, filt, int(M), c->tw_win, c->twr_win, status};
  if (d.precision == 2) launch_filter<double>(d, a, stream);
  else launch_filter<float>(d, a, stream);
  return check_launch(c, "k_filter");
}

gw_status gw_generate_batch_runpsd(gw_ctx* c, uint64_t seed, uint64_t batch_index, int64_t B, const float* bg,
                                   int64_t L_bg, const float* filt, int64_t crop, float* out, float* params_f32,
                                   uint32_t* status, void* workspace, int64_t workspace_bytes, hipStream_t stream) {
  GW_CHECK_CTX(c);
  gw_status s = check_batch_args(c, B, bg, L_bg, out, params_f32, status, workspace, workspace_bytes);
  if (s != GW_OK || B == 0) return s;
  if (!filt || !aligned4(filt)) return fail(c, GW_EINVAL, "filter NULL or misaligned");
  if (c->dc.N > 32768) return fail(c, GW_EUNSUPPORTED, "the per-run mode needs N <= 32768");
  if (crop < 0 || (crop & 1) || 2 * crop >= c->dc.N) return fail(c, GW_EINVAL, "crop must be even with 2 crop < N");
  if (batch_index > (UINT64_MAX - uint64_t(B)) / uint64_t(B)) return fail(c, GW_EINVAL, "batch_index overflows");
  s = enqueue_batch(c, seed, batch_index, nullptr, B, bg, L_bg, out, params_f32, status, workspace, kStageParams,
                    stream);
  if (s != GW_OK) return s;
  char* ws = static_cast<char*>(workspace);
  WinArgs a = win_args(c);
  a.src = bg;
  a.L_bg = L_bg;
  a.offset = reinterpret_cast<int64_t*>(ws + ws_params_bytes(B));
  a.params = reinterpret_cast<double*>(ws);
  a.B = B;
  a.psd = filt;
  a.out = out;
  a.status = status;
  char* wfp = ws + ws_params_bytes(B) + ws_offset_bytes(B) + ws_psd_bytes(c->dc, B);
  a.wf = reinterpret_cast<const WfScalars*>(wfp);
  a.dsc = reinterpret_cast<const DetScalars*>(wfp + ws_wf_bytes(B));
  a.crop = int(crop);
  launch_window_prec<4>(c->dc, B * c->dc.n_det, a, stream);
  return check_launch(c, "k_window<per-run filter>");
}

// ------------------------------------------- view pairs and oversampling
gw_status gw_generate_batch_pairs(gw_ctx* c, uint64_t seed, uint64_t batch_index, int64_t B, const float* bg,
                                  int64_t L_bg, float* out_ref, float* out_shift, float* params_f32, uint32_t* status,
                                  void* workspace, int64_t workspace_bytes, hipStream_t stream) {
  GW_CHECK_CTX(c);
  gw_status s = check_batch_args(c, B, bg, L_bg, out_shift, params_f32, status, workspace, workspace_bytes);
  if (s != GW_OK || B == 0) return s;
  if (!out_ref || !aligned16(out_ref)) return fail(c, GW_EINVAL, "out_ref NULL or misaligned");
  if (batch_index > (UINT64_MAX - uint64_t(B)) / uint64_t(B)) return fail(c, GW_EINVAL, "batch_index overflows");
  return enqueue_batch(c, seed, batch_index, nullptr, B, bg, L_bg, out_shift, params_f32, status, workspace, kStageAll,
                       stream, 1u, out_ref);
}

gw_status gw_generate_batch_oversampled(gw_ctx* c, uint64_t seed, uint64_t batch_index, int64_t B, int32_t ext_k,
                                        const float* bg, int64_t L_bg, float* out, float* params_f32,
                                        uint32_t* status, void* workspace, int64_t workspace_bytes,
                                        hipStream_t stream) {
  GW_CHECK_CTX(c);
  if (ext_k < 1 || ext_k > 65536) return fail(c, GW_EINVAL, "ext_k must be in 1..65536");
  gw_status s = check_batch_args(c, B, bg, L_bg, out, params_f32, status, workspace, workspace_bytes);
  if (s != GW_OK || B == 0) return s;
  if (batch_index > (UINT64_MAX - uint64_t(B)) / uint64_t(B)) return fail(c, GW_EINVAL, "batch_index overflows");
  return enqueue_batch(c, seed, batch_index, nullptr, B, bg, L_bg, out, params_f32, status, workspace, kStageAll,
                       stream, uint32_t(ext_k));
}

}  // extern "C"
