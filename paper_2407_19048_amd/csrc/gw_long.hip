// Long windows (N > 32768 samples, e.g. long-duration binary-neutron-star
// signals): the half-length complex transform of NC = N/2 points no longer
// fits in one workgroup's LDS and runs as a four-step FFT through HBM, with
// NC = N1 x N2, N1 the row length (one workgroup transform in LDS) and
// N2 = NC/N1 in {4, 8, 16, 32} (in registers).  N1 = 8192 up to N = 2^19
// (two workgroups of 512 threads share a CU), 16384 for N = 2^20 (N2 = 32).
// With c[m] = y[2m] + i y[2m+1]:
//
//   forward  columns  w[k2][m1] = W_NC^(m1 k2) sum_m2 c[m1 + N1 m2] W_N2^(m2 k2)
//            rows     X[k2 + N2 k1] = sum_m1 w[k2][m1] W_N1^(m1 k1)   (in place)
//   bins     real-spectrum unpack of the pair (k, NC - k), in-register
//            signal, whitening, repack for the inverse (in place, on the
//            transposed layout X'[k2][k1] = X[k2 + N2 k1])
//   inverse  rows     u[k2][m1] = sum_k1 Z[k2 + N2 k1] W_N1^(-m1 k1)  (in place)
//            columns  c[m1 + N1 m2] = (1/NC) sum_k2 W_N2^(-m2 k2) W_NC^(-m1 k2) u[k2][m1]
//
// The thread of column m1 reads u[k2][m1] for every k2 and writes
// c[m1 + N1 m2] for every m2: the same complex positions, so the inverse
// also runs in place.  Every pass works inside the caller's output buffer
// (N floats = NC complex per window); no other memory is needed.
#include <hip/hip_runtime.h>

#include <string>

#include "gw_fft.hpp"
#include "gw_physics.hpp"
#include "gw_internal.hpp"
#include "gw_items.hpp"
#include "../../include/gwgen.h"

using namespace gw;

namespace {

// Waves per SIMD the row kernels are compiled for: two 512-thread workgroups
// (N1 = 8192) or one 1024-thread workgroup (N1 = 16384) per CU, 128 VGPRs.
constexpr int kRowWaves = 4;

// In-register DFT of length R (natural order in and out), DIR = -1 forward.
template <int R, int DIR, class T>
__device__ __forceinline__ void dft_small(cpx<T>* a) {
  if constexpr (R == 2) dft2<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a);
  else if constexpr (R == 8) dft8<DIR>(a);
  else if constexpr (R == 16) dft16<DIR>(a);
  else {
    static_assert(R == 32, "N2 in {4, 8, 16, 32}");
    cpx<T> e[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      e[i] = a[2 * i];
      o[i] = a[2 * i + 1];
    }
    dft16<DIR>(e);
    dft16<DIR>(o);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      T s, c;
      sincospi_t(T(2 * k) / T(32), &s, &c);  // exp(DIR 2 pi i k / 32)
      const cpx<T> w = {c, T(DIR) * s};
      const cpx<T> t = cmul(o[k], w);
      a[k] = cadd(e[k], t);
      a[k + 16] = csub(e[k], t);
    }
  }
}

struct LongArgs {
  WinArgs w;           // cf, tables, per-sample data, psd, status; out = the in-place buffer
  const void* twc;     // cpx<float>[N2][N1]: exp(-2 pi i m1 k2 / NC) at [k2][m1]
  const void* twr;     // cpx<float>[NC/2 + 1]: exp(-2 pi i k / N)
  const void* tw1;     // cpx<float>[N1]: exp(-2 pi i n / N1)
  const float* x;      // real input of the forward columns (strain rows or the background)
  int NC, N2, l2n2;    // NC = N1 N2, l2n2 = log2(N2)
  // bin tables in the transposed layout (bin k at (k mod N2) N1 + k / N2):
  const double* kc_t;        // k^(1/3)
  const double* lk_t;        // ln(k)/3
  const cpx<float>* twr_t;   // exp(-2 pi i k / N)
};

// x row of window item bd (SRC 0: strain [B][D][N]; SRC 1, 2: background at o + P)
template <int SRC>
__device__ __forceinline__ const float* long_input(const LongArgs& a, int64_t bd) {
  const DevCfg& cf = a.w.cf;
  const int64_t b = bd / cf.n_det;
  const int d = int(bd - b * cf.n_det);
  if constexpr (SRC == 0) return a.x + bd * int64_t(cf.N);
  else return a.x + int64_t(d) * a.w.L_bg + load_const(a.w.offset + b) + cf.P;
}

// Forward columns: one thread per column m1, grid (N1/256, B*D).
template <int N1, int N2, int SRC>
__global__ __launch_bounds__(256) void k_long_cols_fwd(LongArgs a) {
  const int m1 = blockIdx.x * 256 + threadIdx.x;
  const int64_t bd = blockIdx.y;
  const float* x = long_input<SRC>(a, bd);
  float2* buf = reinterpret_cast<float2*>(a.w.out) + bd * a.NC;
  const cpx<float>* twc = reinterpret_cast<const cpx<float>*>(a.twc);
  cpx<float> v[N2];
#pragma unroll
  for (int m2 = 0; m2 < N2; ++m2) {
    float2 q;
    __builtin_memcpy(&q, x + 2 * (int64_t(m1) + int64_t(N1) * m2), sizeof(q));
    v[m2] = {q.x, q.y};
  }
  dft_small<N2, -1>(v);
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    const cpx<float> w = k2 ? cmul(v[k2], twc[k2 * N1 + m1]) : v[k2];
    buf[int64_t(k2) * N1 + m1] = {w.x, w.y};
  }
}

// Inverse columns: twiddle, inverse DFT over k2, scale 1/NC, store real
// samples in place; SRC 2 adds the noise window.
template <int N1, int N2, int SRC>
__global__ __launch_bounds__(256) void k_long_cols_inv(LongArgs a) {
  const int m1 = blockIdx.x * 256 + threadIdx.x;
  const int64_t bd = blockIdx.y;
  float2* buf = reinterpret_cast<float2*>(a.w.out) + bd * a.NC;
  const cpx<float>* twc = reinterpret_cast<const cpx<float>*>(a.twc);
  cpx<float> v[N2];
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    const float2 q = buf[int64_t(k2) * N1 + m1];
    const cpx<float> u = {q.x, q.y};
    v[k2] = k2 ? twmul<+1>(u, twc[k2 * N1 + m1]) : u;
  }
  dft_small<N2, +1>(v);
  const float sc = 1.f / float(a.NC);
  const float* nz = nullptr;
  if constexpr (SRC == 2) nz = long_input<2>(a, bd);
#pragma unroll
  for (int m2 = 0; m2 < N2; ++m2) {
    const int64_t m = int64_t(m1) + int64_t(N1) * m2;
    float2 y = {v[m2].x * sc, v[m2].y * sc};
    if constexpr (SRC == 2) {
      y.x += nz[2 * m];
      y.y += nz[2 * m + 1];
    }
    buf[m] = y;
  }
}

// Row transforms of length N1 in place: grid B*D*N2 workgroups of N1/16.
template <int N1, int DIR>
__global__ __launch_bounds__(N1 / 16, kRowWaves) void k_long_rows(LongArgs a) {
  constexpr int NT = N1 / 16, LS = LdsSize<N1>::value;
  __shared__ float lds[2 * LS];
  const int t = threadIdx.x;
  float2* row = reinterpret_cast<float2*>(a.w.out) + int64_t(blockIdx.x) * N1;
  PowTwiddle<float, N1, 0> tw{reinterpret_cast<const cpx<float>*>(a.tw1)};
  cpx<float> v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const float2 q = row[t + NT * j];
    v[fft_in_slot<N1, 0>(j)] = {q.x, q.y};
  }
  block_fft<float, N1, DIR, false, 0>(v, lds, lds + LS, t, tw);
#pragma unroll
  for (int e = 0; e < 16; ++e) row[fft_out_index<N1, 0>(t, e)] = {v[e].x, v[e].y};
}

// Inject: pack the given projected spectrum for the inverse transform, one
// thread per pair (k, NC - k), k in [0, NC/2], reading hdet by k:
// grid (ceil((NC/2 + 1)/256), B*D).  The packed pair lands at its place in
// the transposed layout X'[k2][k1] = X[k2 + N2 k1] of the inverse rows.
template <int N1>
__global__ __launch_bounds__(256) void k_long_inject(LongArgs a, const float* hdet) {
  const int64_t bd = blockIdx.y;
  const int NC = a.NC, N2 = a.N2;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k > NC / 2) return;
  float2* buf = reinterpret_cast<float2*>(a.w.out) + bd * NC;
  const int km = NC - k;
  auto pos = [&](int kk) { kk &= NC - 1; return int64_t(kk & (N2 - 1)) * N1 + (kk >> a.l2n2); };
  const cpx<float> W = reinterpret_cast<const cpx<float>*>(a.twr)[k];  // exp(-2 pi i k / N)
  const float2* h = reinterpret_cast<const float2*>(hdet) + bd * (NC + 1);
  const float2 h0 = h[k], h1 = h[km];
  // irfft ignores Im at DC and Nyquist
  const cpx<float> Yk = {h0.x, k == 0 ? 0.f : h0.y};
  const cpx<float> Ym = {h1.x, k == 0 ? 0.f : h1.y};
  const cpx<float> p = cscale(cadd(Yk, cconj(Ym)), 0.5f);
  const cpx<float> q = twmul<+1>(cscale(csub(Yk, cconj(Ym)), 0.5f), W);
  buf[pos(k)] = {p.x - q.y, p.y + q.x};
  if (k != 0 && km != k) buf[pos(km)] = {p.x + q.y, -p.y + q.x};
}

// Bins: the real-spectrum unpack of each pair (k, NC - k), k in [0, NC/2],
// then (SRC 1) the in-register signal, the whitening gain and the repack for
// the inverse; SRC 0 whitens only.  Thread (k1, r) takes the element at row
// r, column k1 of X'[k2][k1] = X[k2 + N2 k1], i.e. k = r + N2 k1, or its
// mirror NC - k (row N2 - r, column N1 - 1 - k1) when k > NC/2, so that a
// wavefront reads and writes runs of consecutive (or reversed) columns of two
// rows, and reads the bin tables in the same transposed layout.  Rows 0 and
// N2/2 pair with themselves and use half their columns.  Two pairs per
// thread, columns k1 and k1 + 256 (grid (N1/512, B*D, N2/2 + 1)): both pairs'
// inputs are loaded before either is computed, so the second pair's loads
// overlap the first pair's arithmetic.  Idle lanes load a real pair too (k is
// clamped into range) and only skip their stores.
template <int N1, class TP, int SRC>
__global__ __launch_bounds__(256) void k_long_bins(LongArgs a) {
  static_assert(SRC == 0 || SRC == 1, "whiten or fused");
  constexpr int J = 2;
  const int64_t bd = blockIdx.y;
  const DevCfg& cf = a.w.cf;
  const int NC = a.NC, N2 = a.N2;
  const int r = blockIdx.z;
  const int64_t b = bd / cf.n_det;
  const int d = int(bd - b * cf.n_det);
  float2* buf = reinterpret_cast<float2*>(a.w.out) + bd * NC;
  const float* psd = a.w.psd + bd * cf.Fw;
  auto pos = [&](int kk) { kk &= NC - 1; return int64_t(kk & (N2 - 1)) * N1 + (kk >> a.l2n2); };
  __shared__ uint32_t sflag;
  if (threadIdx.x == 0) sflag = 0u;
  __syncthreads();
  int k[J];
  bool ok[J];
  float2 qa[J], qb[J];
  cpx<float> W[J];
  float g[J][4];
  double kc[J][2], lk[J][2];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k1 = blockIdx.x * (256 * J) + 256 * j + threadIdx.x;  // < N1
    const int kr = r + N2 * k1;
    ok[j] = (r == 0) ? (k1 <= N1 / 2) : (2 * r == N2) ? (k1 < N1 / 2) : true;
    k[j] = min(kr, NC - kr);
    const int km = NC - k[j];
    const int64_t pk = pos(k[j]), pm = pos(km);
    qa[j] = buf[pk];
    qb[j] = buf[pm];
    W[j] = a.twr_t[pk];
    const int ia = psd_index(cf, k[j], NC), ib = psd_index(cf, km, NC);
    g[j][0] = psd[ia];
    g[j][1] = psd[ia + 1];
    g[j][2] = psd[ib];
    g[j][3] = psd[ib + 1];
    if constexpr (SRC == 1) {
      kc[j][0] = a.kc_t[pk];
      lk[j][0] = a.lk_t[pk];
      kc[j][1] = a.kc_t[pm];
      lk[j][1] = a.lk_t[pm];
    }
  }
  float cpl = 0.f, cxx = 0.f;
  double tauT = 0.0;
  WfScalars wsh;
  if constexpr (SRC == 1) {
    wsh = load_const(a.w.wf + b);
    const DetScalars dsh = load_const(a.w.dsc + (b * cf.n_det + d));
    cpl = float(dsh.fp * 0.5 * (1.0 + wsh.cosi * wsh.cosi));
    cxx = float(dsh.fx * wsh.cosi);
    tauT = dsh.tau * cf.invT;
  }
  uint32_t flag = 0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int kk = k[j], km = NC - kk;
    const cpx<float> A = {qa[j].x, qa[j].y}, Bm = {qb[j].x, qb[j].y};
    const cpx<float> s = cadd(A, cconj(Bm));
    const cpx<float> u = cmul(W[j], csub(A, cconj(Bm)));
    cpx<float> Xk = {0.5f * (s.x + u.y), 0.5f * (s.y - u.x)};
    cpx<float> Xm = {0.5f * (s.x - u.y), 0.5f * (-s.y - u.x)};
    if constexpr (SRC == 1) {
      Xk = cadd(Xk, signal_bin_at<float, TP, false>(cf, wsh, cpl, cxx, tauT, kk, kc[j][0], lk[j][0]));
      if (km != kk) Xm = cadd(Xm, signal_bin_at<float, TP, false>(cf, wsh, cpl, cxx, tauT, km, kc[j][1], lk[j][1]));
    }
    uint32_t fj = 0;
    const cpx<float> Yk = cscale(Xk, whiten_gain_at<float>(cf, g[j][0], g[j][1], kk, NC, fj));
    cpx<float> Ym = cscale(Xm, whiten_gain_at<float>(cf, g[j][2], g[j][3], km, NC, fj));
    if (km == kk) Ym = Yk;
    const cpx<float> p = cscale(cadd(Yk, cconj(Ym)), 0.5f);
    const cpx<float> q = twmul<+1>(cscale(csub(Yk, cconj(Ym)), 0.5f), W[j]);
    if (ok[j]) {
      buf[pos(kk)] = {p.x - q.y, p.y + q.x};
      if (kk != 0 && km != kk) buf[pos(km)] = {p.x + q.y, -p.y + q.x};
      flag |= fj;
    }
  }
  if (flag) atomicOr(&sflag, flag);
  __syncthreads();
  if (threadIdx.x == 0 && sflag && a.w.status) atomicOr(a.w.status + b, sflag);
}

// Global inputs of one pair of packed-spectrum bins (k, km = NC - k),
// k <= NC/2: the real-FFT twiddle exp(-2 pi i k / N), the bin tables of both
// bins (SRC 1) and the PSD values around both bins.  pk, pm: positions of k
// and km in the transposed bin tables.
struct LongPairIn {
  cpx<float> W;
  double kc[2], lk[2];
  float g[4];
};

template <int SRC>
__device__ __forceinline__ LongPairIn long_pair_fetch(const LongArgs& a, const float* psd, int k, int64_t pk,
                                                      int64_t pm) {
  const DevCfg& cf = a.w.cf;
  const int NC = a.NC, km = NC - k;
  LongPairIn in;
  in.W = a.twr_t[pk];
  if constexpr (SRC == 1) {
    in.kc[0] = a.kc_t[pk];
    in.lk[0] = a.lk_t[pk];
    in.kc[1] = a.kc_t[pm];
    in.lk[1] = a.lk_t[pm];
  }
  const int ia = psd_index(cf, k, NC), ib = psd_index(cf, km, NC);
  in.g[0] = psd[ia];
  in.g[1] = psd[ia + 1];
  in.g[2] = psd[ib];
  in.g[3] = psd[ib + 1];
  return in;
}

// One pair of packed-spectrum bins (k, km = NC - k), k <= NC/2: A = Z[k] and
// Bm = Z[km] in; out, the packed spectrum of the whitened window (SRC 1 with
// the in-register signal added) at the same two bins.
template <class TP, int SRC>
__device__ __forceinline__ void long_pair(const LongArgs& a, const WfScalars& wsh, float cpl, float cxx, double tauT,
                                          const LongPairIn& in, int k, cpx<float>& A, cpx<float>& Bm, uint32_t& flag) {
  const DevCfg& cf = a.w.cf;
  const int NC = a.NC, km = NC - k;
  const cpx<float> W = in.W;  // exp(-2 pi i k / N)
  const cpx<float> s = cadd(A, cconj(Bm));
  const cpx<float> u = cmul(W, csub(A, cconj(Bm)));
  cpx<float> Xk = {0.5f * (s.x + u.y), 0.5f * (s.y - u.x)};
  cpx<float> Xm = {0.5f * (s.x - u.y), 0.5f * (-s.y - u.x)};
  if constexpr (SRC == 1) {
    Xk = cadd(Xk, signal_bin_at<float, TP, false>(cf, wsh, cpl, cxx, tauT, k, in.kc[0], in.lk[0]));
    if (km != k) Xm = cadd(Xm, signal_bin_at<float, TP, false>(cf, wsh, cpl, cxx, tauT, km, in.kc[1], in.lk[1]));
  }
  const cpx<float> Yk = cscale(Xk, whiten_gain_at<float>(cf, in.g[0], in.g[1], k, NC, flag));
  cpx<float> Ym = cscale(Xm, whiten_gain_at<float>(cf, in.g[2], in.g[3], km, NC, flag));
  if (km == k) Ym = Yk;
  const cpx<float> p = cscale(cadd(Yk, cconj(Ym)), 0.5f);
  const cpx<float> q = twmul<+1>(cscale(csub(Yk, cconj(Ym)), 0.5f), W);
  A = {p.x - q.y, p.y + q.x};
  Bm = {p.x + q.y, -p.y + q.x};
}

// Rows, bins and inverse rows of one row pair in one workgroup (replacing
// three passes through HBM).  Bin k = r + N2 c sits at row r, column c of the
// transposed spectrum, and its partner NC - k at row N2 - r, column N1 - 1 - c
// (row 0 and row N2/2 pair with themselves: columns N1 - c and N1 - 1 - c).
// Grid: B*D*(N2/2 + 1) workgroups of N1/16 threads; workgroup (item, r) owns
// rows r and N2 - r.  Two-row pairs: the spectrum of row r goes back to its
// row of the buffer; thread t writes, and later reads back, exactly the
// columns t + NT j (the output layout of the transform covers them), so the
// round trip needs no barrier and holds no registers while row N2 - r is
// transformed and stored to LDS in natural order.  Each thread then pairs
// its row-r columns with their partners read from LDS, writes row r's
// results to the buffer and row N2 - r's to LDS in place (every LDS word is
// read and written by one thread only); then the inverse transforms of row
// N2 - r (from LDS) and of row r (from its own writes).  Rows are left
// unscaled, as the separate row passes leave them.
template <int N1, class TP, int SRC>
__global__ __launch_bounds__(N1 / 16, kRowWaves) void k_long_rowpair(LongArgs a) {
  static_assert(SRC == 0 || SRC == 1, "whiten or fused");
  constexpr int NT = N1 / 16, LS = LdsSize<N1>::value;
  __shared__ float lds[2 * LS];
  __shared__ uint32_t sflag;
  float* sre = lds;
  float* sim = lds + LS;
  const int t = threadIdx.x;
  const DevCfg& cf = a.w.cf;
  const int NC = a.NC, N2 = a.N2;
  const int npair = N2 / 2 + 1;
  const int64_t bd = blockIdx.x / npair;
  const int rA = int(blockIdx.x - bd * npair);
  const int rB = rA == 0 ? 0 : N2 - rA;
  const int64_t b = bd / cf.n_det;
  const int d = int(bd - b * cf.n_det);
  float2* buf = reinterpret_cast<float2*>(a.w.out) + bd * NC;
  float2* rowA = buf + int64_t(rA) * N1;
  float2* rowB = buf + int64_t(rB) * N1;
  const float* psd = a.w.psd + bd * cf.Fw;
  const cpx<float>* tw1 = reinterpret_cast<const cpx<float>*>(a.tw1);
  // a fresh table pointer per transform (see opaque)
  auto tw = [&]() { return PowTwiddle<float, N1, 0>{opaque(tw1)}; };
  if (t == 0) sflag = 0u;
  float cpl = 0.f, cxx = 0.f;
  double tauT = 0.0;
  WfScalars wsh;
  if constexpr (SRC == 1) {
    wsh = load_const(a.w.wf + b);
    const DetScalars dsh = load_const(a.w.dsc + (b * cf.n_det + d));
    cpl = float(dsh.fp * 0.5 * (1.0 + wsh.cosi * wsh.cosi));
    cxx = float(dsh.fx * wsh.cosi);
    tauT = dsh.tau * cf.invT;
  }
  uint32_t flag = 0;
  cpx<float> v[16];
  // Each phase below takes its own copy of the lane index and row pointers
  // (fresh_lane, fresh): without them the compiler shares the index and
  // address arithmetic of the five transforms and keeps it live throughout,
  // beyond the 128 registers a 1024-thread workgroup allows.
  auto load_row = [&](float2* row) {
    const int tl = fresh_lane(t);
    float2* r = fresh(row);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float2 q = r[tl + NT * j];
      v[fft_in_slot<N1, 0>(j)] = {q.x, q.y};
    }
  };
  auto store_row = [&](float2* row) {
    const int tl = fresh_lane(t);
    float2* r = fresh(row);
#pragma unroll
    for (int e = 0; e < 16; ++e) r[fft_out_index<N1, 0>(tl, e)] = {v[e].x, v[e].y};
  };
  auto store_lds = [&]() {
    const int tl = fresh_lane(t);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = lpad<float>(fft_out_index<N1, 0>(tl, e));
      sre[i] = v[e].x;
      sim[i] = v[e].y;
    }
  };
  // forward transform of row rA
  load_row(rowA);
  block_fft<float, N1, -1, false, 0>(v, sre, sim, fresh_lane(t), tw());
  if (rA == rB) {
    // self-paired row (uniform over the workgroup): spectrum to LDS, pairs
    // in LDS, inverse transform from LDS
    lds_barrier();
    store_lds();
    lds_barrier();
    const int tl = fresh_lane(t);
    // column of iteration j and its mirror; the pair's global inputs are
    // fetched one iteration ahead (clamped to the lower bin, so that every
    // iteration loads a valid pair) to overlap their latency
    auto cols = [&](int j, int& c, int& cm, int& k) {
      c = tl + NT * j;
      cm = rA == 0 ? ((N1 - c) & (N1 - 1)) : (N1 - 1 - c);
      k = rA + N2 * c;
      if (k > NC - k) {  // the partner's thread handles the pair; fetch it anyway
        const int x = c;
        c = cm;
        cm = x;
        k = NC - k;
      }
    };
    int c, cm, k;
    cols(0, c, cm, k);
    LongPairIn nxt = long_pair_fetch<SRC>(a, psd, k, int64_t(rA) * N1 + c, int64_t(rA) * N1 + cm);
#pragma unroll 1
    for (int j = 0; j < 16; ++j) {
      const LongPairIn cur = nxt;
      const int cj = c, cmj = cm, kj = k;
      const bool mine = rA + N2 * (tl + NT * j) <= NC - (rA + N2 * (tl + NT * j));
      if (j + 1 < 16) {
        cols(j + 1, c, cm, k);
        nxt = long_pair_fetch<SRC>(a, psd, k, int64_t(rA) * N1 + c, int64_t(rA) * N1 + cm);
      }
      if (!mine) continue;  // the partner's thread handles the pair
      const int km = NC - kj;
      const int ic = lpad<float>(cj), im = lpad<float>(cmj);
      cpx<float> A = {sre[ic], sim[ic]}, Bm = {sre[im], sim[im]};
      long_pair<TP, SRC>(a, wsh, cpl, cxx, tauT, cur, kj, A, Bm, flag);
      sre[ic] = A.x;
      sim[ic] = A.y;
      if (kj != 0 && km != kj) {
        sre[im] = Bm.x;
        sim[im] = Bm.y;
      }
    }
    lds_barrier();
    block_fft<float, N1, +1, true, 0>(v, sre, sim, fresh_lane(t), tw());
    store_row(rowA);
  } else {
    // row rA's spectrum back to its row (columns t + NT j of this thread);
    // row rB transformed and stored to LDS
    store_row(rowA);
    load_row(rowB);
    lds_barrier();
    block_fft<float, N1, -1, false, 0>(v, sre, sim, fresh_lane(t), tw());
    lds_barrier();
    store_lds();
    lds_barrier();
    {
      const int tl = fresh_lane(t);
      float2* ra = fresh(rowA);
      // the pair's global inputs (own row-r bin, tables, PSD values) are
      // fetched one iteration ahead to overlap their latency
      struct Ahead {
        float2 q;
        LongPairIn in;
      };
      auto fetch = [&](int j) {
        const int c = tl + NT * j;
        const int cm = N1 - 1 - c;
        const int k = rA + N2 * c, km = NC - k;
        const int64_t pa = int64_t(rA) * N1 + c, pb = int64_t(rB) * N1 + cm;
        Ahead h;
        h.q = ra[c];  // this thread's own write above
        h.in = k < km ? long_pair_fetch<SRC>(a, psd, k, pa, pb) : long_pair_fetch<SRC>(a, psd, km, pb, pa);
        return h;
      };
      Ahead nxt = fetch(0);
#pragma unroll 1
      for (int j = 0; j < 16; ++j) {
        const Ahead cur = nxt;
        if (j + 1 < 16) nxt = fetch(j + 1);
        const int c = tl + NT * j;
        const int cm = N1 - 1 - c;
        const int k = rA + N2 * c, km = NC - k;
        const int im = lpad<float>(cm);
        cpx<float> P = {cur.q.x, cur.q.y}, Q = {sre[im], sim[im]};
        if (k < km) long_pair<TP, SRC>(a, wsh, cpl, cxx, tauT, cur.in, k, P, Q, flag);
        else long_pair<TP, SRC>(a, wsh, cpl, cxx, tauT, cur.in, km, Q, P, flag);
        ra[c] = {P.x, P.y};
        sre[im] = Q.x;
        sim[im] = Q.y;
      }
    }
    lds_barrier();
    block_fft<float, N1, +1, true, 0>(v, sre, sim, fresh_lane(t), tw());
    store_row(rowB);
    // row rA: its bins as this thread wrote them, in the transform's input layout
    load_row(rowA);
    lds_barrier();
    block_fft<float, N1, +1, false, 0>(v, sre, sim, fresh_lane(t), tw());
    store_row(rowA);
  }
  if (flag) atomicOr(&sflag, flag);
  __syncthreads();
  if (t == 0 && sflag && a.w.status) atomicOr(a.w.status + b, sflag);
}

template <int N1, int SRC>
void launch_cols_fwd(const LongArgs& a, int64_t items, hipStream_t st) {
  const dim3 grid(unsigned(N1 / 256), unsigned(items));
  if constexpr (N1 == 16384) {  // only N = 2^20 uses rows of 16384
    hipLaunchKernelGGL((k_long_cols_fwd<N1, 32, SRC>), grid, dim3(256), 0, st, a);
  } else {
    switch (a.N2) {
      case 4: hipLaunchKernelGGL((k_long_cols_fwd<N1, 4, SRC>), grid, dim3(256), 0, st, a); break;
      case 8: hipLaunchKernelGGL((k_long_cols_fwd<N1, 8, SRC>), grid, dim3(256), 0, st, a); break;
      case 16: hipLaunchKernelGGL((k_long_cols_fwd<N1, 16, SRC>), grid, dim3(256), 0, st, a); break;
      default: hipLaunchKernelGGL((k_long_cols_fwd<N1, 32, SRC>), grid, dim3(256), 0, st, a); break;
    }
  }
}

template <int N1, int SRC>
void launch_cols_inv(const LongArgs& a, int64_t items, hipStream_t st) {
  const dim3 grid(unsigned(N1 / 256), unsigned(items));
  if constexpr (N1 == 16384) {  // only N = 2^20 uses rows of 16384
    hipLaunchKernelGGL((k_long_cols_inv<N1, 32, SRC>), grid, dim3(256), 0, st, a);
  } else {
    switch (a.N2) {
      case 4: hipLaunchKernelGGL((k_long_cols_inv<N1, 4, SRC>), grid, dim3(256), 0, st, a); break;
      case 8: hipLaunchKernelGGL((k_long_cols_inv<N1, 8, SRC>), grid, dim3(256), 0, st, a); break;
      case 16: hipLaunchKernelGGL((k_long_cols_inv<N1, 16, SRC>), grid, dim3(256), 0, st, a); break;
      default: hipLaunchKernelGGL((k_long_cols_inv<N1, 32, SRC>), grid, dim3(256), 0, st, a); break;
    }
  }
}

// The passes of one window stage at row length N1 (see long_window).
template <int N1>
void long_passes(const DevCfg& d, int src, const LongArgs& a, const float* hdet, int64_t items, hipStream_t st) {
  const dim3 bins_grid(unsigned(N1 / 512), unsigned(items), unsigned(a.N2 / 2 + 1));
  const dim3 inject_grid(unsigned((a.NC / 2 + 1 + 255) / 256), unsigned(items));
  const dim3 rows_grid(unsigned(items * a.N2));
  if (src == 2) {
    hipLaunchKernelGGL((k_long_inject<N1>), inject_grid, dim3(256), 0, st, a, hdet);
    hipLaunchKernelGGL((k_long_rows<N1, +1>), rows_grid, dim3(N1 / 16), 0, st, a);
    launch_cols_inv<N1, 2>(a, items, st);
    return;
  }
  if (src == 0) launch_cols_fwd<N1, 0>(a, items, st);
  else launch_cols_fwd<N1, 1>(a, items, st);
  if (d.ord_win) {
    // rows, bins and inverse rows fused per row pair
    const dim3 pair_grid(unsigned(items * (a.N2 / 2 + 1)));
    if (src == 0) hipLaunchKernelGGL((k_long_rowpair<N1, double, 0>), pair_grid, dim3(N1 / 16), 0, st, a);
    else if (d.precision == 0) hipLaunchKernelGGL((k_long_rowpair<N1, float, 1>), pair_grid, dim3(N1 / 16), 0, st, a);
    else hipLaunchKernelGGL((k_long_rowpair<N1, double, 1>), pair_grid, dim3(N1 / 16), 0, st, a);
    launch_cols_inv<N1, 0>(a, items, st);
    return;
  }
  hipLaunchKernelGGL((k_long_rows<N1, -1>), rows_grid, dim3(N1 / 16), 0, st, a);
  if (src == 0) {
    hipLaunchKernelGGL((k_long_bins<N1, double, 0>), bins_grid, dim3(256), 0, st, a);
  } else if (d.precision == 0) {
    hipLaunchKernelGGL((k_long_bins<N1, float, 1>), bins_grid, dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_long_bins<N1, double, 1>), bins_grid, dim3(256), 0, st, a);
  }
  hipLaunchKernelGGL((k_long_rows<N1, +1>), rows_grid, dim3(N1 / 16), 0, st, a);
  launch_cols_inv<N1, 0>(a, items, st);
}

}  // namespace

namespace gw {

int long_row_length(int NC) { return NC / 8192 <= 32 ? 8192 : 16384; }

// The window stage for N > 32768: SRC 0 whitens strain rows x, SRC 1 is the
// fused batch (x = background), SRC 2 injects hdet into the background
// noise.  w.out is [items][N] and doubles as the transform buffer.
gw_status long_window(gw_ctx* c, int src, const WinArgs& w, const float* x, const float* hdet, int64_t items,
                      hipStream_t st) {
  const DevCfg& d = c->dc;
  LongArgs a;
  a.w = w;
  a.twc = c->tw_long;
  a.twr = c->twr_win;
  a.tw1 = c->tw_win;
  a.x = x;
  a.NC = d.N / 2;
  const int N1 = long_row_length(a.NC);
  a.N2 = a.NC / N1;
  a.l2n2 = 0;
  while ((1 << a.l2n2) < a.N2) ++a.l2n2;
  const char* tabs = static_cast<const char*>(c->long_tabs);
  a.kc_t = reinterpret_cast<const double*>(tabs);
  a.lk_t = reinterpret_cast<const double*>(tabs + sizeof(double) * size_t(a.NC));
  a.twr_t = reinterpret_cast<const cpx<float>*>(tabs + 2 * sizeof(double) * size_t(a.NC));
  if (items <= 0) return GW_OK;
  if (items > 65535) return ctx_fail(c, GW_EINVAL, "long windows: at most 65535 (sample, detector) items per call");
  if (!c->long_tabs) return ctx_fail(c, GW_EUNSUPPORTED, "long windows need the binary32 tables");
  if (a.N2 < 4 || a.N2 > 32 || a.N2 * N1 != a.NC) return ctx_fail(c, GW_EUNSUPPORTED, "long windows: bad split");
  if (N1 == 8192) long_passes<8192>(d, src, a, hdet, items, st);
  else long_passes<16384>(d, src, a, hdet, items, st);
  return ctx_check_launch(c, src == 2 ? "long inject" : "long window");
}

}  // namespace gw
