// Per-item device code shared by the batch kernels and the persistent
// ragged kernels: the window item (rfft -> signal -> whiten -> irfft) and the
// Welch item, each run by the NC/16 threads of a (sub-)block on its own LDS
// planes.
#pragma once
#include <hip/hip_runtime.h>

#include "gw_fft.hpp"
#include "gw_physics.hpp"
#include "../../include/gwgen.h"

namespace gw {

// ---------------------------------------- window kernels (FFT of length N)
// Prior draws for global sample index g (the densities of Table 1 with the
// ranges in c), the window's background offset in [0, span), status
// initialisation, and the per-sample constants of the fused window kernel.
// Row 11 of the parameters receives p11.  With ext_k sky positions per
// intrinsic draw, g is sky position g % ext_k of intrinsic draw g / ext_k:
// every row is drawn at counter index g / ext_k, and alpha, delta, psi and
// the offset use the sub-counter g % ext_k (ext_k = 1: ordinary draws).
__device__ __forceinline__ void draw_sample(const DevCfg& c, uint64_t seed, uint64_t g, int64_t i, int64_t B,
                                            int64_t span, double p11, double* params, int64_t* offset,
                                            float* params_f32, uint32_t* status, WfScalars* wf, DetScalars* dsc,
                                            uint32_t ext_k = 1u) {
#pragma clang fp contract(off)
  const uint64_t gi = g / ext_k;
  const uint32_t j = uint32_t(g - gi * ext_k);
  double u[11];
#pragma unroll
  for (int s = 0; s < 11; ++s) u[s] = philox_uniform(seed, gi, uint32_t(s), (s >= 6 && s <= 8) ? j : 0u);
  const double uo = philox_uniform(seed, gi, 12u, j);
  double p[12];
  if (c.approximant == 2) {
    // sine-Gaussian: f0 and Q uniform, hrss log-uniform
    p[0] = c.f0r[0] + u[0] * (c.f0r[1] - c.f0r[0]);
    p[1] = c.Qr[0] + u[1] * (c.Qr[1] - c.Qr[0]);
    p[2] = exp(log(c.hrssr[0]) + u[2] * (log(c.hrssr[1]) - log(c.hrssr[0])));
    p[3] = 0.0;
    p[4] = 0.0;
  } else {
    p[0] = c.mc[0] + u[0] * (c.mc[1] - c.mc[0]);
    p[1] = c.q[0] + u[1] * (c.q[1] - c.q[0]);
    p[2] = c.chi[0] + u[2] * (c.chi[1] - c.chi[0]);
    p[3] = c.chi[0] + u[3] * (c.chi[1] - c.chi[0]);
    const double a3 = c.dl[0] * c.dl[0] * c.dl[0], b3 = c.dl[1] * c.dl[1] * c.dl[1];
    p[4] = pow(a3 + u[4] * (b3 - a3), 1.0 / 3.0);
  }
  p[5] = acos(2.0 * u[5] - 1.0);
  p[6] = 2.0 * kPi * u[6];
  p[7] = asin(2.0 * u[7] - 1.0);
  p[8] = kPi * u[8];
  p[9] = 2.0 * kPi * u[9];
  p[10] = c.T - 1.5 + u[10] * 1.0;
  p[11] = p11;
#pragma unroll
  for (int r = 0; r < 12; ++r) params[r * B + i] = p[r];
  offset[i] = int64_t(floor(uo * double(span)));
  if (params_f32) {
#pragma unroll
    for (int r = 0; r < 12; ++r) params_f32[r * B + i] = float(p[r]);
  }
  if (status) {
    double f_cut;
    if (c.approximant == 2) {
      f_cut = p[0] + 5.0 / (kPi * (p[1] / (sqrt(2.0) * kPi * p[0])));  // f0 + 5/(pi tau)
    } else {
      const double eta = p[1] / ((1.0 + p[1]) * (1.0 + p[1]));
      const double Ms = p[0] * pow(eta, -0.6) * kMsunSec;
      f_cut = c.approximant == 0 ? 1.0 / (pow(6.0, 1.5) * kPi * Ms) : 0.2 / Ms;
    }
    status[i] = f_cut > 0.5 * c.fs ? GW_STATUS_CUT_AT_NYQUIST : 0u;
  }
  if (wf) {
    WfScalars w;
    wf_setup(params, B, i, c, w);
    wf[i] = w;
    for (int d = 0; d < c.n_det; ++d) dsc[i * c.n_det + d] = det_response(c.det[d], w.ra, w.dec, w.psi, w.tc);
  }
}

// Load through the constant address space: for memory that no thread writes
// while the kernel runs.  A uniform address then becomes a scalar load even
// after earlier stores in the same kernel.
template <class T>
__device__ __forceinline__ T load_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  typedef const __attribute__((address_space(4))) uint32_t* cword_ptr;
  const cword_ptr q = (cword_ptr)(p);
  T v;
  uint32_t* o = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 4); ++i) o[i] = q[i];
  return v;
}

struct WinArgs {
  DevCfg cf;
  const float* src;       // strain [B][D][N] (SRC 0, 2) or background (SRC 1)
  int64_t L_bg;
  const float* bg;        // background for inject (SRC 2)
  const int64_t* offset;
  const double* params;
  int64_t B;
  const float* psd;       // [B][D][Fw]
  float* out;
  uint32_t* status;
  const double* kcbrt;
  const double* lnk3;
  const double* k53;      // k^(-5/3) (SRC 3)
  const void* tw;         // cpx<T>[N/2], exp(-2 pi i n / (N/2))
  const void* twr;        // cpx<T>[N/4 + 1], exp(-2 pi i k / N)
  const WfScalars* wf;    // [B] (SRC 1, 3)
  const DetScalars* dsc;  // [B][D] (SRC 1, 3)
  const float* nodes;     // [B][2][1024] surrogate node values (SRC 3)
  const float* logmm;     // [B] predicted log10 mismatch (SRC 3)
  float logmm_max;        // fallback threshold (SRC 3)
  int crop;               // samples dropped at each end of the output (SRC 4; even)
  float* out2;            // SRC 5: the reference views [B][D][N]
  double t_ref;           // SRC 5: the reference view's signal time
};

// Surrogate node grid: 1024 points log-spaced in Mf over [2e-3, 0.2].
constexpr int kSurrNodes = 1024;
constexpr double kSurrLnMfLo = -6.2146080984221914;   // ln(2e-3)
constexpr double kSurrDlog = 4.6051701859880914 / 1023.0;  // ln(0.2/2e-3)/(NN-1)

// Lower PSD bin for window bin k, clamped so that it and the next bin exist
// for every k in [0, N/2] (the PSD has L/2 + 1 bins, L/2 = (N/2) / ratio).
__device__ __forceinline__ int psd_index(const DevCfg& cf, int k, int NC) {
  return min(k >> cf.log2_ratio, (NC >> cf.log2_ratio) - 1);
}

// Whitening factor for window bin k in [0, N/2] from the PSD values
// s0 = psd[i], s1 = psd[i + 1], i = psd_index(k); sets status bits.
template <class T>
__device__ __forceinline__ T whiten_gain_at(const DevCfg& cf, float s0, float s1, int k, int NC, uint32_t& flag) {
  if (k == 0 || k >= NC || k < cf.kmin) return T(0);
  const int i = k >> cf.log2_ratio;
  const T tt = T(k - (i << cf.log2_ratio)) * T(cf.inv_ratio);
  const T S = (T(1) - tt) * T(s0) + tt * T(s1);
  if (!isfinite(S)) { flag |= GW_STATUS_NONFINITE_PSD; return T(0); }
  if (!(S > T(0))) { flag |= GW_STATUS_NONPOSITIVE_PSD; return T(0); }
  return rsqrt_t(T(cf.fs) * S * T(0.5));
}

template <class T>
__device__ __forceinline__ T whiten_gain(const DevCfg& cf, const float* psd, int k, int NC, uint32_t& flag) {
  const int i = psd_index(cf, k, NC);
  return whiten_gain_at<T>(cf, psd[i], psd[i + 1], k, NC, flag);
}

// Gain g = filt[k] of a precomputed whitening filter; sets status bits.
template <class T>
__device__ __forceinline__ T filter_gain_at(float g, uint32_t& flag) {
  if (!isfinite(g)) { flag |= GW_STATUS_NONFINITE_PSD; return T(0); }
  return T(g);
}

// Projected signal (DFT coefficients) at window bin k, generated in registers.
// Projected sine-Gaussian at bin k: fs sg_G0 [G(f - f0)(cpl - i cxx) e^{-2 pi i rm}
// + G(f + f0)(cpl + i cxx) e^{-2 pi i rp}], rm/rp = k tau/T -/+ phi0/(2 pi).
template <class T, class TP>
__device__ __forceinline__ cpx<T> burst_bin(const DevCfg& cf, const WfScalars& w, T cpl, T cxx, double tauT, int k) {
  const double f = double(k) * cf.invT;
  const T xm = T(f - w.sg_f0), xp = T(f + w.sg_f0);
  const T gm = exp(-T(w.sg_pt2) * xm * xm), gp = exp(-T(w.sg_pt2) * xp * xp);
  const TP base = frac1(TP(k) * TP(tauT));
  T sm, cm, sp, cp;
  sincos_rev(T(frac1(base - TP(w.sg_rphi))), &sm, &cm);
  sincos_rev(T(frac1(base + TP(w.sg_rphi))), &sp, &cp);
  const T A = T(cf.fs) * T(w.sg_G0);
  return {A * (gm * (cpl * cm - cxx * sm) + gp * (cpl * cp + cxx * sp)),
          A * (gp * (cxx * cp - cpl * sp) - gm * (cpl * sm + cxx * cm))};
}

// Same, with k^(1/3) and ln(k)/3 given by the caller (kc, lk).
template <class T, class TP, bool FULL>
__device__ __forceinline__ cpx<T> signal_bin_at(const DevCfg& cf, const WfScalars& w, T cpl, T cxx, double tauT,
                                                int k, double kc, double lk) {
  if (k <= 0 || k < cf.kmin || k >= w.kend) return {T(0), T(0)};
  if (cf.approximant == 2) return burst_bin<T, TP>(cf, w, cpl, cxx, tauT, k);
  TP rev = wf_phase_rev<TP, FULL>(w, k, kc, lk, cf.invT) + TP(w.pconst) + TP(k) * TP(tauT);
  rev = frac1(rev);
  T s, c;
  sincos_rev(T(rev), &s, &c);
  const T A = T(cf.fs) * wf_amplitude<T>(w, k, kc, cf.invT);
  // fs A (cpl - i cxx)(c - i s)
  return {A * (cpl * c - cxx * s), -A * (cpl * s + cxx * c)};
}

template <class T, class TP, bool FULL>
__device__ __forceinline__ cpx<T> signal_bin(const DevCfg& cf, const WinArgs& a, const WfScalars& w, T cpl, T cxx,
                                             double tauT, int k) {
  if (k <= 0 || k < cf.kmin || k >= w.kend) return {T(0), T(0)};
  if (cf.approximant == 2) return burst_bin<T, TP>(cf, w, cpl, cxx, tauT, k);
  const double kc = a.kcbrt[k], lk = a.lnk3[k];
  TP rev = wf_phase_rev<TP, FULL>(w, k, kc, lk, cf.invT) + TP(w.pconst) + TP(k) * TP(tauT);
  rev = frac1(rev);
  T s, c;
  sincos_rev(T(rev), &s, &c);
  const T A = T(cf.fs) * wf_amplitude<T>(w, k, kc, cf.invT);
  // fs A (cpl - i cxx)(c - i s)
  return {A * (cpl * c - cxx * s), -A * (cpl * s + cxx * c)};
}

// Projected signal at window bin k from surrogate node values: binary64
// Newtonian phase + interpolated phase residual (revolutions), amplitude
// A_N(f_k) times the interpolated ratio.
// Node values staged in LDS: typed as such, so that their gathers compile to
// LDS reads rather than generic (flat) loads, which would also wait for the
// global loads issued ahead.
typedef const __attribute__((address_space(3))) float* lds_cfptr;

template <class T>
__device__ __forceinline__ cpx<T> signal_bin_surr(const DevCfg& cf, const WinArgs& a, const WfScalars& w,
                                                  lds_cfptr nd, T cpl, T cxx, double tauT, int k) {
  if (k <= 0 || k < cf.kmin || k >= w.kend) return {T(0), T(0)};
  const double lk3 = a.lnk3[k], k53 = a.k53[k];
  // u = (ln(Ms k / T) - ln Mf_lo) / dlog, ln(Ms/T) = 3 ln v1 - ln pi
  const float u = float((3.0 * w.lnv1 - 1.1447298858494002 - kSurrLnMfLo + 3.0 * lk3) * (1.0 / kSurrDlog));
  const float uc = fminf(fmaxf(u, 0.f), float(kSurrNodes - 1));
  const int i = min(int(uc), kSurrNodes - 2);
  const float tt = uc - float(i);
  const float ratio = (1.f - tt) * nd[i] + tt * nd[i + 1];
  const float dpsi = (1.f - tt) * nd[kSurrNodes + i] + tt * nd[kSurrNodes + i + 1];
  // Newtonian phase cN k^(-5/3) from the table: one binary64 product per bin
  double rev = w.cN * k53 + double(dpsi) * (1.0 / (2.0 * kPi)) + w.pconst + double(k) * tauT;
  rev = frac1(rev);
  T sn, cs;
  sincos_rev(T(rev), &sn, &cs);
  // A_N(f_k) = A0T k^(-7/6) = A0T k^(-5/3) k^(1/2)
  const T kf = T(k);
  const T A = T(cf.fs) * T(w.A0T) * T(k53) * (kf * rsqrt_t(kf)) * T(ratio);
  return {A * (cpl * cs - cxx * sn), -A * (cpl * sn + cxx * cs)};
}

// One window item (sample b, detector d) handled by the NC/16 threads t of a
// (sub-)block, with its own LDS planes.
// SRC 0: whiten strain (x = strain row).  SRC 1: background + in-register
// signal + whiten (x = background at o + P).  SRC 3: as SRC 1 with the signal
// from surrogate node values (plain model where the predicted mismatch
// exceeds the threshold).  SRC 2: inject (hrow = hdet row, nz = noise window).
// SRC 4: as SRC 1 whitened with a fixed per-run filter (psd = filter row of
// N/2 + 1 gains), storing samples [crop, N - crop) only.  SRC 5: the view
// pair of one item: as SRC 1 into o, then, from the same noise spectrum kept
// in registers, the same window with the signal at t_ref into o2.
// `active` false: compute on the given (valid) item but store nothing, so
// that idle sub-blocks still meet every block barrier.
template <class T, class TP, bool FULL, int NC, int SRC, int ORD>
__device__ __forceinline__ void window_item(const DevCfg& cf, const WinArgs& a, int t, int64_t b, int d,
                                            const float* x, const float* hrow, const float* nz, const float* psd,
                                            float* o, const cpx<T>* twtab, const cpx<T>* twr, T* sre, T* sim,
                                            bool active, uint32_t* sflag, float* snodes = nullptr,
                                            float* o2 = nullptr) {
  constexpr int NT = NC / 16;
  static_assert(SRC >= 0 && SRC <= 5, "source");
  constexpr bool SIG = SRC == 1 || SRC == 5;  // in-register plain-model signal
  PowTwiddle<T, NC, ORD> tw{twtab};
  if constexpr (SRC == 3) {
    // the sample's node values go to LDS once (snodes: 2 x 1024 floats of
    // LDS); the barriers of the forward transform below make them visible to
    // the whole (sub-)block
    const float* src = a.nodes + b * 2 * kSurrNodes;
    for (int i = t; i < 2 * kSurrNodes; i += NT) snodes[i] = src[i];
  }
  cpx<T> v[16];
  uint32_t flag = 0;
  if constexpr (SRC != 2) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      float2 q;
      __builtin_memcpy(&q, x + 2 * (t + NT * j), sizeof(q));
      v[fft_in_slot<NC, ORD>(j)] = {T(q.x), T(q.y)};
    }
    // fresh lane indices and a fresh table pointer per transform: otherwise
    // the compiler shares the forward and inverse transforms' index
    // arithmetic and twiddle loads and keeps them live in between
    block_fft<T, NC, -1, false, ORD>(v, sre, sim, fresh_lane(t), tw);
    lds_barrier();
    const int tn = fresh_lane(t);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = lpad<T>(fft_out_index<NC, ORD>(tn, e));
      sre[i] = v[e].x;
      sim[i] = v[e].y;
    }
    lds_barrier();
  }
  // SRC 5: this thread's share of the noise spectrum, for the second view
  cpx<T> keep[SRC == 5 ? 16 : 1];
  if constexpr (SRC == 5) {
#pragma unroll
    for (int e = 0; e < 16; ++e) keep[e] = v[e];
  }

  T cpl = T(0), cxx = T(0);
  double tauT = 0.0;
  WfScalars wsh;
  if constexpr (SIG || SRC == 3 || SRC == 4) wsh = load_const(a.wf + b);
  bool use_surr = false;
  lds_cfptr nd = nullptr;
  if constexpr (SRC == 3) {
    // a NaN prediction fails the test and falls back to the plain model
    use_surr = load_const(a.logmm + b) <= a.logmm_max;
    nd = (lds_cfptr)snodes;  // staged before the forward transform
    if (active && !use_surr && t == 0 && d == 0 && a.status)
      atomicOr(a.status + b, uint32_t(GW_STATUS_SURROGATE_FALLBACK));
  }
  double tauT_ref = 0.0;  // SRC 5: the reference view's time shift
  if constexpr (SIG || SRC == 3 || SRC == 4) {
    const DetScalars dsh = load_const(a.dsc + (b * cf.n_det + d));
    cpl = T(dsh.fp * 0.5 * (1.0 + wsh.cosi * wsh.cosi));
    cxx = T(dsh.fx * wsh.cosi);
    tauT = dsh.tau * cf.invT;
    if constexpr (SRC == 5) tauT_ref = (dsh.tau - wsh.tc + a.t_ref) * cf.invT;  // same delays, signal at t_ref
  }
  const float2* hsrc = reinterpret_cast<const float2*>(hrow);

  // Global inputs of the pair (k, NC - k): the twiddle and what the two bins
  // need (PSD values, filter gains, or the signal to inject), fetched one
  // pair ahead so that their latency overlaps the previous pair's work.
  struct PairIn {
    cpx<T> W;
    float g[4];
  };
  auto fetch = [&](int k) {
    k = min(k, NC / 2);
    const int km = NC - k;
    PairIn q;
    q.W = twr[k];  // exp(-2 pi i k / N)
    if constexpr (SRC == 2) {
      const float2 h0 = hsrc[k], h1 = hsrc[km];
      q.g[0] = h0.x;
      q.g[1] = h0.y;
      q.g[2] = h1.x;
      q.g[3] = h1.y;
    } else if constexpr (SRC == 4) {
      q.g[0] = psd[k];
      q.g[1] = psd[km];
      q.g[2] = q.g[3] = 0.f;
    } else {
      const int ia = psd_index(cf, k, NC), ib = psd_index(cf, km, NC);
      q.g[0] = psd[ia];
      q.g[1] = psd[ia + 1];
      q.g[2] = psd[ib];
      q.g[3] = psd[ib + 1];
    }
    return q;
  };
  // the pair's spectrum values (k, NC - k) from LDS
  auto load_pair = [&](int k, cpx<T>& A, cpx<T>& Bm) {
    if constexpr (SRC != 2) {
      const int ia = lpad<T>(k), ib = lpad<T>((NC - k) & (NC - 1));
      A = {sre[ia], sim[ia]};
      Bm = {sre[ib], sim[ib]};
    }
  };
  // unpack, signal, gain and repack of the pair: zk, zm go to bins k, NC - k
  auto pair_out = [&](const PairIn& cur, int k, cpx<T> A, cpx<T> Bm, cpx<T>& zk, cpx<T>& zm) {
    const int km = NC - k;
    const cpx<T> W = cur.W;
    cpx<T> Yk, Ym;
    if constexpr (SRC == 2) {
      Yk = {T(cur.g[0]), T(cur.g[1])};
      Ym = {T(cur.g[2]), T(cur.g[3])};
      if (k == 0) { Yk.y = T(0); Ym.y = T(0); }  // irfft ignores Im at DC and Nyquist
    } else {
      const cpx<T> s = cadd(A, cconj(Bm));
      const cpx<T> u = cmul(W, csub(A, cconj(Bm)));
      cpx<T> Xk = {T(0.5) * (s.x + u.y), T(0.5) * (s.y - u.x)};
      cpx<T> Xm = {T(0.5) * (s.x - u.y), T(0.5) * (-s.y - u.x)};
      if constexpr (SIG || SRC == 4) {
        Xk = cadd(Xk, signal_bin<T, TP, FULL>(cf, a, wsh, cpl, cxx, tauT, k));
        if (km != k) Xm = cadd(Xm, signal_bin<T, TP, FULL>(cf, a, wsh, cpl, cxx, tauT, km));
      } else if constexpr (SRC == 3) {
        if (use_surr) {
          Xk = cadd(Xk, signal_bin_surr<T>(cf, a, wsh, nd, cpl, cxx, tauT, k));
          if (km != k) Xm = cadd(Xm, signal_bin_surr<T>(cf, a, wsh, nd, cpl, cxx, tauT, km));
        } else {
          Xk = cadd(Xk, signal_bin<T, TP, FULL>(cf, a, wsh, cpl, cxx, tauT, k));
          if (km != k) Xm = cadd(Xm, signal_bin<T, TP, FULL>(cf, a, wsh, cpl, cxx, tauT, km));
        }
      }
      if constexpr (SRC == 4) {
        // fixed per-run filter row [NC + 1] (zero outside the kept band)
        Yk = cscale(Xk, filter_gain_at<T>(cur.g[0], flag));
        Ym = cscale(Xm, filter_gain_at<T>(cur.g[1], flag));
      } else {
        Yk = cscale(Xk, whiten_gain_at<T>(cf, cur.g[0], cur.g[1], k, NC, flag));
        Ym = cscale(Xm, whiten_gain_at<T>(cf, cur.g[2], cur.g[3], km, NC, flag));
      }
      if (km == k) Ym = Yk;
    }
    // inverse packing: Z'_k = p + i q, Z'_{NC-k} = conj(p) + i conj(q)
    const cpx<T> p = cscale(cadd(Yk, cconj(Ym)), T(0.5));
    const cpx<T> q = twmul<+1>(cscale(csub(Yk, cconj(Ym)), T(0.5)), W);
    zk = {p.x - q.y, p.y + q.x};
    zm = {p.x + q.y, -p.y + q.x};
  };
  auto store_pair = [&](int k, cpx<T> zk, cpx<T> zm) {
    const int km = NC - k;
    const int ia = lpad<T>(k);
    sre[ia] = zk.x;
    sim[ia] = zk.y;
    if (k != 0 && km != k) {
      const int ib = lpad<T>(km);
      sre[ib] = zm.x;
      sim[ib] = zm.y;
    }
  };

  // pairs, inverse transform and store of one output window ov
  auto emit = [&](float* ov) {
  // pairs (k, NC - k) for k = t + NT i in [0, NC/2] (NC/2 = 8 NT): two per
  // loop trip, whose LDS reads are issued together and whose arithmetic
  // chains interleave; the last one (k = NC/2) belongs to thread 0 alone
  PairIn n0 = fetch(t), n1 = fetch(t + NT);
#pragma unroll 1
  for (int i = 0; i < 8; i += 2) {
    const int k0 = t + NT * i, k1 = k0 + NT;
    const PairIn c0 = n0, c1 = n1;
    n0 = fetch(k0 + 2 * NT);
    n1 = fetch(k1 + 2 * NT);
    cpx<T> A0 = {}, B0 = {}, A1 = {}, B1 = {}, z0k, z0m, z1k, z1m;
    load_pair(k0, A0, B0);
    load_pair(k1, A1, B1);
    pair_out(c0, k0, A0, B0, z0k, z0m);
    pair_out(c1, k1, A1, B1, z1k, z1m);
    store_pair(k0, z0k, z0m);
    store_pair(k1, z1k, z1m);
  }
  if (t == 0) {  // n0 = fetch(NC/2)
    cpx<T> A = {}, Bm = {}, zk, zm;
    load_pair(NC / 2, A, Bm);
    pair_out(n0, NC / 2, A, Bm, zk, zm);
    store_pair(NC / 2, zk, zm);
  }
  lds_barrier();
  block_fft<T, NC, +1, true, ORD>(v, sre, sim, fresh_lane(t), PowTwiddle<T, NC, ORD>{opaque(twtab)});
  const T sc = T(1) / T(NC);
  if (active) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int n = fft_out_index<NC, ORD>(t, e);
      float2 y = {float(v[e].x * sc), float(v[e].y * sc)};
      if constexpr (SRC == 2) {
        y.x += nz[2 * n];
        y.y += nz[2 * n + 1];
      }
      if constexpr (SRC == 4) {
        // cropped store: samples [crop, N - crop), crop even
        const int m = n - (a.crop >> 1);
        if (m >= 0 && m < NC - a.crop) reinterpret_cast<float2*>(ov)[m] = y;
      } else {
        reinterpret_cast<float2*>(ov)[n] = y;
      }
    }
  }
  };
  emit(o);
  if constexpr (SRC == 5) {
    // reference view: the noise spectrum back to LDS, the signal at t_ref
    lds_barrier();  // the inverse transform's last LDS reads are done
    const int tk = fresh_lane(t);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = lpad<T>(fft_out_index<NC, ORD>(tk, e));
      sre[i] = keep[e].x;
      sim[i] = keep[e].y;
    }
    lds_barrier();
    tauT = tauT_ref;
    emit(o2);
  }
  if (active && flag) atomicOr(sflag, flag);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Twiddles of passes 1.. kept in registers for the whole segment loop.
template <class T, int NC, int ORD> struct RegTwiddle {
  cpx<T> p[FftPlan<NC>::NPASS][16];
  __device__ __forceinline__ void init(const cpx<T>* __restrict__ tab, int t) {
    init_pass<1>(tab, t);
    init_pass<2>(tab, t);
    if constexpr (FftPlan<NC>::NPASS == 4) init_pass<3>(tab, t);
  }
  template <int PASS> __device__ __forceinline__ void init_pass(const cpx<T>* __restrict__ tab, int t) {
    constexpr int R = PassInfo<NC, PASS, ORD>::R, NS = PassInfo<NC, PASS, ORD>::NS, NT = NC / 16;
#pragma unroll
    for (int m = 0; m < 16 / R; ++m) {
      const int k = (t + NT * m) & (NS - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) p[PASS][m * R + r] = tab[(r * k) * (NC / (NS * R))];
    }
  }
  template <int PASS> __device__ __forceinline__ cpx<T> get(int m, int r, int) const {
    return p[PASS][m * PassInfo<NC, PASS, ORD>::R + r];
  }
};

// Welch PSD of one (sample, detector) stretch x = background + o, by the
// NC/16 threads t of a (sub-)block: K periodic-Hann segments of L = NC samples
// at stride L/2.  Segments 2p and 2p+1 go through ONE complex FFT as real and
// imaginary parts; since |A_k|^2 + |B_k|^2 = (|X_k|^2 + |X_{L-k}|^2)/2 for
// X = FFT(a + i b), the accumulated |X|^2 is folded once at the end.
// With ACC wider than T (mixed precision) every transform's |X|^2 is added
// to ACC totals.  With ACC equal to T it is summed in two levels, runs of
// kWelchRun transforms and then the run sums, so that the rounding error
// grows with kWelchRun + K/(2 kWelchRun) terms rather than K/2.  The fold and
// the normalisation are done in ACC.
template <class T, class ACC, int NC, int ORD>
__device__ __forceinline__ void welch_item(int K, double norm, int t, const float* x, float* out, const cpx<T>* twtab,
                                           T* sre, T* sim, bool active) {
  constexpr int NT = NC / 16;
  constexpr int LS = LdsSize<NC>::value;
  static_assert(NC * sizeof(ACC) <= 2 * LS * sizeof(T), "fold buffer must fit in the FFT buffer");
  // periodic Hann window sin^2(pi n / L) at n = t + NT r, r < 8; half a
  // segment later it is cos^2 = 1 - sin^2, applied as x - w x
  T w[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const T sp = sinpi_t(T(t + NT * r) / T(NC));
    w[r] = sp * sp;
  }
  RegTwiddle<T, NC, ORD> tw;
  tw.init(twtab, t);
  constexpr bool kWide = sizeof(ACC) > sizeof(T);
  constexpr int kWelchRun = 16;
  ACC tot[16];
  T run[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    tot[e] = ACC(0);
    run[e] = T(0);
  }
  // |X|^2 of transform p (p < 0: the last, single-segment transform)
  auto add_power = [&](const cpx<T>* v, int p) {
    if constexpr (kWide) {
#pragma unroll
      for (int e = 0; e < 16; ++e) tot[e] += ACC(fma_t(v[e].y, v[e].y, v[e].x * v[e].x));
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) run[e] = fma_t(v[e].y, v[e].y, fma_t(v[e].x, v[e].x, run[e]));
      if (p % kWelchRun == kWelchRun - 1) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          tot[e] += run[e];
          run[e] = T(0);
        }
      }
    }
  };
  // Pair p covers [p L, p L + 3L/2).  Its first half-segment was read by
  // pair p-1; the next pair's 16 new values per thread are requested before
  // the current transform so that their latency hides behind it.
  const int npairs = (K + 1) / 2;
  const int nfull = K / 2;  // pairs holding two segments; with K odd the last pair holds one
  float cur[8], na[8], nb[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    cur[r] = x[t + NT * r];
    na[r] = x[t + NT * (r + 8)];
    nb[r] = (K > 1) ? x[NC / 2 + t + NT * (r + 8)] : 0.f;
  }
#pragma unroll 1
  for (int p = 0; p < nfull; ++p) {
    cpx<T> v[16];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      v[fft_in_slot<NC, ORD>(r)] = {w[r] * T(cur[r]), w[r] * T(na[r])};
      v[fft_in_slot<NC, ORD>(r + 8)] = {T(na[r]) - w[r] * T(na[r]), T(nb[r]) - w[r] * T(nb[r])};
      cur[r] = nb[r];
    }
    const float* xn = x + int64_t(p + 1) * NC;
    if (p + 1 < nfull) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        na[r] = xn[t + NT * (r + 8)];
        nb[r] = xn[NC / 2 + t + NT * (r + 8)];
      }
    } else if (p + 1 < npairs) {
#pragma unroll
      for (int r = 0; r < 8; ++r) na[r] = xn[t + NT * (r + 8)];
    }
    if (p > 0) lds_barrier();
    block_fft<T, NC, -1, false, ORD>(v, sre, sim, t, tw);
    add_power(v, p);
  }
  if (nfull < npairs) {
    // the last segment alone: real input, zero imaginary part
    cpx<T> v[16];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      v[fft_in_slot<NC, ORD>(r)] = {w[r] * T(cur[r]), T(0)};
      v[fft_in_slot<NC, ORD>(r + 8)] = {T(na[r]) - w[r] * T(na[r]), T(0)};
    }
    if (nfull > 0) lds_barrier();
    block_fft<T, NC, -1, false, ORD>(v, sre, sim, t, tw);
    add_power(v, -1);
  }
  lds_barrier();
  ACC* fold = reinterpret_cast<ACC*>(sre);
#pragma unroll
  for (int e = 0; e < 16; ++e) fold[fft_out_index<NC, ORD>(t, e)] = tot[e] + ACC(run[e]);
  lds_barrier();
  if (active) {
    for (int k = t; k <= NC / 2; k += NT) {
      const ACC s = (fold[k] + fold[(NC - k) & (NC - 1)]) * ACC(0.5);
      const ACC ck = (k == 0 || k == NC / 2) ? ACC(1) : ACC(2);
      out[k] = float(s * ck * ACC(norm));
    }
  }
}

}  // namespace gw
