// Device-side physics of the generator: counter-based prior draws, the
// per-sample waveform constants, the per-bin waveform phase and amplitude,
// and the detector response.
//
// Waveform models (section 3.1 of the AMPLFI paper uses an aligned-spin
// IMR model whose inspiral is TaylorF2 to 3.5PN order):
//   approximant 0 -- TaylorF2, 3.5PN phase with 1.5PN spin-orbit and 2PN
//     spin1-spin2 terms, Newtonian amplitude, cut at the Schwarzschild ISCO;
//   approximant 1 -- closed-form inspiral-merger-ringdown: TaylorF2 below
//     f_t = f_RD/2, above it b0 + b1 f + atan((f - f_RD)/f_damp) joined with
//     value and slope continuity; power-law then Lorentzian amplitude; ringdown
//     from the remnant (aligned-spin final-spin fit, radiated-energy fit,
//     fundamental l=m=2 quasi-normal-mode fit); cut at f = 0.2/M.
// The phase is evaluated in revolutions; precision mode 1 and 2 keep it in
// binary64 and reduce it modulo one before a binary32 (mode 1) or binary64
// (mode 2) sine/cosine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gw {

// frac(x) in [0, 1)
__device__ __forceinline__ float frac1(float x) { return x - floorf(x); }
__device__ __forceinline__ double frac1(double x) { return x - floor(x); }

// precision-generic math
__device__ __forceinline__ void sincospi_t(float x, float* s, float* c) { sincospif(x, s, c); }
// sin and cos of 2 pi x for x already reduced to [0, 1): the hardware
// sine/cosine take revolutions (max abs error 1.3e-7 measured on gfx950 over
// [0, 1)); binary64 uses the library routine
__device__ __forceinline__ void sincos_rev(float x, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(x);
  *c = __builtin_amdgcn_cosf(x);
}
__device__ __forceinline__ void sincos_rev(double x, double* s, double* c) { sincospi(2.0 * x, s, c); }
__device__ __forceinline__ void sincospi_t(double x, double* s, double* c) { sincospi(x, s, c); }
__device__ __forceinline__ float sinpi_t(float x) { return sinpif(x); }
__device__ __forceinline__ double sinpi_t(double x) { return sinpi(x); }
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }
// reciprocals: binary32 hardware approximation (about 1 ulp); binary64
// hardware seed refined by two Newton steps to full precision
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float pow_t(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double pow_t(double x, double y) { return pow(x, y); }

constexpr double kPi = 3.14159265358979323846;
constexpr double kMsunSec = 4.925490947641267e-6;                 // G Msun / c^3
constexpr double kMpcSec = 3.085677581491367e22 / 299792458.0;    // Mpc / c
constexpr double kClight = 299792458.0;
constexpr double kStrainScale = 1180591620717411303424.0;         // 2^70
constexpr double kGammaE = 0.5772156649015329;

struct DetGeom {
  double D[6];  // detector tensor xx, xy, xz, yy, yz, zz
  double r[3];  // vertex [m], Earth-fixed
};

struct DevCfg {
  int n_det, N, F, P, L, S, K, Fw, ratio, log2_ratio, approximant, precision, kmin;
  int ord_win, ord_welch;  // FFT radix order of the window and Welch kernels (0: small radix last)
  int occ_welch;           // waves per SIMD the Welch kernel is compiled for (2 or 3)
  double fs, T, invT, f_min, inv_ratio;
  double mc[2], q[2], chi[2], dl[2];
  double f0r[2], Qr[2], hrssr[2];  // sine-Gaussian prior ranges (approximant 2)
  DetGeom det[4];
};

// ---------------------------------------------------------------- Philox
struct U4 { uint32_t a, b, c, d; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.a, hi0 = __umulhi(0xD2511F53u, c.a);
    const uint32_t lo1 = 0xCD9E8D57u * c.c, hi1 = __umulhi(0xCD9E8D57u, c.c);
    c = U4{hi1 ^ c.b ^ k0, lo1, hi0 ^ c.d ^ k1, lo0};
  }
  return c;
}

// binary64 uniform in (0, 1) from the first two words
__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t index, uint32_t stream,
                                                 uint32_t sub = 0u) {
  U4 o = philox4x32_10(U4{uint32_t(index), uint32_t(index >> 32), stream, sub},
                       uint32_t(seed), uint32_t(seed >> 32));
  return (double(o.a >> 5) * 67108864.0 + double(o.b >> 6) + 0.5) * 0x1p-53;
}

// ------------------------------------------------------- waveform constants
struct WfScalars {
  double v1, lnv1;      // v_k = v1 k^(1/3);  ln v_k = lnv1 + ln(k)/3
  double a[8];          // phase polynomial in revolutions: sum (a_k + b_k ln v) v^(k-5)
  double b5, b6;
  double pconst;        // (-phi_c - pi/4) / (2 pi)
  double A0T;           // amplitude A(f_k) = A0T k^(-7/6)
  double mr_b0, mr_b1;  // merger-ringdown phase in revolutions: b0 + b1 f + atan(x)/(2 pi)
  double f_rd, inv_fdamp;
  double At, Ard, ft, fdamp2;
  double Apl;           // At (f_t T)^(2/3): power-law amplitude Apl k^(-2/3) between f_t and f_RD
  double cN;            // Newtonian phase in revolutions at bin k: cN k^(-5/3)
  // sine-Gaussian (approximant 2): G(x) = sg_G0 exp(-sg_pt2 x^2), phase phi0 / (2 pi)
  double sg_f0, sg_pt2, sg_G0, sg_rphi;
  int kend, kt, krd;    // band end; first bins with f >= f_t and f >= f_RD
  int cut_nyquist;
  double cosi, tc, ra, dec, psi;
};

// first bin k in [0, kmax] with k/T >= f (k/T formed by a correctly rounded
// division, as the binary64 grid f_k = k/T is formed)
__device__ __forceinline__ int first_bin_at_or_above(double f, double T, int kmax) {
  double x = f * T;
  if (!(x > 0.0)) return 0;
  if (x >= double(kmax)) return kmax;
  int k = int(ceil(x));
  while (k > 0 && double(k - 1) / T >= f) --k;
  while (k < kmax && double(k) / T < f) ++k;
  return k;
}

__device__ __forceinline__ void pn_coefficients(double eta, double q, double chi1, double chi2,
                                                double* c, double* lg) {
  const double dm = (1.0 - q) / (1.0 + q);
  const double chis = 0.5 * (chi1 + chi2), chia = 0.5 * (chi1 - chi2);
  const double pi = kPi;
  for (int k = 0; k < 8; ++k) { c[k] = 0.0; lg[k] = 0.0; }
  c[0] = 1.0;
  c[2] = 3715.0 / 756.0 + 55.0 * eta / 9.0;
  c[3] = -16.0 * pi + (113.0 / 3.0) * dm * chia + (113.0 / 3.0 - 76.0 * eta / 3.0) * chis;
  c[4] = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta * eta / 72.0
         - (395.0 / 4.0) * eta * chi1 * chi2;
  const double p5 = pi * (38645.0 / 756.0 - 65.0 * eta / 9.0);
  // psi5 (1 + 3 ln(v / v_lso)), v_lso = 6^(-1/2):  ln v_lso = -ln(6)/2
  c[5] = p5 * (1.0 + 1.5 * log(6.0));
  lg[5] = 3.0 * p5;
  const double c6 = 11583231236531.0 / 4694215680.0 - 640.0 * pi * pi / 3.0
                    - (6848.0 / 21.0) * kGammaE
                    + (-15737765635.0 / 3048192.0 + 2255.0 * pi * pi / 12.0) * eta
                    + 76055.0 * eta * eta / 1728.0 - 127825.0 * eta * eta * eta / 1296.0;
  c[6] = c6 - (6848.0 / 21.0) * log(4.0);
  lg[6] = -(6848.0 / 21.0);
  c[7] = pi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0 - 74045.0 * eta * eta / 756.0);
}

// TaylorF2 intrinsic phase P(f) [rad] and dP/df, full binary64, direct powers
__device__ __forceinline__ void tf2_phase_and_slope(double f, double Ms, double eta, const double* c,
                                                    const double* lg, double* P, double* dP) {
  const double v = cbrt(kPi * Ms * f), lnv = log(v);
  double s = 0.0, ds = 0.0;
  for (int k = 0; k < 8; ++k) {
    const double ck = c[k] + lg[k] * lnv;
    s += ck * pow(v, double(k - 5));
    ds += ((k - 5) * ck + lg[k]) * pow(v, double(k - 6));
  }
  const double pre = 3.0 / (128.0 * eta);
  *P = pre * s;
  *dP = pre * ds * v / (3.0 * f);
}

__device__ __forceinline__ void wf_setup(const double* __restrict__ params, int64_t B, int64_t b,
                                         const DevCfg& cf, WfScalars& w) {
  if (cf.approximant == 2) {
    // sine-Gaussian: rows 0 f0, 1 Q, 2 hrss, 5 iota, 9 phi0, 10 t0
    const double f0 = params[0 * B + b], Q = params[1 * B + b], hrss = params[2 * B + b];
    w.ra = params[6 * B + b];
    w.dec = params[7 * B + b];
    w.psi = params[8 * B + b];
    w.tc = params[10 * B + b];
    w.cosi = cos(params[5 * B + b]);
    const double tau = Q / (sqrt(2.0) * kPi * f0);
    const double A = kStrainScale * hrss / sqrt(tau * sqrt(0.5 * kPi));
    w.sg_f0 = f0;
    w.sg_pt2 = kPi * kPi * tau * tau;
    w.sg_G0 = A * 0.5 * sqrt(kPi) * tau;
    w.sg_rphi = params[9 * B + b] / (2.0 * kPi);
    w.kend = cf.N / 2;
    w.kt = w.krd = w.kend;
    w.cut_nyquist = f0 + 5.0 / (kPi * tau) >= 0.5 * cf.fs ? 1 : 0;
    return;
  }
  const double mc = params[0 * B + b], q = params[1 * B + b];
  const double chi1 = params[2 * B + b], chi2 = params[3 * B + b];
  const double dl = params[4 * B + b], iota = params[5 * B + b];
  w.ra = params[6 * B + b];
  w.dec = params[7 * B + b];
  w.psi = params[8 * B + b];
  const double phic = params[9 * B + b];
  w.tc = params[10 * B + b];
  w.cosi = cos(iota);
  const double eta = q / ((1.0 + q) * (1.0 + q));
  const double M = mc * pow(eta, -0.6);
  const double Ms = M * kMsunSec;
  double c[8], lg[8];
  pn_coefficients(eta, q, chi1, chi2, c, lg);
  const double rev = 3.0 / (128.0 * eta) / (2.0 * kPi);
  for (int k = 0; k < 8; ++k) w.a[k] = rev * c[k];
  w.b5 = rev * lg[5];
  w.b6 = rev * lg[6];
  w.v1 = cbrt(kPi * Ms * cf.invT);
  w.lnv1 = log(w.v1);
  w.cN = w.a[0] / (w.v1 * w.v1 * w.v1 * w.v1 * w.v1);
  w.pconst = (-phic - 0.25 * kPi) / (2.0 * kPi);
  const double A0 = kStrainScale * sqrt(5.0 / 24.0) * pow(kPi, -2.0 / 3.0) *
                    pow(mc * kMsunSec, 5.0 / 6.0) / (dl * kMpcSec);
  w.A0T = A0 * pow(cf.T, 7.0 / 6.0);
  const int knyq = cf.N / 2;
  double f_cut;
  if (cf.approximant == 0) {
    f_cut = 1.0 / (pow(6.0, 1.5) * kPi * Ms);
    w.kend = first_bin_at_or_above(f_cut, cf.T, knyq);
    w.kt = w.kend;
    w.krd = w.kend;
    w.mr_b0 = w.mr_b1 = w.f_rd = w.inv_fdamp = 0.0;
    w.At = w.Ard = w.ft = w.fdamp2 = w.Apl = 0.0;
  } else {
    f_cut = 0.2 / Ms;
    w.kend = first_bin_at_or_above(f_cut, cf.T, knyq);
    // remnant: aligned-spin final-spin fit, non-spinning radiated-energy fit
    const double a_tot = (chi1 + chi2 * q * q) / (1.0 + q * q);
    double af = a_tot - 0.1229 * a_tot * a_tot * eta + 0.4537 * a_tot * eta * eta
                - 2.8904 * a_tot * eta + 2.0 * sqrt(3.0) * eta - 3.5171 * eta * eta
                + 2.5763 * eta * eta * eta;
    af = fmin(fmax(af, -0.99), 0.99);
    const double erad = 0.0559745 * eta + 0.580951 * eta * eta - 0.960673 * eta * eta * eta
                        + 3.35241 * eta * eta * eta * eta;
    const double Mf = Ms * (1.0 - erad);
    const double omega = 1.5251 - 1.1568 * pow(1.0 - af, 0.1292);
    const double Q = 0.7 + 1.4187 * pow(1.0 - af, -0.4990);
    const double f_rd = omega / (2.0 * kPi * Mf);
    const double f_damp = f_rd / (2.0 * Q);
    const double f_t = 0.5 * f_rd;
    double Pt, dPt;
    tf2_phase_and_slope(f_t, Ms, eta, c, lg, &Pt, &dPt);
    const double x_t = (f_t - f_rd) / f_damp;
    const double b1 = dPt - (1.0 / f_damp) / (1.0 + x_t * x_t);
    const double b0 = Pt - b1 * f_t - atan(x_t);
    w.mr_b0 = b0 / (2.0 * kPi);
    w.mr_b1 = b1 / (2.0 * kPi);
    w.f_rd = f_rd;
    w.inv_fdamp = 1.0 / f_damp;
    const double At = A0 * pow(f_t, -7.0 / 6.0);
    w.At = At;
    w.Ard = At * pow(f_rd / f_t, -2.0 / 3.0);
    w.ft = f_t;
    w.fdamp2 = f_damp * f_damp;
    w.Apl = At * pow(f_t * cf.T, 2.0 / 3.0);
    w.kt = min(first_bin_at_or_above(f_t, cf.T, knyq), w.kend);
    w.krd = min(first_bin_at_or_above(f_rd, cf.T, knyq), w.kend);
  }
  w.cut_nyquist = f_cut > 0.5 * cf.fs ? 1 : 0;
}

// Waveform phase in revolutions (without the time shift) at bin k.  TP is
// binary64 for precision modes 1 and 2 and binary32 for mode 0; FULL selects
// a binary64 arctangent for the (bounded) ringdown term (mode 2).
template <class TP, bool FULL>
__device__ __forceinline__ TP wf_phase_rev(const WfScalars& w, int k, double kcbrt, double lnk3, double invT) {
  if (k < w.kt) {
    const TP v = TP(w.v1) * TP(kcbrt);
    const TP lnv = TP(w.lnv1) + TP(lnk3);
    const TP iv = rcp_t(v);
    const TP iv2 = iv * iv;
    const TP iv5 = iv2 * iv2 * iv;
    const TP p = TP(w.a[0]) +
                 v * v * (TP(w.a[2]) +
                          v * (TP(w.a[3]) +
                               v * (TP(w.a[4]) +
                                    v * ((TP(w.a[5]) + TP(w.b5) * lnv) +
                                         v * ((TP(w.a[6]) + TP(w.b6) * lnv) + v * TP(w.a[7]))))));
    return p * iv5;
  }
  const double f = double(k) * invT;
  const double x = (f - w.f_rd) * w.inv_fdamp;
  if constexpr (FULL) return TP(w.mr_b0) + TP(w.mr_b1) * TP(f) + TP(atan(x) * (1.0 / (2.0 * kPi)));
  else return TP(w.mr_b0) + TP(w.mr_b1) * TP(f) + TP(atanf(float(x)) * float(1.0 / (2.0 * kPi)));
}

// Amplitude at bin k: A0T k^(-7/6) below f_t, At (f/f_t)^(-2/3) =
// Apl k^(-2/3) up to f_RD (both from the k^(1/3) table), then the Lorentzian.
template <class TA>
__device__ __forceinline__ TA wf_amplitude(const WfScalars& w, int k, double kcbrt, double invT) {
  if (k < w.kt) return TA(w.A0T) * rsqrt_t(TA(kcbrt)) * rcp_t(TA(k));
  if (k < w.krd) {
    const TA kc = TA(kcbrt);
    return TA(w.Apl) * rcp_t(kc * kc);
  }
  const TA d = TA(double(k) * invT) - TA(w.f_rd);
  return TA(w.Ard) * TA(w.fdamp2) * rcp_t(d * d + TA(w.fdamp2));
}

// -------------------------------------------------------- detector response
struct DetScalars { double fp, fx, tau; };

__device__ __forceinline__ DetScalars det_response(const DetGeom& g, double ra, double dec, double psi, double tc) {
  const double sr = sin(ra), cr = cos(ra), sd = sin(dec), cd = cos(dec);
  const double sp = sin(psi), cp = cos(psi);
  const double et[3] = {sd * cr, sd * sr, -cd};
  const double ep[3] = {-sr, cr, 0.0};
  double p[3], qv[3];
  for (int i = 0; i < 3; ++i) {
    p[i] = cp * et[i] + sp * ep[i];
    qv[i] = -sp * et[i] + cp * ep[i];
  }
  const double* D = g.D;
  const double Dm[3][3] = {{D[0], D[1], D[2]}, {D[1], D[3], D[4]}, {D[2], D[4], D[5]}};
  double fp = 0.0, fx = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      fp += Dm[i][j] * (p[i] * p[j] - qv[i] * qv[j]);
      fx += Dm[i][j] * (p[i] * qv[j] + qv[i] * p[j]);
    }
  const double n[3] = {cd * cr, cd * sr, sd};
  const double dt = -(n[0] * g.r[0] + n[1] * g.r[1] + n[2] * g.r[2]) / kClight;
  return DetScalars{fp, fx, tc + dt};
}

}  // namespace gw
