// Block-level FFT for gfx950: one workgroup transforms NC complex points,
// each of NT = NC/16 threads holding 16 of them in registers.
//
// Structure: Stockham auto-sort radix-R passes (radix 16 first, then 16s,
// then one 2/4/8 pass when NC is not a power of 16).  Data is exchanged
// between passes through LDS, in separate real/imaginary planes padded (see
// pad_at) so that each pass's reads and writes are free of bank conflicts.
//
// Register layout of a thread t:
//   before the first pass   v[r]     = x[t + NT*r]                (r < 16)
//   after the last pass     v[m*R+r] = X[t + NT*m + r*NC/R]       (R = last radix)
// A thread therefore reads and writes coalesced global memory at both ends,
// with no transpose.
#pragma once
#include <hip/hip_runtime.h>

namespace gw {

template <class T> struct cpx { T x, y; };

template <class T> __device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T> __device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T> __device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
template <class T> __device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by DIR*i (DIR = -1: by -i, DIR = +1: by +i)
template <int DIR, class T> __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}
// a * w for DIR = -1, a * conj(w) for DIR = +1 (w is a forward twiddle)
template <int DIR, class T> __device__ __forceinline__ cpx<T> twmul(cpx<T> a, cpx<T> w) {
  if constexpr (DIR < 0) return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
  else return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

// Returns p unchanged, but the compiler can no longer prove two loads through
// it the same: table loads stay next to the transform that uses them instead
// of being shared with (and kept live across) other transforms of the same
// kernel or loop iterations.  p points to global memory and is laundered as a
// global pointer, so that loads through it remain global loads: through a
// generic pointer they would become flat loads, which also count against the
// LDS wait counter and make every LDS barrier wait for them.
template <class T>
__device__ __forceinline__ const T* opaque(const T* p) {
  typedef const __attribute__((address_space(1))) T* gptr;
  gptr g = (gptr)p;
  asm volatile("" : "+s"(g));
  return (const T*)g;
}

// p (uniform over the workgroup) unchanged, but addresses derived from it are
// not shared with (and kept live across) other phases of the kernel that use
// the same pointer.
template <class T>
__device__ __forceinline__ T* fresh(T* p) {
  typedef __attribute__((address_space(1))) T* gptr;
  const uint64_t u = reinterpret_cast<uint64_t>(p);
  // readfirstlane works on (signed) int: widen its result as unsigned, or a
  // low word with the top bit set would sign-extend into the high word
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(u))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(u >> 32))));
  const uint64_t s = uint64_t(lo) | (uint64_t(hi) << 32);
  gptr g = (gptr)reinterpret_cast<T*>(s);
  asm volatile("" : "+s"(g));
  return (T*)g;
}

// The lane index t, unchanged, as a value the compiler cannot prove equal to
// t elsewhere: index and LDS-address arithmetic of one phase is then not
// shared with (and kept live across) the other phases.
__device__ __forceinline__ int fresh_lane(int t) {
  asm volatile("" : "+v"(t));
  return t;
}

// Workgroup barrier for the LDS exchanges: waits only for this wave's LDS
// operations (lgkmcnt) before s_barrier.  __syncthreads() also waits for
// every outstanding global load, which would expose the latency of loads
// issued ahead of time (next segment, next pass's twiddles) at each pass.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// LDS padding.  LDS has 32 banks of 4 bytes and serves a wavefront access to
// binary32 words 32 lanes per cycle.  In a binary32 plane, index i is stored
// at i + C (i >> 5): a run of 32 consecutive indices (every read of a pass,
// every natural-order access) then covers 32 banks for any C, and C is chosen
// per exchange for the stores of the pass that writes it (FftPad).  binary64
// planes keep one pad element every 16.
// pad_at(base, off) is the padded index of base + off for the index splits
// used here, where (base mod 32) + (off mod 32) < 32, so that the padding of
// base and of the compile-time offset off add up.
template <class T, int C> __device__ __forceinline__ int pad_at(int base, int off) {
  if constexpr (sizeof(T) == 4) {
    return base + C * (base >> 5) + off + C * (off >> 5);
  } else {
    const int i = base + off;
    return i + (i >> 4);
  }
}
// natural-order layout (C = 1)
template <class T> __device__ __forceinline__ int lpad(int i) { return pad_at<T, 1>(i, 0); }
// padding never moves an index beyond NC + NC/16 (C <= 2 in every plan)
template <int NC> struct LdsSize { static constexpr int value = NC + NC / 16; };

// a * exp(DIR * 2 pi i m / 16), m a compile-time constant
template <int M, int DIR, class T> __device__ __forceinline__ cpx<T> w16(cpx<T> a) {
  constexpr int m = ((M % 16) + 16) % 16;
  constexpr T C1 = T(0.92387953251128675613), S1 = T(0.38268343236508977173);
  constexpr T R2 = T(0.70710678118654752440);
  if constexpr (m == 0) return a;
  else if constexpr (m == 4) return mul_i<DIR>(a);
  else if constexpr (m == 8) return {-a.x, -a.y};
  else if constexpr (m == 12) return mul_i<-DIR>(a);
  else if constexpr (m == 2 || m == 6 || m == 10 || m == 14) {
    // exp(DIR i pi m/8) = (cx + DIR i sy)/sqrt2 with cx, sy in {+1,-1}
    constexpr T cx = (m == 2 || m == 14) ? T(1) : T(-1);
    constexpr T sy = (m == 2 || m == 6) ? T(1) : T(-1);
    constexpr T s = T(DIR) * sy;
    return {(a.x * cx - a.y * s) * R2, (a.y * cx + a.x * s) * R2};
  } else {
    // angle = quad * pi/2 + phi, phi = (m & 3) * pi/8 with (m & 3) in {1, 3}
    constexpr int q = m & 3;
    constexpr T cphi = (q == 1) ? C1 : S1, sphi = (q == 1) ? S1 : C1;
    constexpr int quad = m >> 2;
    constexpr T c = quad == 0 ? cphi : quad == 1 ? -sphi : quad == 2 ? -cphi : sphi;
    constexpr T sn = quad == 0 ? sphi : quad == 1 ? cphi : quad == 2 ? -sphi : -cphi;
    constexpr T s = T(DIR) * sn;
    return {a.x * c - a.y * s, a.y * c + a.x * s};
  }
}

template <int DIR, class T> __device__ __forceinline__ void dft2(cpx<T>* a) {
  cpx<T> t0 = a[0];
  a[0] = cadd(t0, a[1]);
  a[1] = csub(t0, a[1]);
}

template <int DIR, class T> __device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  cpx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}
template <int DIR, class T> __device__ __forceinline__ void dft4(cpx<T>* a) { dft4<DIR>(a[0], a[1], a[2], a[3]); }

template <int DIR, class T> __device__ __forceinline__ void dft8(cpx<T>* a) {
  cpx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cpx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  o1 = w16<2, DIR>(o1);
  o2 = w16<4, DIR>(o2);
  o3 = w16<6, DIR>(o3);
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// 16-point DFT as 4 x 4: X[k1 + 4 k2] = sum_n2 W4^(n2 k2) W16^(n2 k1) DFT4_n1(a[4 n1 + n2])[k1]
template <int DIR, class T> __device__ __forceinline__ void dft16(cpx<T>* a) {
  dft4<DIR>(a[0], a[4], a[8], a[12]);
  dft4<DIR>(a[1], a[5], a[9], a[13]);
  dft4<DIR>(a[2], a[6], a[10], a[14]);
  dft4<DIR>(a[3], a[7], a[11], a[15]);
  // after this, a[n2 + 4 k1] holds Y_{n2}[k1]
  a[5] = w16<1, DIR>(a[5]);
  a[9] = w16<2, DIR>(a[9]);
  a[13] = w16<3, DIR>(a[13]);
  a[6] = w16<2, DIR>(a[6]);
  a[10] = w16<4, DIR>(a[10]);
  a[14] = w16<6, DIR>(a[14]);
  a[7] = w16<3, DIR>(a[7]);
  a[11] = w16<6, DIR>(a[11]);
  a[15] = w16<9, DIR>(a[15]);
  dft4<DIR>(a[0], a[1], a[2], a[3]);
  dft4<DIR>(a[4], a[5], a[6], a[7]);
  dft4<DIR>(a[8], a[9], a[10], a[11]);
  dft4<DIR>(a[12], a[13], a[14], a[15]);
  // now a[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4x4 index
  cpx<T> t;
  t = a[1]; a[1] = a[4]; a[4] = t;
  t = a[2]; a[2] = a[8]; a[8] = t;
  t = a[3]; a[3] = a[12]; a[12] = t;
  t = a[6]; a[6] = a[9]; a[9] = t;
  t = a[7]; a[7] = a[13]; a[13] = t;
  t = a[11]; a[11] = a[14]; a[14] = t;
}

template <int R, int DIR, class T> __device__ __forceinline__ void dftR(cpx<T>* a) {
  if constexpr (R == 16) dft16<DIR>(a);
  else if constexpr (R == 8) dft8<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a);
  else dft2<DIR>(a);
}

// Radix plan: NP16 radix-16 passes and, when NC is not a power of 16, one
// pass of radix RL.  ORD 0 runs the small pass last, ORD 1 first (the two
// orderings trade LDS access patterns; an autotuner picks one per size).
template <int NC> struct FftPlan {
  static constexpr int NP16 = (NC >= 65536) ? 4 : (NC >= 4096) ? 3 : (NC >= 256) ? 2 : 1;
  static constexpr int RL = NC / (NP16 == 4 ? 65536 : NP16 == 3 ? 4096 : NP16 == 2 ? 256 : 16);
  static constexpr int NPASS = NP16 + (RL > 1 ? 1 : 0);
  static constexpr int NT = NC / 16;
  static_assert(NC == 1024 || NC == 2048 || NC == 4096 || NC == 8192 || NC == 16384, "unsupported FFT size");
};

template <int NC, int PASS, int ORD = 0> struct PassInfo {
  using P = FftPlan<NC>;
  static constexpr bool SMALL_FIRST = (ORD == 1) && (P::RL > 1);
  static constexpr int R = SMALL_FIRST ? (PASS == 0 ? P::RL : 16) : ((PASS < P::NP16) ? 16 : P::RL);
  static constexpr int p16 = SMALL_FIRST ? (PASS == 0 ? 0 : PASS - 1) : PASS;
  static constexpr int NS = SMALL_FIRST ? (PASS == 0 ? 1 : P::RL * (p16 == 0 ? 1 : p16 == 1 ? 16 : 256))
                                        : ((PASS == 0) ? 1 : (PASS == 1) ? 16 : (PASS == 2) ? 256 : 4096);
};

template <int NC, int ORD> struct PlanEnds {
  static constexpr int RFIRST = PassInfo<NC, 0, ORD>::R;
  static constexpr int RLAST = PassInfo<NC, FftPlan<NC>::NPASS - 1, ORD>::R;
};

// Padding constant of the exchange written by pass PASS.  Its stores form,
// per run of 32 lanes, 32/NS groups of NS consecutive indices NS*R apart
// (NS < 32) or one run of 32 consecutive indices (NS >= 32); C = 32/R puts
// the groups on disjoint banks.  With NS = 1 the stores are R apart and C = 1
// spreads them.
template <int NC, int PASS, int ORD> struct FftPad {
  static constexpr int R = PassInfo<NC, PASS, ORD>::R, NS = PassInfo<NC, PASS, ORD>::NS;
  static constexpr int C = (NS == 1 || NS >= 32) ? 1 : 32 / R;
  static_assert(NS == 1 || NS >= 32 || NS * R >= 32, "groups must be 32 words apart");
  static_assert(C <= 2, "padding must fit in LdsSize");
};

// Register slot of input x[t + NT*j] (j < 16) before the first pass.
template <int NC, int ORD = 0> __host__ __device__ constexpr int fft_in_slot(int j) {
  constexpr int R0 = PlanEnds<NC, ORD>::RFIRST, NB = 16 / R0;
  return (j % NB) * R0 + j / NB;
}

// Output bin held in element e after the last pass.
template <int NC, int ORD = 0> __device__ __forceinline__ int fft_out_index(int t, int e) {
  constexpr int R = PlanEnds<NC, ORD>::RLAST, NT = FftPlan<NC>::NT;
  return t + NT * (e / R) + (e % R) * (NC / R);
}

// Twiddle providers: return the forward twiddle exp(-2 pi i r k / (NS R)).
// Table form: tw[n] = exp(-2 pi i n / NC).
template <class T, int NC, int ORD = 0> struct TableTwiddle {
  const cpx<T>* __restrict__ tw;
  template <int PASS> __device__ __forceinline__ cpx<T> get(int m, int r, int k) const {
    constexpr int R = PassInfo<NC, PASS, ORD>::R, NS = PassInfo<NC, PASS, ORD>::NS;
    return tw[(r * k) * (NC / (NS * R))];
  }
};

// Table form with fewer loads: per butterfly, W, W^2, W^4 and W^8 come from
// the table and the other powers are products of at most three of them
// (rounding error a few ulp).  Used where twiddle loads would otherwise
// dominate the load count and register pressure.
// block_fft requests each pass's table values during the pass before it
// (Base, load), so that their latency is hidden behind that pass.
template <class T, int NC, int ORD = 0> struct PowTwiddle {
  const cpx<T>* __restrict__ tw;
  // table values of one pass: per butterfly m, W^(2^l) for l < NL
  template <int PASS> struct Base {
    static constexpr int R = PassInfo<NC, PASS, ORD>::R, NS = PassInfo<NC, PASS, ORD>::NS, NB = 16 / R;
    static constexpr int NL = (NS == 1) ? 0 : (R >= 16) ? 4 : (R >= 8) ? 3 : (R >= 4) ? 2 : 1;
    cpx<T> b[NB][NL > 0 ? NL : 1];
  };
  template <int PASS> __device__ __forceinline__ Base<PASS> load(int t) const {
    using B = Base<PASS>;
    constexpr int NT = NC / 16, STEP = NC / (B::NS * B::R);
    B q;
#pragma unroll
    for (int m = 0; m < B::NB; ++m) {
      const int i1 = ((t + NT * m) & (B::NS - 1)) * STEP;
#pragma unroll
      for (int l = 0; l < B::NL; ++l) q.b[m][l] = tw[(1 << l) * i1];
    }
    return q;
  }
  // powers W^1 .. W^(R-1) from W, W^2, W^4, W^8
  template <int R> __device__ static __forceinline__ void expand(const cpx<T>* b, cpx<T>* w) {
    w[1] = b[0];
    if constexpr (R >= 4) {
      w[2] = b[1];
      w[3] = cmul(w[2], w[1]);
    }
    if constexpr (R >= 8) {
      w[4] = b[2];
      w[5] = cmul(w[4], w[1]);
      w[6] = cmul(w[4], w[2]);
      w[7] = cmul(w[6], w[1]);
    }
    if constexpr (R >= 16) {
      w[8] = b[3];
      w[9] = cmul(w[8], w[1]);
      w[10] = cmul(w[8], w[2]);
      w[11] = cmul(w[10], w[1]);
      w[12] = cmul(w[8], w[4]);
      w[13] = cmul(w[12], w[1]);
      w[14] = cmul(w[12], w[2]);
      w[15] = cmul(w[14], w[1]);
    }
  }
};

template <class TW> struct TwiddleIsPow { static constexpr bool value = false; };
template <class T, int NC, int ORD> struct TwiddleIsPow<PowTwiddle<T, NC, ORD>> { static constexpr bool value = true; };

// One Stockham pass.  READ: take input from LDS (else registers already hold
// it).  WRITE: scatter the output to LDS (else it stays in registers in the
// final layout).  A barrier separates this pass's LDS reads from its writes;
// the caller must ensure the LDS buffer is free before a pass that WRITEs
// without READing.  pre: the pass's PowTwiddle table values, already loaded.
template <class T, int NC, int PASS, int DIR, bool READ, bool WRITE, int ORD, class TW>
__device__ __forceinline__ void fft_pass(cpx<T>* v, T* sre, T* sim, int t, const TW& tw,
                                         const cpx<T>* pre = nullptr) {
  constexpr int R = PassInfo<NC, PASS, ORD>::R, NS = PassInfo<NC, PASS, ORD>::NS;
  constexpr int NT = NC / 16, NB = 16 / R, STRIDE = NC / R;
  // layout of the buffer read: written by the previous pass, or natural order
  constexpr int CR = (PASS == 0) ? 1 : FftPad<NC, (PASS > 0 ? PASS - 1 : 0), ORD>::C;
  constexpr int CW = FftPad<NC, PASS, ORD>::C;
  if constexpr (READ) {
#pragma unroll
    for (int m = 0; m < NB; ++m) {
      const int j = t + NT * m;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = pad_at<T, CR>(j, r * STRIDE);
        v[m * R + r] = {sre[i], sim[i]};
      }
    }
  }
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    const int j = t + NT * m;
    if constexpr (NS > 1) {
      const int k = j & (NS - 1);
      if constexpr (TwiddleIsPow<TW>::value) {
        cpx<T> w[R];
        TW::template expand<R>(pre + m * TW::template Base<PASS>::NL, w);
#pragma unroll
        for (int r = 1; r < R; ++r) v[m * R + r] = twmul<DIR>(v[m * R + r], w[r]);
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) v[m * R + r] = twmul<DIR>(v[m * R + r], tw.template get<PASS>(m, r, k));
      }
    }
    dftR<R, DIR>(v + m * R);
  }
  if constexpr (WRITE) {
    if constexpr (READ) lds_barrier();
#pragma unroll
    for (int m = 0; m < NB; ++m) {
      const int j = t + NT * m;
      const int k = j & (NS - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = pad_at<T, CW>(base, r * NS);
        sre[i] = v[m * R + r].x;
        sim[i] = v[m * R + r].y;
      }
    }
    lds_barrier();
  }
}

// Whole transform.  FIRST_FROM_LDS: the first pass reads its input from LDS
// in natural order (else v holds it: x[t + NT j] in slot fft_in_slot(j)).
// The result stays in registers in the final layout (see fft_out_index).
// Ends with LDS still being read by other threads: barrier before reusing it.
template <class T, int NC, int DIR, bool FIRST_FROM_LDS, int ORD = 0, class TW>
__device__ __forceinline__ void block_fft(cpx<T>* v, T* sre, T* sim, int t, const TW& tw) {
  using P = FftPlan<NC>;
  if constexpr (TwiddleIsPow<TW>::value) {
    // each pass's table values are requested before the pass ahead of it
    const auto b1 = tw.template load<1>(t);
    fft_pass<T, NC, 0, DIR, FIRST_FROM_LDS, true, ORD>(v, sre, sim, t, tw);
    const auto b2 = tw.template load<2>(t);
    fft_pass<T, NC, 1, DIR, true, true, ORD>(v, sre, sim, t, tw, &b1.b[0][0]);
    if constexpr (P::NPASS == 3) {
      fft_pass<T, NC, 2, DIR, true, false, ORD>(v, sre, sim, t, tw, &b2.b[0][0]);
    } else {
      const auto b3 = tw.template load<3>(t);
      fft_pass<T, NC, 2, DIR, true, true, ORD>(v, sre, sim, t, tw, &b2.b[0][0]);
      fft_pass<T, NC, 3, DIR, true, false, ORD>(v, sre, sim, t, tw, &b3.b[0][0]);
    }
  } else {
    fft_pass<T, NC, 0, DIR, FIRST_FROM_LDS, true, ORD>(v, sre, sim, t, tw);
    if constexpr (P::NPASS == 3) {
      fft_pass<T, NC, 1, DIR, true, true, ORD>(v, sre, sim, t, tw);
      fft_pass<T, NC, 2, DIR, true, false, ORD>(v, sre, sim, t, tw);
    } else {
      fft_pass<T, NC, 1, DIR, true, true, ORD>(v, sre, sim, t, tw);
      fft_pass<T, NC, 2, DIR, true, true, ORD>(v, sre, sim, t, tw);
      fft_pass<T, NC, 3, DIR, true, false, ORD>(v, sre, sim, t, tw);
    }
  }
}

}  // namespace gw
