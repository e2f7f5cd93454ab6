"""Frequency-domain plus/cross waveforms (oracle side).

Section 3.1 of the paper generates aligned-spin inspiral-merger-ringdown
waveforms: a TaylorF2 inspiral phase to 3.5PN order (it cites the review of
Buonanno, Iyer, Ochsner, Pan & Sathyaprakash 2009) joined to a merger and
ringdown ansatz fitted to numerical relativity (IMRPhenomD).  The fitted
IMRPhenomD coefficient tables are not given in the paper, so two models are
defined here:

TaylorF2 (approximant 0).  With v = (pi M f)^(1/3), eta = q/(1+q)^2,
delta_m = (1-q)/(1+q), chi_s = (chi1+chi2)/2, chi_a = (chi1-chi2)/2:

  P(f)   = 3 / (128 eta v^5) * sum_k psi_k v^k                 (k = 0..7)
  Psi(f) = P(f) - phi_c - pi/4
  psi_0 = 1, psi_1 = 0
  psi_2 = 3715/756 + 55 eta/9
  psi_3 = -16 pi + (113/3) delta_m chi_a + (113/3 - 76 eta/3) chi_s
  psi_4 = 15293365/508032 + 27145 eta/504 + 3085 eta^2/72
          - (395/4) eta chi1 chi2
  psi_5 = pi (38645/756 - 65 eta/9) (1 + 3 ln(v / v_lso)),  v_lso = 6^(-1/2)
  psi_6 = 11583231236531/4694215680 - 640 pi^2/3 - (6848/21)(gamma_E + ln 4v)
          + (-15737765635/3048192 + 2255 pi^2/12) eta
          + 76055 eta^2/1728 - 127825 eta^3/1296
  psi_7 = pi (77096675/254016 + 378515 eta/1512 - 74045 eta^2/756)
  spin terms: 1.5PN spin-orbit and the 2PN spin1-spin2 term only.
  amplitude A(f) = S * sqrt(5/24) pi^(-2/3) (G M_c/c^3)^(5/6) / (D_L/c) f^(-7/6)
  with S = 2**70 (an exact power-of-two scale that keeps PSD values inside
  binary32 range; whitened output does not depend on it).
  h+ = A (1 + cos^2 iota)/2 exp(-i Psi),   hx = -i A cos(iota) exp(-i Psi)
  nonzero for f_min <= f < f_ISCO = 1/(6^(3/2) pi M).

IMR-form (approximant 1), a closed-form inspiral-merger-ringdown model:
  remnant spin a_f (Rezzolla et al. 2008 aligned-spin fit, clamped to
  [-0.99, 0.99]); radiated energy E_rad (non-spinning polynomial in eta);
  M_f = M (1 - E_rad); fundamental l = m = 2 quasi-normal mode from the
  Berti, Cardoso & Will 2006 fit: M_f omega = 1.5251 - 1.1568 (1-a_f)^0.1292,
  Q = 0.7 + 1.4187 (1-a_f)^-0.4990, f_RD = omega/(2 pi), f_damp = f_RD/(2Q).
  Phase: P_TF2 for f < f_t = f_RD/2; above, b0 + b1 f + atan((f-f_RD)/f_damp)
  (the phase of a damped sinusoid's transform), b0, b1 fixed by value and
  slope continuity at f_t.  Amplitude: A(f) below f_t;
  A(f_t)(f/f_t)^(-2/3) on [f_t, f_RD); then that value at f_RD times the
  Lorentzian f_damp^2/((f-f_RD)^2 + f_damp^2).  Cut-off f < 0.2/M.

Sine-Gaussian burst (approximant 2; the burst morphology section 7 names as
an extension), central frequency f0, quality Q, root-sum-square strain hrss,
inclination-like polarisation angle iota, phase phi0, peak at t0 = 0:
  h+(t) = A (1 + cos^2 iota)/2 exp(-t^2/tau^2) cos(2 pi f0 t + phi0)
  hx(t) = A cos(iota) exp(-t^2/tau^2) sin(2 pi f0 t + phi0)
  tau = Q / (sqrt(2) pi f0),  A = S hrss / sqrt(tau sqrt(pi/2))
(so that the integral of h+^2 + hx^2 is (S hrss)^2 at iota = 0).  With
G(x) = (sqrt(pi) tau / 2) exp(-pi^2 tau^2 x^2) the transform is
  h+ = A (1 + cos^2 iota)/2 [e^{i phi0} G(f - f0) + e^{-i phi0} G(f + f0)]
  hx = A cos(iota) [-i e^{i phi0} G(f - f0) + i e^{-i phi0} G(f + f0)]
nonzero for f >= f_min, f > 0 (no cut-off).

Pins: the TaylorF2 phase is tied to the post-Newtonian energy and flux
through the stationary-phase relation dPsi/df = 2 pi t(f); the amplitude to
the stationary-phase transform of the quadrupole chirp; the remnant and
ringdown fits to published numerical-relativity and black-hole perturbation
values; continuity of the IMR joins.  Fidelity to IMRPhenomD itself: parity
unpinned (its calibration tables and LALSimulation are not available).
"""

import math

import numpy as np

MSUN_SEC = 4.925490947641267e-6          # G Msun / c^3 [s]
MPC_SEC = 3.085677581491367e22 / 299792458.0   # 1 Mpc / c [s]
STRAIN_SCALE = 2.0 ** 70
GAMMA_E = 0.5772156649015329


def mass_terms(mc, q):
    eta = q / (1.0 + q) ** 2
    M = mc * eta ** (-0.6)
    return eta, M, M * MSUN_SEC


def pn_coefficients(eta, q, chi1, chi2):
    """psi_k for k = 0..7 as (constant, log) pairs: psi_k = c + l * ln(v)."""
    dm = (1.0 - q) / (1.0 + q)
    chis = 0.5 * (chi1 + chi2)
    chia = 0.5 * (chi1 - chi2)
    pi = math.pi
    c = [0.0] * 8
    lg = [0.0] * 8
    c[0] = 1.0
    c[2] = 3715.0 / 756.0 + 55.0 * eta / 9.0
    c[3] = (-16.0 * pi + (113.0 / 3.0) * dm * chia
            + (113.0 / 3.0 - 76.0 * eta / 3.0) * chis)
    c[4] = (15293365.0 / 508032.0 + 27145.0 * eta / 504.0
            + 3085.0 * eta ** 2 / 72.0 - 10.0 * (79.0 / 8.0) * eta * chi1 * chi2)
    p5 = pi * (38645.0 / 756.0 - 65.0 * eta / 9.0)
    v_lso = 6.0 ** -0.5
    # psi5 (1 + 3 ln(v/v_lso)) = psi5 (1 - 3 ln v_lso) + 3 psi5 ln v
    c[5] = p5 * (1.0 - 3.0 * math.log(v_lso))
    lg[5] = 3.0 * p5
    c6 = (11583231236531.0 / 4694215680.0 - 640.0 * pi ** 2 / 3.0
          - (6848.0 / 21.0) * GAMMA_E
          + (-15737765635.0 / 3048192.0 + 2255.0 * pi ** 2 / 12.0) * eta
          + 76055.0 * eta ** 2 / 1728.0 - 127825.0 * eta ** 3 / 1296.0)
    # -(6848/21) ln(4v) = -(6848/21) ln 4 - (6848/21) ln v
    c[6] = c6 - (6848.0 / 21.0) * math.log(4.0)
    lg[6] = -(6848.0 / 21.0)
    c[7] = pi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0
                 - 74045.0 * eta ** 2 / 756.0)
    return c, lg


def taylorf2_phase(f, mc, q, chi1, chi2, pn_terms=8):
    """Intrinsic TaylorF2 phase P(f) (no phi_c, no pi/4, t_c = 0)."""
    f = np.asarray(f, dtype=np.float64)
    eta, _, Ms = mass_terms(mc, q)
    c, lg = pn_coefficients(eta, q, chi1, chi2)
    v = np.cbrt(math.pi * Ms * f)
    lnv = np.log(v)
    s = np.zeros_like(v)
    for k in range(pn_terms):
        s = s + (c[k] + lg[k] * lnv) * v ** k
    return 3.0 / (128.0 * eta * v ** 5) * s


def taylorf2_phase_derivative(f, mc, q, chi1, chi2):
    """dP/df of the full 3.5PN TaylorF2 phase, analytically."""
    f = np.asarray(f, dtype=np.float64)
    eta, _, Ms = mass_terms(mc, q)
    c, lg = pn_coefficients(eta, q, chi1, chi2)
    v = np.cbrt(math.pi * Ms * f)
    lnv = np.log(v)
    # P = 3/(128 eta) sum_k (c_k + l_k ln v) v^(k-5)
    dPdv = np.zeros_like(v)
    for k in range(8):
        dPdv = dPdv + ((k - 5) * (c[k] + lg[k] * lnv) + lg[k]) * v ** (k - 6)
    dPdv *= 3.0 / (128.0 * eta)
    return dPdv * v / (3.0 * f)


def newtonian_amplitude(f, mc, dl):
    """A(f) including the 2**70 strain scale, in seconds (CT Fourier units)."""
    f = np.asarray(f, dtype=np.float64)
    mcs = mc * MSUN_SEC
    dls = dl * MPC_SEC
    return (STRAIN_SCALE * math.sqrt(5.0 / 24.0) * math.pi ** (-2.0 / 3.0)
            * mcs ** (5.0 / 6.0) / dls * f ** (-7.0 / 6.0))


def remnant(q, chi1, chi2):
    """(a_f, E_rad) of the project's IMR-form model."""
    eta = q / (1.0 + q) ** 2
    a_tot = (chi1 + chi2 * q * q) / (1.0 + q * q)
    af = (a_tot - 0.1229 * a_tot ** 2 * eta + 0.4537 * a_tot * eta ** 2
          - 2.8904 * a_tot * eta + 2.0 * math.sqrt(3.0) * eta
          - 3.5171 * eta ** 2 + 2.5763 * eta ** 3)
    af = min(max(af, -0.99), 0.99)
    erad = (0.0559745 * eta + 0.580951 * eta ** 2 - 0.960673 * eta ** 3
            + 3.35241 * eta ** 4)
    return af, erad


def ringdown_frequencies(mc, q, chi1, chi2):
    """(f_RD, f_damp) in Hz for the l = m = 2, n = 0 mode."""
    _, _, Ms = mass_terms(mc, q)
    af, erad = remnant(q, chi1, chi2)
    Mf = Ms * (1.0 - erad)
    omega = 1.5251 - 1.1568 * (1.0 - af) ** 0.1292
    Q = 0.7 + 1.4187 * (1.0 - af) ** (-0.4990)
    f_rd = omega / (2.0 * math.pi * Mf)
    return f_rd, f_rd / (2.0 * Q)


def imr_form_model(f, mc, q, chi1, chi2, dl):
    """(amplitude A(f), intrinsic phase P(f)) of the IMR-form model."""
    f = np.asarray(f, dtype=np.float64)
    f_rd, f_damp = ringdown_frequencies(mc, q, chi1, chi2)
    f_t = 0.5 * f_rd
    P_t = float(taylorf2_phase(f_t, mc, q, chi1, chi2))
    dP_t = float(taylorf2_phase_derivative(f_t, mc, q, chi1, chi2))
    x_t = (f_t - f_rd) / f_damp
    b1 = dP_t - (1.0 / f_damp) / (1.0 + x_t * x_t)
    b0 = P_t - b1 * f_t - math.atan(x_t)
    ins = f < f_t
    phase = np.where(ins, taylorf2_phase(np.where(ins, f, f_t), mc, q, chi1, chi2),
                     b0 + b1 * f + np.arctan((f - f_rd) / f_damp))
    A_t = float(newtonian_amplitude(f_t, mc, dl))
    A_rd = A_t * (f_rd / f_t) ** (-2.0 / 3.0)
    amp = np.where(ins, newtonian_amplitude(np.where(ins, f, f_t), mc, dl),
                   np.where(f < f_rd, A_t * (f / f_t) ** (-2.0 / 3.0),
                            A_rd * f_damp ** 2 / ((f - f_rd) ** 2 + f_damp ** 2)))
    return amp, phase


def sine_gaussian(f, f0, Q, hrss, iota, phi0, f_min):
    """(h+, hx) complex128 of the sine-Gaussian burst on frequencies f (t0 = 0)."""
    f = np.asarray(f, dtype=np.float64)
    tau = Q / (math.sqrt(2.0) * math.pi * f0)
    A = STRAIN_SCALE * hrss / math.sqrt(tau * math.sqrt(math.pi / 2.0))
    G = lambda x: 0.5 * math.sqrt(math.pi) * tau * np.exp(-(math.pi * tau * x) ** 2)
    em = np.exp(1j * phi0) * G(f - f0)
    ep = np.exp(-1j * phi0) * G(f + f0)
    ci = math.cos(iota)
    band = (f >= f_min) & (f > 0)
    hp = np.where(band, A * 0.5 * (1.0 + ci * ci) * (em + ep), 0.0)
    hc = np.where(band, A * ci * (-1j * em + 1j * ep), 0.0)
    return hp.astype(np.complex128), hc.astype(np.complex128)


def frequency_cutoff(approximant, mc, q):
    _, _, Ms = mass_terms(mc, q)
    if approximant == 0:
        return 1.0 / (6.0 ** 1.5 * math.pi * Ms)
    return 0.2 / Ms


def fd_waveform(f, approximant, mc, q, chi1, chi2, dl, iota, phic, f_min):
    """(h+, hx) complex128 on the frequency array f (t_c = 0).

    Zero outside f_min <= f < f_cut; callers zero DC and Nyquist themselves.
    """
    f = np.asarray(f, dtype=np.float64)
    f_cut = frequency_cutoff(approximant, mc, q)
    band = (f >= f_min) & (f < f_cut) & (f > 0)
    fb = np.where(band, f, f_min if f_min > 0 else 1.0)
    if approximant == 0:
        amp = newtonian_amplitude(fb, mc, dl)
        P = taylorf2_phase(fb, mc, q, chi1, chi2)
    else:
        amp, P = imr_form_model(fb, mc, q, chi1, chi2, dl)
    psi = P - phic - math.pi / 4.0
    ci = math.cos(iota)
    e = np.exp(-1j * psi)
    hp = np.where(band, amp * 0.5 * (1.0 + ci * ci) * e, 0.0)
    hc = np.where(band, -1j * amp * ci * e, 0.0)
    return hp.astype(np.complex128), hc.astype(np.complex128)
