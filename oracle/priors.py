"""Prior draws (oracle side).

Follows the prior of the paper's Table 1 (section 5): chirp mass and mass
ratio uniform, luminosity distance uniform in volume (density proportional
to D_L^2), inclination with a sine density, right ascension uniform,
declination with a cosine density, coalescence phase uniform on (0, 2*pi),
polarisation angle uniform on (0, pi).  The workload configurations replace
the ranges of Table 1 and add aligned spins (uniform components), which the
paper's section 5 says it leaves out for now.

Readings where the paper is silent:
  * inclination iota stands in for theta_JN (they coincide for aligned spins);
  * right ascension is used as the Earth-fixed longitude (sidereal time 0);
  * coalescence time t_c (seconds from the window start) is uniform on
    [T - 1.5 s, T - 0.5 s): the merger lands 0.5-1.5 s before the window end;
  * the background offset o (first background sample used by the sample,
    identical for every detector) is uniform over every admissible start:
    o = floor(u * (L_bg - P - N + 1)).

Parameter rows (binary64, [12][B]):
  0 M_c [Msun]  1 q = m2/m1  2 chi1  3 chi2  4 D_L [Mpc]  5 iota  6 alpha
  7 delta  8 psi  9 phi_c  10 t_c [s]  11 reserved (0)
For the sine-Gaussian burst (approximant 2): 0 f0 [Hz] uniform, 1 Q
uniform, 2 hrss log-uniform, 3 and 4 zero, rows 5-10 as above (9 is the
burst phase phi0, 10 its peak time t0); ranges from cfg f0, quality, hrss.
Philox stream ids: the row index for rows 0-10, 12 for the offset.

Extrinsic oversampling (the augmentation the paper's discussion of
sky-location recovery proposes: several sky positions per intrinsic draw):
with k sky positions per intrinsic draw, global sample index g belongs to
intrinsic draw g // k and is its (g % k)-th sky position.  Every row is
drawn at counter index g // k; rows alpha, delta, psi and the background
offset use the Philox sub-counter g % k, the others sub-counter 0.  k = 1
gives the ordinary draws.
"""

import math

import numpy as np

from .rng import philox_uniform

PARAM_NAMES = ("mc", "q", "chi1", "chi2", "dl", "iota", "ra", "dec", "psi",
               "phic", "tc", "reserved")
N_PARAMS = 12
OFFSET_STREAM = 12


SKY_STREAMS = (6, 7, 8, OFFSET_STREAM)


def sample_params(cfg, seed, first_index, B, L_bg, ext_k=1):
    """Draw B samples; returns (params float64 [12][B], offsets int64 [B]).

    cfg keys used: mc, q, chi, dl (each a (lo, hi) pair), t_window,
    psd_length, fs.  ext_k: sky positions per intrinsic draw (see above).
    """
    fs = float(cfg["fs"])
    T = float(cfg["t_window"])
    N = int(round(T * fs))
    P = int(round(float(cfg["psd_length"]) * fs))
    span = L_bg - P - N + 1
    if span <= 0:
        raise ValueError("background shorter than one PSD stretch plus window")
    if ext_k < 1:
        raise ValueError("ext_k must be positive")
    params = np.zeros((N_PARAMS, B), dtype=np.float64)
    offsets = np.zeros(B, dtype=np.int64)
    (mc_a, mc_b), (q_a, q_b) = cfg["mc"], cfg["q"]
    (chi_a, chi_b), (dl_a, dl_b) = cfg["chi"], cfg["dl"]
    for i in range(B):
        g = first_index + i
        gi, j = g // ext_k, g % ext_k
        u = [philox_uniform(seed, gi, s, j if s in SKY_STREAMS else 0) for s in range(11)]
        if int(cfg.get("approximant", 0)) == 2:
            (f_a, f_b), (Q_a, Q_b), (h_a, h_b) = cfg["f0"], cfg["quality"], cfg["hrss"]
            params[0, i] = f_a + u[0] * (f_b - f_a)
            params[1, i] = Q_a + u[1] * (Q_b - Q_a)
            params[2, i] = math.exp(math.log(h_a) + u[2] * (math.log(h_b) - math.log(h_a)))
        else:
            params[0, i] = mc_a + u[0] * (mc_b - mc_a)
            params[1, i] = q_a + u[1] * (q_b - q_a)
            params[2, i] = chi_a + u[2] * (chi_b - chi_a)
            params[3, i] = chi_a + u[3] * (chi_b - chi_a)
            # uniform in volume: CDF (D^3 - a^3) / (b^3 - a^3)
            params[4, i] = (dl_a ** 3 + u[4] * (dl_b ** 3 - dl_a ** 3)) ** (1.0 / 3.0)
        # sine density on (0, pi): cos(iota) uniform on (-1, 1)
        params[5, i] = math.acos(2.0 * u[5] - 1.0)
        params[6, i] = 2.0 * math.pi * u[6]
        # cosine density on (-pi/2, pi/2): sin(delta) uniform on (-1, 1)
        params[7, i] = math.asin(2.0 * u[7] - 1.0)
        params[8, i] = math.pi * u[8]
        params[9, i] = 2.0 * math.pi * u[9]
        params[10, i] = T - 1.5 + u[10] * 1.0
        uo = philox_uniform(seed, gi, OFFSET_STREAM, j)
        offsets[i] = int(math.floor(uo * span))
    return params, offsets
