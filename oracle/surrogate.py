"""Learned waveform surrogate (oracle side): reduced-basis targets, the
physics features of the linear skip path, the MLP forward and backward pass
with bfloat16 rounding at the same points as the GPU, waveform
reconstruction and the noise-weighted mismatch.

The paper does not use a surrogate; it is an addition of this library to the
waveform step of section 3.1 (one of the workload's three system choices).
Readings:

  * Nodes: NN = 1024 points log-spaced in geometric frequency
    Mf = M_total[s] * f over [2e-3, 0.2].  The IMR-form model is
    self-similar in Mf, so targets depend on (q, chi1, chi2) only, and the
    model's cut-off (Mf = 0.2) is fixed on the node grid.
  * Targets at the nodes: amplitude ratio A(f)/A_N(f) to the Newtonian
    amplitude, and phase residual P(f) - P_N(f) with the Newtonian phase
    P_N = 3/(128 eta v^5), v = (pi Mf)^(1/3) (iota = 0, D_L = 1 Mpc,
    t_c = phi_c = 0: the ratio does not depend on them).
  * Coefficients: projections on the leading 64 orthonormal basis vectors
    of each (mean-removed) target set.
  * Skip path: coefficients = A^T phi(theta) + s * z + m, where phi holds
    the PN phase coefficients 3/(128 eta) c_k (k = 2..7), the log
    coefficients 3/(128 eta) l_5 and l_6, and a constant; A is the least
    squares fit; z is the MLP output (standardised residual).  Inside the
    TaylorF2 region the phase residual is linear in phi, so the MLP learns
    only the merger-ringdown part and the amplitude.
  * MLP 4 -> 256 -> 256 -> 256 -> 128, SiLU, input x = 2 (theta - lo)/(hi - lo) - 1.
    Each layer computes z = bf16(h) bf16(W) + b with float accumulation;
    backward rounds dz and W/h to bfloat16 before every product, as the
    GPU kernels do.  Loss: mean squared error over batch and outputs.
  * Reconstruction at a bin f_k: u = (ln(M_s f_k) - ln Mf_lo)/d, linear
    interpolation between nodes in u; A = A_N(f_k) * ratio;
    Psi = P_N(f_k) + dpsi - phi_c - pi/4; zero outside f_min <= f_k < f_cut.
  * Mismatch: <a|b> = 4 df Re sum_{kept} a_k conj(b_k) / S_k over
    f_min <= f_k < f_cut, 0 < k < N/2;  mm = 1 - <a|b>/sqrt(<a|a><b|b>)
    (strict: at the drawn t_c and phi_c).  Reported beside it, the same
    quantity maximised over a time shift and a phase offset of one
    waveform (mismatch_maximised).

  * Reduced basis: the leading right singular vectors of the mean-removed
    target rows, each with its largest-magnitude component made positive
    (the singular vectors are unique only up to sign).
  * Optimiser: AdamW (Loshchilov & Hutter, "Decoupled Weight Decay
    Regularization", ICLR 2019), the optimiser section 5.1 of the paper
    trains with: Adam's moment estimates with bias correction (Kingma & Ba
    2015) and a weight decay applied to the weights themselves rather than
    added to the gradient.  The step size lr multiplies both terms (the
    decay per step is lr * weight_decay).  Biases are not decayed.
  * Mismatch head: log10 of the mismatch predicted linearly from the last
    hidden layer, bf16(silu(z3)) . w + w0, fitted by ridge least squares
    with the penalty ridge * n on every coefficient (the constant too).
  * Fallback routing: a sample keeps the surrogate only where the predicted
    log10 mismatch is <= the threshold; a NaN prediction falls back.

Pins: the MLP backward pass against central differences; basis truncation
error equal to the discarded squared singular values (Eckart-Young) and no
better basis among random ones; a rank-one case; mm(h, h) = 0 and
invariance of mm to overall scale; small-phase-error law mm ~ Var_w(dpsi)/2;
the first AdamW step by hand, equality with Adam in Kingma & Ba's rearranged
form at zero decay, pure exponential decay of the weights at zero gradient;
the ridge head against its normal equations and a hand-solved case.
"""

import math

import numpy as np

from . import waveform

NN = 1024
MF_LO = 2.0e-3
MF_HI = 0.2
N_BASIS = 64
HIDDEN = 256
N_OUT = 2 * N_BASIS
N_FEAT = 9


def node_grid():
    return np.geomspace(MF_LO, MF_HI, NN)


def targets(mc, q, chi1, chi2):
    """(ratio, dpsi) float64 [NN] at the nodes."""
    Mf = node_grid()
    eta, M, Ms = waveform.mass_terms(mc, q)
    f = Mf / Ms
    amp, P = waveform.imr_form_model(f, mc, q, chi1, chi2, 1.0)
    AN = waveform.newtonian_amplitude(f, mc, 1.0)
    v = np.cbrt(math.pi * Mf)
    PN = 3.0 / (128.0 * eta * v ** 5)
    return amp / AN, P - PN


def features(q, chi1, chi2):
    """phi(theta): PN phase coefficients scaled by 3/(128 eta), and 1."""
    eta = q / (1.0 + q) ** 2
    c, lg = waveform.pn_coefficients(eta, q, chi1, chi2)
    pre = 3.0 / (128.0 * eta)
    return np.array([pre * c[2], pre * c[3], pre * c[4], pre * c[5], pre * c[6], pre * c[7],
                     pre * lg[5], pre * lg[6], 1.0])


def bf16(x):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def normalise_inputs(theta, lo, hi):
    theta = np.asarray(theta, dtype=np.float64)
    return (2.0 * (theta - lo) / (hi - lo) - 1.0).astype(np.float32).astype(np.float64)


def mlp_forward(weights, x, emulate_bf16=True):
    """weights: list of (W [in][out], b [out]); returns (out, cache)."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    h = x
    cache = []
    for l, (W, b) in enumerate(weights):
        hin = r(h)
        z = hin @ r(W) + b
        cache.append((hin, z))
        h = silu(z) if l < len(weights) - 1 else z
    return h, cache


def mlp_backward(weights, cache, dout, emulate_bf16=True):
    """Gradients [(dW, db)] for upstream gradient dout of the output."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * len(weights)
    dz = dout
    for l in range(len(weights) - 1, -1, -1):
        W, _ = weights[l]
        hin, z = cache[l]
        if l < len(weights) - 1:
            dz = dz * silu_grad(z)
        dzr = r(dz)
        grads[l] = (hin.T @ dzr, dz.sum(axis=0))
        if l > 0:
            dz = dzr @ r(W).T
    return grads


def mse_loss_and_grad(out, target):
    n = out.size
    d = out - target
    return float(np.sum(d * d) / n), 2.0 * d / n


def interp_nodes(values, Ms, f):
    """Linear interpolation of node values [NN] in ln(Mf) at frequencies f."""
    u = (np.log(Ms * np.asarray(f, dtype=np.float64)) - math.log(MF_LO)) / (
        math.log(MF_HI / MF_LO) / (NN - 1))
    u = np.clip(u, 0.0, NN - 1.0)
    i = np.minimum(np.floor(u).astype(np.int64), NN - 2)
    t = u - i
    return (1.0 - t) * values[i] + t * values[i + 1]


def nodes_from_state(theta, feat, weights, A, zmean, zstd, basis, mean, lo, hi):
    """Node values [B][2][NN] from the surrogate state: coefficients
    phi A + zstd z + zmean with z the MLP output, then mean + coef V."""
    x = normalise_inputs(theta, lo, hi)
    z, _ = mlp_forward(weights, x, emulate_bf16=True)
    coef = feat @ A + zstd * z + zmean
    ratio = mean[0] + coef[:, :N_BASIS] @ basis[0]
    dpsi = mean[1] + coef[:, N_BASIS:] @ basis[1]
    return np.stack([ratio, dpsi], axis=1)


def reconstruct(cfg, p, ratio_nodes, dpsi_nodes):
    """(h+, hx) on the window grid from node values."""
    hp = reconstruct_hp(cfg, p, ratio_nodes, dpsi_nodes)
    ci = math.cos(p[5])
    c2 = 0.5 * (1.0 + ci * ci)
    hc = np.where(np.abs(hp) > 0, -1j * hp * (ci / c2), 0.0) if c2 != 0 else np.zeros_like(hp)
    return hp, hc


def reconstruct_hp(cfg, p, ratio_nodes, dpsi_nodes):
    """h+ on the window grid from node values (iota, D_L, phi_c from p)."""
    from .pipeline import fd_grid
    f = fd_grid(cfg)
    mc, q, dl, iota, phic = p[0], p[1], p[4], p[5], p[9]
    eta, M, Ms = waveform.mass_terms(mc, q)
    f_cut = waveform.frequency_cutoff(1, mc, q)
    band = (f >= cfg["f_min"]) & (f < f_cut) & (f > 0)
    band[-1] = False
    fb = np.where(band, f, cfg["f_min"])
    ratio = interp_nodes(ratio_nodes, Ms, fb)
    dpsi = interp_nodes(dpsi_nodes, Ms, fb)
    v = np.cbrt(math.pi * Ms * fb)
    psi = 3.0 / (128.0 * eta * v ** 5) + dpsi - phic - math.pi / 4.0
    amp = waveform.newtonian_amplitude(fb, mc, dl) * ratio
    ci = math.cos(iota)
    return np.where(band, amp * 0.5 * (1.0 + ci * ci) * np.exp(-1j * psi), 0.0)


def inner(a, b, S, df, kept):
    return 4.0 * df * float(np.real(np.sum(a[kept] * np.conj(b[kept]) / S[kept])))


def mismatch(a, b, S, df, kept):
    ab = inner(a, b, S, df, kept)
    aa = inner(a, a, S, df, kept)
    bb = inner(b, b, S, df, kept)
    if aa <= 0.0 or bb <= 0.0:
        return 0.0
    return 1.0 - ab / math.sqrt(aa * bb)


def overlap_vs_shift(a, b, S, kept, tau):
    """c(tau) = sum over the kept bins of a_k conj(b_k) / S_k e^{2 pi i k tau}:
    the complex overlap of a with b delayed by tau window lengths (b_k
    e^{-2 pi i f_k t}, f_k = k / T, tau = t / T), up to the factor 4 df.
    Its real part is the overlap at coalescence phase 0; a phase offset phi
    multiplies it by e^{i phi}."""
    k = np.nonzero(kept)[0]
    z = a[k] * np.conj(b[k]) / S[k]
    return complex(np.sum(z * np.exp(2j * math.pi * k * tau)))


def mismatch_maximised(a, b, S, df, kept, n_grid=1 << 18):
    """1 - max over a time shift and a phase of the normalised overlap: the
    maximum over the phase of Re(e^{i phi} c(tau)) is |c(tau)|; the maximum
    over tau in [0, 1) (c has period one window) is taken as the best point of
    a grid of n_grid shifts (an inverse DFT of the zero-padded products)
    refined by a bounded scalar search of |c(tau)| within one grid step of it.
    Never above the strict mismatch (tau = 0, phi = 0 is a candidate)."""
    from scipy.optimize import minimize_scalar
    aa = inner(a, a, S, df, kept)
    bb = inner(b, b, S, df, kept)
    if aa <= 0.0 or bb <= 0.0:
        return 0.0
    k = np.nonzero(kept)[0]
    if k.size == 0:
        return 0.0
    z = np.zeros(n_grid, dtype=np.complex128)
    np.add.at(z, k % n_grid, a[k] * np.conj(b[k]) / S[k])
    c = np.fft.ifft(z) * n_grid  # c[n] = c(n / n_grid)
    n0 = int(np.argmax(np.abs(c)))
    step = 1.0 / n_grid
    res = minimize_scalar(lambda tau: -abs(overlap_vs_shift(a, b, S, kept, tau)),
                          bounds=(n0 * step - step, n0 * step + step), method="bounded",
                          options={"xatol": 1e-6 * step})
    best = max(abs(c[n0]), -res.fun, abs(overlap_vs_shift(a, b, S, kept, 0.0)))
    return 1.0 - 4.0 * df * best / math.sqrt(aa * bb)


# ------------------------------------------------------------ training pieces

def reduced_basis(X, n_basis):
    """(mean [n], V [n_basis][n]) of the rows of X: the column mean and the
    leading right singular vectors of X - mean (numpy.linalg.svd), each row of
    V with its largest-magnitude component positive."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(axis=0)
    _, _, Vt = np.linalg.svd(X - mean, full_matrices=False)
    V = Vt[:n_basis].copy()
    big = V[np.arange(V.shape[0]), np.argmax(np.abs(V), axis=1)]
    return mean, V * np.where(big < 0, -1.0, 1.0)[:, None]


def truncation_error(X, mean, V):
    """Squared Frobenius norm of what the basis V leaves out of X - mean."""
    Xc = np.asarray(X, dtype=np.float64) - mean
    R = Xc - (Xc @ V.T) @ V
    return float(np.sum(R * R))


def adamw_step(p, g, m, v, t, lr, weight_decay, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW update of the parameters p with gradient g at step t >= 1;
    m, v are the moment estimates before the step.  Returns (p, m, v)."""
    p, g = np.asarray(p, np.float64), np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    p = p - lr * (m_hat / (np.sqrt(v_hat) + eps) + weight_decay * p)
    return p, m, v


def ridge_head(h, y, ridge):
    """Coefficients [h.shape[1] + 1] (weights, then the constant) minimising
    ||[h 1] w - y||^2 + ridge * n * ||w||^2, solved as the ordinary least
    squares problem of the stacked system [[h 1]; sqrt(ridge n) I] w = [y; 0]
    (numpy.linalg.lstsq)."""
    h = np.asarray(h, np.float64)
    y = np.asarray(y, np.float64)
    n, k = h.shape
    X = np.concatenate([h, np.ones((n, 1))], axis=1)
    A = np.concatenate([X, math.sqrt(ridge * n) * np.eye(k + 1)], axis=0)
    rhs = np.concatenate([y, np.zeros(k + 1)])
    return np.linalg.lstsq(A, rhs, rcond=None)[0]


def predicted_log10_mismatch(weights, x, head):
    """Head output for normalised inputs x [B][4]: the last hidden layer as
    the GPU stores it (bf16 of silu(z3)) times head[:-1], plus head[-1]."""
    _, cache = mlp_forward(weights, x, emulate_bf16=True)
    h3 = cache[-1][0]          # the output layer's (rounded) input
    return h3 @ np.asarray(head[:-1], np.float64) + float(head[-1])


def keeps_surrogate(logmm, threshold):
    """Routing: surrogate where the prediction is <= threshold (NaN falls back)."""
    return np.asarray(logmm) <= threshold
