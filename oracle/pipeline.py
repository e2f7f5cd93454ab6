"""Projection, injection and the whole per-sample generator (oracle side).

Section 3.2 of the paper: a long background chunk stays in accelerator
memory; for each batch, windows are sliced from it, prior draws are turned
into waveforms, the signals are injected, and the batch is whitened with the
estimated spectrum and handed to training together with the parameters.

Readings where the paper is silent:
  * a sample uses background [o, o + P + N): the first P samples feed the
    Welch PSD, the last N are the window's noise; the same o is used for
    every detector, so detectors stay time-coincident;
  * projected DFT coefficients on f_k = k / T, k = 0 .. N/2:
        H_d[k] = fs (F+ h+(f_k) + Fx hx(f_k)) exp(-2 pi i f_k (t_c + dt_d)),
    zero at k = 0 and k = N/2 (fs turns continuous-transform samples into
    DFT coefficients);
  * injection in the time domain, y_d = bg_d[o+P : o+P+N] + irfft_N(H_d);
  * whitened output: float64 [B][D][N].
  * view pairs for self-supervised pre-training (Fig. 2, section 4): the
    shifted view d' is the ordinary sample; the reference view d has the
    same parameters, background window and PSD with t_c set to the fixed
    reference t_ref = T - 1.5 s (the start of the t_c prior), so d' is d
    with the signal delayed by t_c - t_ref in [0, 1 s);
  * uneven batches (several window lengths and sample rates in one batch):
    slot i of a batch of B slots is an ordinary sample of its own class's
    configuration, drawn at global index batch_index * B + i with that
    class's background; parameter row 11 holds the class index.
"""

import numpy as np

from .detectors import antenna_patterns, detector_geometry, time_delays
from .priors import sample_params
from .spectral import interp_psd, run_psd, truncated_filter, welch_psd, whiten, whiten_filtered
from .waveform import fd_waveform, sine_gaussian


def derived_sizes(cfg):
    fs = float(cfg["fs"])
    N = int(round(cfg["t_window"] * fs))
    P = int(round(cfg["psd_length"] * fs))
    L = int(round(cfg["fftlen"] * fs))
    S = int(round((cfg["fftlen"] - cfg["overlap"]) * fs))
    K = (P - L) // S + 1
    return dict(N=N, F=N // 2 + 1, P=P, L=L, S=S, K=K, Fw=L // 2 + 1, r=N // L)


def fd_grid(cfg):
    z = derived_sizes(cfg)
    return np.arange(z["F"], dtype=np.float64) / float(cfg["t_window"])


def waveform_on_grid(cfg, p):
    """h+, hx on the window grid for one parameter column p (len 12)."""
    f = fd_grid(cfg)
    if int(cfg["approximant"]) == 2:
        # rows: 0 f0, 1 Q, 2 hrss, 5 iota, 9 phi0
        hp, hc = sine_gaussian(f, p[0], p[1], p[2], p[5], p[9], float(cfg["f_min"]))
    else:
        hp, hc = fd_waveform(f, int(cfg["approximant"]), p[0], p[1], p[2], p[3],
                             p[4], p[5], p[9], float(cfg["f_min"]))
    hp[0] = hc[0] = 0.0
    hp[-1] = hc[-1] = 0.0
    return hp, hc


def project_detectors(cfg, p, hp, hc):
    """H_d[k] complex128 [D][F] for one sample."""
    f = fd_grid(cfg)
    fs = float(cfg["fs"])
    out = np.zeros((len(cfg["det_ids"]), f.shape[0]), dtype=np.complex128)
    for d, det in enumerate(cfg["det_ids"]):
        D, r = detector_geometry(det)
        fp, fx = antenna_patterns(D, p[6], p[7], p[8])
        tau = p[10] + time_delays(r, p[6], p[7])
        out[d] = fs * (fp * hp + fx * hc) * np.exp(-2j * np.pi * f * tau)
    return out


def inject(cfg, bg, offset, H):
    """y_d = bg_d[o+P : o+P+N] + irfft(H_d) -> float64 [D][N]."""
    z = derived_sizes(cfg)
    N, P = z["N"], z["P"]
    y = np.zeros((H.shape[0], N), dtype=np.float64)
    for d in range(H.shape[0]):
        noise = np.asarray(bg[d, offset + P:offset + P + N], dtype=np.float64)
        y[d] = noise + np.fft.irfft(H[d], n=N)
    return y


def sample_psd(cfg, bg, offset):
    """Welch PSD [D][L/2+1] from the stretch preceding the window."""
    z = derived_sizes(cfg)
    fs = float(cfg["fs"])
    out = np.zeros((bg.shape[0], z["Fw"]), dtype=np.float64)
    for d in range(bg.shape[0]):
        out[d] = welch_psd(bg[d, offset:offset + z["P"]], fs, z["L"], z["S"])
    return out


def generate_sample(cfg, bg, p, offset, return_stages=False):
    """Whitened strain float64 [D][N] for one sample."""
    z = derived_sizes(cfg)
    fs = float(cfg["fs"])
    hp, hc = waveform_on_grid(cfg, p)
    H = project_detectors(cfg, p, hp, hc)
    y = inject(cfg, bg, offset, H)
    psd = sample_psd(cfg, bg, offset)
    out = np.zeros_like(y)
    for d in range(y.shape[0]):
        out[d] = whiten(y[d], interp_psd(psd[d], z["r"]), fs, float(cfg["f_min"]))
    if return_stages:
        return out, dict(hp=hp, hc=hc, H=H, y=y, psd=psd)
    return out


def generate_batch(cfg, bg, params, offsets):
    """Whitened strain float64 [B][D][N] for params [12][B], offsets [B]."""
    z = derived_sizes(cfg)
    B = params.shape[1]
    out = np.zeros((B, len(cfg["det_ids"]), z["N"]), dtype=np.float64)
    for i in range(B):
        out[i] = generate_sample(cfg, bg, params[:, i], int(offsets[i]))
    return out


def ragged_draws(classes, cls, seed, batch_index, bg_lengths, slots=None):
    """Parameters [12][B] and offsets [B] of an uneven batch (columns of
    slots outside `slots` are left zero when `slots` is given)."""
    B = len(cls)
    params = np.zeros((12, B), dtype=np.float64)
    offsets = np.zeros(B, dtype=np.int64)
    for i in (range(B) if slots is None else slots):
        c = int(cls[i])
        p, o = sample_params(classes[c], seed, batch_index * B + i, 1, bg_lengths[c])
        params[:, i] = p[:, 0]
        params[11, i] = float(c)
        offsets[i] = o[0]
    return params, offsets


def generate_ragged(classes, cls, seed, batch_index, bgs, slots=None):
    """Uneven batch.  classes: list of configurations; cls: class index per
    slot [B]; bgs: background per class.  Returns (outputs, params [12][B],
    offsets [B]) with outputs[i] float64 [D][N_i] for every slot, or for the
    slots listed in `slots` (then only their parameter columns are filled)."""
    params, offsets = ragged_draws(classes, cls, seed, batch_index, [b.shape[1] for b in bgs], slots)
    outs = {}
    for i in (range(len(cls)) if slots is None else slots):
        c = int(cls[i])
        outs[i] = generate_sample(classes[c], bgs[c], params[:, i], int(offsets[i]))
    return outs, params, offsets


def run_psds(cfg, bg, n_chunks):
    """Per-run PSD of every detector row [D][L/2+1]: Welch over the first
    n_chunks * K segments of the row (K segments per psd_length stretch)."""
    z = derived_sizes(cfg)
    return np.stack([run_psd(bg[d], float(cfg["fs"]), z["L"], z["S"], n_chunks * z["K"])
                     for d in range(bg.shape[0])])


def run_filters(cfg, psd, M):
    """Truncated whitening filters [D][N/2+1] from per-run PSDs [D][L/2+1]."""
    z = derived_sizes(cfg)
    return np.stack([truncated_filter(interp_psd(psd[d], z["r"]), float(cfg["fs"]), z["N"],
                                      float(cfg["f_min"]), M) for d in range(psd.shape[0])])


def generate_sample_runpsd(cfg, bg, p, offset, filt, crop):
    """Per-run mode: the sample's window (as in generate_sample) whitened with
    the detector's fixed filter, `crop` samples dropped at each end."""
    hp, hc = waveform_on_grid(cfg, p)
    H = project_detectors(cfg, p, hp, hc)
    y = inject(cfg, bg, offset, H)
    return np.stack([whiten_filtered(y[d], filt[d], crop) for d in range(y.shape[0])])


def reference_time(cfg):
    """Fixed signal time of the reference view: the start of the t_c prior."""
    return float(cfg["t_window"]) - 1.5


def generate_pair(cfg, bg, p, offset):
    """(d, d'): reference view and ordinary (shifted) view of one sample."""
    p_ref = np.array(p, dtype=np.float64).copy()
    p_ref[10] = reference_time(cfg)
    return generate_sample(cfg, bg, p_ref, offset), generate_sample(cfg, bg, p, offset)
