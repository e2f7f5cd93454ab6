/*
 * gwgen.h -- C ABI of libgwgen.so, an on-the-fly training-data generator for
 * likelihood-free inference of binary-black-hole mergers on AMD MI355X
 * (gfx950).
 *
 * The generator follows section 3.2 of "Rapid Likelihood Free Inference of
 * Compact Binary Coalescences using Accelerated Hardware" (AMPLFI).  A long
 * detector background is kept resident in device memory.  Each batch draws
 * parameters from the priors of Table 1 (section 5) and generates
 * frequency-domain plus/cross waveforms (section 3.1).  It projects them onto
 * the detectors with antenna patterns and arrival-time delays (the on-device
 * projection that section 6 describes), injects them into the background, and
 * estimates a noise PSD.  Finally it whitens the strain and emits the windows
 * together with the parameters.
 *
 * Conventions shared by every entry point:
 *   - Array arguments are caller-owned DEVICE pointers (for example, memory
 *     allocated by PyTorch).  The library never frees, keeps or reallocates
 *     them.  Pointers must be 16-byte aligned unless stated otherwise.
 *   - Work is queued asynchronously on `stream`.  Nothing synchronises;
 *     results are ready once the caller synchronises that stream.
 *   - Sizes, null pointers, alignment and configuration are checked on the
 *     host before anything is launched.  On a failed check the call returns
 *     GW_EINVAL and launches nothing.  A failed launch returns GW_EHIP;
 *     gw_last_error() then returns HIP's message.
 *   - A bad DATA value (a NaN in the background, a PSD bin <= 0) never fails
 *     a call.  Affected bins are dropped from the whitened output and a
 *     per-sample status bit is set (GW_STATUS_*).
 *   - A gw_ctx is not thread-safe.  Use one per host thread / stream.
 *   - Strain is in units of 2^70 x dimensionless strain.  This exact power of
 *     two keeps PSD values inside binary32 range.  The PSD is in
 *     (2^70)^2 / Hz.  The whitened output is dimensionless and does not depend
 *     on the scale.
 *   - Complex arrays are interleaved (re, im) binary32 pairs.
 */
#ifndef GWGEN_H
#define GWGEN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gw_status;
#define GW_OK            0
#define GW_EINVAL       -1  /* bad argument or configuration               */
#define GW_ENOMEM       -2  /* device allocation failed (allocating calls)  */
#define GW_EHIP         -3  /* a HIP call or kernel launch failed           */
#define GW_EUNSUPPORTED -4  /* valid, but not supported by this library     */

/* Per-sample status bits (uint32), OR-ed over the sample's detectors. */
#define GW_STATUS_NONFINITE_PSD  1u  /* a PSD bin was NaN/Inf (bad background) */
#define GW_STATUS_NONPOSITIVE_PSD 2u /* a kept PSD bin was <= 0                */
#define GW_STATUS_NONFINITE_DATA 4u  /* a window value was NaN/Inf             */
#define GW_STATUS_CUT_AT_NYQUIST 8u  /* waveform cut-off above fs/2            */
#define GW_STATUS_SURROGATE_FALLBACK 16u /* surrogate batch: plain model used  */

#define GW_N_PARAMS 12
#define GW_MAX_DET 4

/* Generator configuration (plain data, copied by gw_create).
 * Priors: M_c, q, chi and D_L ranges replace those of Table 1.  The angles
 * follow Table 1: iota with a sine density, RA uniform on (0, 2 pi),
 * declination with a cosine density, phi_c uniform on (0, 2 pi), psi uniform
 * on (0, pi).  t_c is uniform on [T - 1.5 s, T - 0.5 s).
 * Sizes: N = t_window*fs is the window length.  P = psd_length*fs is the PSD
 * stretch preceding the window.  L = fftlen*fs is the Welch segment length and
 * S = (fftlen - overlap)*fs is the segment stride.  K = (P - L)/S + 1
 * segments are averaged.  Constraints: N and L are powers of two,
 * 2^11 <= N <= 2^20, 2^11 <= L <= 2^12, N/L is an integer, and
 * (P - L) is a multiple of S.  The stride must be L/2 (50 % overlap).
 * Precision mode 2 allows N up to 2^14 (gw_create returns GW_EUNSUPPORTED
 * above).  Windows longer than 2^15 samples run as a four-step transform
 * inside the output buffer, through the six steps and gw_generate_batch; the
 * surrogate, per-run-PSD, view-pair and ragged calls return GW_EUNSUPPORTED
 * for them. */
typedef struct gw_config {
  int32_t n_det;               /* 1..4 */
  int32_t det_id[GW_MAX_DET];  /* 0 = H1, 1 = L1, 2 = V1 */
  double  fs;                  /* sample rate [Hz] */
  double  t_window;            /* window length T [s] */
  double  psd_length;          /* Welch stretch [s] */
  double  fftlen;              /* Welch segment [s] */
  double  overlap;             /* Welch overlap [s] */
  double  f_min;               /* waveform start and whitening low cut [Hz] */
  int32_t approximant;         /* 0 TaylorF2 3.5PN, 1 IMR-form, 2 sine-Gaussian
                                  burst (rows 0-2 of params are f0, Q, hrss) */
  int32_t precision;           /* 0 binary32 throughout, 1 mixed (binary64
                                  waveform phase, time shift and Welch
                                  sums), 2 binary64 */
  double  mc[2], q[2], chi[2], dl[2];   /* prior ranges [Msun], [], [], [Mpc] */
  double  f0[2], quality[2], hrss[2];   /* approximant 2 only: central
                                  frequency [Hz] (uniform, below fs/2),
                                  quality factor (uniform), root-sum-square
                                  strain (log-uniform) */
} gw_config;

typedef struct gw_ctx gw_ctx;
typedef struct gw_surrogate gw_surrogate;

/* Create a context: validate the configuration, build detector geometry and
 * twiddle/power tables on the current HIP device.  Allocates device memory
 * for them (under 1 MB up to N = 2^15, about 32 MB at N = 2^20).  The only
 * other calls that allocate are gw_ragged_create, gw_surrogate_create and
 * gw_surrogate_fit_basis (a temporary Gram buffer); gw_graph_create and
 * gw_ragged_graph_create instantiate HIP graphs. */
gw_status gw_create(const gw_config* cfg, gw_ctx** out);
gw_status gw_destroy(gw_ctx* ctx);
const char* gw_strerror(gw_status s);
/* Message of the last failure seen by this context (HIP string or a
 * description of the rejected argument).  Valid until the next call. */
const char* gw_last_error(const gw_ctx* ctx);

/* gw_query keys. */
#define GW_Q_N        0   /* window samples                          */
#define GW_Q_F        1   /* window rfft bins N/2+1                  */
#define GW_Q_P        2   /* PSD stretch samples                     */
#define GW_Q_L        3   /* Welch segment samples                   */
#define GW_Q_K        4   /* Welch segments                          */
#define GW_Q_FW       5   /* Welch bins L/2+1                        */
#define GW_Q_NDET     6
#define GW_Q_NPARAMS  7
gw_status gw_query(const gw_ctx* ctx, int32_t key, int64_t* value);
/* Bytes of device workspace gw_generate_batch needs for batch size B. */
gw_status gw_workspace_size(const gw_ctx* ctx, int64_t B, int64_t* bytes);

/* sample_params -- prior draws (Table 1, section 5; ranges from gw_config).
 * Draws use the Philox4x32-10 counter-based generator (Salmon et al. 2011).
 * The key is (seed lo, seed hi) and the counter is (g lo, g hi, stream, 0),
 * where g = first_index + i is the global sample index.  Output is therefore
 * independent of how a run is split into batches.
 * params: double [12][B] rows {M_c, q, chi1, chi2, D_L, iota, RA, dec, psi,
 *         phi_c, t_c, 0}.
 * offset: int64 [B] first background sample of sample i, uniform on
 *         [0, L_bg - P - N].  The PSD stretch is [o, o+P); the window is
 *         [o+P, o+P+N).
 * Requires L_bg >= P + N and B >= 0 (B == 0 is a no-op). */
gw_status sample_params(gw_ctx* ctx, uint64_t seed, uint64_t first_index,
                        int64_t B, int64_t L_bg, double* params,
                        int64_t* offset, hipStream_t stream);

/* gen_fd_waveform -- frequency-domain plus/cross polarisations (section
 * 3.1) on f_k = k/T, k = 0..N/2, with t_c = 0.  The result is in
 * continuous-transform units [2^70 s].  It is zero outside
 * f_min <= f_k < f_cut and at k = 0 and k = N/2.  TaylorF2 has
 * f_cut = f_ISCO; IMR-form has f_cut = 0.2/M.
 * params: double [12][B] as written by sample_params.
 * hp, hc: interleaved complex float [B][N/2+1]. */
gw_status gen_fd_waveform(gw_ctx* ctx, const double* params, int64_t B,
                          float* hp, float* hc, hipStream_t stream);

/* project_detectors -- antenna patterns F+, Fx and geocentric delay dt_d for
 * each configured detector, from (RA, dec, psi).  Applied on device as the
 * paper's section 6 describes.  Output:
 *   hdet[b][d][k] = fs (F+ hp + Fx hc) exp(-2 pi i f_k (t_c + dt_d)),
 * i.e. DFT coefficients of the detector strain on the window grid.
 * hdet: interleaved complex float [B][n_det][N/2+1]. */
gw_status project_detectors(gw_ctx* ctx, const double* params,
                            const float* hp, const float* hc, int64_t B,
                            float* hdet, hipStream_t stream);

/* inject -- add each projected signal to its background window (section
 * 3.2): strain[b][d][n] = bg[d][o_b + P + n] + irfft_N(hdet[b][d])[n].
 * bg: float [n_det][L_bg] (row pitch L_bg, 4-byte alignment suffices).
 * offset: int64 [B] (host does not read it; values must lie in
 * [0, L_bg - P - N]).  strain: float [B][n_det][N]. */
gw_status inject(gw_ctx* ctx, const float* bg, int64_t L_bg,
                 const int64_t* offset, const float* hdet, int64_t B,
                 float* strain, hipStream_t stream);

/* welch_psd -- noise PSD fitted to background (section 3.2).  One estimate
 * is made per (sample, detector) from the P samples [o_b, o_b + P) preceding
 * the window.  Welch's method uses K periodic-Hann segments of L samples at
 * stride S, no detrending, a mean over segments, and one-sided density
 * scaling:
 *   psd[k] = c_k/(K fs sum w^2) sum_s |rfft(w seg_s)[k]|^2,
 * with c_k = 2 except at DC and Nyquist, where c_k = 1.
 * offset: int64 [B] device array; the host does not read it, so its values
 * must lie in [0, L_bg - P] (sample_params draws them in [0, L_bg - P - N]).
 * psd: float [B][n_det][L/2+1]. */
gw_status welch_psd(gw_ctx* ctx, const float* bg, int64_t L_bg,
                    const int64_t* offset, int64_t B, float* psd,
                    hipStream_t stream);

/* whiten -- whiten each window with its PSD (section 3.2).  The PSD is
 * interpolated linearly onto the window grid (ratio N/L), then
 *   out = irfft(rfft(strain) / sqrt(fs S(f_k)/2)),
 * keeping f_k >= f_min and 0 < k < N/2.  Bins with a non-finite or
 * non-positive PSD are dropped and flagged.
 * strain, out: float [B][n_det][N] (may alias).  psd: float [B][n_det][L/2+1].
 * status: uint32 [B] or NULL.  It is overwritten with the GW_STATUS_* bits. */
gw_status whiten(gw_ctx* ctx, const float* strain, const float* psd,
                 int64_t B, float* out, uint32_t* status, hipStream_t stream);

/* gw_generate_batch -- the whole per-batch path (section 3.2) in three
 * launches: prior draws, per-(sample, detector) Welch PSDs, then one fused
 * kernel per (sample, detector).  The fused kernel loads the noise window,
 * transforms it, adds the in-register waveform + projection + time shift,
 * whitens, inverse-transforms and stores.  The result equals
 * sample_params -> gen_fd_waveform -> project_detectors -> inject ->
 * welch_psd -> whiten.  The global sample indices are
 * batch_index*B .. batch_index*B + B - 1.
 * out:        float [B][n_det][N] whitened strain.
 * params_f32: float [12][B] parameters for the trainer, or NULL.
 * status:     uint32 [B] or NULL.
 * workspace:  device memory of at least gw_workspace_size(B) bytes.  It
 *             holds params (double [12][B]), offsets and PSDs.  After the
 *             call, the first 96*B bytes hold params as double [12][B] and the
 *             next 8*B bytes hold the int64 offsets. */
gw_status gw_generate_batch(gw_ctx* ctx, uint64_t seed, uint64_t batch_index,
                            int64_t B, const float* bg, int64_t L_bg,
                            float* out, float* params_f32, uint32_t* status,
                            void* workspace, int64_t workspace_bytes,
                            hipStream_t stream);

/* gw_generate_batch_noalloc -- gw_generate_batch for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and results except the
 * workspace: the call uses the library's static device scratch area of
 * GW_SCRATCH_BYTES on the device the context was created on, held until the
 * process ends, and calls no allocator.  B must satisfy
 * gw_workspace_size(B) <= GW_SCRATCH_BYTES (B <= 2600 at 3 detectors with
 * L = 4096), else GW_EINVAL.  Every call on a device shares that device's
 * area, which keeps the last call's contents: calls that overlap in time on
 * one device (other streams or host threads) race, so serialise them; the
 * parameters and offsets are not readable by the caller (use params_f32). */
#define GW_SCRATCH_BYTES (64ll << 20)
gw_status gw_generate_batch_noalloc(gw_ctx* ctx, uint64_t seed, uint64_t batch_index, int64_t B,
                                    const float* bg, int64_t L_bg, float* out, float* params_f32,
                                    uint32_t* status, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Per-run PSD mode (section 3.2 fits one noise spectrum to the background
 * chunk held on the accelerator): one Welch PSD per detector for the run,
 * turned into a truncated whitening filter, then batches that only
 * generate, inject and whiten.
 * ------------------------------------------------------------------------ */
/* Bytes of workspace gw_run_psd needs. */
gw_status gw_run_psd_workspace_size(const gw_ctx* ctx, int64_t n_chunks, int64_t* bytes);
/* Welch PSD of each detector row over its first n_chunks*K segments
 * (segment s starts at s*S), computed as the mean of n_chunks psd_length
 * stretches starting at c*K*S.  bg: float [n_det][L_bg] (4-byte aligned);
 * psd: float [n_det][L/2+1].  Requires (n_chunks-1)*K*S + P <= L_bg. */
gw_status gw_run_psd(gw_ctx* ctx, const float* bg, int64_t L_bg, int64_t n_chunks, float* psd,
                     void* workspace, int64_t workspace_bytes, hipStream_t stream);
/* Truncated whitening filter per detector: the gain 1/sqrt(fs S/2) on the
 * window grid (S linearly interpolated from psd [n_det][L/2+1]; zero below
 * f_min, at DC and at Nyquist), its impulse response (inverse real
 * transform of length N) multiplied by cos^2(pi n / M) for circular lags
 * |n| < M/2 and by 0 elsewhere, then the magnitude of the forward transform.
 * filt: float [n_det][N/2+1].  M even, 2 <= M < N (M = fduration * fs).
 * status: uint32 [n_det] or NULL; overwritten with each detector's
 * GW_STATUS_NONFINITE_PSD / GW_STATUS_NONPOSITIVE_PSD bits (such bins get
 * zero gain before truncation). */
gw_status gw_whiten_filter(gw_ctx* ctx, const float* psd, int64_t M, float* filt, uint32_t* status,
                           hipStream_t stream);
/* gw_generate_batch with the fixed filters in place of per-sample Welch
 * PSDs: same prior draws and windows (same seed gives the same parameters
 * and offsets), whitening Y_k = X_k filt[d][k], and the first and last
 * `crop` samples of each window dropped (crop even, 2 crop < N; normally
 * M/2).  out: float [B][n_det][N - 2 crop].  Workspace as for
 * gw_generate_batch (its PSD region is unused). */
gw_status gw_generate_batch_runpsd(gw_ctx* ctx, uint64_t seed, uint64_t batch_index, int64_t B,
                                   const float* bg, int64_t L_bg, const float* filt, int64_t crop,
                                   float* out, float* params_f32, uint32_t* status,
                                   void* workspace, int64_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Views for self-supervised pre-training and extrinsic oversampling.
 * ------------------------------------------------------------------------ */
/* View pairs (Fig. 2 and section 4): out_shift is exactly gw_generate_batch's
 * output; out_ref has the same parameters, background windows and PSDs with
 * the signal at the fixed reference time t_ref = T - 1.5 s (the start of the
 * t_c prior), so each shifted view is its reference view with the signal
 * delayed by t_c - t_ref in [0, 1 s).  Both float [B][n_det][N]. */
gw_status gw_generate_batch_pairs(gw_ctx* ctx, uint64_t seed, uint64_t batch_index, int64_t B,
                                  const float* bg, int64_t L_bg, float* out_ref, float* out_shift,
                                  float* params_f32, uint32_t* status, void* workspace,
                                  int64_t workspace_bytes, hipStream_t stream);
/* gw_generate_batch with ext_k sky positions per intrinsic draw (the
 * augmentation in the extrinsic parameters proposed in section 6): global
 * sample g is sky position g % ext_k of intrinsic draw g / ext_k.  Every
 * parameter row is drawn at Philox index g / ext_k; alpha, delta, psi and
 * the background offset use the Philox sub-counter g % ext_k (the fourth
 * counter word), the other rows sub-counter 0.  ext_k = 1 gives exactly
 * gw_generate_batch; 1 <= ext_k <= 65536. */
gw_status gw_generate_batch_oversampled(gw_ctx* ctx, uint64_t seed, uint64_t batch_index, int64_t B,
                                        int32_t ext_k, const float* bg, int64_t L_bg, float* out,
                                        float* params_f32, uint32_t* status, void* workspace,
                                        int64_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Captured batch pipelines (HIP graphs).  A gw_graph replays the kernels of
 * one batch with the pointers given at creation; every launch then advances
 * a batch counter kept in the workspace, so replay r (counting from 0 after
 * creation or gw_graph_set_batch(b0)) produces exactly what the eager call
 * with batch_index = b0 + r produces.  The caller keeps bg, out, params_f32,
 * status and workspace alive and unmoved while the graph exists.  Creation
 * captures on a private stream and synchronises; tune (gw_set_tuning /
 * gw_autotune) before creating a graph, since the graph keeps the kernel
 * variants chosen at capture.
 * ------------------------------------------------------------------------ */
typedef struct gw_graph gw_graph;
/* Graph of gw_generate_batch(seed, first_batch + r, B, ...). */
gw_status gw_graph_create(gw_ctx* ctx, uint64_t seed, uint64_t first_batch,
                          int64_t B, const float* bg, int64_t L_bg,
                          float* out, float* params_f32, uint32_t* status,
                          void* workspace, int64_t workspace_bytes,
                          gw_graph** graph);
/* Replay one batch on `stream` (asynchronous). */
gw_status gw_graph_launch(gw_graph* graph, hipStream_t stream);
/* Queue a reset of the batch counter to batch_index on `stream`. */
gw_status gw_graph_set_batch(gw_graph* graph, uint64_t batch_index, hipStream_t stream);
const char* gw_graph_last_error(const gw_graph* graph);
gw_status gw_graph_destroy(gw_graph* graph);

/* Kernel variants.  GW_TUNE_ORD_*: 0 puts the FFT's small radix pass last,
 * 1 puts it first (same result up to rounding; which is faster depends on
 * the size).  GW_TUNE_OCC_WELCH: 2 or 3 waves per SIMD for the Welch kernel
 * (3 caps it at 168 VGPRs, which the binary32 kernels meet without spills
 * at L = 4096).  Binary64 kernels (precision 2) have one variant.  For
 * windows longer than 2^15 samples GW_TUNE_ORD_WINDOW selects the structure
 * of the four-step window stage instead: 1 fuses the row transforms, the
 * bins and the inverse row transforms into one pass per row pair, 0 runs
 * them as three passes.  Defaults (before gw_autotune): OCC_WELCH 3 for
 * binary32 transforms of L = 4096, else 2; ORD_WINDOW 1 for N = 16384 or
 * N > 32768 with binary32 transforms, else 0; ORD_WELCH 0. */
#define GW_TUNE_ORD_WINDOW 1
#define GW_TUNE_ORD_WELCH  2
#define GW_TUNE_OCC_WELCH  3
gw_status gw_set_tuning(gw_ctx* ctx, int32_t key, int64_t value);
gw_status gw_get_tuning(const gw_ctx* ctx, int32_t key, int64_t* value);
/* Autotuner: runs one batch of size B, then times the Welch kernel under
 * each (radix order, occupancy) and the fused window kernel under each radix
 * order, over `reps` launches each on a private stream (synchronous), in
 * three interleaved rounds, and keeps the fastest.  report (host double [6],
 * nullable) receives, per variant, the best round's mean ms of Welch
 * (order 0, occ 2), (1, 2), (0, 3), (1, 3), then window order 0 and 1.
 * Overwrites out and workspace. */
gw_status gw_autotune(gw_ctx* ctx, int64_t B, const float* bg, int64_t L_bg,
                      float* out, void* workspace, int64_t workspace_bytes,
                      int32_t reps, double* report);

/* ------------------------------------------------------------------------
 * Uneven (ragged) batches: signals of several size classes in one batch.
 * Each class is a full gw_config (its own fs, t_window, psd_length, fftlen,
 * f_min); all classes share n_det, det_id, approximant, prior ranges and
 * precision (0 or 1), and need N >= 2 L.  Up to GW_RAGGED_MAX_CLASSES
 * classes.  The class of each of the B signal slots is fixed when the
 * handle is created (host array cls[B]); parameters, offsets and noise are
 * drawn per batch exactly as gw_generate_batch draws them for the class's
 * configuration at global index batch_index*B + i, with parameter row 11
 * set to the class index.  Each stage is ONE persistent launch over all
 * classes: a Welch kernel and a fused window kernel pull groups of
 * (signal, detector) items of one class from an atomic queue, largest
 * transforms first; small transforms share a workgroup as sub-blocks.
 * Output: one flat float buffer; signal i occupies [n_det][N_i] floats from
 * out_offset[i] (gw_ragged_offsets).
 * ------------------------------------------------------------------------ */
#define GW_RAGGED_MAX_CLASSES 8
typedef struct gw_ragged gw_ragged;
/* Validate the classes, build the work plan (descriptors, queues, tables)
 * on the current device.  Allocates device memory; not for the hot path. */
gw_status gw_ragged_create(const gw_config* classes, int32_t n_classes,
                           const int32_t* cls, int64_t B, gw_ragged** out);
gw_status gw_ragged_destroy(gw_ragged* r);
const char* gw_ragged_last_error(const gw_ragged* r);
#define GW_RQ_B          0  /* signal slots                                  */
#define GW_RQ_OUT_FLOATS 1  /* floats of the flat output                     */
#define GW_RQ_PSD_FLOATS 2  /* floats of the flat PSD region                 */
#define GW_RQ_WORKSPACE  3  /* workspace bytes                               */
#define GW_RQ_PSD_OFFSET 4  /* byte offset of the PSD region in the workspace */
#define GW_RQ_NCLASSES   5
gw_status gw_ragged_query(const gw_ragged* r, int32_t key, int64_t* value);
/* Host arrays [B+1]: float offsets of each signal's output block and of its
 * [n_det][L/2+1] PSD block (the last entry is the total). */
gw_status gw_ragged_offsets(const gw_ragged* r, int64_t* out_offset, int64_t* psd_offset);
/* One ragged batch.  bg, L_bg: host arrays [n_classes] of device
 * background pointers (float [n_det][L_bg[c]], 4-byte aligned) and lengths;
 * classes with equal fs normally share one background.  out: float
 * [GW_RQ_OUT_FLOATS]; params_f32: float [12][B] or NULL; status: uint32
 * [B] or NULL.  Workspace layout: params double [12][B], offsets int64 [B],
 * then per-sample constants, the queue/batch counters, and the PSDs from
 * byte GW_RQ_PSD_OFFSET. */
gw_status gw_generate_ragged(gw_ragged* r, uint64_t seed, uint64_t batch_index,
                             const float* const* bg, const int64_t* L_bg,
                             float* out, float* params_f32, uint32_t* status,
                             void* workspace, int64_t workspace_bytes,
                             hipStream_t stream);
/* Graph of gw_generate_ragged(seed, first_batch + r, ...); see gw_graph. */
gw_status gw_ragged_graph_create(gw_ragged* r, uint64_t seed, uint64_t first_batch,
                                 const float* const* bg, const int64_t* L_bg,
                                 float* out, float* params_f32, uint32_t* status,
                                 void* workspace, int64_t workspace_bytes,
                                 gw_graph** graph);
/* Ragged kernel variants: radix orders as for gw_set_tuning, the
 * persistent grid of each stage in workgroups per compute unit (1..8), and
 * each stage's issue mode.  Window mode: 0 one persistent launch over all
 * classes (default), 1 one launch per class (largest first) with one
 * NC/16-thread workgroup per item.  Welch mode: 0 one persistent launch, 1
 * one launch per class (largest transform first, default) with one
 * L/16-thread workgroup per item at 3 waves per SIMD; the Welch grid only
 * applies to mode 0. */
#define GW_RTUNE_ORD_WINDOW 1
#define GW_RTUNE_ORD_WELCH  2
#define GW_RTUNE_GRID_WINDOW 3
#define GW_RTUNE_GRID_WELCH  4
#define GW_RTUNE_WINDOW_MODE 5
#define GW_RTUNE_WELCH_MODE  6
gw_status gw_ragged_set_tuning(gw_ragged* r, int32_t key, int64_t value);
gw_status gw_ragged_get_tuning(const gw_ragged* r, int32_t key, int64_t* value);
/* Autotuner of the ragged stages (synchronous, private stream): times the
 * Welch stage over radix order x grid {1, 2, 4 per CU} in mode 0 and radix
 * order in mode 1, and the window stage over issue mode x radix order,
 * `reps` launches each, in three interleaved rounds, and keeps the fastest.
 * report (host double [12], nullable): the best round's mean ms of Welch
 * mode 0 (order 0, grid 1, 2, 4), (order 1, grid 1, 2, 4), then window
 * (mode 0, order 0), (0, 1), (1, 0), (1, 1), then Welch mode 1 (order 0),
 * (order 1).  Overwrites out and workspace. */
gw_status gw_ragged_autotune(gw_ragged* r, const float* const* bg, const int64_t* L_bg,
                             float* out, void* workspace, int64_t workspace_bytes,
                             int32_t reps, double* report);


/* ------------------------------------------------------------------------
 * Learned waveform surrogate (an addition of this library to the waveform
 * step of section 3.1; approximant 1 only).  A 4-256-256-256-128 MLP with
 * bfloat16 MFMA forward/backward kernels (binary32 accumulation, binary32
 * master weights, AdamW) maps (M_c, q, chi1, chi2) to 64 + 64 reduced-basis
 * coefficients of the amplitude ratio A/A_N and phase residual P - P_N on
 * 1024 nodes log-spaced in geometric frequency Mf in [2e-3, 0.2].
 * Coefficients = A^T phi(theta) + zstd * z + zmean, where phi holds the PN
 * phase-coefficient functions (a least-squares skip path) and z is the MLP
 * output.  Training data come from the plain IMR-form model of this library.
 * A linear head on the last hidden layer predicts log10 of the mismatch; the
 * fused surrogate batch falls back to the plain model where it exceeds a
 * threshold.  The handle owns its weights and scratch for up to max_batch
 * rows; all data buffers are caller-owned device memory unless noted.
 * ------------------------------------------------------------------------ */
#define GW_SURR_NODES 1024
#define GW_SURR_OUT 128
#define GW_SURR_FEAT 9
#define GW_SURR_HIDDEN 256

gw_status gw_surrogate_create(gw_ctx* ctx, int64_t max_batch, gw_surrogate** out);
gw_status gw_surrogate_destroy(gw_surrogate* s);
const char* gw_surrogate_last_error(const gw_surrogate* s);
/* number of floats in the flat weight layout [W0 (16x256), b0, W1, b1, W2, b2,
 * W3 (256x128), b3], W stored [in][out] row-major; input rows 4..15 of W0 are
 * padding and stay zero */
int64_t gw_surrogate_n_weights(void);
gw_status gw_surrogate_set_weights(gw_surrogate* s, const float* host_flat, int64_t n);   /* host array; resets Adam */
gw_status gw_surrogate_get_weights(gw_surrogate* s, float* host_flat, int64_t n);         /* host array */
/* targets of the plain model at the nodes: ratio, dpsi float [B][1024];
 * feat double [B][9] (phi) */
gw_status gw_surrogate_targets(gw_surrogate* s, const double* params, int64_t B, float* ratio, float* dpsi,
                               double* feat, hipStream_t stream);
/* reduced basis (64 per target) from the first n target rows; synchronous */
gw_status gw_surrogate_fit_basis(gw_surrogate* s, const float* ratio, const float* dpsi, int64_t n, hipStream_t stream);
/* coefficients C float [n][128] (64 amplitude then 64 phase) */
gw_status gw_surrogate_project(gw_surrogate* s, const float* ratio, const float* dpsi, int64_t n, float* C,
                               hipStream_t stream);
/* least-squares skip path and standardisation; Z float [n][128] receives the
 * standardised residual targets; synchronous */
gw_status gw_surrogate_fit_skip(gw_surrogate* s, const double* feat, const float* C, int64_t n, float* Z,
                                hipStream_t stream);
gw_status gw_surrogate_standardise(gw_surrogate* s, const double* feat, const float* C, int64_t n, float* Z,
                                   hipStream_t stream);
/* theta float [B][4] = (M_c, q, chi1, chi2); out/z float [B][128] */
gw_status gw_surrogate_forward(gw_surrogate* s, const float* theta, int64_t B, float* out, hipStream_t stream);
/* gradients of the mean-squared loss (flat layout, device float) and the
 * summed squared error (device float[1] or NULL); no update */
gw_status gw_surrogate_gradients(gw_surrogate* s, const float* theta, const float* z, int64_t B, float* grads,
                                 float* loss, hipStream_t stream);
/* One AdamW step (section 5.1 trains with AdamW; Loshchilov & Hutter 2019)
 * on a batch of B <= max_batch: gradients of the mean-squared loss, moment
 * estimates m, v with bias correction, then for every weight
 *   p <- p - lr (m_hat / (sqrt(v_hat) + eps) + weight_decay p);
 * biases are updated without the decay term.  lr >= 0, weight_decay >= 0.
 * loss: device float[1] receiving the summed squared error, or NULL. */
gw_status gw_surrogate_train_step(gw_surrogate* s, const float* theta, const float* z, int64_t B, float lr,
                                  float weight_decay, float* loss, hipStream_t stream);
/* AdamW hyper-parameters (defaults beta1 0.9, beta2 0.999, eps 1e-8);
 * 0 <= beta < 1, eps > 0.  Kept in the checkpoint. */
gw_status gw_surrogate_set_adam(gw_surrogate* s, double beta1, double beta2, double eps);
/* last hidden layer float [B][256] */
gw_status gw_surrogate_hidden(gw_surrogate* s, const float* theta, int64_t B, float* h3, hipStream_t stream);
gw_status gw_surrogate_set_head(gw_surrogate* s, const float* host_head, int64_t n);      /* 257 floats */
/* Ridge fit of the mismatch head (synchronous): the coefficients w of
 * [h3 1] minimising ||[h3 1] w - y||^2 + ridge n ||w||^2 with
 * y = log10(max(mm, 1e-12)).  h3: device float [n][256] (last hidden layer,
 * gw_surrogate_hidden); mm: host double [n] measured mismatches (finite);
 * ridge >= 0. */
gw_status gw_surrogate_fit_head(gw_surrogate* s, const float* h3, const double* mm_host, int64_t n, double ridge);
/* node values float [B][2][1024] and predicted log10 mismatch float [B] (or NULL) */
gw_status gw_surrogate_nodes(gw_surrogate* s, const double* params, int64_t B, float* nodes, float* logmm,
                             hipStream_t stream);
/* h+, hx (interleaved complex float [B][N/2+1]) from node values; same
 * conventions and band as gen_fd_waveform */
gw_status gw_surrogate_waveform(gw_surrogate* s, const double* params, const float* nodes, int64_t B, float* hp,
                                float* hc, hipStream_t stream);
/* noise-weighted mismatch 1 - <a|b>/sqrt(<a|a><b|b>), <a|b> = 4 df Re sum
 * a conj(b)/S over f_min <= f_k < f_cut (IMR-form cut from params, or all
 * bins below Nyquist if params is NULL), 0 < k < N/2.  ha, hb interleaved
 * complex float [B][N/2+1]; psd float [N/2+1]; mm double [B]; all device
 * memory owned by the caller.  B = 0 returns GW_OK without reading any
 * buffer (they may be NULL); a NULL buffer otherwise is GW_EINVAL. */
gw_status gw_mismatch(gw_ctx* ctx, const float* ha, const float* hb, const float* psd, const double* params,
                      int64_t B, double* mm, hipStream_t stream);
/* The same mismatch maximised over a time shift t and a phase offset phi of
 * hb (the reported surrogate accuracy, beside the strict value above):
 * 1 - max over t, phi of <a|b e^{i phi - 2 pi i f t}>/sqrt(<a|a><b|b>), with
 * t over one window (the overlap has period T in t).  The best of the N/2
 * shifts t = n T/(N/2) (one inverse transform of the weighted products) is
 * refined by three parabolic steps (spacings 1, 1/4 and 1/16 of a shift) on
 * the directly summed overlap (binary64 sums).  The zero shift is always a
 * candidate, so the result is at most gw_mismatch's up to rounding.  Same
 * arguments, layouts and ownership as gw_mismatch; B = 0 launches nothing.
 * GW_EUNSUPPORTED for binary64 transforms (precision 2) or N > 32768. */
gw_status gw_mismatch_max(gw_ctx* ctx, const float* ha, const float* hb, const float* psd, const double* params,
                          int64_t B, double* mm, hipStream_t stream);
/* Bytes of workspace gw_generate_batch_surrogate needs for batch size B. */
gw_status gw_workspace_size_surrogate(const gw_ctx* ctx, int64_t B, int64_t* bytes);
/* gw_generate_batch with the waveform taken from the surrogate: prior draws,
 * surrogate node values and predicted log10 mismatch, Welch PSDs, then the
 * fused window kernel building each bin's signal from the node values
 * (binary64 Newtonian phase + interpolated residual).  Samples whose predicted
 * log10 mismatch exceeds log10_mm_max use the plain model instead and get
 * GW_STATUS_SURROGATE_FALLBACK.  Workspace: gw_workspace_size_surrogate(B)
 * bytes, laid out as for gw_generate_batch followed by the node values. */
gw_status gw_generate_batch_surrogate(gw_ctx* ctx, gw_surrogate* s, uint64_t seed, uint64_t batch_index,
                                      int64_t B, const float* bg, int64_t L_bg, float* out, float* params_f32,
                                      uint32_t* status, float log10_mm_max, void* workspace,
                                      int64_t workspace_bytes, hipStream_t stream);
/* Set the non-network state from host arrays: basis float [2][64][1024],
 * mean double [2][1024], skip path A float [9][128], zmean/zstd float [128],
 * head float [257] (weights: gw_surrogate_set_weights). */
gw_status gw_surrogate_set_state(gw_surrogate* s, const float* basis, const double* mean, const float* A,
                                 const float* zmean, const float* zstd, const float* head);
/* The same state copied to host arrays (synchronous). */
gw_status gw_surrogate_get_state(gw_surrogate* s, float* basis, double* mean, float* A, float* zmean,
                                 float* zstd, float* head);
/* Host checkpoint file: basis, skip path, standardisation, head, weights and
 * the optimiser state (AdamW moments, step counter, hyper-parameters), so
 * that training resumed after gw_surrogate_load continues exactly as without
 * the interruption.  Synchronous.  Load returns GW_EINVAL for a bad or
 * truncated file. */
gw_status gw_surrogate_save(gw_surrogate* s, const char* path);
gw_status gw_surrogate_load(gw_surrogate* s, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* GWGEN_H */
