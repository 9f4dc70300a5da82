/*
 * fcx — online all-to-all functional connectivity on one MI355X (gfx950).
 *
 * A session holds one connectivity estimate over a sliding window of trials
 * (the user-set number of averaged trials of the connectivity plug-in,
 * Sec. 2.5).  Each pushed trial [N nodes][M samples] is tapered and
 * transformed at the band bins only; its spectra are cached in a device ring
 * so a trial is never transformed twice (the reuse of stored per-trial
 * results, Sec. 2.4); running sums over the window are updated in place —
 * the new trial added, the evicted one subtracted — and the band-averaged
 * network of every enabled metric is refreshed.  The metrics are those of the
 * supplementary metric section: COH, IMAGCOHY, PLV, PLI, WPLI, USPLI,
 * debiased squared WPLI, COR and XCOR.  Only pairs i < j are computed
 * (undirected half, Sec. 2.4).
 *
 * Conventions (where the paper is silent):
 *   CSD_ij = X_i conj(X_j); IMCOH_ji = -IMCOH_ij.
 *   Band bins: k_lo = floor(f_lo F / fs), k_hi = floor(f_hi F / fs),
 *              inclusive, clamped to [0, F/2].
 *   Taper: periodic Hann 0.5 - 0.5 cos(2 pi n / M), or DPSS (unit energy,
 *          weights = concentration ratios); zero padding to F.
 *   Multitaper trial CSD/PSD: sum_l lam_l X_il conj(X_jl) / sum_l lam_l.
 *   sign(0) = 0; a metric whose denominator is exactly 0 is 0; the unit
 *   phasor of 0 is 0; USPLI and DSWPLI are NaN while K < 2.
 *   DSWPLI = ((sum Im)^2 - sum Im^2) / ((sum |Im|)^2 - sum Im^2)  (the
 *   debiased estimator the metric is named for).
 *   COR = mean over the window of each trial's Pearson correlation.
 *   XCOR = mean over the window of each trial's largest cross-correlation
 *          over the lags -L..L: for lag tau >= 0 the XCOR equation with node
 *          i advanced by tau against node j (its energy over the overlap,
 *          node j's over all M samples), for -tau the same with the nodes
 *          exchanged (so XCOR_ij = XCOR_ji); 0 where a denominator is 0.
 *          The lag of the maximum is not kept.
 *   Band value = arithmetic mean of the per-bin values.
 *
 * Network layout: packed upper triangle without diagonal, row-major:
 *   idx(i, j) = i (2N - i - 1) / 2 + (j - i - 1),  0 <= i < j < N,
 *   P = N (N - 1) / 2 entries per metric.
 *
 * Errors: every call returns an fcx_status; no exception crosses the ABI.
 * Handles are checked against a table, so a closed handle gives
 * FCX_E_CLOSED rather than undefined behaviour.  A session is used by one
 * thread at a time; different sessions may be used concurrently.
 */
#ifndef FCX_H
#define FCX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcx_session fcx_session;
typedef struct fcx_server fcx_server;

typedef enum {
    FCX_OK = 0,
    FCX_E_INVAL = 1,      /* bad argument or configuration                        */
    FCX_E_NOMEM = 2,      /* device or host allocation failed                     */
    FCX_E_DEVICE = 3,     /* a HIP runtime call failed                            */
    FCX_E_NOTREADY = 4,   /* no trial yet, or K < 2 for USPLI / DSWPLI            */
    FCX_E_BUSY = 5,       /* server: the session does not fit the HBM budget now  */
    FCX_E_CLOSED = 6,     /* the handle was closed                                */
    FCX_E_NONFINITE = 7   /* a pushed trial held NaN/Inf and was rejected         */
} fcx_status;

/* metric mask bits; fcx_read_network takes exactly one of them */
enum {
    FCX_COH = 1, FCX_IMCOH = 2, FCX_PLV = 4, FCX_PLI = 8,
    FCX_WPLI = 16, FCX_USPLI = 32, FCX_DSWPLI = 64, FCX_COR = 128, FCX_XCOR = 256
};
enum { FCX_TAPER_HANN = 0, FCX_TAPER_DPSS = 1 };
/* operand precision of the batch Gram sums (fcx_push_batch / fcx_resync) */
enum { FCX_GRAM_FP32 = 0, FCX_GRAM_BF16 = 1, FCX_GRAM_BF16X3 = 2 };
/* arithmetic of spectra and outputs: float32 or float64 */
enum { FCX_ELEM_F32 = 0, FCX_ELEM_F64 = 1 };

typedef struct {
    uint32_t struct_size;   /* sizeof(fcx_config), for forward compatibility      */
    int32_t n_nodes;        /* N, 2 <= N <= 65536                                  */
    int32_t n_samples;      /* M samples per trial, 2 <= M <= 8192                 */
    int32_t window_trials;  /* W, trials averaged (FIFO window), 1 <= W <= 32767   */
    int32_t n_fft;          /* F >= M, zero-padded DFT length                      */
    double fs_hz;           /* sampling rate                                       */
    double f_lo_hz;         /* band, inclusive bins (see conventions)              */
    double f_hi_hz;
    int32_t taper;          /* FCX_TAPER_*                                         */
    int32_t dpss_k;         /* number of DPSS tapers (1..8), DPSS only             */
    double dpss_nw;         /* time-bandwidth product NW, DPSS only                */
    uint32_t metrics;       /* OR of metric bits, non-zero                         */
    int32_t gram_precision; /* FCX_GRAM_*                                          */
    int32_t elem;           /* FCX_ELEM_*; input x and outputs use this type       */
    int32_t xcor_max_lag;   /* XCOR lags -L..L; 0: L = M - 1. Needs M + L <= 2048 */
} fcx_config;

/* Fill *cfg with defaults (Hann, all 8 metrics, FP32 Gram, F32). */
void fcx_config_init(fcx_config *cfg);

/* Device bytes a session with this configuration allocates (ring of W+1
 * spectra slots, running sums, COR sample ring, outputs, staging).
 * Returns -1 for an invalid configuration. */
int64_t fcx_footprint_bytes(const fcx_config *cfg);

/* Algorithmic HBM bytes of the pair update of one push: every running sum the
 * enabled metrics keep is read and written once per pair and bin (FP64 CSD,
 * |Im| and Im^2 sums; unit-phasor sums as int32 fixed point for FP32 sessions
 * with W <= 256, else FP64; sign sums as int8 for W <= 127, else int16), the
 * COR sum (FP64) once per pair, and each enabled metric's band mean written
 * once per pair.  Node data (spectra, power sums) are not counted.  Returns -1
 * for an invalid configuration. */
int64_t fcx_pair_update_bytes(const fcx_config *cfg);

/* Number of band bins, or -1 for an invalid configuration. */
int32_t fcx_band_bins(const fcx_config *cfg, int32_t *k_lo, int32_t *k_hi);

/*
 * Open a session on the current HIP device (Sec. 2.4: the connectivity
 * library's metric routines and the container of the resulting networks
 * behind an API; Sec. 2.5: the connectivity plug-in's settings, the number of
 * averaged trials W and the frequency band).  hip_stream is a hipStream_t to
 * order all the session's work on (NULL: the session creates its own).  The
 * library owns every device buffer it allocates here and frees them in
 * fcx_close.
 * Errors: FCX_E_INVAL (configuration), FCX_E_NOMEM, FCX_E_DEVICE.
 */
fcx_status fcx_open(const fcx_config *cfg, void *hip_stream, fcx_session **out);

/*
 * Push one trial x[N][M] (Sec. 2.5: each trial the averaging plug-in cuts
 * goes to the connectivity plug-in; SI-1 PSD/CSD: its spectra; Sec. 2.4: the
 * sums over trials kept up to date, stored per-trial values reused) (row
 * stride ld >= M elements; float for ELEM_F32, double for ELEM_F64).  x_on_device = 0: x is host memory, copied before
 * the call returns, so the caller may reuse it at once.  x_on_device = 1:
 * x is device memory that must stay valid until fcx_sync returns.
 * The push is stream-ordered and returns before the GPU work finishes.  It
 * is atomic: a trial holding NaN/Inf is detected on the device before any
 * running sum changes, is dropped, and the next fcx_sync or
 * fcx_read_network reports FCX_E_NONFINITE once.
 * Errors: FCX_E_INVAL, FCX_E_CLOSED, FCX_E_DEVICE.
 */
fcx_status fcx_push_trial(fcx_session *s, const void *x, int64_t ld, int x_on_device);

/*
 * Replace the window with n_trials trials (trial k at x + k*trial_stride,
 * node rows ld apart), n_trials <= W, and compute its networks in one batch
 * pass (SI-1 metric equations over a set of trials; Sec. 2.4: the metrics of
 * all trials at once): Re of the cross-spectral Gram and the unit-phasor Gram
 * on the matrix cores in the session's gram_precision, Im(X_i conj X_j) in
 * FP64 with its sign, |Im|, Im^2 and Im sums on the vector units.  Inputs must be finite
 * (checked on the device; a non-finite batch leaves the session empty and
 * reports FCX_E_NONFINITE at the next sync).  Strides are in elements of
 * cfg.elem.  A device-resident batch (x_on_device = 1) is transformed in one
 * launch per kernel; host trials are uploaded one at a time.  The batch
 * writes the band-mean networks directly; the running sums (which the batch
 * pass uses as scratch) are rebuilt from the cached window, in one pass, by
 * the next sliding push, per-bin read or fcx_resync.  A session with COR and
 * gram_precision FCX_GRAM_BF16 allocates, on its first batch call, a BF16
 * copy of a window of z-scored samples (W * N * Mz * 2 bytes, Mz = M rounded
 * up to a multiple of 32; not counted by fcx_footprint_bytes), kept until
 * fcx_close; FCX_E_NOMEM if that allocation fails.
 */
fcx_status fcx_push_batch(fcx_session *s, const void *x, int64_t n_trials, int64_t trial_stride,
                          int64_t ld, int x_on_device);

/*
 * Copy the current network of one metric into out (host or device memory)
 * (Sec. 2.4: the network container; Sec. 3.2: the frequency bins of an edge
 * averaged).
 * per_bin = 0: band mean, out_len >= P.  per_bin = 1: [B][P], out_len >= B*P
 * (COR and XCOR are broadband and always [P]).  Element type follows
 * cfg.elem; XCOR is computed in FP32 (an FP32 FFT per pair) for both,
 * except at the lags where the overlap holds under 1/1024 of the advanced
 * node's energy, which are summed directly in FP64.
 * *k_trials_out (may be NULL) receives K, the trials in the window.
 * Synchronous.  Returns FCX_E_NOTREADY (and fills NaN) for USPLI/DSWPLI
 * while K < 2 and when no trial was pushed; FCX_E_NONFINITE once after a
 * rejected push (the output is still the valid current network).
 */
fcx_status fcx_read_network(fcx_session *s, uint32_t metric, void *out, int64_t out_len,
                            int out_on_device, int per_bin, int32_t *k_trials_out);

/* Wait for the session's queued work (stream ordering; not a step of the
 * paper's method).  Returns FCX_E_NONFINITE once after a rejected push. */
fcx_status fcx_sync(fcx_session *s);

/* Rebuild every running sum from the cached trials of the window in one
 * pass (Sec. 2.4: the sums over the stored per-trial values): per pair and
 * bin the K cached trials are added oldest first with the sliding update's
 * own per-trial arithmetic, so the sums equal, bit for bit, those of pushing
 * the window's trials into an empty session, and each state element is
 * written once (XCOR's window sum is recomputed trial by trial).  Used after
 * a batch pass and to discard the rounding a very long run accumulates.
 * Synchronous.  Errors: FCX_E_CLOSED, FCX_E_DEVICE. */
fcx_status fcx_resync(fcx_session *s);

/* Release the session and every device buffer it owns; the handle becomes
 * invalid (FCX_E_CLOSED afterwards).  Not a step of the paper's method. */
fcx_status fcx_close(fcx_session *s);

/* The hipStream_t the session orders its work on. */
fcx_status fcx_session_stream(fcx_session *s, void **hip_stream);

/* Trials pushed and accepted so far, and trials rejected as non-finite. */
fcx_status fcx_session_counts(fcx_session *s, int64_t *accepted, int64_t *rejected);

/*
 * Kernel timing: when enabled, every launch of the listed kernels is
 * bracketed by HIP events on the session stream; fcx_kernel_time returns the
 * number of timed launches and their summed duration in milliseconds
 * (pending events are resolved, which synchronises the stream).
 */
enum { FCX_K_SPECTRA = 0, FCX_K_PSD = 1, FCX_K_PAIR_UPDATE = 2, FCX_K_COR = 3,
       FCX_K_PAIR_BATCH = 4, FCX_K_ZNORM = 5, FCX_K_XCOR = 6, FCX_K_COUNT = 7 };
fcx_status fcx_set_timing(fcx_session *s, int enable);
fcx_status fcx_kernel_time(fcx_session *s, int kernel, int64_t *launches, double *total_ms);

/* Host DPSS tapers: tapers[K][M] (unit energy) and concentration ratios[K]. */
fcx_status fcx_dpss(int32_t M, double NW, int32_t K, double *tapers, double *ratios);

const char *fcx_status_str(fcx_status st);

/*
 * HBM streaming probe: dst[i] = src[i] for n_bytes (multiple of 16) on the
 * given stream; used to calibrate traffic counters and the achievable copy
 * bandwidth.  Device pointers.
 */
fcx_status fcx_probe_copy(void *dst, const void *src, int64_t n_bytes, void *hip_stream);

/*
 * Read-modify-write probe of the pair state layout of an FP32 all-8 session:
 * buf (device, 41 * n_elems bytes) holds four FP64 planes, two int32 planes
 * and one int8 plane of n_elems elements, in that order; every element of
 * every plane is read, incremented and written once per call (non-temporal
 * hint, as the pair update uses).  Enqueued on hip_stream; the caller times
 * it.  Errors: FCX_E_INVAL, FCX_E_DEVICE.
 */
fcx_status fcx_probe_rmw(void *buf, int64_t n_elems, void *hip_stream);

/*
 * Matrix-core probe: 8192 wavefronts each run `iters` rounds of independent
 * MFMA chains on register operands (kind 0: v_mfma_f32_16x16x4_f32, 8
 * chains; 1: v_mfma_f32_32x32x2_f32, 4 chains; 2: v_mfma_f32_16x16x32_bf16,
 * 8 chains) and write one float per lane to out (device, >= 524288 floats).
 * *flops receives the floating-point operations of the call.  Enqueued on
 * hip_stream; the caller times it.  Errors: FCX_E_INVAL, FCX_E_DEVICE.
 */
fcx_status fcx_probe_mfma(int32_t kind, int32_t iters, float *out, double *flops, void *hip_stream);

/* ------------------------------------------------------------------------
 * Network post-processing for display (results sections and the online
 * pipeline: every network is normalised by its maximum edge weight, only the
 * strongest fraction of its edges is drawn, and nodes are sized by their
 * degree in that thresholded network).
 *
 * w is one packed upper-triangle FP32 network of n_nodes nodes (P =
 * n(n-1)/2 edges, pair (i, j), i < j, at i(2n-i-1)/2 + j-i-1), e.g. the
 * device output of fcx_read_network.  Over its finite edges E (USPLI and
 * DSWPLI are NaN below two trials):
 *   max_abs     = max |w_e|
 *   w_norm_e    = w_e / max_abs  (FP32 division; 0 when max_abs = 0;
 *                 non-finite edges copied)
 *   k           = min(ceil(fraction * P), |E|)
 *   threshold   = |w| of the k-th strongest edge (+inf when k = 0)
 *   selected_e  = 1 iff e in E and |w_e| >= threshold (ties are all kept,
 *                 so n_selected >= k; equal when the weights are distinct)
 *   degree_i    = selected edges at node i
 *   strength_i  = sum of |w_norm_e| over them (summed exactly in units of
 *                 2^-32, stored as FP32)
 * Strength is taken on |w| so that signed ImCoh keeps its strongest negative
 * edges.  w, w_norm [P], selected [P] (bytes), degree and strength [n] are
 * device pointers; any output may be NULL; w_norm may equal w (in place).
 * The call enqueues its kernels on hip_stream (NULL: the default stream),
 * waits for them and fills *info (may be NULL).  The first call on a device
 * allocates a control block of about 1 MB that is kept until the process
 * ends; calls on one device are serialised on it.  Errors: FCX_E_INVAL for
 * n_nodes outside [2, 65536], a NULL w or a fraction outside [0, 1];
 * FCX_E_NOMEM / FCX_E_DEVICE from HIP.
 * ------------------------------------------------------------------------ */
typedef struct {
    float max_abs;
    float threshold;
    int64_t k;
    int64_t n_finite;
    int64_t n_selected;
} fcx_select_info;

fcx_status fcx_network_select(int32_t n_nodes, const float *w, double fraction, float *w_norm,
                              uint8_t *selected, int32_t *degree, float *strength, fcx_select_info *info,
                              void *hip_stream);

/* fcx_network_select_noalloc: the same selection for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, outputs and errors are those
 * of fcx_network_select, with these differences:
 *   - no hipMalloc, hipFree or other allocating call is made: the control
 *     block (about 0.7 MB) is a device array inside the library, one copy per
 *     device, held until the process ends; its address is looked up on the
 *     first call on a device (FCX_E_DEVICE if that fails; FCX_E_INVAL for a
 *     device index of 64 or more);
 *   - the largest network is 65536 nodes (FCX_E_INVAL above; the size of the
 *     array's per-node counters);
 *   - with info == NULL the call only enqueues its kernels on hip_stream and
 *     returns (no wait, nothing copied back: usable under graph capture);
 *     with info non-NULL it waits for the stream and fills *info.
 * Every call on a device shares that device's array and leaves its contents
 * behind (each call clears what it needs first, with a kernel): calls whose
 * work overlaps on one device (different streams, or host threads racing on
 * one stream) corrupt each other's results.  The caller owns w and the
 * outputs. */
fcx_status fcx_network_select_noalloc(int32_t n_nodes, const float *w, double fraction, float *w_norm,
                                      uint8_t *selected, int32_t *degree, float *strength,
                                      fcx_select_info *info, void *hip_stream);

/* ------------------------------------------------------------------------
 * Stream front end (the noise-reduction and averaging plug-ins of the online
 * pipeline, Sec. 2.5): a linear-phase FIR filter applied block by block by
 * FFT convolution with overlap-add, all channels in parallel, and trials cut
 * around the rising edges of a trigger channel, ready to push.
 * ------------------------------------------------------------------------ */
typedef struct fcx_stream fcx_stream;
enum { FCX_FIR_LOWPASS = 0, FCX_FIR_HIGHPASS = 1, FCX_FIR_BANDPASS = 2 };

/*
 * Windowed-sinc FIR design (Hamming window, odd length T, symmetric: linear
 * phase with group delay (T-1)/2).  Lowpass f1; highpass f1 (spectral
 * inversion); bandpass f1..f2.  Scaled to gain 1 at DC, at Nyquist, or at
 * the band centre.  n_taps = 0 takes the odd T >= 3.3 fs / transition_hz.
 * taps (host, capacity cap) receives the coefficients; taps = NULL only
 * reports the length in *n_taps_out.  Errors: FCX_E_INVAL (cut-offs outside
 * (0, fs/2), f2 <= f1 for a bandpass, an even n_taps, cap < T).
 */
fcx_status fcx_fir_design(int32_t kind, double fs_hz, double f1_hz, double f2_hz, double transition_hz,
                          int32_t n_taps, double *taps, int32_t cap, int32_t *n_taps_out);

typedef struct {
    uint32_t struct_size;      /* sizeof(fcx_stream_config)                          */
    int32_t n_channels;        /* C data channels (all filtered)                     */
    int32_t block_len;         /* samples per pushed block                           */
    int32_t n_taps;            /* T, odd; block_len + T - 1 <= 4096                  */
    const double *taps;        /* host, T coefficients (copied by fcx_stream_open)   */
    float trigger_threshold;   /* an event where trig[n-1] < thr <= trig[n]          */
    int32_t pre_samples;       /* trial = raw times n0 - pre .. n0 + post - 1        */
    int32_t post_samples;      /* (>= 1)                                             */
} fcx_stream_config;

/* Open a stream on the current device; work is ordered on hip_stream (NULL:
 * the default stream).  Errors: FCX_E_INVAL, FCX_E_NOMEM, FCX_E_DEVICE. */
fcx_status fcx_stream_open(const fcx_stream_config *cfg, void *hip_stream, fcx_stream **out);

/*
 * Push the next block: x [C][block_len] (device, row stride ld >= block_len)
 * and the trigger channel trig [block_len] (device).  The data are filtered
 * (the output lags by D = (T-1)/2 samples; optional y [C][block_len] device
 * receives the filtered block).  Every trial whose window is complete is
 * written, filtered and shifted by D (so it covers the raw times around its
 * event), to trials [k][C][pre + post] (device, up to cap trials), in event
 * order; *n_trials gets their number.  *n_dropped (may be NULL) counts the
 * events whose window starts before the stream or that exceeded cap.
 * Synchronous.  Errors: FCX_E_INVAL, FCX_E_CLOSED, FCX_E_DEVICE.
 */
fcx_status fcx_stream_push(fcx_stream *s, const float *x, int64_t ld, const float *trig, float *y,
                           float *trials, int32_t cap, int32_t *n_trials, int32_t *n_dropped);
fcx_status fcx_stream_close(fcx_stream *s);

/* ------------------------------------------------------------------------
 * Time-resolved phase connectivity from the analytic signal: the approach
 * the paper sets against its own in Sec. 4 (restrict every node to a narrow
 * band with a temporal filter, form the analytic signal by the Hilbert
 * transform, and estimate connectivity from the instantaneous phase and
 * amplitude), on one segment of N nodes x M samples at a time:
 *
 *   y_i   = h * x_i, the full causal convolution of the zero-extended
 *           segment (length M + T - 1)
 *   z_i   = analytic signal of y_i over F points (the smallest power of
 *           two >= max(M + T - 1, 256), zero padded): spectrum x 1 at DC
 *           and F/2, x 2 at the positive frequencies, 0 at the negative
 *           ones; samples D .. D + M - 1 with D = (T - 1) / 2 (so Re z_i is
 *           the delay-compensated filtered segment)
 *   windows of win_len samples starting at 0, hop, 2 hop, ... (while they
 *           fit in M): the seven spectral metrics of the session (COH,
 *           IMCOH, PLV, PLI, WPLI, USPLI, DSWPLI, same conventions) with the
 *           window's samples in the role of the trials, i.e. from the
 *           instantaneous cross-spectra z_i(t) conj(z_j(t)) and powers
 *           |z_i(t)|^2.
 * ------------------------------------------------------------------------ */
typedef struct fcx_hilbert fcx_hilbert;

typedef struct {
    uint32_t struct_size;      /* sizeof(fcx_hilbert_config)                         */
    int32_t n_nodes;           /* N, 2 <= N <= 65536                                 */
    int32_t n_samples;         /* M >= 1 samples per segment; M + T - 1 <= 4096      */
    int32_t n_taps;            /* T, odd (1 with taps {1}: no filter)                */
    const double *taps;        /* host, T coefficients (copied), e.g. fcx_fir_design */
    int32_t win_len;           /* samples per window, 1..M; 0: M (one window)        */
    int32_t win_hop;           /* samples between window starts; 0: win_len          */
    uint32_t metrics;          /* OR of FCX_COH .. FCX_DSWPLI, non-zero              */
    int32_t gram_precision;    /* FCX_GRAM_* of the cross-spectrum Gram sums         */
} fcx_hilbert_config;

/* Open on the current device; work is ordered on hip_stream (NULL: the
 * default stream).  Errors: FCX_E_INVAL, FCX_E_NOMEM, FCX_E_DEVICE. */
fcx_status fcx_hilbert_open(const fcx_hilbert_config *cfg, void *hip_stream, fcx_hilbert **out);

/* Number of windows per segment and the transform length F (either pointer
 * may be NULL). */
fcx_status fcx_hilbert_info(fcx_hilbert *h, int32_t *n_windows, int32_t *fft_len);

/*
 * One segment: x [N][M] (device FP32, row stride ld >= M).  out (device
 * FP32) receives metric m (bit 1 << m) of window w for pair (i, j) at
 * out[(w * 7 + m) * P + idx(i, j)], P = N (N - 1) / 2, for the requested
 * metrics (the other rows are not written).  z (device, may be NULL)
 * receives the analytic signal as [M][N] complex FP32 (re, im).  The call
 * only enqueues work on the handle's stream.  Nodes 2k and 2k + 1 share one
 * transform: a non-finite input sample makes the analytic signals of both
 * non-finite and the metrics of their pairs meaningless (the zero-denominator
 * rules may turn them into 0 rather than NaN); other pairs are unaffected.
 * Errors: FCX_E_INVAL (NULL x or out, ld < M), FCX_E_CLOSED, FCX_E_DEVICE.
 */
fcx_status fcx_hilbert_run(fcx_hilbert *h, const float *x, int64_t ld, float *out, float *z);
fcx_status fcx_hilbert_close(fcx_hilbert *h);

/* ------------------------------------------------------------------------
 * Serving: many concurrent sessions, continuous batching (the online
 * pipeline's plug-ins joined by buffers, Sec. 2.5, for many sessions at once;
 * the batching itself is not in the paper).
 *
 * A server owns an HBM budget.  fcx_server_open admits a session only if its
 * footprint fits what is left (FCX_E_BUSY otherwise; retry after another
 * session closes).  A served session's footprint is
 * fcx_server_footprint_bytes: the plain session's buffers with
 * FCX_SERVER_MAX_GROUP - 1 more ring slots, plus two input buffers of
 * FCX_SERVER_MAX_GROUP trials (the uploads of one tick run on a copy stream
 * while the previous tick computes).  Submitted trials of all sessions are gathered by a
 * server thread into ticks: one tick runs the spectra, power and pair-update
 * work of every session with pending trials as a few batched launches whose
 * workgroups drain a shared list of (session, tile) items, so sessions of
 * different N and W overlap on the device.  A session's queued trials (up to
 * FCX_SERVER_MAX_GROUP finite ones) are coalesced into one pass over its
 * running sums, read once and written once, the trials applied in
 * submission order with the single push's arithmetic; a non-finite trial
 * goes alone and is rejected as by fcx_push_trial.  Each result equals the
 * same session run alone, bit for bit.  fcx_read_network, fcx_sync and
 * fcx_resync on a served session first wait until every trial submitted
 * before them is applied (a session is used from one thread at a time).
 * Served sessions compute in float32 and without XCOR (FCX_E_INVAL
 * otherwise).
 * ------------------------------------------------------------------------ */
#define FCX_SERVER_MAX_GROUP 8
/* Device bytes a session with this configuration holds when served (its
 * ring has W + FCX_SERVER_MAX_GROUP slots, so a coalesced group never
 * overwrites a trial it still evicts; plus the two tick input buffers).
 * Returns -1 for a configuration the server does not take. */
int64_t fcx_server_footprint_bytes(const fcx_config *cfg);
fcx_status fcx_server_create(int64_t hbm_budget_bytes, fcx_server **out);
fcx_status fcx_server_open(fcx_server *srv, const fcx_config *cfg, fcx_session **out);
/* Copy x (host, [N][M] with row stride ld) and queue it; *ticket identifies it. */
fcx_status fcx_server_submit(fcx_server *srv, fcx_session *s, const void *x, int64_t ld,
                             uint64_t *ticket);
/* done = 1 once the trial's update finished on the device; latency_s is
 * submit -> completion observed by the server thread (host monotonic clock). */
fcx_status fcx_server_poll(fcx_server *srv, uint64_t ticket, int *done, double *latency_s);
/* Wait until every submitted trial is done. */
fcx_status fcx_server_drain(fcx_server *srv);
/* Budget accounting: bytes admitted, bytes left, sessions open. */
fcx_status fcx_server_usage(fcx_server *srv, int64_t *used, int64_t *left, int32_t *n_sessions);
/* hold = 1: submissions are queued but no tick is formed (the queues fill,
 * so the next ticks coalesce whole bursts); hold = 0 lets the server thread
 * run again.  fcx_server_drain returns FCX_E_BUSY while held with trials
 * pending; reading, syncing or closing a served session and
 * fcx_server_destroy release the hold (they need the trials applied). */
fcx_status fcx_server_hold(fcx_server *srv, int hold);
/* Ticks run, trials applied, the largest coalesced group and the summed
 * device time of the finished ticks (ms; from the tick's first kernel being
 * able to start to its last one finishing, on the server's stream) so far.
 * Any pointer may be NULL. */
fcx_status fcx_server_counts(fcx_server *srv, int64_t *ticks, int64_t *trials, int64_t *max_group,
                             double *busy_ms);
/* Close a session opened on this server (drains its pending trials). */
fcx_status fcx_server_close_session(fcx_server *srv, fcx_session *s);
fcx_status fcx_server_destroy(fcx_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* FCX_H */
