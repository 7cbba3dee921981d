/*
 * spiir.h - C ABI of the MI355X (gfx950) SPIIR filter-bank library.
 *
 * The operation (Chu et al., "The SPIIR online coherent pipeline ...",
 * Section II.B.1, Eq. zk and the text before it): a template is approximated by
 * the summed response of first-order complex IIR filters, filter k having
 * feedback a_k, feedforward b_k and an integer delay d_k.  For whitened real
 * input x[n] (one stream per detector) the library computes
 *
 *     y_k[n] = a_k * y_k[n-1] + b_k * x[n - d_k]        (complex, per filter)
 *     z_t[n] = sum over the filters k of template t of y_k[n]
 *
 * i.e. the complex SNR series of every template, and from it the largest |z_t|
 * per window and its position (the per-template, per-second candidate of the
 * trigger selection in Section II.C.1).  Filter state and input history are
 * carried across calls, so a stream can be fed in packets of any length
 * (Section II.A: data arrive in one-second packets).  Zero state and zero input
 * precede the first packet.
 *
 * Conventions for every entry point:
 *  - Complex numbers are interleaved float pairs (re, im), i.e. complex64.
 *  - "host" pointers are read during the call only; the caller keeps ownership.
 *    "device" pointers are HIP device memory owned by the caller; the library
 *    reads or writes them asynchronously on the given stream, so they must stay
 *    valid until that stream has reached the call.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *    asynchronously; a device fault surfaces as SPIIR_E_HIP from a later call.
 *  - Argument errors are detected on the host before anything is enqueued; the
 *    call then returns a non-zero status, changes nothing, and spiir_last_error()
 *    describes the problem.  No C++ exception crosses this interface.
 *  - A bank is not re-entrant: use one bank from one host thread and one stream
 *    at a time.
 */
#ifndef SPIIR_H
#define SPIIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spiir_bank spiir_bank; /* opaque: device coefficients, state, history */

typedef enum {
    SPIIR_OK = 0,
    SPIIR_E_INVAL = 1,       /* invalid argument (shape, range, NULL, non-finite) */
    SPIIR_E_NOMEM = 2,       /* host or device allocation failed */
    SPIIR_E_HIP = 3,         /* a HIP runtime call failed (including earlier async faults) */
    SPIIR_E_STATE = 4,       /* call not valid in the bank's current state */
    SPIIR_E_UNSUPPORTED = 5  /* valid request outside what this build implements */
} spiir_status;

typedef enum {
    SPIIR_MODE_FP32_SCAN = 0,  /* plain recurrence, float32 state and arithmetic */
    SPIIR_MODE_BF16_BLOCK = 1  /* time-blocked form, split-bf16 matrix-core products */
} spiir_mode;

typedef struct {
    int32_t n_detectors;      /* D >= 1 independent input streams sharing the bank */
    int32_t max_chunk;        /* largest packet length n accepted by spiir_filter_chunk */
    int32_t max_delay;        /* input history kept per detector; 0 = largest d_k.
                                 Must be >= every d_k and <= 8191 */
    int32_t peak_window;      /* samples per peak window of spiir_filter_chunk;
                                 0 = one window per packet */
    int32_t mode;             /* spiir_mode */
    int32_t filters_per_lane; /* FP32 scan: filters held per GPU lane, 1, 2, 4 or 8; 0 = 4 */
    int32_t time_tile;        /* FP32 scan schedule.  -1 or 0: one wave per filter group
                                 walks the whole packet (see balance_wgs).  16..4096
                                 (multiple of 16): the persistent work-queue scan with
                                 packets cut into time tiles of this many samples */
    int32_t block_len;        /* block form: time-block length L, 64, 128 or 256; 0 = 128 */
    double long_pole_abs_a;   /* block form: a tile of 16 filters (of one template) carries
                                 its block-to-block state in FP64 when any of them has
                                 |a_k| above this, in FP32 otherwise; <= 0 = 0.999 */
    int32_t ckpt_stride;      /* differentiation: samples per checkpoint segment,
                                 a multiple of 128; 0 = 2048 */
    int32_t balance_wgs;      /* FP32 scan with time_tile -1 or 0: 0 = one wave per filter
                                 group; 1..8 = balanced static schedule with this many
                                 resident workgroups (of four waves) per compute unit,
                                 capped by what fits, used when a packet of max_chunk
                                 samples and its history fit one LDS window: every wave
                                 gets an equal share of the work, filter groups being
                                 cut in time between two waves where needed.  Every
                                 planned workgroup must be resident at once (the count
                                 is clamped to the kernel's occupancy); waves that
                                 share the GPU with other work may make a hand-off wait
                                 hit its bound (see wait_spins) */
    int32_t wait_spins;       /* FP32 scan, persistent or balanced schedule: bound of a wait
                                 for the state another wave hands over, in polls of about
                                 128 clocks; 0 = 4194304.  A wait that hits the bound lets
                                 the wave go on with a stale state: the library counts it
                                 (spiir_bank_info.scan_wait_timeouts) and every later
                                 spiir_filter_chunk / spiir_forward / spiir_backward on the
                                 bank returns SPIIR_E_STATE until spiir_bank_reset.  Small
                                 values exist to test that path */
} spiir_opts;

/* Fill `opts` with defaults: 1 detector, max_chunk 2048, max_delay 0 (from the bank),
 * one peak window per packet, FP32 scan, 4 filters per lane, no time split, no balanced
 * schedule, L = 128, 0.999, checkpoint stride 2048, wait bound 4194304 polls. */
void spiir_opts_default(spiir_opts *opts);

/*
 * Create a bank from host arrays (copied; the caller keeps and frees them).
 *   n_templates  T >= 1
 *   offsets      host int32[T+1], offsets[0] = 0, non-decreasing; template t owns
 *                filters offsets[t] .. offsets[t+1]-1 (F = offsets[T] >= 0)
 *   a, b         host complex64[F]: feedback and feedforward coefficients (the
 *                filter triplet of Section II.B.1); |a_k| < 1, all finite
 *   delay        host int32[F]: d_k in [0, max_delay] samples
 *   opts         may be NULL for defaults
 *   stream       stream used for the uploads
 *   out          receives the bank; NULL on failure
 * Allocates all device memory the bank will use: later calls allocate nothing.
 * Filter state and history start at zero.
 */
spiir_status spiir_bank_create(int32_t n_templates, const int32_t *offsets, const float *a,
                               const float *b, const int32_t *delay, const spiir_opts *opts,
                               void *stream, spiir_bank **out);

/* Release the bank's device memory (synchronises the bank's last stream).  NULL is ignored. */
spiir_status spiir_bank_destroy(spiir_bank *bank);

/* Zero the filter state and the input history of every detector: the next packet
 * is the start of a new stream.  Also clears the count of hand-off waits that hit their
 * bound (after waiting for the bank's last stream and `stream`, so that no earlier launch
 * can raise it afterwards). */
spiir_status spiir_bank_reset(spiir_bank *bank, void *stream);

/* Shape of a bank, for callers sizing their buffers. */
typedef struct {
    int32_t n_templates, n_detectors, max_chunk, max_delay, peak_window, mode;
    int64_t n_filters;
    int64_t device_bytes;     /* device memory held by the bank */
    int32_t n_slices;         /* FP32 scan work units (filter groups of one template) */
    int32_t filters_per_lane;
    int32_t time_tile;        /* 0 when the scan is not time-split */
    int32_t scan_waves;       /* grid of the persistent scan */
    int32_t block_len;
    int32_t n_long_pole;      /* block form: filters with |a_k| above long_pole_abs_a
                                 (counted from the coefficients given at creation) */
    int32_t scan_wait_timeouts; /* state hand-off waits (persistent or balanced scan) that hit their
                                   bound since creation or the last reset: the stream's results
                                   from that packet on are invalid; 0 normally */
    int32_t balance_waves;    /* waves per detector of the balanced schedule; 0 when the
                                 scan does not use it */
    int64_t block_mfma_flop_per_column; /* block form: matrix-core flop of its two products
                                 (input-to-state and output, three split products each)
                                 per column, i.e. per detector and block of L samples;
                                 0 for the FP32 scan */
} spiir_bank_info;

/* Fill `info`.  Waits for the bank's last stream (to read the wait-timeout count). */
spiir_status spiir_bank_get_info(const spiir_bank *bank, spiir_bank_info *info);

/*
 * Filter one packet of n samples per detector through the bank (Eq. zk,
 * Section II.B.1), advancing the stream.
 *   x       device float32 [D][n] (row stride n)
 *   n       1 <= n <= max_chunk; if peak_window > 0, n must be a multiple of it
 *   z       device complex64 [D][T][n], or NULL: the SNR series of every template
 *   peak    device float32 [D][T][W], or NULL: max |z_t| in each window of the
 *           packet (W = n / peak_window, or 1)
 *   argmax  device int32 [D][T][W], or NULL: index in the window of that maximum;
 *           among equal |z|^2 the lowest index.  |z|^2 is re*re + im*im rounded
 *           in float32 without fused multiply-add, and peak = sqrtf of it.
 * peak and argmax must both be given or both be NULL.
 * Returns SPIIR_E_STATE, enqueueing nothing, once an earlier launch on the bank had a
 * state hand-off wait hit its bound (see spiir_opts.wait_spins), until spiir_bank_reset.
 */
spiir_status spiir_filter_chunk(spiir_bank *bank, const float *x, int32_t n, float *z,
                                float *peak, int32_t *argmax, void *stream);

/*
 * Largest |z| per window of a complex series, and its position (the one-candidate-
 * per-template-per-window rule of Section II.C.1, trigger selection).
 *   z       device complex64 [rows][n]
 *   window  >= 1; the last window of a row may be shorter (ragged)
 *   peak    device float32 [rows][ceil(n/window)]
 *   argmax  device int32   [rows][ceil(n/window)], index within the window
 * Same tie and rounding rules as spiir_filter_chunk.  rows = 0 or n = 0 is a no-op.
 */
spiir_status spiir_peaks(const float *z, int64_t rows, int32_t n, int32_t window, float *peak,
                         int32_t *argmax, void *stream);

/*
 * ---- Trigger selection (Section II.C.1) ----
 * E|z_t|^2 for stationary white input of unit variance (the whitened strain of
 * Section II.A), per template, in FP64 on the host from the coefficients given at bank
 * creation (spiir_bank_trigger_weights uses the current device coefficients):
 *   E|z_t|^2 = sum_{k,l in t} Re[ b_k conj(b_l) conj(a_l)^(d_k-d_l) / (1 - a_k conj(a_l)) ]
 * (pairs ordered so that d_k >= d_l).  power: host double [T].  Synchronous.
 */
spiir_status spiir_bank_noise_power(const spiir_bank *bank, double *power);

/*
 * The weights spiir_triggers takes, weight_t = 2 / E|z_t|^2 (0 for a template whose
 * E|z_t|^2 is 0), computed on the GPU in FP64 with the same pair sum as
 * spiir_bank_noise_power but from the bank's current device coefficients (so they
 * follow spiir_bank_set_coeffs).  Enqueued on `stream`; allocates nothing.
 *   weight  device float32 [T]
 */
spiir_status spiir_bank_trigger_weights(const spiir_bank *bank, float *weight, void *stream);

/*
 * Single-detector candidates of Section II.C.1: at every sample the template with
 * the largest normalised SNR^2  rho2_t = |z_t|^2 * weight_t  (|z|^2 = re*re + im*im,
 * every product and sum rounded to float32; weight_t = 2 / E|z_t|^2 normalises each
 * quadrature to unit variance) is a candidate when rho2 > threshold^2; a template
 * keeps at most one candidate per window of `window` samples, the largest (lowest
 * sample on ties; lowest template on ties across templates).
 *   z        device complex64 [n_det][n_templates][n]
 *   weight   device float32 [n_templates]
 *   work     device uint64 [n_det][n_templates][W], W = ceil(n/window): scratch
 *   snr      device float32 [n_det][n_templates][W]: sqrtf(rho2) of the kept candidate, 0 if none
 *   index    device int32   [n_det][n_templates][W]: its sample in [0, n), -1 if none
 */
spiir_status spiir_triggers(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                            const float *weight, float threshold, int32_t window, void *work,
                            float *snr, int32_t *index, void *stream);

/*
 * spiir_triggers without the `work` argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as spiir_triggers; the key slots
 * live in a workspace the library keeps on every device it runs on (8 MiB, held until
 * the process ends), so the call allocates nothing.
 *   n_det * n_templates * ceil(n / window) must be <= 1048576, else SPIIR_E_INVAL
 *   (nothing enqueued).
 *   stream must belong to the calling thread's current device.
 * The first call on a device looks up that device's workspace address (not a stream
 * operation).  Every call on one device shares its workspace: calls that overlap in
 * time on one device (other streams, other host threads) race and give undefined
 * results; calls on one stream are ordered and safe.  The slots are cleared by a
 * kernel at the start of every call.
 */
spiir_status spiir_triggers_noalloc(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                                    const float *weight, float threshold, int32_t window,
                                    float *snr, int32_t *index, void *stream);

/*
 * ---- Signal-consistency statistic (Section II.C.1) ----
 * The correlation of each template with itself,
 *   R_t[j] = sum_m u_t[m+j] conj(u_t[m]),  j = 0..nj   (R_t[-j] = conj(R_t[j])),
 * of the template's impulse response u_t[m] = sum_k b_k a_k^(m-d_k) [m >= d_k]; in
 * closed form (a geometric sum per pair of filters), in FP64 on the GPU from the
 * bank's coefficients (float32 values promoted exactly).  R_t[0] = E|z_t|^2 for unit
 * white input.
 *   nj  1..4096
 *   R   device double [T][nj+1][2] (complex128, interleaved)
 * Synchronous: allocates, fills and frees temporary device copies of the coefficients.
 */
spiir_status spiir_bank_autocorr(const spiir_bank *bank, int32_t nj, double *R, void *stream);

/*
 * xi^2 at candidate samples (Section II.C.1): for row (detector, template) and its
 * candidate sample c,
 *   xi^2 = sum_{j=-nj..nj} |v[c+j] - v[c] A[j]|^2 / sum_{j=-nj..nj} (2 - 2|A[j]|^2),
 * A[j] = R_t[j] / R_t[0], v = z * sqrt(2 / R_t[0]) (unit variance per quadrature for unit
 * white input, so that noise alone gives a reduced chi-square of mean 1).  Sums in FP64.
 *   z      device complex64 [n_det][n_templates][n]
 *   index  device int32 [n_det][n_templates][n_win]: candidate sample in [0, n), -1 = none
 *          (the `index` output of spiir_triggers)
 *   R      device double [n_templates][nj+1][2] from spiir_bank_autocorr with the same nj
 *   xi2    device float32 [n_det][n_templates][n_win]; NaN where there is no candidate or
 *          c - nj < 0 or c + nj >= n (the caller keeps enough of the series around it)
 */
spiir_status spiir_xi2(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                       const int32_t *index, int32_t n_win, const double *R, int32_t nj, float *xi2,
                       void *stream);

/*
 * The detector average xi^2_C = (1/N_d) sum_J xi_J^2 of Section II.C.1 at coherent
 * candidates.  For the candidate of detector I, template t, window w at sample
 * c = index[I][t][w] with sky direction p = pix[I][t][w] (the coherent stage's best
 * direction, e.g. spiir_coherent's pix with one, unshifted, time shift), detector J is
 * read at its arrival time in that direction, s_J = c + tau[p][J] - tau[p][I], and xi_J^2
 * is spiir_xi2's statistic of series z[J][t] at s_J (FP64 sums).
 *   z        device complex64 [n_det][n_templates][n], 1 <= n_det <= 8
 *   index    device int32 [n_det][n_templates][n_win], -1 = no candidate
 *   pix      device int32 [n_det][n_templates][n_win], -1 = no direction
 *   tau      device int32 [n_pix][n_det]: the arrival-time offsets spiir_coherent used
 *   R        device double [n_templates][nj+1][2] from spiir_bank_autocorr with the same nj
 *   xi2_det  device float32 [n_det][n_templates][n_win][n_det] (last index J), or NULL
 *   xi2_c    device float32 [n_det][n_templates][n_win]: the mean over J, in detector order
 * NaN where there is no candidate, p is outside [0, n_pix), or some s_J - nj < 0 or
 * s_J + nj >= n.
 */
spiir_status spiir_xi2_network(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                               const int32_t *index, const int32_t *pix, int32_t n_win,
                               const int32_t *tau, int32_t n_pix, const double *R, int32_t nj,
                               float *xi2_det, float *xi2_c, void *stream);

/*
 * ---- Coherent search (Section II.C.1, Eq. llr_form; null statistic of the appendix) ----
 * For every candidate (detector I, template t, window w) at sample c = index[I][t][w],
 * every time shift k and every sky direction p, detector J contributes
 *   v_J = z[J][t][s_J],  s_J = c + tau[p][J] - tau[p][I] + shifts[k][(J-I) mod n_det] - shifts[k][0]
 * (background events shift the other detectors' series relative to the candidate's
 * detector: column r of the shift table applies to the detector r places after I),
 * and with the orthogonal matrix U[p] (N_d x N_d, the SVD factor of the noise-weighted
 * detector response; its first two columns span the signal plane)
 *   rho_C^2 = sum_{i<2} |sum_J U[p][J][i] v_J|^2,   rho_N^2 = sum_J |v_J|^2 - rho_C^2.
 * Per (candidate, shift) the direction with the largest rho_C^2 is kept (lowest p on
 * ties).  Float32 arithmetic.
 *   z       device complex64 [n_det][n_templates][n], 2 <= n_det <= 8
 *   index   device int32 [n_det][n_templates][n_win], -1 = no candidate (spiir_triggers)
 *   U       device float32 [n_pix][n_det][n_det] (row J, column i)
 *   tau     device int32 [n_pix][n_det]: arrival-time offsets in samples
 *   shifts  device int32 [n_shift][n_det]: background time shifts by relative detector
 *           position (all zero: foreground)
 *   snr2, null2  device float32 [n_det][n_templates][n_win][n_shift]: rho_C^2, rho_N^2
 *   pix     device int32 same shape: the direction; -1 (and NaN above) where there is no
 *           candidate or some s_J (any direction) leaves [0, n)
 */
spiir_status spiir_coherent(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                            const int32_t *index, int32_t n_win, const float *U, const int32_t *tau,
                            int32_t n_pix, const int32_t *shifts, int32_t n_shift, float *snr2,
                            int32_t *pix, float *null2, void *stream);

/*
 * ---- Differentiation (FP32 scan mode only) ----
 * For fitting coefficients to a target response (the overlap of Eq. overlap,
 * Section II.B.1, between a template and the summed filter response).  These
 * calls run a whole signal from zero state and zero history; they use the bank's
 * stream buffers, so the stream state is undefined afterwards (call
 * spiir_bank_reset before streaming again).  Gradients use the convention
 * dL/dRe(c) + i dL/dIm(c) for a real loss L and complex c (torch's).
 */

/* Number of complex64 values of the checkpoint buffer for a signal of n samples
 * (the filter state at the start of every ckpt_stride-sample segment, per detector). */
spiir_status spiir_ckpt_count(const spiir_bank *bank, int32_t n, int64_t *n_values);

/*
 * Forward pass over a whole signal from zero state: z as in spiir_filter_chunk.
 *   x     device float32 [D][n], 1 <= n <= max_chunk
 *   z     device complex64 [D][T][n]
 *   ckpt  device complex64 [spiir_ckpt_count], or NULL: states for spiir_backward
 */
spiir_status spiir_forward(spiir_bank *bank, const float *x, int32_t n, float *z, float *ckpt,
                           void *stream);

/*
 * Reverse-time adjoint: the gradient of a real loss L with respect to every a_k
 * and b_k, given grad_z = dL/dRe z + i dL/dIm z (device complex64 [D][T][n]) for
 * the z of spiir_forward on the same x with the same coefficients, and that
 * call's checkpoints.  With lambda_k[n] = grad_z_t[n] + conj(a_k) lambda_k[n+1]:
 *   grad_a_k = sum_n lambda_k[n] conj(y_k[n-1]),   grad_b_k = sum_n lambda_k[n] x[n-d_k]
 * summed over detectors.  Inside each checkpoint segment the states are recomputed
 * forward (no per-sample storage).
 *   grad_a, grad_b  device complex64 [F] in the bank's original filter order (overwritten)
 */
spiir_status spiir_backward(spiir_bank *bank, const float *x, int32_t n, const float *grad_z,
                            const float *ckpt, float *grad_a, float *grad_b, void *stream);

/*
 * Replace the coefficients with device arrays a, b (complex64 [F], original filter
 * order); delays and layout are kept.  Enqueued on `stream`; the values are not
 * validated (the caller keeps |a_k| < 1).  In the block mode the matrix-core operands
 * (Section II.B.1's filters unrolled over a time block) are regenerated from the new
 * coefficients on the GPU, also enqueued on `stream`; the stream state is kept either
 * way (call spiir_bank_reset to start a new stream).
 */
spiir_status spiir_bank_set_coeffs(spiir_bank *bank, const float *a, const float *b, void *stream);

/*
 * Kernel timing (diagnostics for roofline reporting).  While enabled, every
 * spiir_filter_chunk brackets the launch of the bank's main filtering kernel (the
 * FP32 scan kernel) with a pair of HIP events on the call's stream, for up to
 * `capacity` launches (the events are created here, not in later calls).
 * spiir_bank_kernel_time waits for the last recorded launch and returns the summed
 * kernel time in milliseconds and the number of timed launches; enabling again
 * restarts the count.  enable = 0 releases the events.
 */
spiir_status spiir_bank_set_timing(spiir_bank *bank, int32_t enable, int32_t capacity);
spiir_status spiir_bank_kernel_time(spiir_bank *bank, double *total_ms, int64_t *launches);

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char *spiir_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPIIR_H */
