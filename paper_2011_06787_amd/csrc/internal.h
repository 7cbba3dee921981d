// Internal declarations shared by the HIP translation units of libspiir.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/spiir.h"

namespace spiir {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kSub = 16;           // samples per register sub-tile of the FP32 scan
constexpr int kScanWaves = 4;      // waves per workgroup of the FP32 scan
constexpr int kMaxDelay = 8191;    // largest supported delay (samples)
constexpr int kWindowFloats = 12288;  // LDS input window of the FP32 scan (floats)
constexpr int kSimdKeys = 1 << 15;  // hardware SIMD ids (HW_ID bits 4..15, XCC id)
constexpr int kPeerTableWords = 8;  // words per SIMD of the balanced scan's progress table
constexpr int kLdsPerCu = 160 * 1024;  // LDS of one compute unit (bytes)

// Device bookkeeping of the persistent FP32 scan (one per bank).
struct ScanQueue {
    uint32_t head;   // next work item to hand out in the current launch
    uint32_t done;   // waves of the current launch that have finished
    uint32_t epoch;  // time tiles every slice completed before the current launch
    uint32_t error;  // sticky count of dependency waits that hit their bound
};

// Block form: one row tile of the input-to-state product (16 filters of one
// template, sorted by delay) and its band of input offsets.
struct WTile {
    int32_t tmpl;
    int32_t f0;        // first filter of the tile, in the template's delay order
    int32_t sigma_lo;  // first input offset (relative to the block start), multiple of 16
    int32_t nks;       // K steps of 16 offsets
    int64_t a_off;     // bf16 offset of the tile's operand blocks
    int64_t g0;        // first filter of the tile in the bank's sorted-padded order
};

// Block form: per-template operands of the output product z = [P | M] [Y; H].
struct BTemplate {
    int32_t fpad;      // filters rounded up to 16
    int32_t nks_p;     // K steps of the state part (2*fpad/16)
    int32_t nks_m;     // K steps of the input part ((L - sigma_lo)/16)
    int32_t sigma_lo;  // first input offset of the input part, multiple of 16
    int64_t a_off;     // bf16 offset of the template's operand blocks
    int64_t y_off;     // element offset of the template's state rows (per detector)
    int64_t g0;        // first filter of the template in the sorted-padded order
};

// One FP32-scan work unit: up to 64 * filters_per_lane filters of one template.
// Its filters occupy `n_slots` consecutive slots of 64 lanes starting at `slot_base`.
// A slice that holds all of its template's filters (`single`) is the template's SNR
// series itself: the scan writes it straight into z.
struct Slice {
    int32_t tmpl;
    int32_t slot_base;
    int32_t n_slots;
    int32_t single;
};

// Balanced FP32-scan schedule: one entry of a wave's work list, the slice's samples
// [phi0 n, phi1 n) with phi in units of 1/65536 of the packet (rounded down to whole
// sub-tiles in the kernel).  A slice cut between two waves has phi1 < 65536 on the
// wave that runs its first part (at the start of that wave's list) and phi0 > 0 on
// the wave that continues it (at the end of its list); `flag` indexes their hand-off.
struct Seg {
    int32_t slice;
    int32_t phi0;
    int32_t phi1;
    int32_t flag;   // -1 when the slice is not cut
};
constexpr int32_t kPhiOne = 65536;

struct Bank {
    // shape
    int32_t n_templates = 0;
    int64_t n_filters = 0;
    int32_t n_det = 1;
    int32_t max_chunk = 0;
    int32_t hist_len = 0;      // input history kept per detector (>= every delay)
    int32_t peak_window = 0;
    int32_t mode = SPIIR_MODE_FP32_SCAN;
    int32_t fpl = 4;           // filters per lane (FP32 scan)
    int32_t block_len = 128;
    double long_pole = 0.999;
    int32_t scan_tile = 2048;  // samples per LDS input window of the one-shot FP32 scan
    int32_t time_tile = 256;   // samples per work item of the persistent scan; 0 = one-shot
    int32_t scan_waves = 0;    // resident waves of the persistent scan (grid size)
    bool balanced = false;     // one-shot scan runs the balanced static schedule
    int32_t balance_per_cu = 0;  // requested resident workgroups per compute unit
    int32_t balance_unit = 0;    // waves per detector with one workgroup per compute unit
    int32_t balance_waves = 0;   // waves per detector of the balanced schedule
    int32_t balance_lds = 0;     // dynamic LDS per workgroup of the balanced scan (bytes)
    int32_t n_splits = 0;        // slices cut between two waves (per detector)
    int32_t ckpt_stride = 2048;  // differentiation: samples per checkpoint segment
    int32_t bwd_max_seg = 0;     // segments of a max_chunk signal (adjoint partial sums sized for it)

    // FP32 scan layout
    int32_t n_slices = 0;
    int64_t n_slots = 0;       // slots of 64 lanes
    float2 *d_a = nullptr;     // [n_slots*64]
    float2 *d_b = nullptr;     // [n_slots*64]
    int32_t *d_delay = nullptr;  // [n_slots*64]
    int32_t *d_perm = nullptr;   // [n_slots*64]: original filter index, -1 for padding
    Slice *d_slices = nullptr;   // [n_slices]
    int32_t *d_tmpl_slices = nullptr;  // [T+1]: slices of template t are [off[t], off[t+1])
    float2 *d_state = nullptr;   // [D][n_slots*64]
    float *d_hist = nullptr;     // [D][hist_len]
    float2 *d_partial = nullptr; // [D][n_slices][max_chunk]
    int32_t *d_multi_tmpl = nullptr;  // templates with other than one slice, ascending
    int32_t n_multi = 0;
    ScanQueue *d_queue = nullptr;
    uint32_t *d_flags = nullptr; // [D][n_slices]: tiles completed (epoch-relative)
    Seg *d_segs = nullptr;             // balanced schedule: work lists of all waves
    int32_t *d_seg_off = nullptr;      // [balance_waves+1]: list of wave w is [off[w], off[w+1])
    uint32_t *d_split_flags = nullptr; // [D][n_splits]: launches whose first part has published
    float2 *d_split_cand = nullptr;    // [D][n_splits]: peak candidate (|z|^2, index bits) that
                                       // the first part leaves for a window it does not finish
    ScanQueue *d_bqueue = nullptr;     // balanced schedule: launch epoch, finished waves, timeouts
    uint32_t *d_simd_tab = nullptr;    // balanced schedule: per-SIMD progress of co-resident waves
    float2 *d_bwd_part = nullptr;      // adjoint per-segment sums [D][bwd_max_seg][6][lanes]
    uint32_t wait_spins = 1u << 22;    // bound of a state hand-off wait (polls)
    uint32_t *h_wait_flag = nullptr;   // pinned host word: set by a wait that hit its bound
    uint32_t *d_wait_flag = nullptr;   // its device alias
    std::vector<int32_t> h_slice_slots;  // slots of every slice (host copy, for planning)
    int32_t *d_order = nullptr;  // [D*n_slices]: det*n_slices + slice, largest slices first
    int32_t *d_slice_order = nullptr;  // [n_slices]: slices, largest first

    // block form (split-bf16 matrix-core products)
    int32_t hist_pad = 0;        // history samples kept in the split input, multiple of 16
    int32_t n_wtiles = 0;
    int32_t max_wg_band = 0;     // widest input band over groups of 4 consecutive tiles
    int64_t n_fpad = 0;          // filters in sorted-padded order
    int64_t y_per_det = 0;       // state-row elements per detector (NBmax * sum 2*fpad)
    int32_t n_long_pole = 0;
    WTile *d_wtiles = nullptr;
    BTemplate *d_btmpl = nullptr;
    uint16_t *d_wa = nullptr;    // input-to-state operand blocks (bf16 hi/lo)
    uint16_t *d_pa = nullptr;    // output operand blocks (bf16 hi/lo)
    double2 *d_aL = nullptr;     // [n_fpad] a^L in FP64
    int32_t *d_lp = nullptr;     // [n_fpad] 1 if |a| > long_pole
    double2 *d_state64 = nullptr;  // [D][n_fpad] carried state
    uint16_t *d_yt = nullptr;    // [2][D][y_per_det]: state entering each block, bf16 hi / lo planes
    int64_t xs_stride = 0;       // per-detector length of the split input
    uint16_t *d_xs = nullptr;    // [2][D][xs_stride]: input from -hist_pad, bf16 hi / lo planes
    float2 *d_zbuf = nullptr;    // [D][T][max_chunk] when the caller passes no z
    float2 *d_ga = nullptr;      // [n_fpad] coefficients in sorted-padded order (0 for padding)
    float2 *d_gb = nullptr;
    int32_t *d_gd = nullptr;     // [n_fpad] delays in sorted-padded order (padding: past every band)
    int32_t *d_wblk = nullptr;   // [n_wblocks] tile of every input-to-state operand block
    int64_t n_wblocks = 0;
    int64_t block_flop_per_col = 0;   // matrix-core flop of both products per column
    int32_t max_p_blocks = 0;    // output-operand blocks of the largest template: state part
    int32_t max_m_blocks = 0;    // and input part
    int32_t out_ksplit = 1;      // workgroups sharing one output tile's K steps
    float2 *d_zpart = nullptr;   // [out_ksplit][D][T][n] partial outputs when out_ksplit > 1

    int64_t device_bytes = 0;
    hipStream_t last_stream = nullptr;

    // host copy of the bank (noise power on request)
    std::vector<int32_t> h_offsets, h_delay;
    std::vector<float> h_a, h_b;

    // optional kernel timing
    std::vector<hipEvent_t> ev_start, ev_stop;
    int64_t timed = 0;
    std::vector<void *> allocations;
};

// Launchers (enqueue only; arguments already validated).
size_t scan_fp32_lds_bytes(int32_t tile, int32_t hist_len);
size_t scan_persistent_lds_bytes(int32_t tile, int32_t hist_len);
hipError_t prepare_scan_fp32(Bank &bk);
// True when the scan launch for these arguments is the balanced schedule, which then
// also finds the peaks of every single-slice template (and writes nothing for them
// when z is not asked for): the slice sum then skips those templates.
bool scan_fuses_singles(const Bank &bk, int32_t n, bool with_ckpt, bool with_peaks);
// Single-slice templates go straight into z (when given) in every schedule.
hipError_t launch_scan_fp32(const Bank &bk, const float *x, int32_t n, float2 *ckpt, float2 *z,
                            float *peak, int32_t *argmax, hipStream_t s);
size_t backward_lds_bytes(int32_t stride, int32_t hist_len, int32_t fpl);
hipError_t prepare_backward(const Bank &bk);
hipError_t launch_backward(const Bank &bk, const float *x, int32_t n, const float2 *gz,
                           const float2 *ckpt, float2 *grad_a, float2 *grad_b, hipStream_t s);
hipError_t launch_set_coeffs(const Bank &bk, const float2 *a, const float2 *b, hipStream_t s);
hipError_t launch_hist_update(const Bank &bk, const float *x, int32_t n, hipStream_t s);
hipError_t launch_reduce_peaks(const Bank &bk, int32_t n, float2 *z, float *peak,
                               int32_t *argmax, const float *x, bool fused, hipStream_t s);
hipError_t launch_peaks(const float2 *z, int64_t rows, int32_t n, int32_t window, float *peak,
                        int32_t *argmax, hipStream_t s);
hipError_t launch_zero(void *ptr, int64_t bytes, hipStream_t s);
hipError_t launch_triggers(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                           const float *weight, float threshold, int32_t window,
                           unsigned long long *work, float *snr, int32_t *index, hipStream_t s);
// Key slots (64-bit) of the workspace spiir_triggers_noalloc keeps on every device.
constexpr int64_t kTriggerScratchSlots = int64_t(1) << 20;
hipError_t launch_triggers_noalloc(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                                   const float *weight, float threshold, int32_t window,
                                   float *snr, int32_t *index, hipStream_t s);
hipError_t launch_block_bf16(const Bank &bk, const float *x, int32_t n, float2 *z, hipStream_t s);
hipError_t launch_autocorr(int32_t n_templates, const int32_t *offsets, const float2 *a,
                           const float2 *b, const int32_t *d, int32_t nj, double2 *R, hipStream_t s);
hipError_t launch_coherent(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                           const int32_t *index, int32_t n_win, const float *U, const int32_t *tau,
                           int32_t n_pix, const int32_t *shifts, int32_t n_shift, float *snr2,
                           int32_t *pix, float *null2, hipStream_t s);
hipError_t launch_xi2(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                      const int32_t *index, int32_t n_win, const double2 *R, int32_t nj, float *xi2,
                      hipStream_t s);
hipError_t launch_xi2_network(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                              const int32_t *index, const int32_t *pix, int32_t n_win,
                              const int32_t *tau, int32_t n_pix, const double2 *R, int32_t nj,
                              float *xi2_det, float *xi2_c, hipStream_t s);
hipError_t launch_trigger_weights(const Bank &bk, float *weight, hipStream_t s);
hipError_t launch_block_operands(const Bank &bk, hipStream_t s);
hipError_t launch_block_set_coeffs(const Bank &bk, const float2 *a, const float2 *b, hipStream_t s);
int32_t block_state_xwin(const Bank &bk);
int32_t block_output_ksplit(const Bank &bk, int32_t min_k_steps);
size_t block_state_lds_bytes(const Bank &bk);
hipError_t prepare_block_bf16(const Bank &bk);
spiir_status plan_block(Bank &bk, const int32_t *offsets, const float *a, const float *b,
                        const int32_t *delay, hipStream_t s, std::string &err);

}  // namespace spiir
