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

// Device bookkeeping of the persistent FP32 scan (one per bank).
struct ScanQueue {
    uint32_t head;   // next work item to hand out in the current launch
    uint32_t done;   // waves of the current launch that have finished
    uint32_t epoch;  // time tiles every slice completed before the current launch
    uint32_t error;  // sticky count of dependency waits that hit their bound
};

// One FP32-scan work unit: up to 64 * filters_per_lane filters of one template.
// Its filters occupy `n_slots` consecutive slots of 64 lanes starting at `slot_base`.
struct Slice {
    int32_t tmpl;
    int32_t slot_base;
    int32_t n_slots;
    int32_t pad;
};

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
    ScanQueue *d_queue = nullptr;
    uint32_t *d_flags = nullptr; // [D][n_slices]: tiles completed (epoch-relative)
    int32_t *d_order = nullptr;  // [D*n_slices]: det*n_slices + slice, largest slices first

    int64_t device_bytes = 0;
    hipStream_t last_stream = nullptr;

    // optional kernel timing
    std::vector<hipEvent_t> ev_start, ev_stop;
    int64_t timed = 0;
    std::vector<void *> allocations;
};

// Launchers (enqueue only; arguments already validated).
size_t scan_fp32_lds_bytes(int32_t tile, int32_t hist_len);
size_t scan_persistent_lds_bytes(int32_t tile, int32_t hist_len);
hipError_t prepare_scan_fp32(Bank &bk);
hipError_t launch_scan_fp32(const Bank &bk, const float *x, int32_t n, hipStream_t s);
hipError_t launch_hist_update(const Bank &bk, const float *x, int32_t n, hipStream_t s);
hipError_t launch_reduce_peaks(const Bank &bk, int32_t n, float2 *z, float *peak,
                               int32_t *argmax, hipStream_t s);
hipError_t launch_peaks(const float2 *z, int64_t rows, int32_t n, int32_t window, float *peak,
                        int32_t *argmax, hipStream_t s);
hipError_t launch_zero(void *ptr, int64_t bytes, hipStream_t s);

}  // namespace spiir
