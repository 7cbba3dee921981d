// Template sum, peak search and input-history update.
//
// reduce_peaks: z_t[n] = sum over the slices of template t of the slice partials
// (Eq. zk's sum over a template's filters, Section II.B.1), optionally written
// out, and per window the largest |z_t| with its position (one candidate per
// template per window, Section II.C.1).  |z|^2 is formed as re*re + im*im with
// every product and the sum rounded to float32 (no contraction) so that the
// decision is reproducible; among equal |z|^2 the lowest index wins.  The
// block-wide arg-max reduction uses wave shuffles and one LDS exchange.
#include <algorithm>
#include <climits>
#include <mutex>

#include "internal.h"

namespace spiir {
namespace {

constexpr int kPeakThreads = 256;
constexpr int kUnroll = 4;

struct Best {
    float p;
    int32_t i;
};

__device__ __forceinline__ Best better(Best a, Best b) {
    // larger |z|^2; on a tie the lower index (indices are unique within a window)
    return (b.p > a.p || (b.p == a.p && b.i < a.i)) ? b : a;
}

__device__ __forceinline__ float abs2_rn(float re, float im) {
    // two rounded products and a rounded sum: never contracted into an fma
#pragma clang fp contract(off)
    const float rr = re * re;
    const float ii = im * im;
    return rr + ii;
}

__device__ __forceinline__ Best block_best(Best v, Best *scratch) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Best o;
        o.p = __shfl_xor(v.p, off);
        o.i = __shfl_xor(v.i, off);
        v = better(v, o);
    }
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0) scratch[wave] = v;
    __syncthreads();
    Best r = scratch[0];
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) r = better(r, scratch[w]);
    __syncthreads();  // scratch may be reused by the next window
    return r;
}

// One block per row (template x detector) of the rows listed in `rows` (all rows
// when NULL; `n_list` of them).  The row's series is the sum of its template's slice
// partials (`tmpl_parts` non-NULL) or the row itself.  A template with exactly one
// slice was written into z by the scan: with z given it is read from there.
// With `hist` non-NULL the grid has one more workgroup per detector (blockIdx.x ==
// n_list) that moves the detector's input history past the packet x (what
// hist_update_kernel does), saving a launch after the scan; `hist` and `x` are then
// both non-NULL.
__global__ __launch_bounds__(kPeakThreads) void reduce_peaks_kernel(
    const float2 *__restrict__ src_all, const int32_t *__restrict__ tmpl_parts, int32_t parts_per_det,
    int32_t part_stride, int32_t n, int32_t n_rows_per_det, float2 *__restrict__ z,
    float *__restrict__ peak, int32_t *__restrict__ argmax, int32_t window, int32_t n_win,
    float *__restrict__ hist, int32_t hist_len, const float *__restrict__ x,
    const int32_t *__restrict__ rows, int32_t n_list) {
    __shared__ Best scratch[kPeakThreads / kWave];
    const int det = blockIdx.y;
    if ((int)blockIdx.x == n_list) {
        // the history workgroup: every old value is read before any is written
        constexpr int kPer = (kMaxDelay + kPeakThreads) / kPeakThreads;
        float *h = hist + (int64_t)det * hist_len;
        const float *xd = x + (int64_t)det * n;
        float v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int j = threadIdx.x + k * kPeakThreads;
            v[k] = 0.0f;
            if (j < hist_len) {
                const int pos = n - hist_len + j;
                v[k] = pos >= 0 ? xd[pos] : h[hist_len + pos];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int j = threadIdx.x + k * kPeakThreads;
            if (j < hist_len) h[j] = v[k];
        }
        return;
    }
    if (z == nullptr && peak == nullptr) return;   // only the history was asked for
    const int t = rows != nullptr ? rows[blockIdx.x] : (int)blockIdx.x;
    int p0, np;
    if (tmpl_parts != nullptr) {
        p0 = tmpl_parts[t];
        np = tmpl_parts[t + 1] - p0;
    } else {  // the rows themselves are the series
        p0 = t;
        np = 1;
    }
    const int64_t row = (int64_t)det * n_rows_per_det + t;
    const bool in_z = tmpl_parts != nullptr && np == 1 && z != nullptr;
    const float2 *src = in_z ? z + row * n
                             : src_all + ((int64_t)det * parts_per_det + p0) * part_stride;
    float2 *zr = z != nullptr && !in_z ? z + row * n : nullptr;
    if (zr == nullptr && peak == nullptr) return;
    for (int w = 0; w < n_win; ++w) {
        const int lo = w * window;
        const int hi = min(lo + window, n);
        Best b{-1.0f, INT_MAX};
        // kUnroll samples per thread and pass, their loads issued together; the slices are
        // added in order for every sample, so the sums do not depend on the unrolling
        for (int i0 = lo + threadIdx.x; i0 < hi; i0 += kUnroll * blockDim.x) {
            float vr[kUnroll], vi[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) vr[u] = vi[u] = 0.0f;
            for (int p = 0; p < np; ++p) {
                float2 v[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int i = i0 + u * (int)blockDim.x;
                    v[u] = i < hi ? src[(int64_t)p * part_stride + i] : make_float2(0.0f, 0.0f);
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    vr[u] += v[u].x;
                    vi[u] += v[u].y;
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i >= hi) break;
                if (zr != nullptr) zr[i] = make_float2(vr[u], vi[u]);
                const float pw = abs2_rn(vr[u], vi[u]);
                if (pw > b.p) {  // i increases per thread: first occurrence kept
                    b.p = pw;
                    b.i = i - lo;
                }
            }
        }
        if (peak != nullptr) {
            const Best r = block_best(b, scratch);
            if (threadIdx.x == 0) {
                peak[row * n_win + w] = sqrtf(r.p);
                argmax[row * n_win + w] = r.i;
            }
        }
    }
}

// hist[det][j] <- the last hist_len samples of (old history ++ packet).
// One block per detector; all reads finish before any write (in-place update).
constexpr int kHistThreads = 1024;
constexpr int kHistPerThread = (kMaxDelay + kHistThreads) / kHistThreads;

__global__ __launch_bounds__(kHistThreads) void hist_update_kernel(float *__restrict__ hist,
                                                                   int32_t hist_len,
                                                                   const float *__restrict__ x,
                                                                   int32_t n) {
    const int det = blockIdx.x;
    float *h = hist + (int64_t)det * hist_len;
    const float *xd = x + (int64_t)det * n;
    float v[kHistPerThread];
#pragma unroll
    for (int k = 0; k < kHistPerThread; ++k) {
        const int j = threadIdx.x + k * kHistThreads;
        v[k] = 0.0f;
        if (j < hist_len) {
            const int pos = n - hist_len + j;  // stream position relative to the packet
            v[k] = pos >= 0 ? xd[pos] : h[hist_len + pos];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kHistPerThread; ++k) {
        const int j = threadIdx.x + k * kHistThreads;
        if (j < hist_len) h[j] = v[k];
    }
}

// Trigger selection (Section II.C.1).  Pass 1: a workgroup covers S samples of one
// detector and all templates: thread (sample s, group g) scans templates g, g +
// 256/S, ... (a wave reads 64/S template rows of S consecutive samples; S = 32 for
// long streams, 8 for short packets so that the launch still fills the chip), then
// one thread per sample takes the largest normalised SNR^2 over the
// groups (lowest template on ties) and, above threshold, offers it to that template's
// window slot with a 64-bit atomic max of (rho2 bits << 32 | ~sample): the largest
// rho2 wins, then the lowest sample, whatever the order of the offers.  Pass 2 decodes
// the slots.
constexpr int kTrigThreads = 256;

template <int S>
__global__ __launch_bounds__(kTrigThreads) void trigger_keys_kernel(
    const float2 *__restrict__ z, int32_t n_templates, int32_t n, const float *__restrict__ weight,
    float thr2, int32_t window, int32_t n_win, unsigned long long *__restrict__ keys) {
    constexpr int kTrigGroups = kTrigThreads / S;
    __shared__ float sbest[kTrigGroups][S];
    __shared__ int sidx[kTrigGroups][S];
    const int det = blockIdx.y;
    const int sl = threadIdx.x % S, g = threadIdx.x / S;
    const int i = blockIdx.x * S + sl;
    float best = -1.0f;
    int bt = INT32_MAX;
    if (i < n) {
        const float2 *zd = z + (int64_t)det * n_templates * n + i;
        // increasing templates and a strict comparison: the lowest template of a tie
#pragma unroll 4
        for (int t = g; t < n_templates; t += kTrigGroups) {
            const float2 v = zd[(int64_t)t * n];
            const float r2 = __fmul_rn(abs2_rn(v.x, v.y), weight[t]);
            if (r2 > best) {
                best = r2;
                bt = t;
            }
        }
    }
    sbest[g][sl] = best;
    sidx[g][sl] = bt;
    __syncthreads();
    if (threadIdx.x < S && i < n) {
        for (int q = 1; q < kTrigGroups; ++q) {
            const float v = sbest[q][sl];
            const int t = sidx[q][sl];
            if (v > best || (v == best && t < bt)) {
                best = v;
                bt = t;
            }
        }
        if (bt != INT32_MAX && best > thr2) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(best) << 32) |
                                           (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
            atomicMax(keys + ((int64_t)det * n_templates + bt) * n_win + i / window, key);
        }
    }
}

// Trigger weight 2 / E|z_t|^2 of every template for unit white input, from the bank's
// device coefficients in FP64 (Section II.C.1 normalises each quadrature of the SNR to
// unit variance):  E|z_t|^2 = sum over ordered pairs (k, l) of the template's filters of
// Re[ b_p conj(b_q) conj(a_q)^(d_p - d_q) / (1 - a_p conj(a_q)) ]  with (p, q) the pair
// ordered so that d_p >= d_q.  One workgroup per template: thread k walks every l;
// padding entries (b = 0) add nothing.  The filters of template t are the entries
// [lo, hi) of the coefficient arrays: the slot lanes of its slices (FP32 scan layout,
// `slices` non-NULL) or [g0, g0 + fpad) of the delay-sorted layout (block form).
struct Cd {
    double r, i;
};
__device__ __forceinline__ Cd cmul(Cd a, Cd b) { return Cd{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

constexpr int kWeightThreads = 256;

__global__ __launch_bounds__(kWeightThreads) void trigger_weight_kernel(
    const float2 *__restrict__ ca, const float2 *__restrict__ cb, const int32_t *__restrict__ cd,
    const Slice *__restrict__ slices, const int32_t *__restrict__ tmpl_slices,
    const BTemplate *__restrict__ btmpl, float *__restrict__ weight) {
    __shared__ double part[kWeightThreads / kWave];
    const int t = blockIdx.x;
    int64_t lo = 0, hi = 0;
    if (slices != nullptr) {
        const int s0 = tmpl_slices[t], s1 = tmpl_slices[t + 1];
        if (s1 > s0) {
            lo = (int64_t)slices[s0].slot_base * kWave;
            hi = (int64_t)(slices[s1 - 1].slot_base + slices[s1 - 1].n_slots) * kWave;
        }
    } else {
        lo = btmpl[t].g0;
        hi = lo + btmpl[t].fpad;
    }
    double acc = 0.0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += kWeightThreads) {
        const float2 bk = cb[k];
        if (bk.x == 0.0f && bk.y == 0.0f) continue;
        for (int64_t l = lo; l < hi; ++l) {
            const float2 bl = cb[l];
            if (bl.x == 0.0f && bl.y == 0.0f) continue;
            const bool kp = cd[k] >= cd[l];
            const int64_t p = kp ? k : l, q = kp ? l : k;
            const Cd ap{(double)ca[p].x, (double)ca[p].y};
            const Cd aq{(double)ca[q].x, -(double)ca[q].y};                 // conj(a_q)
            const Cd num = cmul(Cd{(double)cb[p].x, (double)cb[p].y},
                                Cd{(double)cb[q].x, -(double)cb[q].y});     // b_p conj(b_q)
            Cd pw{1.0, 0.0}, base = aq;
            for (int e = cd[p] - cd[q]; e > 0; e >>= 1) {
                if (e & 1) pw = cmul(pw, base);
                base = cmul(base, base);
            }
            const Cd nu = cmul(num, pw);
            const Cd den{1.0 - (ap.r * aq.r - ap.i * aq.i), -(ap.r * aq.i + ap.i * aq.r)};
            acc += (nu.r * den.r + nu.i * den.i) / (den.r * den.r + den.i * den.i);
        }
    }
    for (int off = kWave / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kWeightThreads / kWave; ++w) tot += part[w];
        weight[t] = tot > 0.0 ? (float)(2.0 / tot) : 0.0f;
    }
}

__global__ void zero_u64_kernel(unsigned long long *__restrict__ p, int64_t count) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0ull;
}

__global__ void trigger_decode_kernel(const unsigned long long *__restrict__ keys, int64_t count,
                                      float *__restrict__ snr, int32_t *__restrict__ index) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long key = keys[k];
        if (key == 0ull) {
            snr[k] = 0.0f;
            index[k] = -1;
        } else {
            snr[k] = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
            index[k] = (int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
        }
    }
}

__global__ void zero_kernel(float4 *__restrict__ p, int64_t n4) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace

hipError_t launch_reduce_peaks(const Bank &bk, int32_t n, float2 *z, float *peak, int32_t *argmax,
                               const float *x, bool fused, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int32_t window = bk.peak_window > 0 ? bk.peak_window : n;
    const int32_t n_win = (n + window - 1) / window;
    const bool hist = bk.hist_len > 0 && x != nullptr;
    // after a scan that finished its single-slice templates, only the others are left
    const int32_t n_list = fused ? bk.n_multi : bk.n_templates;
    const bool rows = z != nullptr || peak != nullptr;
    const int32_t grid_x = (rows ? n_list : 0) + (hist ? 1 : 0);
    if (grid_x == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_peaks_kernel, dim3(grid_x, bk.n_det), dim3(kPeakThreads), 0, s,
                       bk.d_partial, bk.d_tmpl_slices, bk.n_slices, bk.max_chunk, n,
                       bk.n_templates, z, peak, argmax, window, n_win,
                       hist ? bk.d_hist : nullptr, bk.hist_len, x,
                       fused ? bk.d_multi_tmpl : nullptr, rows ? n_list : 0);
    return hipGetLastError();
}

hipError_t launch_peaks(const float2 *z, int64_t rows, int32_t n, int32_t window, float *peak,
                        int32_t *argmax, hipStream_t s) {
    if (rows <= 0 || n <= 0) return hipSuccess;
    const int32_t n_win = (n + window - 1) / window;
    // rows are split over grid.x (<= 2^31-1) and grid.y (detector slot, here 1 row block)
    const int64_t max_x = 1 << 30;
    for (int64_t r0 = 0; r0 < rows; r0 += max_x) {
        const int64_t cnt = rows - r0 < max_x ? rows - r0 : max_x;
        hipLaunchKernelGGL(reduce_peaks_kernel, dim3((unsigned)cnt, 1), dim3(kPeakThreads), 0, s,
                           z + r0 * n, nullptr, 0, n, n, (int32_t)cnt, nullptr,
                           peak + r0 * n_win, argmax + r0 * n_win, window, n_win, nullptr, 0,
                           nullptr, nullptr, (int32_t)cnt);
    }
    return hipGetLastError();
}

hipError_t launch_hist_update(const Bank &bk, const float *x, int32_t n, hipStream_t s) {
    if (n <= 0 || bk.hist_len == 0) return hipSuccess;
    hipLaunchKernelGGL(hist_update_kernel, dim3(bk.n_det), dim3(kHistThreads), 0, s, bk.d_hist,
                       bk.hist_len, x, n);
    return hipGetLastError();
}

hipError_t launch_triggers(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                           const float *weight, float threshold, int32_t window,
                           unsigned long long *work, float *snr, int32_t *index, hipStream_t s) {
    const int32_t n_win = (n + window - 1) / window;
    const int64_t count = (int64_t)n_det * n_templates * n_win;
    if (count == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    // clear the slots with a kernel (graph-safe)
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, work, count);
    const float thr2 = threshold * threshold;
    if ((int64_t)(n / 32) * n_det >= 1024)
        hipLaunchKernelGGL(trigger_keys_kernel<32>, dim3((n + 31) / 32, n_det), dim3(kTrigThreads),
                           0, s, z, n_templates, n, weight, thr2, window, n_win, work);
    else
        hipLaunchKernelGGL(trigger_keys_kernel<8>, dim3((n + 7) / 8, n_det), dim3(kTrigThreads),
                           0, s, z, n_templates, n, weight, thr2, window, n_win, work);
    hipLaunchKernelGGL(trigger_decode_kernel, dim3((unsigned)blocks), dim3(256), 0, s, work, count,
                       snr, index);
    return hipGetLastError();
}

namespace {

// Key slots of spiir_triggers_noalloc: a library-owned workspace for callers that
// cannot allocate.  Every GPU holds its own copy until the process ends; every call
// on one GPU shares it.  In host code the name is a stand-in for the device copy, so
// kernels get the address looked up per device below, never the name itself.
static __device__ __align__(256) unsigned long long scratch[kTriggerScratchSlots];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per device.
hipError_t scratch_address(unsigned long long **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<unsigned long long *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t launch_triggers_noalloc(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                                   const float *weight, float threshold, int32_t window,
                                   float *snr, int32_t *index, hipStream_t s) {
    const int64_t count = (int64_t)n_det * n_templates * ((n + window - 1) / window);
    if (count > kTriggerScratchSlots) return hipErrorInvalidValue;   // checked by the caller
    unsigned long long *work = nullptr;
    const hipError_t e = scratch_address(&work);
    if (e != hipSuccess) return e;
    // the same kernels as launch_triggers; the slots are cleared there by a kernel
    return launch_triggers(z, n_det, n_templates, n, weight, threshold, window, work, snr, index,
                           s);
}

hipError_t launch_trigger_weights(const Bank &bk, float *weight, hipStream_t s) {
    if (bk.n_templates <= 0) return hipSuccess;
    if (bk.mode == SPIIR_MODE_BF16_BLOCK)
        hipLaunchKernelGGL(trigger_weight_kernel, dim3(bk.n_templates), dim3(kWeightThreads), 0, s,
                           bk.d_ga, bk.d_gb, bk.d_gd, nullptr, nullptr, bk.d_btmpl, weight);
    else
        hipLaunchKernelGGL(trigger_weight_kernel, dim3(bk.n_templates), dim3(kWeightThreads), 0, s,
                           bk.d_a, bk.d_b, bk.d_delay, bk.d_slices, bk.d_tmpl_slices, nullptr,
                           weight);
    return hipGetLastError();
}

hipError_t launch_zero(void *ptr, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    // callers pass 16-byte multiples (allocations are rounded up)
    const int64_t n4 = bytes / 16;
    const int64_t blocks64 = (n4 + 255) / 256;
    const unsigned blocks = (unsigned)(blocks64 < 4096 ? (blocks64 > 0 ? blocks64 : 1) : 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, static_cast<float4 *>(ptr), n4);
    return hipGetLastError();
}

}  // namespace spiir
