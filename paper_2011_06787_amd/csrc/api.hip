// C-ABI of libspiir: argument validation, bank layout planning and launches.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <thread>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

struct spiir_bank {
    spiir::Bank bk;
};

namespace {

thread_local std::string g_error;

spiir_status fail(spiir_status st, const std::string &msg) {
    g_error = msg;
    return st;
}

#define SPIIR_HIP(expr)                                                                      \
    do {                                                                                     \
        const hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                                \
            return fail(SPIIR_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

int64_t round16(int64_t bytes) { return (bytes + 15) & ~int64_t(15); }

// Device allocation tracked by the bank (freed in destroy).
template <typename T>
spiir_status dev_alloc(spiir::Bank &bk, T **ptr, int64_t count) {
    *ptr = nullptr;
    const int64_t bytes = round16(std::max<int64_t>(count, 1) * (int64_t)sizeof(T));
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPIIR_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                       hipGetErrorString(e));
    }
    bk.allocations.push_back(p);
    bk.device_bytes += bytes;
    *ptr = static_cast<T *>(p);
    return SPIIR_OK;
}

void free_all(spiir::Bank &bk) {
    for (void *p : bk.allocations) (void)hipFree(p);
    bk.allocations.clear();
    if (bk.h_wait_flag != nullptr) (void)hipHostFree(bk.h_wait_flag);
    bk.h_wait_flag = bk.d_wait_flag = nullptr;
}

// A state hand-off wait of an earlier launch hit its bound: the waiting wave went on
// with a stale state, so the stream's results are invalid until the next reset.
spiir_status check_waits(const spiir::Bank &bk) {
    if (bk.h_wait_flag != nullptr && __atomic_load_n(bk.h_wait_flag, __ATOMIC_ACQUIRE) != 0u)
        return fail(SPIIR_E_STATE,
                    "a state hand-off wait of an earlier FP32 scan launch hit its bound "
                    "(wait_spins); the stream's results are invalid until spiir_bank_reset");
    return SPIIR_OK;
}

void release_events(spiir::Bank &bk) {
    for (hipEvent_t e : bk.ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : bk.ev_stop) (void)hipEventDestroy(e);
    bk.ev_start.clear();
    bk.ev_stop.clear();
    bk.timed = 0;
}

template <typename T>
spiir_status upload(T *dst, const std::vector<T> &src, hipStream_t s) {
    if (src.empty()) return SPIIR_OK;
    SPIIR_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return SPIIR_OK;
}

#define SPIIR_TRY(expr)                                                                      \
    do {                                                                                     \
        const spiir_status st_ = (expr);                                                     \
        if (st_ != SPIIR_OK) return st_;                                                     \
    } while (0)

// Plan the FP32-scan layout.  A template of F_t filters takes the minimum
// ceil(F_t/64) slots of 64 lanes; these are split into ceil(slots/fpl) slices of
// near-equal slot counts (<= fpl each).  Inside a template, filters are ordered by
// d mod 64 and dealt to the slices in that order (each next filter to the slice
// with the lowest fill ratio); within a slice they are dealt by d mod 32 over its
// half-waves (see below), so the lanes of a half-wave read the input window at
// well-spread LDS banks.
spiir_status plan_scan(spiir::Bank &bk, const int32_t *offsets, const float *a, const float *b,
                       const int32_t *delay, hipStream_t s) {
    const int32_t T = bk.n_templates;
    std::vector<spiir::Slice> slices;
    std::vector<int32_t> tmpl_slices(T + 1, 0);
    std::vector<std::vector<int32_t>> members;   // filter indices per slice, in sorted order
    for (int32_t t = 0; t < T; ++t) {
        tmpl_slices[t] = (int32_t)slices.size();
        const int32_t lo = offsets[t], hi = offsets[t + 1];
        const int32_t f = hi - lo;
        if (f == 0) continue;
        std::vector<int32_t> idx(f);
        std::iota(idx.begin(), idx.end(), lo);
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int32_t p, int32_t q) { return (delay[p] & 63) < (delay[q] & 63); });
        const int32_t slots = (f + spiir::kWave - 1) / spiir::kWave;
        const int32_t ns = (slots + bk.fpl - 1) / bk.fpl;
        std::vector<int32_t> cap(ns);
        for (int32_t p = 0; p < ns; ++p) cap[p] = (slots / ns + (p < slots % ns ? 1 : 0)) * spiir::kWave;
        std::vector<std::vector<int32_t>> part(ns);
        for (int32_t i = 0; i < f; ++i) {
            int32_t best = -1;
            double best_fill = 2.0;
            for (int32_t p = 0; p < ns; ++p) {
                if ((int32_t)part[p].size() >= cap[p]) continue;
                const double fill = (double)part[p].size() / cap[p];
                if (fill < best_fill) {
                    best_fill = fill;
                    best = p;
                }
            }
            part[best].push_back(idx[i]);
        }
        for (int32_t p = 0; p < ns; ++p) {
            spiir::Slice sl{};
            sl.tmpl = t;
            sl.single = ns == 1 ? 1 : 0;
            sl.n_slots = (int32_t)((part[p].size() + spiir::kWave - 1) / spiir::kWave);
            slices.push_back(sl);
            members.push_back(std::move(part[p]));
        }
    }
    tmpl_slices[T] = (int32_t)slices.size();
    // templates the slice-sum kernel always visits (none or several slices)
    std::vector<int32_t> multi;
    for (int32_t t = 0; t < T; ++t)
        if (tmpl_slices[t + 1] - tmpl_slices[t] != 1) multi.push_back(t);
    bk.n_multi = (int32_t)multi.size();
    int64_t slot = 0;
    for (auto &sl : slices) {
        sl.slot_base = (int32_t)slot;
        slot += sl.n_slots;
    }
    if (slot * spiir::kWave > INT32_MAX)
        return fail(SPIIR_E_UNSUPPORTED, "bank too large for the FP32 scan layout");
    bk.n_slices = (int32_t)slices.size();
    bk.n_slots = slot;
    bk.h_slice_slots.resize(slices.size());
    for (size_t si = 0; si < slices.size(); ++si) bk.h_slice_slots[si] = slices[si].n_slots;
    const int64_t lanes = slot * spiir::kWave;
    std::vector<float2> ha(lanes, make_float2(0.f, 0.f)), hb(lanes, make_float2(0.f, 0.f));
    std::vector<int32_t> hd(lanes, 0), hp(lanes, -1);
    constexpr int32_t kHalf = spiir::kWave / 2;   // lanes whose LDS reads are served together
    for (size_t si = 0; si < slices.size(); ++si) {
        std::vector<int32_t> mem = members[si];
        const int32_t m = slices[si].n_slots;
        // LDS input reads: lane reads window[n - d]; two lanes of one half-wave whose delays
        // agree mod 32 hit the same bank.  Sorted by d mod 32 and dealt over the slice's 2m
        // half-waves, each residue is spread as evenly as its count allows.
        std::stable_sort(mem.begin(), mem.end(),
                         [&](int32_t p, int32_t q) { return (delay[p] & 31) < (delay[q] & 31); });
        for (size_t i = 0; i < mem.size(); ++i) {
            const int32_t hw = (int32_t)(i % (size_t)(2 * m));     // half-wave
            const int64_t g = (int64_t)(slices[si].slot_base + hw % m) * spiir::kWave +
                              (hw / m) * kHalf + (int64_t)(i / (size_t)(2 * m));
            const int32_t k = mem[i];
            ha[g] = make_float2(a[2 * (int64_t)k], a[2 * (int64_t)k + 1]);
            hb[g] = make_float2(b[2 * (int64_t)k], b[2 * (int64_t)k + 1]);
            hd[g] = delay[k];
            hp[g] = k;
        }
        // padding lanes (b = 0) read the address of the half-wave's first lane: no new bank
        for (int32_t hw = 0; hw < 2 * m; ++hw) {
            const int64_t g0 = (int64_t)(slices[si].slot_base + hw % m) * spiir::kWave +
                               (hw / m) * kHalf;
            for (int32_t l = 1; l < kHalf; ++l)
                if (hp[g0 + l] < 0 && hp[g0] >= 0) hd[g0 + l] = hd[g0];
        }
    }
    SPIIR_TRY(dev_alloc(bk, &bk.d_a, lanes));
    SPIIR_TRY(dev_alloc(bk, &bk.d_b, lanes));
    SPIIR_TRY(dev_alloc(bk, &bk.d_delay, lanes));
    SPIIR_TRY(dev_alloc(bk, &bk.d_perm, lanes));
    SPIIR_TRY(dev_alloc(bk, &bk.d_slices, std::max<int64_t>(bk.n_slices, 1)));
    SPIIR_TRY(dev_alloc(bk, &bk.d_tmpl_slices, T + 1));
    SPIIR_TRY(dev_alloc(bk, &bk.d_multi_tmpl, std::max<int64_t>(bk.n_multi, 1)));
    SPIIR_TRY(dev_alloc(bk, &bk.d_state, lanes * bk.n_det));
    SPIIR_TRY(dev_alloc(bk, &bk.d_partial,
                        std::max<int64_t>((int64_t)bk.n_det * bk.n_slices * bk.max_chunk, 1)));
    SPIIR_TRY(dev_alloc(bk, &bk.d_queue, 1));
    SPIIR_TRY(dev_alloc(bk, &bk.d_flags, std::max<int64_t>((int64_t)bk.n_det * bk.n_slices, 4)));
    SPIIR_TRY(dev_alloc(bk, &bk.d_order, std::max<int64_t>((int64_t)bk.n_det * bk.n_slices, 1)));
    // persistent-scan hand-out order inside a time tile: largest slices first
    std::vector<int32_t> order((size_t)bk.n_det * bk.n_slices);
    for (int32_t dd = 0; dd < bk.n_det; ++dd)
        for (int32_t si = 0; si < bk.n_slices; ++si) order[(size_t)dd * bk.n_slices + si] = dd * bk.n_slices + si;
    std::stable_sort(order.begin(), order.end(), [&](int32_t p, int32_t q) {
        return slices[p % bk.n_slices].n_slots > slices[q % bk.n_slices].n_slots;
    });
    SPIIR_TRY(upload(bk.d_order, order, s));
    std::vector<int32_t> sorder(bk.n_slices);
    std::iota(sorder.begin(), sorder.end(), 0);
    std::stable_sort(sorder.begin(), sorder.end(), [&](int32_t p, int32_t q) {
        return slices[p].n_slots > slices[q].n_slots;
    });
    SPIIR_TRY(dev_alloc(bk, &bk.d_slice_order, std::max<int64_t>(bk.n_slices, 1)));
    SPIIR_TRY(upload(bk.d_slice_order, sorder, s));
    SPIIR_TRY(upload(bk.d_a, ha, s));
    SPIIR_TRY(upload(bk.d_b, hb, s));
    SPIIR_TRY(upload(bk.d_delay, hd, s));
    SPIIR_TRY(upload(bk.d_perm, hp, s));
    SPIIR_TRY(upload(bk.d_slices, slices, s));
    SPIIR_TRY(upload(bk.d_tmpl_slices, tmpl_slices, s));
    if (!multi.empty()) SPIIR_TRY(upload(bk.d_multi_tmpl, multi, s));
    // the host staging vectors die at return: wait for the copies
    SPIIR_HIP(hipStreamSynchronize(s));
    return SPIIR_OK;
}

// Balanced schedule of the FP32 scan: the wrap-around rule for preemptive
// scheduling on identical machines applied to the slices of one detector.  A slice
// of m slots costs m + kReduceSlots slot-units of work per packet (the lane
// reduction of every sub-tile is worth about 0.45 slot).  The wave count W is a
// whole number c of workgroups on every compute unit (so that every SIMD holds the
// same number of equal waves), with c as large as allowed while the mean load
// C = P / W stays at or above the largest slice, so that a cut slice spans only two
// waves.  Waves are filled in order up to C; a slice that does not fit is cut at
// the sample fraction that fills the wave: its later part closes this wave's list,
// its earlier part opens the next wave's list.
constexpr double kReduceSlots = 0.45;

spiir_status plan_balanced(spiir::Bank &bk, hipStream_t s) {
    const int32_t S = bk.n_slices;
    double P = 0.0, pmax = 0.0;
    for (int32_t i = 0; i < S; ++i) {
        const double p = bk.h_slice_slots[i] + kReduceSlots;
        P += p;
        pmax = std::max(pmax, p);
    }
    const int64_t unit = std::max(1, bk.balance_unit);
    int64_t c = pmax > 0 ? (int64_t)std::floor(P / (pmax * (double)unit)) : 1;
    c = std::min<int64_t>(c, std::max(1, bk.balance_per_cu));
    int64_t W = c >= 1 ? c * unit
                       : std::max<int64_t>(1, pmax > 0 ? (int64_t)std::floor(P / pmax) : 1);
    // LDS request: the input window, padded so that c workgroups fit on a compute unit
    // and c + 1 do not; the dispatcher then places exactly c on every compute unit
    const int64_t cc = std::max<int64_t>(c, 1);
    const int64_t pad = ((int64_t)spiir::kLdsPerCu * 2 / (2 * cc + 1)) / 512 * 512;
    bk.balance_lds = (int32_t)std::min<int64_t>(
        spiir::kLdsPerCu,
        std::max<int64_t>((int64_t)spiir::scan_fp32_lds_bytes(bk.max_chunk, bk.hist_len), pad));
    const double C = P / (double)W;
    std::vector<std::vector<spiir::Seg>> lists((size_t)W);
    int64_t w = 0;
    double fill = 0.0;
    int32_t splits = 0;
    const double eps = 1e-9 * std::max(1.0, C);
    for (int32_t i = 0; i < S; ++i) {
        const double p = bk.h_slice_slots[i] + kReduceSlots;
        const double room = C - fill;
        if (w == W - 1 || p <= room + eps) {
            lists[(size_t)w].push_back(spiir::Seg{i, 0, spiir::kPhiOne, -1});
            fill += p;
        } else if (room <= eps) {
            ++w;
            lists[(size_t)w].push_back(spiir::Seg{i, 0, spiir::kPhiOne, -1});
            fill = p;
        } else {
            // earlier part (fraction (p - room) / p of the packet) opens wave w+1
            const int32_t phi = (int32_t)std::min<int64_t>(
                spiir::kPhiOne - 1,
                std::max<int64_t>(1, std::llround((p - room) / p * spiir::kPhiOne)));
            lists[(size_t)w].push_back(spiir::Seg{i, phi, spiir::kPhiOne, splits});
            ++w;
            lists[(size_t)w].push_back(spiir::Seg{i, 0, phi, splits});
            ++splits;
            fill = p - room;
        }
        if (fill >= C - eps && w < W - 1 && i + 1 < S) {
            ++w;
            fill = 0.0;
        }
    }
    std::vector<spiir::Seg> segs;
    std::vector<int32_t> off((size_t)W + 1, 0);
    for (int64_t k = 0; k < W; ++k) {
        off[(size_t)k] = (int32_t)segs.size();
        segs.insert(segs.end(), lists[(size_t)k].begin(), lists[(size_t)k].end());
    }
    off[(size_t)W] = (int32_t)segs.size();
    bk.balance_waves = (int32_t)W;
    bk.n_splits = splits;
    SPIIR_TRY(dev_alloc(bk, &bk.d_segs, std::max<int64_t>((int64_t)segs.size(), 1)));
    SPIIR_TRY(dev_alloc(bk, &bk.d_seg_off, W + 1));
    SPIIR_TRY(dev_alloc(bk, &bk.d_split_flags, std::max<int64_t>((int64_t)bk.n_det * splits, 4)));
    SPIIR_TRY(dev_alloc(bk, &bk.d_split_cand, std::max<int64_t>((int64_t)bk.n_det * splits, 1)));
    SPIIR_TRY(dev_alloc(bk, &bk.d_bqueue, 1));
    SPIIR_TRY(dev_alloc(bk, &bk.d_simd_tab, (int64_t)spiir::kSimdKeys * spiir::kPeerTableWords));
    SPIIR_TRY(upload(bk.d_segs, segs, s));
    SPIIR_TRY(upload(bk.d_seg_off, off, s));
    SPIIR_HIP(hipStreamSynchronize(s));   // the host vectors die at return
    return SPIIR_OK;
}

spiir_status zero_stream_state(spiir::Bank &bk, hipStream_t s) {
    if (bk.mode == SPIIR_MODE_BF16_BLOCK)
        SPIIR_HIP(spiir::launch_zero(bk.d_state64, round16(std::max<int64_t>(bk.n_fpad, 1) * bk.n_det *
                                                           (int64_t)sizeof(double2)), s));
    else
        SPIIR_HIP(spiir::launch_zero(bk.d_state, round16(bk.n_slots * spiir::kWave * bk.n_det *
                                                         (int64_t)sizeof(float2)), s));
    if (bk.hist_len > 0)
        SPIIR_HIP(spiir::launch_zero(bk.d_hist,
                                     round16((int64_t)bk.hist_len * bk.n_det * (int64_t)sizeof(float)),
                                     s));
    return SPIIR_OK;
}

// Work-queue counters and per-slice progress flags of the persistent scan.
spiir_status zero_queue(spiir::Bank &bk, hipStream_t s) {
    SPIIR_HIP(spiir::launch_zero(bk.d_queue, round16(sizeof(spiir::ScanQueue)), s));
    SPIIR_HIP(spiir::launch_zero(bk.d_flags,
                                 round16(std::max<int64_t>((int64_t)bk.n_det * bk.n_slices, 4) *
                                         (int64_t)sizeof(uint32_t)), s));
    if (bk.balanced) {
        SPIIR_HIP(spiir::launch_zero(bk.d_bqueue, round16(sizeof(spiir::ScanQueue)), s));
        SPIIR_HIP(spiir::launch_zero(bk.d_simd_tab,
                                     round16((int64_t)spiir::kSimdKeys * spiir::kPeerTableWords *
                                             (int64_t)sizeof(uint32_t)),
                                     s));
        SPIIR_HIP(spiir::launch_zero(bk.d_split_flags,
                                     round16(std::max<int64_t>((int64_t)bk.n_det * bk.n_splits, 4) *
                                             (int64_t)sizeof(uint32_t)), s));
    }
    return SPIIR_OK;
}

}  // namespace

extern "C" {

void spiir_opts_default(spiir_opts *opts) {
    if (opts == nullptr) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->n_detectors = 1;
    opts->max_chunk = 2048;
    opts->max_delay = 0;
    opts->peak_window = 0;
    opts->mode = SPIIR_MODE_FP32_SCAN;
    opts->filters_per_lane = 4;
    opts->time_tile = 0;
    opts->block_len = 128;
    opts->long_pole_abs_a = 0.999;
    opts->ckpt_stride = 2048;
    opts->balance_wgs = 0;
    opts->wait_spins = 0;
}

const char *spiir_last_error(void) { return g_error.c_str(); }

spiir_status spiir_bank_create(int32_t n_templates, const int32_t *offsets, const float *a,
                               const float *b, const int32_t *delay, const spiir_opts *opts_in,
                               void *stream, spiir_bank **out) {
    try {
        if (out == nullptr) return fail(SPIIR_E_INVAL, "out is NULL");
        *out = nullptr;
        spiir_opts opts;
        spiir_opts_default(&opts);
        if (opts_in != nullptr) opts = *opts_in;
        if (n_templates < 1) return fail(SPIIR_E_INVAL, "n_templates must be >= 1");
        if (offsets == nullptr) return fail(SPIIR_E_INVAL, "offsets is NULL");
        if (offsets[0] != 0) return fail(SPIIR_E_INVAL, "offsets[0] must be 0");
        for (int32_t t = 0; t < n_templates; ++t)
            if (offsets[t + 1] < offsets[t])
                return fail(SPIIR_E_INVAL, "offsets must be non-decreasing (template " +
                                               std::to_string(t) + ")");
        const int64_t F = offsets[n_templates];
        if (F > 0 && (a == nullptr || b == nullptr || delay == nullptr))
            return fail(SPIIR_E_INVAL, "a, b and delay must be non-NULL when the bank has filters");
        if (opts.n_detectors < 1) return fail(SPIIR_E_INVAL, "n_detectors must be >= 1");
        if (opts.max_chunk < 1) return fail(SPIIR_E_INVAL, "max_chunk must be >= 1");
        if (opts.max_delay < 0 || opts.max_delay > spiir::kMaxDelay)
            return fail(SPIIR_E_INVAL, "max_delay must be in [0, " +
                                           std::to_string(spiir::kMaxDelay) + "]");
        if (opts.peak_window < 0) return fail(SPIIR_E_INVAL, "peak_window must be >= 0");
        if (opts.mode != SPIIR_MODE_FP32_SCAN && opts.mode != SPIIR_MODE_BF16_BLOCK)
            return fail(SPIIR_E_INVAL, "unknown mode");
        const int block_len = opts.block_len == 0 ? 128 : opts.block_len;
        const int ckpt_stride = opts.ckpt_stride == 0 ? 2048 : opts.ckpt_stride;
        if (ckpt_stride < 128 || ckpt_stride % 128 != 0)
            return fail(SPIIR_E_INVAL, "ckpt_stride must be a positive multiple of 128");
        if (opts.mode == SPIIR_MODE_BF16_BLOCK) {
            if (block_len != 64 && block_len != 128 && block_len != 256)
                return fail(SPIIR_E_INVAL, "block_len must be 64, 128 or 256");
            if (opts.max_chunk % block_len != 0)
                return fail(SPIIR_E_INVAL, "block form: max_chunk must be a multiple of block_len");
            if (opts.peak_window > 0 && opts.peak_window % block_len != 0)
                return fail(SPIIR_E_INVAL, "block form: peak_window must be a multiple of block_len");
        }
        int fpl = opts.filters_per_lane == 0 ? 4 : opts.filters_per_lane;
        if (fpl != 1 && fpl != 2 && fpl != 4 && fpl != 8)
            return fail(SPIIR_E_INVAL, "filters_per_lane must be 1, 2, 4 or 8");
        const int time_tile = opts.time_tile;
        if (time_tile != -1 && time_tile != 0 &&
            (time_tile < spiir::kSub || time_tile > 4096 || time_tile % spiir::kSub != 0))
            return fail(SPIIR_E_INVAL, "time_tile must be -1, 0 or a multiple of 16 in [16, 4096]");
        if (opts.balance_wgs < 0 || opts.balance_wgs > 8)
            return fail(SPIIR_E_INVAL, "balance_wgs must be in [0, 8]");
        if (opts.wait_spins < 0) return fail(SPIIR_E_INVAL, "wait_spins must be >= 0");
        int32_t dmax = 0;
        for (int64_t k = 0; k < F; ++k) {
            const double ar = a[2 * k], ai = a[2 * k + 1], br = b[2 * k], bi = b[2 * k + 1];
            if (!std::isfinite(ar) || !std::isfinite(ai) || !std::isfinite(br) || !std::isfinite(bi))
                return fail(SPIIR_E_INVAL, "non-finite coefficient at filter " + std::to_string(k));
            if (ar * ar + ai * ai >= 1.0)
                return fail(SPIIR_E_INVAL, "|a| >= 1 at filter " + std::to_string(k));
            if (delay[k] < 0) return fail(SPIIR_E_INVAL, "negative delay at filter " + std::to_string(k));
            dmax = std::max(dmax, delay[k]);
        }
        const int32_t hist_len = opts.max_delay > 0 ? opts.max_delay : dmax;
        if (dmax > hist_len)
            return fail(SPIIR_E_INVAL, "delay " + std::to_string(dmax) + " exceeds max_delay " +
                                           std::to_string(hist_len));
        if (hist_len > spiir::kMaxDelay)
            return fail(SPIIR_E_UNSUPPORTED, "delays above " + std::to_string(spiir::kMaxDelay) +
                                                 " samples are not supported");
        if (opts.peak_window > opts.max_chunk)
            return fail(SPIIR_E_INVAL, "peak_window larger than max_chunk");

        auto *h = new (std::nothrow) spiir_bank;
        if (h == nullptr) return fail(SPIIR_E_NOMEM, "host allocation failed");
        spiir::Bank &bk = h->bk;
        bk.n_templates = n_templates;
        bk.n_filters = F;
        bk.n_det = opts.n_detectors;
        bk.max_chunk = opts.max_chunk;
        bk.hist_len = hist_len;
        bk.peak_window = opts.peak_window;
        bk.mode = opts.mode;
        bk.fpl = fpl;
        bk.time_tile = time_tile > 0 ? time_tile : 0;
        bk.balance_per_cu = opts.balance_wgs;
        bk.balanced = time_tile <= 0 && opts.balance_wgs > 0 &&
                         (int64_t)bk.max_chunk + hist_len + spiir::kSub <= spiir::kWindowFloats;
        bk.block_len = block_len;
        bk.ckpt_stride = ckpt_stride;
        if (opts.wait_spins > 0) bk.wait_spins = (uint32_t)opts.wait_spins;
        bk.h_offsets.assign(offsets, offsets + n_templates + 1);
        if (F > 0) {
            bk.h_a.assign(a, a + 2 * F);
            bk.h_b.assign(b, b + 2 * F);
            bk.h_delay.assign(delay, delay + F);
        }
        bk.long_pole = opts.long_pole_abs_a > 0 ? opts.long_pole_abs_a : 0.999;
        int32_t tile = spiir::kWindowFloats - hist_len - spiir::kSub;
        tile = std::min(tile, bk.max_chunk);
        tile = std::max(spiir::kSub, tile / spiir::kSub * spiir::kSub);
        bk.scan_tile = tile;
        hipStream_t s = static_cast<hipStream_t>(stream);
        spiir_status st = dev_alloc(bk, &bk.d_hist, std::max<int64_t>((int64_t)bk.hist_len * bk.n_det, 4));
        if (st == SPIIR_OK && bk.mode == SPIIR_MODE_BF16_BLOCK) {
            std::string err;
            st = spiir::plan_block(bk, offsets, a, b, delay, s, err);
            if (st != SPIIR_OK) fail(st, err);
            if (st == SPIIR_OK) {
                if (spiir::block_state_lds_bytes(bk) > 150 * 1024) {
                    st = fail(SPIIR_E_UNSUPPORTED, "block form: input band too wide for LDS");
                } else {
                    const hipError_t e = spiir::prepare_block_bf16(bk);
                    if (e != hipSuccess)
                        st = fail(SPIIR_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
                }
            }
        } else if (st == SPIIR_OK) {
            // the flag a bounded hand-off wait raises when it gives up, in pinned host
            // memory so that later calls read it without synchronising
            void *hp = nullptr, *dp = nullptr;
            if (hipHostMalloc(&hp, 64, hipHostMallocMapped) != hipSuccess) {
                (void)hipGetLastError();
                st = fail(SPIIR_E_NOMEM, "hipHostMalloc of the wait flag failed");
            } else {
                bk.h_wait_flag = static_cast<uint32_t *>(hp);
                *bk.h_wait_flag = 0u;
                const hipError_t e = hipHostGetDevicePointer(&dp, hp, 0);
                if (e != hipSuccess)
                    st = fail(SPIIR_E_HIP, std::string("hipHostGetDevicePointer: ") + hipGetErrorString(e));
                bk.d_wait_flag = static_cast<uint32_t *>(dp);
            }
        }
        if (st == SPIIR_OK && bk.mode != SPIIR_MODE_BF16_BLOCK) {
            st = plan_scan(bk, offsets, a, b, delay, s);
            if (st == SPIIR_OK) {
                hipError_t e = spiir::prepare_scan_fp32(bk);
                // the backward kernel's LDS window (segment + history) must fit
                if (e == hipSuccess &&
                    spiir::backward_lds_bytes(bk.ckpt_stride, bk.hist_len, bk.fpl) <= 160 * 1024)
                    e = spiir::prepare_backward(bk);
                if (e != hipSuccess)
                    st = fail(SPIIR_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
            }
            if (st == SPIIR_OK && bk.balanced) st = plan_balanced(bk, s);
            // per-segment partial sums of the adjoint, when a signal can span several
            // checkpoint segments (the segments are then walked in parallel)
            bk.bwd_max_seg = (bk.max_chunk + bk.ckpt_stride - 1) / bk.ckpt_stride;
            if (st == SPIIR_OK && bk.bwd_max_seg > 1)
                st = dev_alloc(bk, &bk.d_bwd_part,
                               (int64_t)bk.n_det * bk.bwd_max_seg * 6 * bk.n_slots * spiir::kWave);
            if (st == SPIIR_OK) st = zero_queue(bk, s);
        }
        if (st == SPIIR_OK) st = zero_stream_state(bk, s);
        if (st == SPIIR_OK) {
            const hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = fail(SPIIR_E_HIP, std::string("hipStreamSynchronize: ") +
                                                            hipGetErrorString(e));
        }
        if (st != SPIIR_OK) {
            free_all(bk);
            delete h;
            return st;
        }
        bk.last_stream = s;
        *out = h;
        return SPIIR_OK;
    } catch (const std::bad_alloc &) {
        return fail(SPIIR_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(SPIIR_E_INVAL, e.what());
    }
}

spiir_status spiir_bank_destroy(spiir_bank *h) {
    if (h == nullptr) return SPIIR_OK;
    spiir_status st = SPIIR_OK;
    const hipError_t e = hipStreamSynchronize(h->bk.last_stream);
    if (e != hipSuccess) st = fail(SPIIR_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    release_events(h->bk);
    free_all(h->bk);
    delete h;
    return st;
}

spiir_status spiir_bank_set_timing(spiir_bank *h, int32_t enable, int32_t capacity) {
    if (h == nullptr) return fail(SPIIR_E_INVAL, "bank is NULL");
    spiir::Bank &bk = h->bk;
    SPIIR_HIP(hipStreamSynchronize(bk.last_stream));
    release_events(bk);
    if (!enable) return SPIIR_OK;
    if (capacity < 1 || capacity > (1 << 20)) return fail(SPIIR_E_INVAL, "capacity must be in [1, 2^20]");
    bk.ev_start.resize(capacity);
    bk.ev_stop.resize(capacity);
    for (int32_t i = 0; i < capacity; ++i) {
        hipError_t e1 = hipEventCreate(&bk.ev_start[i]);
        hipError_t e2 = hipEventCreate(&bk.ev_stop[i]);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            bk.ev_start.resize(i);
            bk.ev_stop.resize(i);
            release_events(bk);
            return fail(SPIIR_E_HIP, "hipEventCreate failed");
        }
    }
    return SPIIR_OK;
}

spiir_status spiir_bank_kernel_time(spiir_bank *h, double *total_ms, int64_t *launches) {
    if (h == nullptr || total_ms == nullptr || launches == nullptr)
        return fail(SPIIR_E_INVAL, "bank, total_ms or launches is NULL");
    spiir::Bank &bk = h->bk;
    *total_ms = 0.0;
    *launches = 0;
    if (bk.ev_start.empty()) return fail(SPIIR_E_STATE, "timing is not enabled");
    const int64_t n = std::min<int64_t>(bk.timed, (int64_t)bk.ev_start.size());
    if (n > 0) SPIIR_HIP(hipEventSynchronize(bk.ev_stop[n - 1]));
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        float ms = 0.0f;
        SPIIR_HIP(hipEventElapsedTime(&ms, bk.ev_start[i], bk.ev_stop[i]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = n;
    return SPIIR_OK;
}

spiir_status spiir_bank_reset(spiir_bank *h, void *stream) {
    if (h == nullptr) return fail(SPIIR_E_INVAL, "bank is NULL");
    spiir::Bank &bk = h->bk;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (bk.h_wait_flag != nullptr) {
        // No launch still in flight may raise the flag after it is cleared.  The hand-off
        // bookkeeping restarts as at creation: a wave that gave up on a wait may have
        // left a flag behind the count the next launch expects.
        SPIIR_HIP(hipStreamSynchronize(bk.last_stream));
        SPIIR_HIP(hipStreamSynchronize(s));
        SPIIR_TRY(zero_queue(bk, s));
        SPIIR_HIP(hipStreamSynchronize(s));
        __atomic_store_n(bk.h_wait_flag, 0u, __ATOMIC_RELEASE);
    }
    bk.last_stream = s;
    return zero_stream_state(bk, s);
}

spiir_status spiir_bank_get_info(const spiir_bank *h, spiir_bank_info *info) {
    if (h == nullptr || info == nullptr) return fail(SPIIR_E_INVAL, "bank or info is NULL");
    const spiir::Bank &bk = h->bk;
    std::memset(info, 0, sizeof(*info));
    info->n_templates = bk.n_templates;
    info->n_detectors = bk.n_det;
    info->max_chunk = bk.max_chunk;
    info->max_delay = bk.hist_len;
    info->peak_window = bk.peak_window;
    info->mode = bk.mode;
    info->n_filters = bk.n_filters;
    info->device_bytes = bk.device_bytes;
    info->n_slices = bk.n_slices;
    info->filters_per_lane = bk.fpl;
    info->time_tile = bk.time_tile;
    info->scan_waves = bk.scan_waves;
    info->balance_waves = bk.balanced ? bk.balance_waves : 0;
    info->block_len = bk.block_len;
    info->n_long_pole = bk.n_long_pole;
    info->block_mfma_flop_per_column = bk.mode == SPIIR_MODE_BF16_BLOCK ? bk.block_flop_per_col : 0;
    if (bk.d_queue != nullptr) {
        spiir::ScanQueue q{};
        SPIIR_HIP(hipStreamSynchronize(bk.last_stream));
        SPIIR_HIP(hipMemcpy(&q, bk.d_queue, sizeof(q), hipMemcpyDeviceToHost));
        info->scan_wait_timeouts = (int32_t)q.error;
    }
    if (bk.d_bqueue != nullptr) {
        spiir::ScanQueue q{};
        SPIIR_HIP(hipStreamSynchronize(bk.last_stream));
        SPIIR_HIP(hipMemcpy(&q, bk.d_bqueue, sizeof(q), hipMemcpyDeviceToHost));
        info->scan_wait_timeouts += (int32_t)q.error;
    }
    return SPIIR_OK;
}

spiir_status spiir_filter_chunk(spiir_bank *h, const float *x, int32_t n, float *z, float *peak,
                                int32_t *argmax, void *stream) {
    if (h == nullptr) return fail(SPIIR_E_INVAL, "bank is NULL");
    spiir::Bank &bk = h->bk;
    if (n < 0 || n > bk.max_chunk)
        return fail(SPIIR_E_INVAL, "n must be in [0, max_chunk=" + std::to_string(bk.max_chunk) + "]");
    if (n == 0) return SPIIR_OK;
    if (x == nullptr) return fail(SPIIR_E_INVAL, "x is NULL");
    if ((peak == nullptr) != (argmax == nullptr))
        return fail(SPIIR_E_INVAL, "peak and argmax must both be given or both be NULL");
    if (peak != nullptr && bk.peak_window > 0 && n % bk.peak_window != 0)
        return fail(SPIIR_E_INVAL, "n must be a multiple of peak_window");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (bk.mode == SPIIR_MODE_BF16_BLOCK) {
        if (n % bk.block_len != 0)
            return fail(SPIIR_E_INVAL, "block form: n must be a multiple of block_len=" +
                                           std::to_string(bk.block_len));
        bk.last_stream = s;
        float2 *zz = z != nullptr ? reinterpret_cast<float2 *>(z) : bk.d_zbuf;
        const bool timing = bk.timed < (int64_t)bk.ev_start.size();
        if (timing) SPIIR_HIP(hipEventRecord(bk.ev_start[bk.timed], s));
        SPIIR_HIP(spiir::launch_block_bf16(bk, x, n, zz, s));
        if (timing) {
            SPIIR_HIP(hipEventRecord(bk.ev_stop[bk.timed], s));
            ++bk.timed;
        }
        SPIIR_HIP(spiir::launch_hist_update(bk, x, n, s));
        if (peak != nullptr) {
            const int32_t window = bk.peak_window > 0 ? bk.peak_window : n;
            SPIIR_HIP(spiir::launch_peaks(zz, (int64_t)bk.n_det * bk.n_templates, n, window, peak,
                                          argmax, s));
        }
        return SPIIR_OK;
    }
    SPIIR_TRY(check_waits(bk));
    bk.last_stream = s;
    const bool timing = bk.timed < (int64_t)bk.ev_start.size();
    if (timing) SPIIR_HIP(hipEventRecord(bk.ev_start[bk.timed], s));
    float2 *zz = reinterpret_cast<float2 *>(z);
    SPIIR_HIP(spiir::launch_scan_fp32(bk, x, n, nullptr, zz, peak, argmax, s));
    if (timing) {
        SPIIR_HIP(hipEventRecord(bk.ev_stop[bk.timed], s));
        ++bk.timed;
    }
    // slice sums, peaks and the history update in one launch
    SPIIR_HIP(spiir::launch_reduce_peaks(bk, n, zz, peak, argmax, x,
                                         spiir::scan_fuses_singles(bk, n, false, peak != nullptr),
                                         s));
    return SPIIR_OK;
}

spiir_status spiir_bank_noise_power(const spiir_bank *h, double *power) {
    if (h == nullptr || power == nullptr) return fail(SPIIR_E_INVAL, "bank or power is NULL");
    const spiir::Bank &bk = h->bk;
    const int32_t T = bk.n_templates;
    auto work = [&](int32_t t0, int32_t t1) {
        for (int32_t t = t0; t < t1; ++t) {
            double acc = 0.0;
            const int32_t lo = bk.h_offsets[t], hi = bk.h_offsets[t + 1];
            for (int32_t k = lo; k < hi; ++k)
                for (int32_t l = lo; l < hi; ++l) {
                    const int32_t p = bk.h_delay[k] >= bk.h_delay[l] ? k : l;
                    const int32_t q = p == k ? l : k;
                    const std::complex<double> ap(bk.h_a[2 * p], bk.h_a[2 * p + 1]);
                    const std::complex<double> aq(bk.h_a[2 * q], -bk.h_a[2 * q + 1]);   // conj(a_q)
                    const std::complex<double> bp(bk.h_b[2 * p], bk.h_b[2 * p + 1]);
                    const std::complex<double> bq(bk.h_b[2 * q], -bk.h_b[2 * q + 1]);   // conj(b_q)
                    std::complex<double> pw(1.0, 0.0), base = aq;
                    for (int32_t e = bk.h_delay[p] - bk.h_delay[q]; e > 0; e >>= 1) {
                        if (e & 1) pw *= base;
                        base *= base;
                    }
                    acc += (bp * bq * pw / (1.0 - ap * aq)).real();
                }
            power[t] = acc;
        }
    };
    const int32_t nt = (int32_t)std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 64u));
    std::vector<std::thread> pool;
    std::atomic<int32_t> next{0};
    for (int32_t w = 0; w < nt; ++w)
        pool.emplace_back([&]() {
            for (int32_t t; (t = next.fetch_add(1)) < T;) work(t, t + 1);
        });
    for (auto &th : pool) th.join();
    return SPIIR_OK;
}

spiir_status spiir_bank_trigger_weights(const spiir_bank *h, float *weight, void *stream) {
    if (h == nullptr || weight == nullptr) return fail(SPIIR_E_INVAL, "bank or weight is NULL");
    SPIIR_HIP(spiir::launch_trigger_weights(h->bk, weight, static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

spiir_status spiir_triggers(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                            const float *weight, float threshold, int32_t window, void *work,
                            float *snr, int32_t *index, void *stream) {
    if (n_det < 0 || n_templates < 0 || n < 0) return fail(SPIIR_E_INVAL, "sizes must be >= 0");
    if (window < 1) return fail(SPIIR_E_INVAL, "window must be >= 1");
    if (!std::isfinite(threshold) || threshold < 0.0f)
        return fail(SPIIR_E_INVAL, "threshold must be finite and >= 0");
    if ((int64_t)n_det * n_templates * n == 0) return SPIIR_OK;
    if (z == nullptr || weight == nullptr || work == nullptr || snr == nullptr || index == nullptr)
        return fail(SPIIR_E_INVAL, "z, weight, work, snr and index must be non-NULL");
    SPIIR_HIP(spiir::launch_triggers(reinterpret_cast<const float2 *>(z), n_det, n_templates, n,
                                     weight, threshold, window,
                                     static_cast<unsigned long long *>(work), snr, index,
                                     static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

spiir_status spiir_triggers_noalloc(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                                    const float *weight, float threshold, int32_t window,
                                    float *snr, int32_t *index, void *stream) {
    if (n_det < 0 || n_templates < 0 || n < 0) return fail(SPIIR_E_INVAL, "sizes must be >= 0");
    if (window < 1) return fail(SPIIR_E_INVAL, "window must be >= 1");
    if (!std::isfinite(threshold) || threshold < 0.0f)
        return fail(SPIIR_E_INVAL, "threshold must be finite and >= 0");
    if ((int64_t)n_det * n_templates * n == 0) return SPIIR_OK;
    const int64_t slots = (int64_t)n_det * n_templates * (((int64_t)n + window - 1) / window);
    if (slots > spiir::kTriggerScratchSlots)
        return fail(SPIIR_E_INVAL, "n_det * n_templates * ceil(n / window) = " +
                                       std::to_string(slots) + " exceeds the " +
                                       std::to_string(spiir::kTriggerScratchSlots) +
                                       " slots of the library's trigger workspace");
    if (z == nullptr || weight == nullptr || snr == nullptr || index == nullptr)
        return fail(SPIIR_E_INVAL, "z, weight, snr and index must be non-NULL");
    SPIIR_HIP(spiir::launch_triggers_noalloc(reinterpret_cast<const float2 *>(z), n_det,
                                             n_templates, n, weight, threshold, window, snr, index,
                                             static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

spiir_status spiir_bank_autocorr(const spiir_bank *h, int32_t nj, double *R, void *stream) {
    if (h == nullptr || R == nullptr) return fail(SPIIR_E_INVAL, "bank or R is NULL");
    if (nj < 1 || nj > 4096) return fail(SPIIR_E_INVAL, "nj must be in [1, 4096]");
    const spiir::Bank &bk = h->bk;
    const int32_t T = bk.n_templates;
    const int64_t F = bk.n_filters;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // temporary device copies of the coefficients in template order
    int32_t *d_off = nullptr, *d_d = nullptr;
    float2 *d_a = nullptr, *d_b = nullptr;
    auto release = [&]() {
        (void)hipFree(d_off);
        (void)hipFree(d_d);
        (void)hipFree(d_a);
        (void)hipFree(d_b);
    };
    const size_t fb = (size_t)std::max<int64_t>(F, 1);
    if (hipMalloc((void **)&d_off, sizeof(int32_t) * (T + 1)) != hipSuccess ||
        hipMalloc((void **)&d_d, sizeof(int32_t) * fb) != hipSuccess ||
        hipMalloc((void **)&d_a, sizeof(float2) * fb) != hipSuccess ||
        hipMalloc((void **)&d_b, sizeof(float2) * fb) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(SPIIR_E_NOMEM, "autocorr: temporary device allocation failed");
    }
    hipError_t e = hipMemcpyAsync(d_off, bk.h_offsets.data(), sizeof(int32_t) * (T + 1),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && F > 0)
        e = hipMemcpyAsync(d_d, bk.h_delay.data(), sizeof(int32_t) * F, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && F > 0)
        e = hipMemcpyAsync(d_a, bk.h_a.data(), sizeof(float2) * F, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && F > 0)
        e = hipMemcpyAsync(d_b, bk.h_b.data(), sizeof(float2) * F, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = spiir::launch_autocorr(T, d_off, d_a, d_b, d_d, nj, reinterpret_cast<double2 *>(R), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) return fail(SPIIR_E_HIP, std::string("autocorr: ") + hipGetErrorString(e));
    return SPIIR_OK;
}

spiir_status spiir_xi2(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                       const int32_t *index, int32_t n_win, const double *R, int32_t nj, float *xi2,
                       void *stream) {
    if (n_det < 0 || n_templates < 0 || n < 0 || n_win < 0)
        return fail(SPIIR_E_INVAL, "sizes must be >= 0");
    if (nj < 1 || nj > 4096) return fail(SPIIR_E_INVAL, "nj must be in [1, 4096]");
    if ((int64_t)n_det * n_templates * n_win == 0) return SPIIR_OK;
    if (z == nullptr || index == nullptr || R == nullptr || xi2 == nullptr)
        return fail(SPIIR_E_INVAL, "z, index, R and xi2 must be non-NULL");
    SPIIR_HIP(spiir::launch_xi2(reinterpret_cast<const float2 *>(z), n_det, n_templates, n, index,
                                n_win, reinterpret_cast<const double2 *>(R), nj, xi2,
                                static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

spiir_status spiir_xi2_network(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                               const int32_t *index, const int32_t *pix, int32_t n_win,
                               const int32_t *tau, int32_t n_pix, const double *R, int32_t nj,
                               float *xi2_det, float *xi2_c, void *stream) {
    if (n_det < 1 || n_det > 8) return fail(SPIIR_E_INVAL, "n_det must be in [1, 8]");
    if (n_templates < 0 || n < 0 || n_win < 0 || n_pix < 0)
        return fail(SPIIR_E_INVAL, "sizes must be >= 0");
    if (nj < 1 || nj > 4096) return fail(SPIIR_E_INVAL, "nj must be in [1, 4096]");
    if ((int64_t)n_templates * n_win == 0) return SPIIR_OK;
    if (z == nullptr || index == nullptr || pix == nullptr || R == nullptr || xi2_c == nullptr ||
        (n_pix > 0 && tau == nullptr))
        return fail(SPIIR_E_INVAL, "z, index, pix, tau, R and xi2_c must be non-NULL");
    SPIIR_HIP(spiir::launch_xi2_network(reinterpret_cast<const float2 *>(z), n_det, n_templates, n,
                                        index, pix, n_win, tau, n_pix,
                                        reinterpret_cast<const double2 *>(R), nj, xi2_det, xi2_c,
                                        static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

spiir_status spiir_coherent(const float *z, int32_t n_det, int32_t n_templates, int32_t n,
                            const int32_t *index, int32_t n_win, const float *U, const int32_t *tau,
                            int32_t n_pix, const int32_t *shifts, int32_t n_shift, float *snr2,
                            int32_t *pix, float *null2, void *stream) {
    if (n_det < 2 || n_det > 8) return fail(SPIIR_E_INVAL, "n_det must be in [2, 8]");
    if (n_templates < 0 || n < 0 || n_win < 0 || n_pix < 0 || n_shift < 0)
        return fail(SPIIR_E_INVAL, "sizes must be >= 0");
    if ((int64_t)n_templates * n_win * n_shift == 0) return SPIIR_OK;
    if (z == nullptr || index == nullptr || shifts == nullptr || snr2 == nullptr ||
        pix == nullptr || null2 == nullptr || (n_pix > 0 && (U == nullptr || tau == nullptr)))
        return fail(SPIIR_E_INVAL, "z, index, U, tau, shifts and the outputs must be non-NULL");
    SPIIR_HIP(spiir::launch_coherent(reinterpret_cast<const float2 *>(z), n_det, n_templates, n, index,
                                     n_win, U, tau, n_pix, shifts, n_shift, snr2, pix, null2,
                                     static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

spiir_status spiir_ckpt_count(const spiir_bank *h, int32_t n, int64_t *n_values) {
    if (h == nullptr || n_values == nullptr) return fail(SPIIR_E_INVAL, "bank or n_values is NULL");
    const spiir::Bank &bk = h->bk;
    if (bk.mode != SPIIR_MODE_FP32_SCAN)
        return fail(SPIIR_E_UNSUPPORTED, "differentiation needs the FP32 scan mode");
    if (n < 0) return fail(SPIIR_E_INVAL, "n must be >= 0");
    const int64_t n_seg = (n + bk.ckpt_stride - 1) / bk.ckpt_stride;
    *n_values = (int64_t)bk.n_det * n_seg * bk.n_slots * spiir::kWave;
    return SPIIR_OK;
}

namespace {
spiir_status check_diff_call(const spiir::Bank &bk, const float *x, int32_t n) {
    if (bk.mode != SPIIR_MODE_FP32_SCAN)
        return fail(SPIIR_E_UNSUPPORTED, "differentiation needs the FP32 scan mode");
    if (n < 1 || n > bk.max_chunk)
        return fail(SPIIR_E_INVAL, "n must be in [1, max_chunk=" + std::to_string(bk.max_chunk) + "]");
    if (x == nullptr) return fail(SPIIR_E_INVAL, "x is NULL");
    return SPIIR_OK;
}
}  // namespace

spiir_status spiir_forward(spiir_bank *h, const float *x, int32_t n, float *z, float *ckpt,
                           void *stream) {
    if (h == nullptr) return fail(SPIIR_E_INVAL, "bank is NULL");
    spiir::Bank &bk = h->bk;
    SPIIR_TRY(check_diff_call(bk, x, n));
    if (z == nullptr) return fail(SPIIR_E_INVAL, "z is NULL");
    SPIIR_TRY(check_waits(bk));
    hipStream_t s = static_cast<hipStream_t>(stream);
    bk.last_stream = s;
    SPIIR_TRY(zero_stream_state(bk, s));
    float2 *zz = reinterpret_cast<float2 *>(z);
    SPIIR_HIP(spiir::launch_scan_fp32(bk, x, n, reinterpret_cast<float2 *>(ckpt), zz, nullptr,
                                      nullptr, s));
    SPIIR_HIP(spiir::launch_reduce_peaks(bk, n, zz, nullptr, nullptr, nullptr,
                                         spiir::scan_fuses_singles(bk, n, true, false), s));
    return SPIIR_OK;
}

spiir_status spiir_backward(spiir_bank *h, const float *x, int32_t n, const float *grad_z,
                            const float *ckpt, float *grad_a, float *grad_b, void *stream) {
    if (h == nullptr) return fail(SPIIR_E_INVAL, "bank is NULL");
    spiir::Bank &bk = h->bk;
    SPIIR_TRY(check_diff_call(bk, x, n));
    if (grad_z == nullptr || ckpt == nullptr || grad_a == nullptr || grad_b == nullptr)
        return fail(SPIIR_E_INVAL, "grad_z, ckpt, grad_a and grad_b must be non-NULL");
    if (spiir::backward_lds_bytes(bk.ckpt_stride, bk.hist_len, bk.fpl) > 160 * 1024)
        return fail(SPIIR_E_UNSUPPORTED, "ckpt_stride + max_delay too large for the adjoint window");
    SPIIR_TRY(check_waits(bk));
    hipStream_t s = static_cast<hipStream_t>(stream);
    bk.last_stream = s;
    SPIIR_HIP(spiir::launch_backward(bk, x, n, reinterpret_cast<const float2 *>(grad_z),
                                     reinterpret_cast<const float2 *>(ckpt),
                                     reinterpret_cast<float2 *>(grad_a),
                                     reinterpret_cast<float2 *>(grad_b), s));
    return SPIIR_OK;
}

spiir_status spiir_bank_set_coeffs(spiir_bank *h, const float *a, const float *b, void *stream) {
    if (h == nullptr) return fail(SPIIR_E_INVAL, "bank is NULL");
    spiir::Bank &bk = h->bk;
    if (bk.n_filters > 0 && (a == nullptr || b == nullptr)) return fail(SPIIR_E_INVAL, "a or b is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    bk.last_stream = s;
    if (bk.mode == SPIIR_MODE_BF16_BLOCK)
        SPIIR_HIP(spiir::launch_block_set_coeffs(bk, reinterpret_cast<const float2 *>(a),
                                                 reinterpret_cast<const float2 *>(b), s));
    else
        SPIIR_HIP(spiir::launch_set_coeffs(bk, reinterpret_cast<const float2 *>(a),
                                           reinterpret_cast<const float2 *>(b), s));
    return SPIIR_OK;
}

spiir_status spiir_peaks(const float *z, int64_t rows, int32_t n, int32_t window, float *peak,
                         int32_t *argmax, void *stream) {
    if (rows < 0 || n < 0) return fail(SPIIR_E_INVAL, "rows and n must be >= 0");
    if (window < 1) return fail(SPIIR_E_INVAL, "window must be >= 1");
    if (rows == 0 || n == 0) return SPIIR_OK;
    if (z == nullptr || peak == nullptr || argmax == nullptr)
        return fail(SPIIR_E_INVAL, "z, peak and argmax must be non-NULL");
    SPIIR_HIP(spiir::launch_peaks(reinterpret_cast<const float2 *>(z), rows, n, window, peak, argmax,
                                  static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

}  // extern "C"
