// FP32 scan of the SPIIR filter bank (Eq. zk, Section II.B.1, read per filter):
//     y_k[n] = a_k y_k[n-1] + b_k x[n-d_k],   partial_s[n] = sum_{k in slice s} y_k[n]
//
// Work decomposition.  A slice is up to 64*MAXM filters of one template.  One
// wavefront owns one slice for one detector and walks the whole packet in time:
// lane l holds the slice's filters of slots 0..m-1 (coefficients and state in
// registers), so every lane runs m independent recurrences.  Four waves share a
// workgroup and the LDS copy of the detector's input window
//     x[n0 - hist_len, n0 + tile)     (history ring followed by the packet)
// which covers every delay: filter k at sample n reads window[n - n0 + hist_len - d_k].
// Time advances in register sub-tiles of kSub samples.  Each lane accumulates
// the sum of its own filters per sample; the 64 lane partials of a sub-tile are
// then reduced in registers by a transpose-reduce across lanes (lane-half swaps,
// then row rotations and mirrors within 16-lane rows): every step halves the
// samples a lane holds and doubles the lanes summed, so 16 lanes end with the
// slice's partial template sum of one sample each.  No LDS is used for it.  A
// second kernel adds the slices of each template.
//
// Arithmetic per filter-sample: 2 mul + 4 fma (complex a*y + b*x with real x)
// and 2 adds into the lane sum (none for a lane's first filter): at most 8 VALU
// lane-operations for the paper's 12 flops.
//
// Schedules.  The static kernel gives one slice to each wave.  When the packet and
// its history fit one LDS window, the balanced kernel (on request) instead runs a
// fixed set of resident waves, each with a host-planned list of equal total work in
// which slices may be cut in time between two waves.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "internal.h"

namespace spiir {
namespace {

static_assert(kSub == 16, "the lane reduction halves 16 samples four times");

// Cross-lane data movement for the reduction.  DPP controls (within rows of 16
// lanes): rotate by 8 (partner l^8), mirror within 8 lanes (partner 7-i), and
// quad permutations swapping neighbours at distance 1 and 2.
constexpr int kDppRowRor8 = 0x128;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// a in the lower, b in the upper half-wave exchanged: every lane gets the sum of one
// of the two values over itself and its partner in the other half
__device__ __forceinline__ float swap32_sum(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// the same between the two 16-lane rows of each half-wave
__device__ __forceinline__ float swap16_sum(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sample of the sub-tile whose 64-lane total reduce_lanes leaves in this lane: the
// two swap steps are traced on the sample offsets they select (8 and 4), the two
// DPP steps select by lane bits 3 and 2.
__device__ __forceinline__ int reduce_sample(int lane) {
    const auto h8 = __builtin_amdgcn_permlane32_swap(0u, 8u, false, false);
    const auto h4 = __builtin_amdgcn_permlane16_swap(0u, 4u, false, false);
    return (int)h8[0] + (int)h4[0] + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}

// Sum acc[s] over the 64 lanes for all 16 samples s; the lane receives the total of
// sample reduce_sample(lane) (all four lanes of a quad hold the same one).
__device__ __forceinline__ float2 reduce_lanes(const float2 (&acc)[kSub], int lane) {
    float2 w[8];
#pragma unroll
    for (int s = 0; s < 8; ++s)
        w[s] = make_float2(swap32_sum(acc[s].x, acc[s + 8].x), swap32_sum(acc[s].y, acc[s + 8].y));
    float2 u[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
        u[s] = make_float2(swap16_sum(w[s].x, w[s + 4].x), swap16_sum(w[s].y, w[s + 4].y));
    const bool b3 = (lane & 8) != 0;
    float2 t[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const float2 send = b3 ? u[s] : u[s + 2];
        const float2 keep = b3 ? u[s + 2] : u[s];
        t[s] = make_float2(keep.x + dpp_move<kDppRowRor8>(send.x),
                           keep.y + dpp_move<kDppRowRor8>(send.y));
    }
    const bool b2 = (lane & 4) != 0;
    const float2 send = b2 ? t[0] : t[1];
    const float2 keep = b2 ? t[1] : t[0];
    float2 v = make_float2(keep.x + dpp_move<kDppRowHalfMirror>(send.x),
                           keep.y + dpp_move<kDppRowHalfMirror>(send.y));
    v.x += dpp_move<kDppQuadXor1>(v.x);
    v.y += dpp_move<kDppQuadXor1>(v.y);
    v.x += dpp_move<kDppQuadXor2>(v.x);
    v.y += dpp_move<kDppQuadXor2>(v.y);
    return v;
}

__device__ __forceinline__ void lds_fence() {
    // orders this wave's LDS writes before its later LDS reads (and vice versa)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Copy the input window x[n0 - hist_len, n0 + T) of one detector into LDS:
// positions before the packet come from the history ring.  Loads are issued in
// batches of kBatch per thread before their LDS stores, so that many global loads
// are in flight at once instead of one latency per element.
constexpr int kBatch = 16;

__device__ __forceinline__ void load_window(float *__restrict__ win, const float *__restrict__ xd,
                                            const float *__restrict__ hd, int hist_len, int n0,
                                            int T, int tid, int nthreads) {
    const int total = T + hist_len;
    for (int b0 = 0; b0 < total; b0 += kBatch * nthreads) {
        float v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = b0 + k * nthreads + tid;
            const int pos = n0 - hist_len + i;
            v[k] = 0.0f;
            if (i < total) v[k] = pos >= 0 ? xd[pos] : hd[hist_len + pos];
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = b0 + k * nthreads + tid;
            if (i < total) win[i] = v[k];
        }
    }
}

// Returns the slice's sum of sample s0 + reduce_sample(lane), which the first lane of
// every quad also stores at out[reduce_sample(lane)] when out is given.
template <int MAXM, int M, bool TAIL>
__device__ __forceinline__ float2 sub_tile_m(const float *__restrict__ win, int red_sample,
                                           int lane, int s0, int valid,
                                           const float (&ar)[MAXM], const float (&ai)[MAXM],
                                           const float (&br)[MAXM], const float (&bi)[MAXM],
                                           const int (&base)[MAXM], float (&yr)[MAXM],
                                           float (&yi)[MAXM], float2 *__restrict__ out) {
    // M >= 1 filters per lane: in a full sub-tile the lane sums start from the first
    // filter's outputs (no zero fill, no first add)
    float2 acc[kSub];
    if (TAIL) {
#pragma unroll
        for (int s = 0; s < kSub; ++s) acc[s] = make_float2(0.0f, 0.0f);
    }
    // The kSub inputs of filter j+1 are read from LDS while filter j computes, so a
    // wave waits for LDS once per sub-tile instead of once per pair of samples (the
    // scheduling barriers keep the compiler from sinking the reads next to their
    // uses).  Reads past `valid` in a tail stay inside the window's kSub padding.
    float xb[2][kSub];   // filter j reads xb[j & 1] (a compile-time index: no copies)
#pragma unroll
    for (int s = 0; s < kSub; ++s) xb[0][s] = win[base[0] + s0 + s];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        {
            if (j + 1 < M) {
#pragma unroll
                for (int s = 0; s < kSub; ++s) xb[(j + 1) & 1][s] = win[base[j + 1] + s0 + s];
            }
            __builtin_amdgcn_sched_barrier(0);
            float r = yr[j], im = yi[j];
#pragma unroll
            for (int s = 0; s < kSub; ++s) {
                if (!TAIL || s < valid) {
                    const float xv = xb[j & 1][s];
                    const float nr = fmaf(ar[j], r, fmaf(-ai[j], im, br[j] * xv));
                    const float ni = fmaf(ar[j], im, fmaf(ai[j], r, bi[j] * xv));
                    r = nr;
                    im = ni;
                    if (!TAIL && j == 0) {
                        acc[s] = make_float2(r, im);
                    } else {
                        acc[s].x += r;
                        acc[s].y += im;
                    }
                }
            }
            yr[j] = r;
            yi[j] = im;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const float2 v = reduce_lanes(acc, lane);
    if (out != nullptr && (lane & 3) == 0 && (!TAIL || red_sample < valid)) out[red_sample] = v;
    return v;
}

// One sub-tile for a wave whose slice has m (1..MAXM, wave-uniform) filters per lane:
// a scalar branch to the variant compiled for exactly m.
template <int MAXM, bool TAIL>
__device__ __forceinline__ float2 sub_tile(const float *__restrict__ win, int red_sample, int lane,
                                         int m, int s0, int valid, const float (&ar)[MAXM],
                                         const float (&ai)[MAXM], const float (&br)[MAXM],
                                         const float (&bi)[MAXM], const int (&base)[MAXM],
                                         float (&yr)[MAXM], float (&yi)[MAXM],
                                         float2 *__restrict__ out) {
#define SPIIR_SUB_TILE(M)                                                                    \
    case M:                                                                                  \
        if constexpr (M <= MAXM)                                                             \
            return sub_tile_m<MAXM, M, TAIL>(win, red_sample, lane, s0, valid, ar, ai, br, bi,  \
                                             base, yr, yi, out);                             \
        break;
    switch (m) {
        SPIIR_SUB_TILE(1)
        SPIIR_SUB_TILE(2)
        SPIIR_SUB_TILE(3)
        SPIIR_SUB_TILE(4)
        SPIIR_SUB_TILE(5)
        SPIIR_SUB_TILE(6)
        SPIIR_SUB_TILE(7)
        SPIIR_SUB_TILE(8)
    default: break;
    }
#undef SPIIR_SUB_TILE
    return make_float2(0.0f, 0.0f);
}

// Run fn(std::integral_constant<int, M>{}) for the wave-uniform filter count m in
// 1..MAXM: a caller's whole sub-tile loop is compiled once per filter count, so the
// loop makes no per-sub-tile dispatch (5% of the balanced kernel's time on the
// realistic bank when the switch sat inside the loop).
template <int MAXM, typename Fn>
__device__ __forceinline__ void with_m(int m, Fn &&fn) {
#define SPIIR_WITH_M(M)                                                                      \
    case M:                                                                                  \
        if constexpr (M <= MAXM) fn(std::integral_constant<int, M>{});                      \
        break;
    switch (m) {
        SPIIR_WITH_M(1)
        SPIIR_WITH_M(2)
        SPIIR_WITH_M(3)
        SPIIR_WITH_M(4)
        SPIIR_WITH_M(5)
        SPIIR_WITH_M(6)
        SPIIR_WITH_M(7)
        SPIIR_WITH_M(8)
    default: break;
    }
#undef SPIIR_WITH_M
}

template <int MAXM>
__global__ __launch_bounds__(kWave *kScanWaves) void scan_fp32_kernel(
    const float2 *__restrict__ ca, const float2 *__restrict__ cb, const int32_t *__restrict__ cd,
    float2 *__restrict__ state, const Slice *__restrict__ slices,
    const int32_t *__restrict__ slice_order, int32_t n_slices,
    int64_t lanes_total, const float *__restrict__ x, int32_t n, const float *__restrict__ hist,
    int32_t hist_len, float2 *__restrict__ partial, int32_t part_stride, int32_t tile_len,
    float2 *__restrict__ ckpt, int32_t ckpt_stride, int32_t n_seg, float2 *__restrict__ z,
    int32_t n_tmpl) {
    extern __shared__ float smem[];
    float *win = smem;
    // wave-uniform values live in scalar registers (readfirstlane), so that the
    // per-slot tests below are scalar branches
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int red_sample = reduce_sample(lane);
    const int det = blockIdx.y;
    // slices go out largest first, so the waves of a workgroup carry equal work
    const int rank = blockIdx.x * kScanWaves + wave;
    const bool active = rank < n_slices;
    const int sidx = active ? __builtin_amdgcn_readfirstlane(slice_order[rank]) : 0;
    Slice sl = active ? slices[sidx] : Slice{0, 0, 0, 0};
    sl.tmpl = __builtin_amdgcn_readfirstlane(sl.tmpl);
    sl.slot_base = __builtin_amdgcn_readfirstlane(sl.slot_base);
    sl.n_slots = __builtin_amdgcn_readfirstlane(sl.n_slots);
    sl.single = __builtin_amdgcn_readfirstlane(sl.single);
    const int m = sl.n_slots;

    float ar[MAXM], ai[MAXM], br[MAXM], bi[MAXM], yr[MAXM], yi[MAXM];
    int base[MAXM];
    float2 *st = state + (int64_t)det * lanes_total;
#pragma unroll
    for (int j = 0; j < MAXM; ++j) {
        if (j < m) {
            const int64_t g = (int64_t)(sl.slot_base + j) * kWave + lane;
            const float2 a = ca[g], b = cb[g], y = st[g];
            ar[j] = a.x; ai[j] = a.y; br[j] = b.x; bi[j] = b.y; yr[j] = y.x; yi[j] = y.y;
            base[j] = hist_len - cd[g];
        } else {
            ar[j] = ai[j] = br[j] = bi[j] = yr[j] = yi[j] = 0.0f;
            base[j] = 0;
        }
    }

    const float *xd = x + (int64_t)det * n;
    const float *hd = hist + (int64_t)det * hist_len;
    float2 *pout = sl.single && z != nullptr
                       ? z + ((int64_t)det * n_tmpl + sl.tmpl) * n
                       : partial + ((int64_t)det * n_slices + sidx) * part_stride;
    // optional checkpoints: the state entering every ckpt_stride-sample segment
    float2 *ck = ckpt != nullptr ? ckpt + (int64_t)det * n_seg * lanes_total : nullptr;
    if (ck != nullptr && active) {
#pragma unroll
        for (int j = 0; j < MAXM; ++j)
            if (j < m) ck[(int64_t)(sl.slot_base + j) * kWave + lane] = make_float2(yr[j], yi[j]);
    }

    for (int n0 = 0; n0 < n; n0 += tile_len) {
        const int T = min(tile_len, n - n0);
        __syncthreads();  // every wave is done with the previous window
        load_window(win, xd, hd, hist_len, n0, T, threadIdx.x, blockDim.x);
        __syncthreads();
        if (!active) continue;
        const int full = T & ~(kSub - 1);
        with_m<MAXM>(m, [&](auto mc) {
            constexpr int M = decltype(mc)::value;
            for (int s0 = 0; s0 < full; s0 += kSub) {
                sub_tile_m<MAXM, M, false>(win, red_sample, lane, s0, kSub, ar, ai, br, bi, base,
                                           yr, yi, pout + n0 + s0);
                const int e = n0 + s0 + kSub;
                if (ck != nullptr && e % ckpt_stride == 0 && e < n) {
                    float2 *cs = ck + (int64_t)(e / ckpt_stride) * lanes_total;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        cs[(int64_t)(sl.slot_base + j) * kWave + lane] = make_float2(yr[j], yi[j]);
                }
            }
        });
        if (full < T)
            sub_tile<MAXM, true>(win, red_sample, lane, m, full, T - full, ar, ai, br, bi, base, yr,
                                 yi, pout + n0 + full);
    }
    if (active) {
#pragma unroll
        for (int j = 0; j < MAXM; ++j)
            if (j < m) st[(int64_t)(sl.slot_base + j) * kWave + lane] = make_float2(yr[j], yi[j]);
    }
}

// Cross-XCD hand-off of filter state inside one launch.  The state travels through
// device-scope atomic accesses (coherent across XCDs, not held in the non-coherent
// caches); the producer waits until those stores have completed before it moves
// the flag (a device-scope atomic), and the consumer spins on the flag before it
// loads the state.  The wait is bounded (`spins` polls of about 128 clocks); a wait
// that hits the bound is counted in the bank's queue record and raises a flag in
// host memory, which the library's next call reads (it then refuses to go on until
// the stream is reset: the waiting wave went on with a stale state).
struct WaitBound {
    uint32_t spins;
    uint32_t *host_flag;   // device alias of a word in pinned host memory
};

__device__ __forceinline__ float2 load_coherent(const float2 *p) {
    const uint64_t v = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, v);
}

__device__ __forceinline__ void store_coherent(float2 *p, float2 v) {
    __hip_atomic_store(reinterpret_cast<uint64_t *>(p), __builtin_bit_cast(uint64_t, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wait_memory() {
    // every memory operation this wave issued so far has completed (s_waitcnt with all
    // counters at zero); no cache maintenance.  The fences keep the compiler from
    // moving memory accesses across the wait.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Wait until *flag has reached `target` (counts are compared modulo 2^32); lane 0
// polls, the other lanes wait at the following wave-wide operations.
__device__ __forceinline__ void wait_flag(const uint32_t *flag, uint32_t target, int lane,
                                          uint32_t *error, WaitBound wb) {
    if (lane == 0) {
        uint32_t spins = 0;
        while ((int32_t)(__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                         target) < 0) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins >= wb.spins) {
                __hip_atomic_fetch_add(error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(wb.host_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                break;
            }
        }
    }
    wait_memory();
}

// Issue priority among the waves of the balanced schedule that share a SIMD.  They
// carry equal planned work, but the SIMD's arbiter favours the older wave, which
// then finishes long before its younger neighbour (about a quarter of the launch
// on the realistic bank), and the SIMD runs one wave for the rest of the launch.
// Each wave therefore publishes its progress (planned cost of the sub-tiles done)
// in a per-SIMD table every kPeerPeriod sub-tiles and sets its priority to the
// number of co-resident waves that are ahead of it, so the wave that lags is served
// first.  The table lives in global memory but only waves of one compute unit
// share an entry, so workgroup-scope accesses suffice; a stale read only delays a
// priority change.  Entry (kPeerWords words per SIMD): progress of arrival slots
// 0..kPeerSlots-1, then the number of waves registered.  A wave past the last slot
// stays at the default priority.
constexpr uint32_t kPeerPeriod = 8;
constexpr uint32_t kPeerSlots = 4;
constexpr uint32_t kPeerWords = kPeerTableWords;

struct SimdPeers {
    uint32_t *tab;
    uint32_t slot;
    uint32_t done;
    uint32_t tick;
    uint32_t seen;   // lane k < kPeerSlots: slot k of the table as read at the previous exchange
};

__device__ __forceinline__ uint32_t simd_key() {
    // HW_ID bits 4..15: SIMD, pipe, CU, shader array and engine; XCC_ID: the XCD
    const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);
    const uint32_t xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);
    return ((hw >> 4) & 0xFFFu) | ((xcc & 7u) << 12);
}

__device__ __forceinline__ SimdPeers simd_join(uint32_t *table, int lane) {
    SimdPeers p{table + (size_t)simd_key() * kPeerWords, 0u, 0u, 0u, 0u};
    uint32_t slot = 0;
    if (lane == 0)
        slot = __hip_atomic_fetch_add(p.tab + kPeerSlots, 1u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
    p.slot = __builtin_amdgcn_readfirstlane(slot);
    return p;
}

__device__ __forceinline__ void set_priority(uint32_t level) {
    if (level == 0) __builtin_amdgcn_s_setprio(0);
    else if (level == 1) __builtin_amdgcn_s_setprio(1);
    else if (level == 2) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(3);
}

// After a sub-tile of planned cost `cost`; every kPeerPeriod sub-tiles: compare with
// the table read at the previous exchange (its loads have long returned), set the
// priority, publish the progress and read the table again.
__device__ __forceinline__ void simd_step(SimdPeers &p, uint32_t cost, int lane) {
    if (p.slot >= kPeerSlots) return;
    p.done += cost;
    if (++p.tick % kPeerPeriod != 0) return;
    // one slot per lane: the waves ahead are the lanes whose slot beats this progress
    const uint64_t ahead = __builtin_amdgcn_ballot_w64((uint32_t)lane < kPeerSlots && p.seen > p.done);
    set_priority((uint32_t)__builtin_popcountll(ahead));
    if (lane == 0)
        __hip_atomic_store(p.tab + p.slot, p.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if ((uint32_t)lane < kPeerSlots)
        p.seen = __hip_atomic_load(p.tab + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void simd_leave(SimdPeers &p, int lane) {
    __builtin_amdgcn_s_setprio(0);
    if (lane == 0) {
        if (p.slot < kPeerSlots)
            __hip_atomic_store(p.tab + p.slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_sub(p.tab + kPeerSlots, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// First sample of the sub-tile that starts at fraction phi of a packet of n samples.
__device__ __forceinline__ int phi_sample(int32_t phi, int32_t n) {
    if (phi >= kPhiOne) return n;
    const int t = (int)(((int64_t)phi * n + kPhiOne / 2) >> 16);
    return min(n, t) & ~(kSub - 1);
}

// Peak search of a single-slice template inside the balanced scan (one candidate per
// template per window, Section II.C.1), with the slice-sum kernel's decision: |z|^2
// as two rounded products and a rounded sum, the largest value winning and the
// lowest index among equal ones.  It runs when a wave has finished its part
// [t0, t1) of the slice: the wave reads back the series it has just written (from
// its own compute unit's L2) one window at a time, so the sub-tile loop carries
// no extra registers.  Windows are whole sub-tiles or the whole packet; a window
// that a cut splits is closed by the later part, from the candidate the earlier
// part leaves next to its state.

// Outputs of the fused peak search (peak NULL: not fused).
struct FusedPeaks {
    float *peak;       // [D][T][n_win]
    int32_t *argmax;   // [D][T][n_win]
    float2 *cand;      // [D][n_splits]
    int32_t window;
    int32_t n_win;
};

struct PeakBest {
    float p;    // |z|^2 (-1 before the first sample)
    int32_t i;  // index in the window
};

__device__ __forceinline__ float abs2_rn(float re, float im) {
#pragma clang fp contract(off)
    const float rr = re * re;
    const float ii = im * im;
    return rr + ii;
}

__device__ __forceinline__ PeakBest peak_better(PeakBest a, PeakBest b) {
    return (b.p > a.p || (b.p == a.p && b.i < a.i)) ? b : a;
}

__device__ __forceinline__ void segment_peaks(const float2 *__restrict__ row, int t0, int t1, int n,
                                           int window, const float2 *cand_in,
                                           float2 *cand_out, float *__restrict__ pk,
                                           int32_t *__restrict__ am, int lane) {
    constexpr int kRb = 8;   // loads in flight per lane
    wait_memory();           // this wave's stores of the series have completed
    PeakBest best{-1.0f, INT_MAX};
    if (cand_in != nullptr) {
        const float2 c = load_coherent(cand_in);
        best = PeakBest{c.x, __float_as_int(c.y)};
    }
    int cw = t0 / window;
    for (int w0 = t0; w0 < t1;) {
        const int wlo = cw * window;
        const int wend = min(wlo + window, t1);
        PeakBest b{-1.0f, INT_MAX};
        for (int i0 = w0; i0 < wend; i0 += kRb * kWave) {
            float2 v[kRb];
#pragma unroll
            for (int k = 0; k < kRb; ++k) {
                const int i = i0 + k * kWave + lane;
                v[k] = i < wend ? load_coherent(row + i) : make_float2(0.0f, 0.0f);
            }
#pragma unroll
            for (int k = 0; k < kRb; ++k) {
                const int i = i0 + k * kWave + lane;
                const float p = abs2_rn(v[k].x, v[k].y);
                if (i < wend && p > b.p) {   // a lane's samples increase: first one kept
                    b.p = p;
                    b.i = i - wlo;
                }
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            PeakBest o;
            o.p = __shfl_xor(b.p, off);
            o.i = __shfl_xor(b.i, off);
            b = peak_better(b, o);
        }
        best = peak_better(best, b);
        if (wend == wlo + window || wend == n) {
            if (lane == 0) {
                pk[cw] = sqrtf(best.p);
                am[cw] = best.i;
            }
            best = PeakBest{-1.0f, INT_MAX};
            ++cw;
        } else if (lane == 0) {
            // the segment ends inside the window: the later part finishes it
            store_coherent(cand_out, make_float2(best.p, __int_as_float(best.i)));
        }
        w0 = wend;
    }
}

// Balanced static schedule of the one-shot scan.  The host cuts the detector's
// slices into equal shares of work, one per resident wave (the wrap-around rule
// for preemptive scheduling on identical machines: fill wave after wave up to the
// mean load; a slice that does not fit is cut in time, its later part closing the
// current wave's list and its earlier part opening the next one).  Every SIMD then
// carries the same load whatever the slice sizes, and the earlier part of a cut
// slice runs first in its wave while the later part runs last in its own, so the
// state hand-off between them rarely waits.  The window x[-hist_len, n) of the
// workgroup's detector is loaded into LDS once for all its waves.
// Waves per SIMD the balanced kernel must fit in registers: its planner places a
// whole number of workgroups (one wave per SIMD each) on every compute unit, and the
// best counts are 3 at 8 filters per lane and up to 4 at 2 or 4.
constexpr int balanced_min_waves(int maxm) { return maxm >= 8 ? 3 : 4; }

template <int MAXM>
__global__ __launch_bounds__(kWave *kScanWaves) __attribute__((amdgpu_waves_per_eu(
    balanced_min_waves(MAXM)))) void scan_fp32_balanced_kernel(
    const float2 *__restrict__ ca, const float2 *__restrict__ cb, const int32_t *__restrict__ cd,
    float2 *__restrict__ state, const Slice *__restrict__ slices, int32_t n_slices,
    const Seg *__restrict__ segs, const int32_t *__restrict__ seg_off, int32_t waves_per_det,
    int32_t n_splits, uint32_t *__restrict__ flags, ScanQueue *__restrict__ queue,
    int64_t lanes_total, const float *__restrict__ x, int32_t n, const float *__restrict__ hist,
    int32_t hist_len, float2 *__restrict__ partial, int32_t part_stride, float2 *__restrict__ ckpt,
    int32_t ckpt_stride, int32_t n_seg, uint32_t *__restrict__ simd_tab, WaitBound wb,
    float2 *__restrict__ z, int32_t n_tmpl, FusedPeaks fp) {
    extern __shared__ float smem[];
    float *win = smem;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int red_sample = reduce_sample(lane);
    const int det = blockIdx.y;
    const uint32_t epoch =
        __hip_atomic_load(&queue->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float *xd = x + (int64_t)det * n;
    const float *hd = hist + (int64_t)det * hist_len;
    load_window(win, xd, hd, hist_len, 0, n, threadIdx.x, blockDim.x);
    __syncthreads();
    SimdPeers peers = simd_join(simd_tab, lane);
    float2 *st = state + (int64_t)det * lanes_total;
    float2 *ck = ckpt != nullptr ? ckpt + (int64_t)det * n_seg * lanes_total : nullptr;
    uint32_t *fl = flags + (int64_t)det * n_splits;
    const int w = blockIdx.x * kScanWaves + wave;
    const int e0 = w < waves_per_det ? __builtin_amdgcn_readfirstlane(seg_off[w]) : 0;
    const int e1 = w < waves_per_det ? __builtin_amdgcn_readfirstlane(seg_off[w + 1]) : 0;
    for (int e = e0; e < e1; ++e) {
        Seg sg = segs[e];
        sg.slice = __builtin_amdgcn_readfirstlane(sg.slice);
        sg.phi0 = __builtin_amdgcn_readfirstlane(sg.phi0);
        sg.phi1 = __builtin_amdgcn_readfirstlane(sg.phi1);
        sg.flag = __builtin_amdgcn_readfirstlane(sg.flag);
        Slice sl = slices[sg.slice];
        sl.tmpl = __builtin_amdgcn_readfirstlane(sl.tmpl);
        sl.slot_base = __builtin_amdgcn_readfirstlane(sl.slot_base);
        sl.n_slots = __builtin_amdgcn_readfirstlane(sl.n_slots);
        sl.single = __builtin_amdgcn_readfirstlane(sl.single);
        const int m = sl.n_slots;
        const int t0 = sg.phi0 > 0 ? phi_sample(sg.phi0, n) : 0;
        const int t1 = phi_sample(sg.phi1, n);
        float ar[MAXM], ai[MAXM], br[MAXM], bi[MAXM], yr[MAXM], yi[MAXM];
        int base[MAXM];
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
            if (j < m) {
                const int64_t g = (int64_t)(sl.slot_base + j) * kWave + lane;
                const float2 a = ca[g], b = cb[g];
                ar[j] = a.x; ai[j] = a.y; br[j] = b.x; bi[j] = b.y;
                base[j] = hist_len - cd[g];
            } else {
                ar[j] = ai[j] = br[j] = bi[j] = 0.0f;
                base[j] = 0;
            }
        }
        if (sg.phi0 > 0) {
            __builtin_amdgcn_s_setprio(0);   // a waiting wave yields the SIMD
            wait_flag(fl + sg.flag, epoch + 1u, lane, &queue->error, wb);
        }
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
            if (j < m) {
                const int64_t g = (int64_t)(sl.slot_base + j) * kWave + lane;
                const float2 y = sg.phi0 > 0 ? load_coherent(st + g) : st[g];
                yr[j] = y.x; yi[j] = y.y;
            } else {
                yr[j] = yi[j] = 0.0f;
            }
        }
        if (ck != nullptr && t0 == 0) {
#pragma unroll
            for (int j = 0; j < MAXM; ++j)
                if (j < m) ck[(int64_t)(sl.slot_base + j) * kWave + lane] = make_float2(yr[j], yi[j]);
        }
        // a single-slice template is its own SNR series: into z when asked for
        float2 *pout = sl.single && z != nullptr
                           ? z + ((int64_t)det * n_tmpl + sl.tmpl) * n
                           : partial + ((int64_t)det * n_slices + sg.slice) * part_stride;
        const int full_end = t1 == n ? (n & ~(kSub - 1)) : t1;
        with_m<MAXM>(m, [&](auto mc) {
            constexpr int M = decltype(mc)::value;
            for (int s0 = t0; s0 < full_end; s0 += kSub) {
                sub_tile_m<MAXM, M, false>(win, red_sample, lane, s0, kSub, ar, ai, br, bi, base,
                                           yr, yi, pout + s0);
                simd_step(peers, 20u * (uint32_t)M + 9u, lane);
                const int eo = s0 + kSub;
                if (ck != nullptr && eo % ckpt_stride == 0 && eo < n) {
                    float2 *cs = ck + (int64_t)(eo / ckpt_stride) * lanes_total;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        cs[(int64_t)(sl.slot_base + j) * kWave + lane] = make_float2(yr[j], yi[j]);
                }
            }
        });
        if (t1 == n && full_end < n)
            sub_tile<MAXM, true>(win, red_sample, lane, m, full_end, n - full_end, ar, ai, br, bi,
                                 base, yr, yi, pout + full_end);
        if (sl.single && fp.peak != nullptr && t1 > t0) {
            const int64_t prow = ((int64_t)det * n_tmpl + sl.tmpl) * fp.n_win;
            float2 *cs = fp.cand + (int64_t)det * n_splits + (sg.flag >= 0 ? sg.flag : 0);
            segment_peaks(pout, t0, t1, n, fp.window,
                          sg.phi0 > 0 && t0 % fp.window != 0 ? cs : nullptr, cs, fp.peak + prow,
                          fp.argmax + prow, lane);
        }
        if (sg.phi1 < kPhiOne) {
            // first part of a cut slice: publish the state (and a peak candidate) for the
            // wave that continues it
#pragma unroll
            for (int j = 0; j < MAXM; ++j)
                if (j < m)
                    store_coherent(st + (int64_t)(sl.slot_base + j) * kWave + lane,
                                   make_float2(yr[j], yi[j]));
            wait_memory();
            if (lane == 0)
                __hip_atomic_store(fl + sg.flag, epoch + 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
#pragma unroll
            for (int j = 0; j < MAXM; ++j)
                if (j < m) st[(int64_t)(sl.slot_base + j) * kWave + lane] = make_float2(yr[j], yi[j]);
        }
    }
    simd_leave(peers, lane);
    // the last wave to finish advances the epoch for the next launch
    if (lane == 0) {
        const uint32_t total = gridDim.x * gridDim.y * kScanWaves;
        const uint32_t old =
            __hip_atomic_fetch_add(&queue->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == total - 1) {
            __hip_atomic_store(&queue->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue->epoch, epoch + 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Persistent variant.  The packet is cut into time tiles of `tile` samples and
// the work items are (detector, slice, tile), handed out in tile-major order
// (largest slices first inside a tile) by an atomic counter, one item per wave at
// a time, so every SIMD gets an equal share however uneven the slices are.  An
// item needs the state its slice reached at the end of the previous tile, which
// another wave, possibly on another XCD, produced: it is handed over as described
// above (coherent state accesses, a flag, a bounded wait).  Items are handed out in order, so the producer of any awaited item is
// already running and the wait ends; it is bounded all the same, and a wait that
// hits the bound is counted in ScanQueue::error.  Flags count tiles since the bank
// was created: a launch knows the count every slice reached before it (`epoch`),
// and the last wave to finish advances the epoch and rewinds the counters for the
// next launch (kernel boundaries order these with the next launch).
template <int MAXM>
__global__ __launch_bounds__(kWave) void scan_fp32_persistent_kernel(
    const float2 *__restrict__ ca, const float2 *__restrict__ cb, const int32_t *__restrict__ cd,
    float2 *__restrict__ state, const Slice *__restrict__ slices, const int32_t *__restrict__ order,
    int32_t n_slices, int32_t n_det, int64_t lanes_total, const float *__restrict__ x, int32_t n,
    const float *__restrict__ hist, int32_t hist_len, float2 *__restrict__ partial,
    int32_t part_stride, int32_t tile, ScanQueue *__restrict__ queue,
    uint32_t *__restrict__ flags, WaitBound wb, float2 *__restrict__ z, int32_t n_tmpl) {
    extern __shared__ float smem[];
    float *win = smem;
    const int lane = threadIdx.x;
    const int red_sample = reduce_sample(lane);
    const uint32_t per_round = (uint32_t)n_det * (uint32_t)n_slices;
    const uint32_t n_tiles = (uint32_t)((n + tile - 1) / tile);
    const uint32_t total = n_tiles * per_round;
    const uint32_t epoch = __hip_atomic_load(&queue->epoch, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        uint32_t item = 0;
        if (lane == 0)
            item = __hip_atomic_fetch_add(&queue->head, 1u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        const uint32_t tau = item / per_round;
        const int code = __builtin_amdgcn_readfirstlane(order[item % per_round]);
        const int det = code / n_slices;
        const int sidx = code % n_slices;
        Slice sl = slices[sidx];
        sl.tmpl = __builtin_amdgcn_readfirstlane(sl.tmpl);
        sl.slot_base = __builtin_amdgcn_readfirstlane(sl.slot_base);
        sl.n_slots = __builtin_amdgcn_readfirstlane(sl.n_slots);
        sl.single = __builtin_amdgcn_readfirstlane(sl.single);
        const int m = sl.n_slots;
        const int n0 = (int)tau * tile;
        const int T = min(tile, n - n0);

        // input window of this tile: history ring followed by the packet
        const float *xd = x + (int64_t)det * n;
        const float *hd = hist + (int64_t)det * hist_len;
        load_window(win, xd, hd, hist_len, n0, T, lane, kWave);

        float ar[MAXM], ai[MAXM], br[MAXM], bi[MAXM], yr[MAXM], yi[MAXM];
        int base[MAXM];
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
            if (j < m) {
                const int64_t g = (int64_t)(sl.slot_base + j) * kWave + lane;
                const float2 a = ca[g], b = cb[g];
                ar[j] = a.x; ai[j] = a.y; br[j] = b.x; bi[j] = b.y;
                base[j] = hist_len - cd[g];
            } else {
                ar[j] = ai[j] = br[j] = bi[j] = 0.0f;
                base[j] = 0;
            }
        }

        // wait until the previous tile of this (detector, slice) has published its state
        uint32_t *flag = flags + (int64_t)det * n_slices + sidx;
        const uint32_t target = epoch + tau;
        wait_flag(flag, target, lane, &queue->error, wb);
        float2 *st = state + (int64_t)det * lanes_total;
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
            if (j < m) {
                const float2 y = load_coherent(st + (int64_t)(sl.slot_base + j) * kWave + lane);
                yr[j] = y.x; yi[j] = y.y;
            } else {
                yr[j] = yi[j] = 0.0f;
            }
        }
        lds_fence();  // window stores visible to every lane of the wave
        float2 *pout = (sl.single && z != nullptr
                            ? z + ((int64_t)det * n_tmpl + sl.tmpl) * n
                            : partial + ((int64_t)det * n_slices + sidx) * part_stride) + n0;
        const int full = T & ~(kSub - 1);
        with_m<MAXM>(m, [&](auto mc) {
            constexpr int M = decltype(mc)::value;
            for (int s0 = 0; s0 < full; s0 += kSub)
                sub_tile_m<MAXM, M, false>(win, red_sample, lane, s0, kSub, ar, ai, br, bi, base,
                                           yr, yi, pout + s0);
        });
        if (full < T)
            sub_tile<MAXM, true>(win, red_sample, lane, m, full, T - full, ar, ai, br, bi, base, yr,
                                 yi, pout + full);
#pragma unroll
        for (int j = 0; j < MAXM; ++j)
            if (j < m)
                store_coherent(st + (int64_t)(sl.slot_base + j) * kWave + lane,
                               make_float2(yr[j], yi[j]));
        // publish: the state stores have completed before the flag moves
        wait_memory();
        if (lane == 0)
            __hip_atomic_store(flag, target + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lds_fence();  // every lane done with the window before the next item overwrites it
    }
    // the last wave to finish prepares the bookkeeping for the next launch
    if (lane == 0) {
        const uint32_t old = __hip_atomic_fetch_add(&queue->done, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            __hip_atomic_store(&queue->head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue->epoch, epoch + n_tiles, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

size_t scan_fp32_lds_bytes(int32_t tile, int32_t hist_len) {
    const int32_t win_floats = ((tile + hist_len + kSub) + 3) & ~3;
    return (size_t)win_floats * sizeof(float);
}

size_t scan_persistent_lds_bytes(int32_t tile, int32_t hist_len) {
    return scan_fp32_lds_bytes(tile, hist_len);
}

namespace {

hipError_t device_cus(int &cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    return hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
}

template <int MAXM>
hipError_t prepare_fpl(Bank &bk) {
    hipError_t e = hipFuncSetAttribute((const void *)scan_fp32_kernel<MAXM>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)scan_fp32_lds_bytes(bk.scan_tile, bk.hist_len));
    if (e != hipSuccess) return e;
    if (bk.balanced) {
        // the launch may pad its LDS request up to the whole LDS of a compute unit (so
        // that exactly the planned number of workgroups fits on each)
        const int lds = (int)scan_fp32_lds_bytes(bk.max_chunk, bk.hist_len);
        e = hipFuncSetAttribute((const void *)scan_fp32_balanced_kernel<MAXM>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsPerCu);
        if (e != hipSuccess) return e;
        int per_cu = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void *)scan_fp32_balanced_kernel<MAXM>, kWave * kScanWaves, lds);
        if (e != hipSuccess) return e;
        e = device_cus(cus);
        if (e != hipSuccess) return e;
        // planner inputs: waves per detector with one workgroup on every compute unit,
        // and the most workgroups per compute unit allowed
        bk.balance_unit = (int32_t)std::max<int64_t>(1, (int64_t)std::max(1, cus) / bk.n_det) *
                          kScanWaves;
        bk.balance_per_cu = std::max(1, std::min(bk.balance_per_cu, per_cu));
    }
    if (bk.time_tile <= 0) return hipSuccess;
    const int lds = (int)scan_persistent_lds_bytes(bk.time_tile, bk.hist_len);
    e = hipFuncSetAttribute((const void *)scan_fp32_persistent_kernel<MAXM>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, (const void *)scan_fp32_persistent_kernel<MAXM>, kWave, lds);
    if (e != hipSuccess) return e;
    e = device_cus(cus);
    if (e != hipSuccess) return e;
    bk.scan_waves = std::max(1, per_cu) * std::max(1, cus);
    return hipSuccess;
}

template <int MAXM>
void launch_fpl(const Bank &bk, const float *x, int32_t n, float2 *ckpt, float2 *z, float *peak,
                int32_t *argmax, hipStream_t s) {
    const int64_t lanes = bk.n_slots * kWave;
    if (bk.time_tile > 0 && ckpt == nullptr) {
        const int64_t items = (int64_t)((n + bk.time_tile - 1) / bk.time_tile) * bk.n_det *
                              bk.n_slices;
        const int grid = (int)std::min<int64_t>(bk.scan_waves, items);
        hipLaunchKernelGGL(scan_fp32_persistent_kernel<MAXM>, dim3(grid), dim3(kWave),
                           scan_persistent_lds_bytes(bk.time_tile, bk.hist_len), s, bk.d_a, bk.d_b,
                           bk.d_delay, bk.d_state, bk.d_slices, bk.d_order, bk.n_slices, bk.n_det,
                           lanes, x, n, bk.d_hist, bk.hist_len, bk.d_partial, bk.max_chunk,
                           bk.time_tile, bk.d_queue, bk.d_flags,
                           WaitBound{bk.wait_spins, bk.d_wait_flag}, z, bk.n_templates);
    } else if (bk.balanced) {
        const bool fuse = peak != nullptr && scan_fuses_singles(bk, n, ckpt != nullptr, true);
        const int32_t window = bk.peak_window > 0 ? bk.peak_window : n;
        const dim3 grid((unsigned)((bk.balance_waves + kScanWaves - 1) / kScanWaves), bk.n_det);
        hipLaunchKernelGGL(scan_fp32_balanced_kernel<MAXM>, grid, dim3(kWave * kScanWaves),
                           (size_t)bk.balance_lds, s, bk.d_a, bk.d_b, bk.d_delay,
                           bk.d_state, bk.d_slices, bk.n_slices, bk.d_segs, bk.d_seg_off,
                           bk.balance_waves, bk.n_splits, bk.d_split_flags, bk.d_bqueue, lanes, x,
                           n, bk.d_hist, bk.hist_len, bk.d_partial, bk.max_chunk, ckpt,
                           bk.ckpt_stride, (n + bk.ckpt_stride - 1) / bk.ckpt_stride,
                           bk.d_simd_tab, WaitBound{bk.wait_spins, bk.d_wait_flag}, z,
                           bk.n_templates,
                           FusedPeaks{fuse ? peak : nullptr, fuse ? argmax : nullptr,
                                      bk.d_split_cand, window, (n + window - 1) / window});
    } else {
        const int32_t tile = bk.scan_tile;
        const dim3 grid((bk.n_slices + kScanWaves - 1) / kScanWaves, bk.n_det);
        hipLaunchKernelGGL(scan_fp32_kernel<MAXM>, grid, dim3(kWave * kScanWaves),
                           scan_fp32_lds_bytes(tile, bk.hist_len), s, bk.d_a, bk.d_b, bk.d_delay,
                           bk.d_state, bk.d_slices, bk.d_slice_order, bk.n_slices, lanes, x, n, bk.d_hist,
                           bk.hist_len, bk.d_partial, bk.max_chunk, tile, ckpt,
                           bk.ckpt_stride, (n + bk.ckpt_stride - 1) / bk.ckpt_stride, z,
                           bk.n_templates);
    }
}

}  // namespace

// One filter per lane (groups of 64, the most waves for a small bank) runs the two-filter
// kernels, every group holding one slot.
hipError_t prepare_scan_fp32(Bank &bk) {
    switch (bk.fpl) {
    case 1:
    case 2: return prepare_fpl<2>(bk);
    case 4: return prepare_fpl<4>(bk);
    case 8: return prepare_fpl<8>(bk);
    default: return hipErrorInvalidValue;
    }
}

bool scan_fuses_singles(const Bank &bk, int32_t n, bool with_ckpt, bool with_peaks) {
    // the same choice of schedule as launch_fpl
    if (!bk.balanced || (bk.time_tile > 0 && !with_ckpt)) return false;
    if (!with_peaks) return true;
    const int32_t window = bk.peak_window > 0 ? bk.peak_window : n;
    return window >= n || window % kSub == 0;
}

hipError_t launch_scan_fp32(const Bank &bk, const float *x, int32_t n, float2 *ckpt, float2 *z,
                            float *peak, int32_t *argmax, hipStream_t s) {
    if (n <= 0 || bk.n_slices == 0) return hipSuccess;
    switch (bk.fpl) {
    case 1:
    case 2: launch_fpl<2>(bk, x, n, ckpt, z, peak, argmax, s); break;
    case 4: launch_fpl<4>(bk, x, n, ckpt, z, peak, argmax, s); break;
    case 8: launch_fpl<8>(bk, x, n, ckpt, z, peak, argmax, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace spiir
