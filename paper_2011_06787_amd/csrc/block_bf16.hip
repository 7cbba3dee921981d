// Time-blocked form of the SPIIR filter bank on the matrix cores (split bf16).
//
// For a block of L samples starting at n0 = bL, the per-filter recurrence of
// Eq. zk (Section II.B.1) unrolls exactly into
//     y_k[n0+j] = a_k^{j+1} y_k[n0-1] + sum_{i<=j} b_k a_k^{j-i} x[n0+i-d_k]
// so, with Y_k[b] = y_k[bL-1] the state entering block b,
//     Y_k[b+1] = a_k^L Y_k[b] + S_k[b],   S_k[b] = sum_{i<L} b_k a_k^{L-1-i} x[bL+i-d_k]
//     z_t[bL+j] = sum_k a_k^{j+1} Y_k[b] + sum_{sigma} M_t[j,sigma] x[bL+sigma]
// with M_t[j,sigma] = sum_{k in t, 0<=sigma+d_k<=j} b_k a_k^{j-sigma-d_k}.  Over all blocks
// these are matrix products against the Hankel view H[sigma][b] = x[bL+sigma] of the
// input, which every filter and template shares:
//   kernel 1 (split_input)   x -> bf16 hi + lo planes (x = hi + lo to ~2^-17)
//   kernel 2 (block_state)   S = W'.H per 16 delay-sorted filters of a template (the
//                            operand W' holds b a^{L-1-i} on the band sigma = i - d_k),
//                            then the block-to-block carry (FP64 for tiles holding a
//                            filter with |a| > 0.999, FP32 otherwise, a^L in FP64),
//                            writing Y as bf16 hi + lo
//   kernel 3 (block_output)  z_t = [P_t | M_t] [Y_t ; H], P_t[j,k] = a_k^{j+1}
// Every product runs as hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation.  Complex operands use the real 2x2 block form; output rows are
// (j, re/im) interleaved so that four accumulator rows are one 16-byte complex pair.
#include <hip/hip_bf16.h>

#include "internal.h"

namespace spiir {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    return *reinterpret_cast<const bf16x8 *>(p);
}

__device__ __forceinline__ f32x16 mma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, f32x16 c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
    return c;
}

__device__ __forceinline__ uint16_t bf16_bits(__hip_bfloat16 v) {
    return __builtin_bit_cast(uint16_t, v);
}

// x (with history) -> xs[plane][det][hist_pad + p], p in [-hist_pad, n + 16)
__global__ void split_input_kernel(const float *__restrict__ x, int32_t n,
                                   const float *__restrict__ hist, int32_t hist_len,
                                   int32_t hist_pad, uint16_t *__restrict__ xs, int64_t xs_stride,
                                   int32_t n_det) {
    const int det = blockIdx.y;
    const int64_t plane = (int64_t)n_det * xs_stride;
    uint16_t *hi = xs + (int64_t)det * xs_stride;
    uint16_t *lo = hi + plane;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < xs_stride;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i - hist_pad;
        float v = 0.0f;
        if (p >= 0 && p < n) v = x[(int64_t)det * n + p];
        else if (p < 0 && p >= -hist_len) v = hist[(int64_t)det * hist_len + hist_len + p];
        const __hip_bfloat16 h = __float2bfloat16(v);
        const __hip_bfloat16 l = __float2bfloat16(v - __bfloat162float(h));
        hi[i] = bf16_bits(h);
        lo[i] = bf16_bits(l);
    }
}

// Block-to-block carry of one chunk of kChunk blocks for the lane's filter f and its
// group q of kChunk/4 consecutive blocks:  Y[b+1] = A Y[b] + S[b]  (A = a^L).
// A two-level scan in two passes: every lane runs its group from a zero state for the
// group's total, the four group totals are combined through LDS (Ystart[q+1] = A^len
// Ystart[q] + T[q]), and each lane then runs its group again from Ystart[q], writing the
// state entering every block as bf16 hi + lo (running the group twice keeps no
// per-block state in registers).  R is double for tiles with a long-pole filter, float
// otherwise.
// AG = A^kGroup (precomputed per filter).
constexpr int kChunk = 64;
constexpr int kGroup = kChunk / 4;

template <typename R>
struct C2 {
    R r, i;
};

template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
    return C2<R>{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}

template <typename R>
__device__ __forceinline__ C2<R> cfma(C2<R> a, C2<R> b, C2<R> c) {   // a*b + c
    return C2<R>{a.r * b.r - a.i * b.i + c.r, a.r * b.i + a.i * b.r + c.i};
}

__device__ __forceinline__ uint32_t pack_bf16(float lo_half, float hi_half) {
    return (uint32_t)bf16_bits(__float2bfloat16(lo_half)) |
           ((uint32_t)bf16_bits(__float2bfloat16(hi_half)) << 16);
}

// write Y (state entering block) as hi and lo planes: (re, im) pairs as 32-bit stores
__device__ __forceinline__ void store_split(uint32_t *yh, uint32_t *yl, float yr, float yi) {
    const float hr = __bfloat162float(__float2bfloat16(yr));
    const float hi = __bfloat162float(__float2bfloat16(yi));
    *yh = pack_bf16(yr, yi);
    *yl = pack_bf16(yr - hr, yi - hi);
}

template <typename R>
__device__ __forceinline__ void carry_chunk(const float (*sl)[kChunk + 1], C2<R> (*tot)[16],
                                            int f, int q, int valid_cols, C2<R> A, C2<R> AG,
                                            C2<R> &y_prev, uint32_t *yh, uint32_t *yl,
                                            int64_t row_len2, int64_t col0) {
    // pass 1: the group's total from a zero state
    const int c_lo = q * kGroup;
    const int len = max(0, min(kGroup, valid_cols - c_lo));
    C2<R> y{0, 0};
    for (int c = 0; c < len; ++c) {
        const C2<R> sv{(R)sl[2 * f][c_lo + c], (R)sl[2 * f + 1][c_lo + c]};
        y = cfma(A, y, sv);
    }
    tot[q][f] = y;
    // sl and tot belong to this wave alone and the four lanes of a filter take the same
    // branch, so a wave-level LDS ordering fence (no barrier) is enough here
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    // combine the group totals: state entering each group, and the chunk's exit state
    C2<R> ystart = y_prev, ynext = y_prev;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int lq = max(0, min(kGroup, valid_cols - qq * kGroup));
        C2<R> p = AG;                                  // A^kGroup for a full group
        if (lq < kGroup) {
            p = C2<R>{1, 0};
            for (int k = 0; k < lq; ++k) p = cmul(p, A);   // A^lq (last chunk only)
        }
        if (qq == q) ystart = ynext;
        ynext = cfma(p, ynext, tot[qq][f]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    y_prev = ynext;
    // pass 2: the states entering the group's blocks, from the group's true start
    y = ystart;
    for (int c = 0; c < len; ++c) {
        const int64_t o = (col0 + c_lo + c) * row_len2;
        store_split(yh + o, yl + o, (float)y.r, (float)y.i);
        const C2<R> sv{(R)sl[2 * f][c_lo + c], (R)sl[2 * f + 1][c_lo + c]};
        y = cfma(A, y, sv);
    }
}

// s_waitcnt with vmcnt = N and lgkmcnt = 0 (gfx9 encoding: vmcnt in bits 3:0 and
// 15:14, expcnt 6:4 left at its maximum, lgkmcnt 11:8)
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// 16-byte LDS read at byte address `addr` (+ imm); the result is tied to an
// explicit lgkmcnt wait by the caller
template <int OFF>
__device__ __forceinline__ bf16x8 lds_read16(uint32_t addr) {
    bf16x8 v;
    asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "i"(OFF));
    return v;
}

// LDS (address space 3) pointer to element `elem` of `smem`, and its byte address
__device__ __forceinline__ __attribute__((address_space(3))) void *lds_elem(uint16_t *smem, int elem) {
    return (__attribute__((address_space(3))) void *)(
        (__attribute__((address_space(3))) uint16_t *)smem + elem);
}

// direct global-to-LDS load of 16 bytes per lane: lane i's bytes from `src` land at
// element `elem` of `smem` (wave-uniform) + 16 x i bytes
__device__ __forceinline__ void lds_dma16(const void *src, uint16_t *smem, int elem) {
    __builtin_amdgcn_global_load_lds(src, lds_elem(smem, elem), 16, 0, 0);
}

__device__ __forceinline__ uint32_t lds_byte_addr(uint16_t *smem) {
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint16_t *)smem;
}

// One workgroup of kStateWaves waves per kStateWaves consecutive tiles; wave w owns
// tile blockIdx.x*kStateWaves + w (16 filters) for every detector in turn.  The
// tile's W' fragments of its first kACache K steps are loaded into registers once and
// serve every chunk of every detector; further steps (a tile of the precision bank has
// 11-16 at L = 128) are read again from memory for every chunk.  For every chunk of
// kChunk blocks the workgroup stages the input range all its tiles read,
//     x[c0 L + P_lo, (c0 + kChunk - 1) L + P_hi)     (P_lo, P_hi: union band of the tiles)
// once into LDS (hi and lo planes), skewed by 8 elements per row of L so that the
// 16-byte fragments of consecutive blocks (columns) start 4 banks apart; the MFMA B
// fragments are then LDS reads instead of strided global reads.  Each wave computes S
// for its tile (two 32-column MFMA tiles sharing each A fragment).  After a barrier the
// same LDS holds the waves' S rows for the carry, so the footprint is the larger of the
// two uses and several workgroups share a CU.
constexpr int kStateWaves = 4;
constexpr int kSlFloats = 32 * (kChunk + 1);   // one wave's S rows
// W' K steps kept in registers: with the two-pass carry, 8 of them fit the 168-register
// budget of three waves per SIMD (4: 11.72-11.76 ms per precision pass, 8: 11.54-11.63)
constexpr int kACache = 8;

__device__ __forceinline__ int skew(int p, int L) { return p + 8 * (p / L); }

__global__ __launch_bounds__(kWave *kStateWaves) __attribute__((amdgpu_waves_per_eu(3)))
void block_state_kernel(
    const WTile *__restrict__ tiles, int32_t n_tiles, const BTemplate *__restrict__ tmpls,
    const uint16_t *__restrict__ wa, const uint16_t *__restrict__ xs, int64_t xs_stride,
    int32_t hist_pad, int32_t n_det, int32_t L, int32_t nb, const double2 *__restrict__ aL,
    const int32_t *__restrict__ lp, double2 *__restrict__ state, int64_t n_fpad,
    uint16_t *__restrict__ yt, int64_t y_per_det, int32_t xwin) {
    extern __shared__ __attribute__((aligned(16))) uint16_t lds[];   // staged input / S rows
    __shared__ C2<double> tot64[kStateWaves][4][16];
    __shared__ C2<float> tot32[kStateWaves][4][16];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int tile0 = blockIdx.x * kStateWaves;
    const int tile_id = tile0 + wave;
    const bool active = tile_id < n_tiles;
    WTile tl = tiles[active ? tile_id : tile0];
    tl.nks = __builtin_amdgcn_readfirstlane(tl.nks);
    const BTemplate bt = tmpls[tl.tmpl];
    // union band of the workgroup's tiles (multiples of 16)
    int p_lo = 1 << 30, p_hi = -(1 << 30);
    for (int id = tile0; id < min(n_tiles, tile0 + kStateWaves); ++id) {
        const WTile tw = tiles[id];
        p_lo = min(p_lo, tw.sigma_lo);
        p_hi = max(p_hi, tw.sigma_lo + 16 * tw.nks);
    }
    uint16_t *sh = lds;
    uint16_t *slo = lds + xwin;
    float(*sl)[kChunk + 1] =
        reinterpret_cast<float(*)[kChunk + 1]>(reinterpret_cast<float *>(lds) + wave * kSlFloats);
    const int col = lane % 32;
    const int kg = (lane / 32) * 8;
    const uint16_t *ap = wa + tl.a_off + (lane % 32) * 16 + kg;
    bf16x8 ach[kACache], acl[kACache];
#pragma unroll
    for (int ks = 0; ks < kACache; ++ks) {
        if (active && ks < tl.nks) {
            ach[ks] = load8(ap + (int64_t)ks * 1024);
            acl[ks] = load8(ap + (int64_t)ks * 1024 + 512);
        } else {
            ach[ks] = bf16x8{};
            acl[ks] = bf16x8{};
        }
    }

    const int f = lane & 15;
    const int q = lane >> 4;
    const int64_t gf = tl.g0 + f;
    const double2 ta = active ? aL[gf] : make_double2(0.0, 0.0);
    // The carry's precision is chosen per tile, for the whole wave: FP64 when any of the
    // tile's 16 filters has |a| above the long-pole threshold.  A per-filter choice made
    // every wave holding both kinds run both carries and both sets of state stores.
    const bool long_pole = __builtin_amdgcn_ballot_w64(active && lp[gf] != 0) != 0;
    const C2<double> A64{ta.x, ta.y};
    const C2<float> A32{(float)ta.x, (float)ta.y};
    C2<double> AG64{1.0, 0.0};
    for (int k = 0; k < kGroup; ++k) AG64 = cmul(AG64, A64);
    C2<float> AG32{1.0f, 0.0f};
    for (int k = 0; k < kGroup; ++k) AG32 = cmul(AG32, A32);
    const int64_t row_len2 = bt.fpad;

    for (int det = 0; det < n_det; ++det) {
        const uint16_t *xh = xs + (int64_t)det * xs_stride + hist_pad;
        const uint16_t *xl = xh + (int64_t)n_det * xs_stride;
        const double2 ys = active ? state[(int64_t)det * n_fpad + gf] : make_double2(0.0, 0.0);
        C2<double> y64{ys.x, ys.y};
        C2<float> y32{(float)ys.x, (float)ys.y};
        uint32_t *yh =
            reinterpret_cast<uint32_t *>(yt + (int64_t)det * y_per_det + bt.y_off) + tl.f0 + f;
        uint32_t *yl = reinterpret_cast<uint32_t *>(yt + (int64_t)(n_det + det) * y_per_det +
                                                    bt.y_off) + tl.f0 + f;
        for (int c0 = 0; c0 < nb; c0 += kChunk) {
            const int cols = min(kChunk, nb - c0);
            const int span = (cols - 1) * L + (p_hi - p_lo);   // multiple of 16
            const int64_t g0 = (int64_t)c0 * L + p_lo;
            __syncthreads();   // previous chunk's S rows no longer read
            {
                // 16-byte unit u of the range goes to slot u + u / R of its plane (R units
                // per row of L, then the skew's one-unit gap); the slots are filled by
                // direct global-to-LDS loads, 64 consecutive slots per instruction, all in
                // flight together.  A gap slot takes a copy of its row's last unit (an
                // in-range address) and is never read.
                const int R = L / 8;
                const int U = span / 8;
                const int slots = U + (U - 1) / R;
                const int n_ins = (slots + kWave - 1) / kWave;
                for (int k = wave; k < 2 * n_ins; k += kStateWaves) {
                    const int plane = k >= n_ins;
                    const int s0 = (k - plane * n_ins) * kWave;
                    const int sl_ = s0 + lane;
                    const int row = sl_ / (R + 1), w = sl_ % (R + 1);
                    const int u = row * R + min(w, R - 1);
                    if (sl_ < slots)
                        lds_dma16((plane ? xl : xh) + g0 + 8 * u, plane ? slo : sh, 8 * s0);
                }
                wait_vm_lgkm0<0>();
            }
            __syncthreads();
            f32x16 acc[2] = {};
            if (active) {
                bool valid[2];
                int rel[2];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    const int b = ct * 32 + col;
                    valid[ct] = b < cols;
                    rel[ct] = (valid[ct] ? b : 0) * L + tl.sigma_lo - p_lo + kg;
                }
                auto step = [&](int ks, const bf16x8 &ah, const bf16x8 &al) {
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct) {
                        bf16x8 bh = {}, bl = {};
                        if (valid[ct]) {
                            const int o = skew(rel[ct] + 16 * ks, L);
                            bh = *reinterpret_cast<const bf16x8 *>(sh + o);
                            bl = *reinterpret_cast<const bf16x8 *>(slo + o);
                        }
                        acc[ct] = mma3(ah, al, bh, bl, acc[ct]);
                    }
                };
#pragma unroll
                for (int ks = 0; ks < kACache; ++ks)
                    if (ks < tl.nks) step(ks, ach[ks], acl[ks]);
                for (int ks = kACache; ks < tl.nks; ++ks) {
                    const bf16x8 ah = load8(ap + (int64_t)ks * 1024);
                    const bf16x8 al = load8(ap + (int64_t)ks * 1024 + 512);
                    step(ks, ah, al);
                }
            }
            __syncthreads();   // staged input no longer read: the LDS now holds S rows
            if (active) {
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        sl[8 * (i / 4) + 4 * (lane / 32) + (i % 4)][ct * 32 + col] = acc[ct][i];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                if (long_pole)
                    carry_chunk<double>(sl, tot64[wave], f, q, cols, A64, AG64, y64, yh, yl,
                                        row_len2, c0);
                else
                    carry_chunk<float>(sl, tot32[wave], f, q, cols, A32, AG32, y32, yh, yl,
                                       row_len2, c0);
            }
        }
        if (active && q == 0)
            state[(int64_t)det * n_fpad + gf] =
                long_pole ? make_double2(y64.r, y64.i) : make_double2((double)y32.r, (double)y32.i);
    }
}

// Output product, one workgroup of RW x CH waves per (template, CH x 128 columns),
// RW = 2L/64; a column is (detector, block).  Wave (r, h) computes output rows
// [64r, 64r+64) x columns [128h, 128h+128) of the tile: 2 x 4 accumulator tiles of
// 32x32.  Per K step of 16 both operands are copied into LDS by direct
// global-to-LDS loads (each lane's 16 bytes land at the instruction's LDS base + 16
// x lane), shared by the waves that need them: the B operand (CH x 128 columns x 16
// entries, hi and lo: CH x 8 KB) and the A rows (RW x 2 row tiles, hi and lo: RW x
// 4 KB); every A byte serves CH x 128 columns.  The loads run three steps ahead in
// a ring of kStages buffers: with fewer steps of matrix-core work in front of them,
// their latency (the block states come from HBM) set the kernel's time.  The fragments are read from LDS with
// explicit waits: the compiler, which cannot tell the ring's stages apart, would
// otherwise wait for every load in flight before each read.
// LDS layout of a stage: A [row tile][plane][32 rows x 16 k] as in global memory,
// then B [plane][column][k half] x 16 bytes; either way the fragment reads of a
// wave cover 1 KB contiguously, without bank conflicts.
// Workgroups are dispatched round-robin over the XCDs (id % kXcds); the mapping
// gives every column tile of a template to the same XCD, one after the other, so
// the template's operand is fetched into that XCD's L2 once.
constexpr int kXcds = 8;
constexpr int kOutCols = 128;   // columns per wave
constexpr int kStages = 4;
constexpr int kALoads = 4;      // 1-KB direct loads of A per row wave per stage

// column waves per workgroup for RW row waves (at most 8 waves per workgroup)
__host__ __device__ constexpr int out_col_waves(int rw) { return rw <= 4 ? 2 : 1; }

__host__ __device__ constexpr int out_stage_elems(int rw) {
    return 2 * rw * 1024 + 2 * 2 * out_col_waves(rw) * kOutCols * 8;
}

size_t block_output_lds_bytes(int rw) { return (size_t)kStages * out_stage_elems(rw) * sizeof(uint16_t); }

// wait for every LDS read of the step, which the MFMAs reading the fragments cannot be
// moved above
__device__ __forceinline__ void wait_frags(bf16x8 &a0, bf16x8 &a1, bf16x8 &a2, bf16x8 &a3,
                                           bf16x8 &b0, bf16x8 &b1, bf16x8 &b2, bf16x8 &b3,
                                           bf16x8 &b4, bf16x8 &b5, bf16x8 &b6, bf16x8 &b7) {
    asm volatile("s_waitcnt lgkmcnt(0)"
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(b0), "+v"(b1), "+v"(b2),
                   "+v"(b3), "+v"(b4), "+v"(b5), "+v"(b6), "+v"(b7));
}

template <int RW>
__global__ __launch_bounds__(RW * out_col_waves(RW) * kWave) void block_output_kernel(
    const BTemplate *__restrict__ tmpls, const uint16_t *__restrict__ pa,
    const uint16_t *__restrict__ yt, int64_t y_per_det, const uint16_t *__restrict__ xs,
    int64_t xs_stride, int32_t hist_pad, int32_t n_det, int32_t L, int32_t nb, int32_t n,
    int32_t n_templates, float *__restrict__ z, int32_t n_col_tiles, int32_t ksplit,
    float *__restrict__ zpart) {
    constexpr int CH = out_col_waves(RW);
    constexpr int kWaves = RW * CH;
    constexpr int kCols = CH * kOutCols;                // columns of the workgroup's tile
    constexpr int kBLoadsWg = 2 * 2 * kCols / kWave;    // 1-KB direct loads of B per stage
    constexpr int kALoadsWg = kALoads * RW;             // and of A
    static_assert(kBLoadsWg % kWaves == 0 && kALoadsWg % kWaves == 0,
                  "every wave issues the same number of loads");
    constexpr int kMyLoads = (kBLoadsWg + kALoadsWg) / kWaves;   // per wave per stage
    constexpr int kStageElems = out_stage_elems(RW);
    extern __shared__ __attribute__((aligned(16))) uint16_t smem_out[];
    const int wg = blockIdx.x;
    const int xcd = wg % kXcds;
    const int seq = wg / kXcds;
    const int units = n_col_tiles * ksplit;   // (column tile, K part) pairs per template
    const int t = (seq / units) * kXcds + xcd;
    const int col_tile = (seq % units) / ksplit;
    const int kpart = (seq % units) % ksplit;
    if (t >= n_templates) return;
    const BTemplate bt = tmpls[t];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int rw = wave % RW, ch = wave / RW;   // row wave, column wave
    const int rt_per = 2 * RW;
    const int kg = (lane / 32) * 8;
    const int ncols = n_det * nb;
    const int64_t row_len = 2 * (int64_t)bt.fpad;
    // this workgroup's K steps: part kpart of the template's, in order
    const int nks_all = bt.nks_p + bt.nks_m;
    const int k_lo = (int)((int64_t)kpart * nks_all / ksplit);
    const int nks = (int)((int64_t)(kpart + 1) * nks_all / ksplit) - k_lo;
    const uint32_t ring = lds_byte_addr(smem_out);

    // global source of the B entries of step ks for column c (8 entries of one plane)
    auto b_src = [&](int ks, int c, int plane, int half) -> const uint16_t * {
        const int cc = min(col_tile * kCols + c, ncols - 1);
        const int det = cc / nb, blk = cc % nb;
        if (ks < bt.nks_p)
            return yt + (int64_t)plane * n_det * y_per_det + (int64_t)det * y_per_det + bt.y_off +
                   (int64_t)blk * row_len + 16 * ks + 8 * half;
        return xs + (int64_t)plane * n_det * xs_stride + (int64_t)det * xs_stride + hist_pad +
               (int64_t)blk * L + bt.sigma_lo + 16 * (ks - bt.nks_p) + 8 * half;
    };
    // this wave's share of the direct loads of step ks into stage ks % kStages: A
    // loads q = wave, wave + kWaves, ... (1 KB each, the step's A rows being
    // contiguous), B loads likewise, each covering items 64q..64q+63 with item
    // e = (plane * kCols + column) * 2 + half: the two halves of a column's 32
    // contiguous bytes go to neighbouring lanes, one cache-line request for both
    auto issue = [&](int ks) {
        const int st = (ks % kStages) * kStageElems;
        const int kstep = k_lo + ks;   // the template's K step
        const uint16_t *asrc = pa + bt.a_off + (int64_t)kstep * rt_per * 1024 + lane * 8;
#pragma unroll
        for (int i = 0; i < kALoadsWg / kWaves; ++i) {
            const int q = wave + i * kWaves;
            lds_dma16(asrc + q * 512, smem_out, st + q * 512);
        }
#pragma unroll
        for (int i = 0; i < kBLoadsWg / kWaves; ++i) {
            const int q = wave + i * kWaves;
            const int e = q * kWave + lane;
            const int c = (e >> 1) % kCols, plane = (e >> 1) / kCols;
            lds_dma16(b_src(kstep, c, plane, e & 1), smem_out, st + 2 * RW * 1024 + q * kWave * 8);
        }
    };

    f32x16 acc[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[r][ct] = f32x16{};

    // byte offsets of this lane's fragments within a stage
    const uint32_t a_frag = (uint32_t)((2 * rw * 1024 + (lane % 32) * 16 + kg) * 2);
    const uint32_t b_frag =
        (uint32_t)((2 * RW * 1024 + ((ch * kOutCols + (lane % 32)) * 2 + kg / 8) * 8) * 2);
    constexpr int kPl = 2 * kCols * 8 * 2;   // bytes from plane 0 to plane 1 of B
#pragma unroll
    for (int i = 0; i < kStages - 1; ++i)
        if (i < nks) issue(i);
    for (int ks = 0; ks < nks; ++ks) {
        // this step's operands have landed once at most the later steps' loads are in
        // flight; after the barrier every wave's part is visible, and the stage read
        // in the previous step (every wave is past its reads) is free for step
        // ks + kStages - 1
        static_assert(kStages == 4, "the waits below assume two later steps in flight");
        const int later = min(nks - 1 - ks, kStages - 2);
        if (later >= 2) wait_vm_lgkm0<2 * kMyLoads>();
        else if (later == 1) wait_vm_lgkm0<kMyLoads>();
        else wait_vm_lgkm0<0>();
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (ks + kStages - 1 < nks) issue(ks + kStages - 1);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t base = ring + (uint32_t)((ks % kStages) * kStageElems * 2);
        const uint32_t pa_ = base + a_frag, pb = base + b_frag;
        bf16x8 ah0 = lds_read16<0>(pa_), al0 = lds_read16<1024>(pa_);
        bf16x8 ah1 = lds_read16<2048>(pa_), al1 = lds_read16<3072>(pa_);
        // B: plane 1 kPl bytes after plane 0; accumulator column tile ct at +32 x 32 x ct
        bf16x8 bh0 = lds_read16<0>(pb), bl0 = lds_read16<kPl>(pb);
        bf16x8 bh1 = lds_read16<1024>(pb), bl1 = lds_read16<kPl + 1024>(pb);
        bf16x8 bh2 = lds_read16<2048>(pb), bl2 = lds_read16<kPl + 2048>(pb);
        bf16x8 bh3 = lds_read16<3072>(pb), bl3 = lds_read16<kPl + 3072>(pb);
        // one wait for all twelve reads: waiting for the first fragments only, and
        // starting on them, measured no faster
        wait_frags(ah0, al0, ah1, al1, bh0, bl0, bh1, bl1, bh2, bl2, bh3, bl3);
        acc[0][0] = mma3(ah0, al0, bh0, bl0, acc[0][0]);
        acc[1][0] = mma3(ah1, al1, bh0, bl0, acc[1][0]);
        acc[0][1] = mma3(ah0, al0, bh1, bl1, acc[0][1]);
        acc[1][1] = mma3(ah1, al1, bh1, bl1, acc[1][1]);
        acc[0][2] = mma3(ah0, al0, bh2, bl2, acc[0][2]);
        acc[1][2] = mma3(ah1, al1, bh2, bl2, acc[1][2]);
        acc[0][3] = mma3(ah0, al0, bh3, bl3, acc[0][3]);
        acc[1][3] = mma3(ah1, al1, bh3, bl3, acc[1][3]);
    }
    // rows (2j + re/im): accumulator entries 4q..4q+3 are (j0 re, j0 im, j0+1 re, j0+1 im)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int c = col_tile * kCols + ch * kOutCols + ct * 32 + (lane % 32);
        if (c >= ncols) continue;
        const int det = c / nb, blk = c % nb;
        // a split K writes its part's partial sums, added in order by block_ksum_kernel
        float *zt = ksplit > 1 ? zpart + (int64_t)kpart * 2 * n_det * n_templates * n : z;
        float *zr = zt + 2 * (((int64_t)det * n_templates + t) * n + (int64_t)blk * L);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 64 * rw + 32 * r + 8 * q + 4 * (lane / 32);
                const int j0 = row / 2;
                const float4 v = make_float4(acc[r][ct][4 * q], acc[r][ct][4 * q + 1],
                                             acc[r][ct][4 * q + 2], acc[r][ct][4 * q + 3]);
                *reinterpret_cast<float4 *>(zr + 2 * j0) = v;
            }
        }
    }
}

// z = sum over the K parts of their partial outputs, in part order (deterministic)
__global__ void block_ksum_kernel(const float4 *__restrict__ zpart, int64_t count, int32_t ksplit,
                                  float4 *__restrict__ z) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        float4 v = zpart[i];
        for (int p = 1; p < ksplit; ++p) {
            const float4 w = zpart[(int64_t)p * count + i];
            v.x += w.x;
            v.y += w.y;
            v.z += w.z;
            v.w += w.w;
        }
        z[i] = v;
    }
}

}  // namespace

// LDS elements per plane of the staged input of block_state_kernel: the widest union
// band of a workgroup's tiles plus kChunk-1 blocks, skewed (8 per L elements).
int32_t block_state_xwin(const Bank &bk) {
    const int L = bk.block_len;
    const int span = (kChunk - 1) * L + bk.max_wg_band;
    return (int32_t)((span + 8 * (span / L + 1) + 15) / 16 * 16);
}

// Workgroups sharing one output tile's K steps: when the (template, column tile) pairs of a
// packet of max_chunk samples are fewer than the compute units, the K steps of each are cut
// into parts (at least 8 steps each, at most 32 parts) whose partial outputs are summed by a
// second launch; otherwise 1.
int32_t block_output_ksplit(const Bank &bk, int32_t min_k_steps) {
    const int rw = 2 * bk.block_len / 64;
    const int64_t ncols = (int64_t)bk.n_det * (bk.max_chunk / bk.block_len);
    const int64_t cols_wg = (int64_t)out_col_waves(rw) * kOutCols;
    const int64_t wgs = std::max<int64_t>(1, (int64_t)bk.n_templates * ((ncols + cols_wg - 1) / cols_wg));
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 256;
    }
    int64_t ks = std::min<int64_t>(cus / wgs, min_k_steps / 8);
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(ks, 32));
}

// dynamic LDS of block_state_kernel: the staged input and, reusing it, the S rows
size_t block_state_lds_bytes(const Bank &bk) {
    return std::max<size_t>((size_t)2 * block_state_xwin(bk) * sizeof(uint16_t),
                            (size_t)kStateWaves * kSlFloats * sizeof(float));
}

hipError_t prepare_block_bf16(const Bank &bk) {
    hipError_t e = hipFuncSetAttribute((const void *)block_state_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)block_state_lds_bytes(bk));
    if (e != hipSuccess) return e;
    const void *out[3] = {(const void *)block_output_kernel<2>, (const void *)block_output_kernel<4>,
                          (const void *)block_output_kernel<8>};
    const int rw[3] = {2, 4, 8};
    for (int k = 0; k < 3; ++k) {
        e = hipFuncSetAttribute(out[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)block_output_lds_bytes(rw[k]));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_block_bf16(const Bank &bk, const float *x, int32_t n, float2 *z, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int L = bk.block_len;
    const int nb = n / L;
    {
        const int64_t blocks = (bk.xs_stride + 255) / 256;
        hipLaunchKernelGGL(split_input_kernel, dim3((unsigned)std::min<int64_t>(blocks, 1024), bk.n_det),
                           dim3(256), 0, s, x, n, bk.d_hist, bk.hist_len, bk.hist_pad, bk.d_xs,
                           bk.xs_stride, bk.n_det);
    }
    if (bk.n_wtiles > 0) {
        const int32_t xwin = block_state_xwin(bk);
        hipLaunchKernelGGL(block_state_kernel,
                           dim3((bk.n_wtiles + kStateWaves - 1) / kStateWaves),
                           dim3(kWave * kStateWaves), block_state_lds_bytes(bk), s,
                           bk.d_wtiles, bk.n_wtiles, bk.d_btmpl, bk.d_wa, bk.d_xs, bk.xs_stride,
                           bk.hist_pad, bk.n_det, L, nb, bk.d_aL, bk.d_lp, bk.d_state64, bk.n_fpad,
                           bk.d_yt, bk.y_per_det, xwin);
    }
    const int ncols = bk.n_det * nb;
    const int64_t groups = (bk.n_templates + kXcds - 1) / kXcds;
    const int32_t ksplit = bk.d_zpart != nullptr ? bk.out_ksplit : 1;
#define SPIIR_BLOCK_OUT(RW)                                                                   \
    const int col_tiles = (ncols + out_col_waves(RW) * kOutCols - 1) / (out_col_waves(RW) * kOutCols); \
    const dim3 grid((unsigned)(groups * kXcds * col_tiles * ksplit));                         \
    hipLaunchKernelGGL(block_output_kernel<RW>, grid, dim3(RW * out_col_waves(RW) * kWave),      \
                       block_output_lds_bytes(RW), s, bk.d_btmpl,                                \
                       bk.d_pa, bk.d_yt, bk.y_per_det, bk.d_xs, bk.xs_stride, bk.hist_pad,       \
                       bk.n_det, L, nb, n, bk.n_templates, reinterpret_cast<float *>(z),         \
                       col_tiles, ksplit, reinterpret_cast<float *>(bk.d_zpart))
    switch (2 * L / 64) {
    case 2: { SPIIR_BLOCK_OUT(2); break; }
    case 4: { SPIIR_BLOCK_OUT(4); break; }
    case 8: { SPIIR_BLOCK_OUT(8); break; }
    default: return hipErrorInvalidValue;
    }
#undef SPIIR_BLOCK_OUT
    if (ksplit > 1) {
        const int64_t count = (int64_t)bk.n_det * bk.n_templates * n / 2;   // float4 per part
        const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
        hipLaunchKernelGGL(block_ksum_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256),
                           0, s, reinterpret_cast<const float4 *>(bk.d_zpart), count, ksplit,
                           reinterpret_cast<float4 *>(z));
    }
    return hipGetLastError();
}

}  // namespace spiir
