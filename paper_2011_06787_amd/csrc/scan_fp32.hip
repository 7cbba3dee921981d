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
// then reduced through a padded LDS transpose (each lane sums 16 rows of one
// sample) and two cross-half shuffles, and 16 lanes write the slice's partial
// template sum for the sub-tile.  A second kernel adds the slices of each template.
//
// Arithmetic per filter-sample: 2 mul + 4 fma (complex a*y + b*x with real x)
// and 2 adds into the lane sum: 8 VALU lane-operations for the paper's 12 flops.
#include "internal.h"

namespace spiir {
namespace {

constexpr int kRedStride = kSub + 1;  // float2 per lane row, padded against bank conflicts
static_assert(kSub == 16, "the lane reduction assumes 4 quarters of 16 lanes");

__device__ __forceinline__ void lds_fence() {
    // orders this wave's LDS writes before its later LDS reads (and vice versa)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

template <int MAXM, bool TAIL>
__device__ __forceinline__ void sub_tile(const float *__restrict__ win, float2 *__restrict__ red,
                                         int lane, int m, int s0, int valid,
                                         const float (&ar)[MAXM], const float (&ai)[MAXM],
                                         const float (&br)[MAXM], const float (&bi)[MAXM],
                                         const int (&base)[MAXM], float (&yr)[MAXM],
                                         float (&yi)[MAXM], float2 *__restrict__ out) {
    float accr[kSub], acci[kSub];
#pragma unroll
    for (int s = 0; s < kSub; ++s) {
        accr[s] = 0.0f;
        acci[s] = 0.0f;
    }
#pragma unroll
    for (int j = 0; j < MAXM; ++j) {
        if (j < m) {  // wave-uniform
            const float *xp = win + base[j] + s0;
            float r = yr[j], im = yi[j];
#pragma unroll
            for (int s = 0; s < kSub; ++s) {
                if (!TAIL || s < valid) {
                    const float xv = xp[s];
                    const float nr = fmaf(ar[j], r, fmaf(-ai[j], im, br[j] * xv));
                    const float ni = fmaf(ar[j], im, fmaf(ai[j], r, bi[j] * xv));
                    r = nr;
                    im = ni;
                    accr[s] += r;
                    acci[s] += im;
                }
            }
            yr[j] = r;
            yi[j] = im;
        }
    }
    // lane -> sample transpose: row `lane` holds this lane's kSub partial sums
#pragma unroll
    for (int s = 0; s < kSub; ++s) red[lane * kRedStride + s] = make_float2(accr[s], acci[s]);
    lds_fence();
    const int q = lane >> 4;     // quarter of the wave: rows 16q .. 16q+15
    const int s = lane & 15;     // sample of the sub-tile this lane reduces
    float vr = 0.0f, vi = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float2 v = red[(q * 16 + i) * kRedStride + s];
        vr += v.x;
        vi += v.y;
    }
    lds_fence();
    vr += __shfl_xor(vr, 16);
    vi += __shfl_xor(vi, 16);
    vr += __shfl_xor(vr, 32);
    vi += __shfl_xor(vi, 32);
    if (lane < kSub && (!TAIL || lane < valid)) out[lane] = make_float2(vr, vi);
}

template <int MAXM>
__global__ __launch_bounds__(kWave *kScanWaves) void scan_fp32_kernel(
    const float2 *__restrict__ ca, const float2 *__restrict__ cb, const int32_t *__restrict__ cd,
    float2 *__restrict__ state, const Slice *__restrict__ slices, int32_t n_slices,
    int64_t lanes_total, const float *__restrict__ x, int32_t n, const float *__restrict__ hist,
    int32_t hist_len, float2 *__restrict__ partial, int32_t part_stride, int32_t tile_len,
    int32_t win_floats) {
    extern __shared__ float smem[];
    float *win = smem;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    float2 *red = reinterpret_cast<float2 *>(smem + win_floats) + wave * kWave * kRedStride;
    const int det = blockIdx.y;
    const int sidx = blockIdx.x * kScanWaves + wave;
    const bool active = sidx < n_slices;
    const Slice sl = active ? slices[sidx] : Slice{0, 0, 0, 0};
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
    float2 *pout = partial + ((int64_t)det * n_slices + sidx) * part_stride;

    for (int n0 = 0; n0 < n; n0 += tile_len) {
        const int T = min(tile_len, n - n0);
        __syncthreads();  // every wave is done with the previous window
        for (int i = threadIdx.x; i < T + hist_len; i += blockDim.x) {
            const int pos = n0 - hist_len + i;
            win[i] = pos >= 0 ? xd[pos] : hd[hist_len + pos];
        }
        __syncthreads();
        if (!active) continue;
        int s0 = 0;
        for (; s0 + kSub <= T; s0 += kSub)
            sub_tile<MAXM, false>(win, red, lane, m, s0, kSub, ar, ai, br, bi, base, yr, yi,
                                  pout + n0 + s0);
        if (s0 < T)
            sub_tile<MAXM, true>(win, red, lane, m, s0, T - s0, ar, ai, br, bi, base, yr, yi,
                                 pout + n0 + s0);
    }
    if (active) {
#pragma unroll
        for (int j = 0; j < MAXM; ++j)
            if (j < m) st[(int64_t)(sl.slot_base + j) * kWave + lane] = make_float2(yr[j], yi[j]);
    }
}

}  // namespace

size_t scan_fp32_lds_bytes(int32_t tile, int32_t hist_len) {
    const int32_t win_floats = ((tile + hist_len + kSub) + 3) & ~3;
    return (size_t)win_floats * sizeof(float) +
           (size_t)kScanWaves * kWave * kRedStride * sizeof(float2);
}

hipError_t prepare_scan_fp32(const Bank &bk) {
    // allow the dynamic LDS this bank's window needs (above the 64 KiB default)
    const int lds = (int)scan_fp32_lds_bytes(bk.scan_tile, bk.hist_len);
    hipError_t e = hipSuccess;
    switch (bk.fpl) {
    case 2: e = hipFuncSetAttribute((const void *)scan_fp32_kernel<2>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
    case 4: e = hipFuncSetAttribute((const void *)scan_fp32_kernel<4>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
    case 8: e = hipFuncSetAttribute((const void *)scan_fp32_kernel<8>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
    default: e = hipErrorInvalidValue;
    }
    return e;
}

hipError_t launch_scan_fp32(const Bank &bk, const float *x, int32_t n, hipStream_t s) {
    if (n <= 0 || bk.n_slices == 0) return hipSuccess;
    const int32_t tile = bk.scan_tile;
    const int32_t win_floats = ((tile + bk.hist_len + kSub) + 3) & ~3;
    const size_t lds = scan_fp32_lds_bytes(tile, bk.hist_len);
    const dim3 grid((bk.n_slices + kScanWaves - 1) / kScanWaves, bk.n_det);
    const dim3 block(kWave * kScanWaves);
    const int64_t lanes = bk.n_slots * kWave;
    switch (bk.fpl) {
    case 2:
        hipLaunchKernelGGL(scan_fp32_kernel<2>, grid, block, lds, s, bk.d_a, bk.d_b, bk.d_delay,
                           bk.d_state, bk.d_slices, bk.n_slices, lanes, x, n, bk.d_hist,
                           bk.hist_len, bk.d_partial, bk.max_chunk, tile, win_floats);
        break;
    case 4:
        hipLaunchKernelGGL(scan_fp32_kernel<4>, grid, block, lds, s, bk.d_a, bk.d_b, bk.d_delay,
                           bk.d_state, bk.d_slices, bk.n_slices, lanes, x, n, bk.d_hist,
                           bk.hist_len, bk.d_partial, bk.max_chunk, tile, win_floats);
        break;
    case 8:
        hipLaunchKernelGGL(scan_fp32_kernel<8>, grid, block, lds, s, bk.d_a, bk.d_b, bk.d_delay,
                           bk.d_state, bk.d_slices, bk.n_slices, lanes, x, n, bk.d_hist,
                           bk.hist_len, bk.d_partial, bk.max_chunk, tile, win_floats);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace spiir
