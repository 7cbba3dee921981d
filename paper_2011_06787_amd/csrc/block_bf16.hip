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
//                            then the block-to-block carry (FP64 where |a| > 0.999,
//                            FP32 otherwise, a^L in FP64), writing Y as bf16 hi + lo
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

// One wave per (tile of 16 filters, detector): S for all blocks, 32 blocks per MFMA
// column tile, then the carry along the blocks by 16 lanes (one filter each).
__global__ __launch_bounds__(kWave) void block_state_kernel(
    const WTile *__restrict__ tiles, const BTemplate *__restrict__ tmpls,
    const uint16_t *__restrict__ wa, const uint16_t *__restrict__ xs, int64_t xs_stride,
    int32_t hist_pad, int32_t n_det, int32_t L, int32_t nb, int32_t nb_max,
    const double2 *__restrict__ aL, const int32_t *__restrict__ lp, double2 *__restrict__ state,
    int64_t n_fpad, uint16_t *__restrict__ yt, int64_t y_per_det) {
    __shared__ float sl[32][33];
    const int lane = threadIdx.x;
    const WTile tl = tiles[blockIdx.x];
    const int det = blockIdx.y;
    const BTemplate bt = tmpls[tl.tmpl];
    const uint16_t *xh = xs + (int64_t)det * xs_stride + hist_pad;
    const uint16_t *xl = xh + (int64_t)n_det * xs_stride;
    const int col = lane % 32;
    const int kg = (lane / 32) * 8;
    const uint16_t *ap = wa + tl.a_off + (lane % 32) * 16 + kg;

    // carried state and transition of this lane's filter (lanes 0..15)
    const int64_t gf = tl.g0 + (lane & 15);
    double2 y = make_double2(0.0, 0.0);
    double2 t = make_double2(0.0, 0.0);
    bool long_pole = false;
    if (lane < 16) {
        y = state[(int64_t)det * n_fpad + gf];
        t = aL[gf];
        long_pole = lp[gf] != 0;
    }
    uint16_t *yh = yt + (int64_t)det * y_per_det + bt.y_off;
    uint16_t *yl = yh + (int64_t)n_det * y_per_det;
    const int64_t row_len = 2 * (int64_t)bt.fpad;

    for (int c0 = 0; c0 < nb; c0 += 32) {
        const int b = c0 + col;
        const bool valid = b < nb;
        f32x16 acc = {};
        const int64_t pbase = (int64_t)b * L + tl.sigma_lo + kg;
        for (int ks = 0; ks < tl.nks; ++ks) {
            const bf16x8 ah = load8(ap + (int64_t)ks * 1024);
            const bf16x8 al = load8(ap + (int64_t)ks * 1024 + 512);
            bf16x8 bh = {}, bl = {};
            if (valid) {
                bh = load8(xh + pbase + 16 * ks);
                bl = load8(xl + pbase + 16 * ks);
            }
            acc = mma3(ah, al, bh, bl, acc);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) sl[8 * (i / 4) + 4 * (lane / 32) + (i % 4)][col] = acc[i];
        __syncthreads();
        if (lane < 16) {
            const int cmax = min(32, nb - c0);
            for (int cc = 0; cc < cmax; ++cc) {
                const int bb = c0 + cc;
                // state entering block bb, split into bf16 hi + lo
                const float yr = (float)y.x, yi = (float)y.y;
                const __hip_bfloat16 hr = __float2bfloat16(yr), hi_ = __float2bfloat16(yi);
                const __hip_bfloat16 lr = __float2bfloat16(yr - __bfloat162float(hr));
                const __hip_bfloat16 li = __float2bfloat16(yi - __bfloat162float(hi_));
                const int64_t o = (int64_t)bb * row_len + 2 * (int64_t)(tl.f0 + lane);
                yh[o] = bf16_bits(hr);
                yh[o + 1] = bf16_bits(hi_);
                yl[o] = bf16_bits(lr);
                yl[o + 1] = bf16_bits(li);
                const float sr = sl[2 * lane][cc], si = sl[2 * lane + 1][cc];
                if (long_pole) {
                    const double nr = t.x * y.x - t.y * y.y + (double)sr;
                    const double ni = t.x * y.y + t.y * y.x + (double)si;
                    y = make_double2(nr, ni);
                } else {
                    const float tr = (float)t.x, ti = (float)t.y;
                    const float nr = fmaf(tr, yr, fmaf(-ti, yi, sr));
                    const float ni = fmaf(tr, yi, fmaf(ti, yr, si));
                    y = make_double2((double)nr, (double)ni);
                }
            }
        }
        __syncthreads();
    }
    if (lane < 16) state[(int64_t)det * n_fpad + gf] = y;
    (void)nb_max;
}

// One workgroup of (2L/64) waves per (template, 64 columns); a column is
// (detector, block).  Wave w computes output rows [64w, 64w+64) x the 64 columns.
__global__ __launch_bounds__(512) void block_output_kernel(
    const BTemplate *__restrict__ tmpls, const uint16_t *__restrict__ pa,
    const uint16_t *__restrict__ yt, int64_t y_per_det, const uint16_t *__restrict__ xs,
    int64_t xs_stride, int32_t hist_pad, int32_t n_det, int32_t L, int32_t nb, int32_t n,
    int32_t n_templates, float *__restrict__ z) {
    const int t = blockIdx.x;
    const BTemplate bt = tmpls[t];
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int rt_per = (2 * L) / 32;             // row tiles of the template
    const int kg = (lane / 32) * 8;
    const int ncols = n_det * nb;
    int det[2], blk[2];
    bool valid[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const int c = blockIdx.y * 64 + ct * 32 + (lane % 32);
        valid[ct] = c < ncols;
        const int cc = valid[ct] ? c : 0;
        det[ct] = cc / nb;
        blk[ct] = cc % nb;
    }
    f32x16 acc[2][2] = {};
    const int64_t row_len = 2 * (int64_t)bt.fpad;
    // state part: K = 2*fpad state entries
    for (int ks = 0; ks < bt.nks_p; ++ks) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint16_t *p = pa + bt.a_off +
                                ((int64_t)ks * rt_per + 2 * wave + r) * 1024 + (lane % 32) * 16 + kg;
            ah[r] = load8(p);
            al[r] = load8(p + 512);
        }
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const uint16_t *q = yt + (int64_t)det[ct] * y_per_det + bt.y_off +
                                (int64_t)blk[ct] * row_len + 16 * ks + kg;
            bh[ct] = load8(q);
            bl[ct] = load8(q + (int64_t)n_det * y_per_det);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) acc[r][ct] = mma3(ah[r], al[r], bh[ct], bl[ct], acc[r][ct]);
    }
    // input part: K = offsets sigma in [sigma_lo, L)
    for (int ks = 0; ks < bt.nks_m; ++ks) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint16_t *p = pa + bt.a_off +
                                ((int64_t)(bt.nks_p + ks) * rt_per + 2 * wave + r) * 1024 +
                                (lane % 32) * 16 + kg;
            ah[r] = load8(p);
            al[r] = load8(p + 512);
        }
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const uint16_t *q = xs + (int64_t)det[ct] * xs_stride + hist_pad +
                                (int64_t)blk[ct] * L + bt.sigma_lo + 16 * ks + kg;
            bh[ct] = load8(q);
            bl[ct] = load8(q + (int64_t)n_det * xs_stride);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) acc[r][ct] = mma3(ah[r], al[r], bh[ct], bl[ct], acc[r][ct]);
    }
    // rows (2j + re/im): accumulator entries 4q..4q+3 are (j0 re, j0 im, j0+1 re, j0+1 im)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        if (!valid[ct]) continue;
        float *zr = z + 2 * (((int64_t)det[ct] * n_templates + t) * n + (int64_t)blk[ct] * L);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 64 * wave + 32 * r + 8 * q + 4 * (lane / 32);
                const int j0 = row / 2;
                float4 v = make_float4(acc[r][ct][4 * q], acc[r][ct][4 * q + 1],
                                       acc[r][ct][4 * q + 2], acc[r][ct][4 * q + 3]);
                *reinterpret_cast<float4 *>(zr + 2 * j0) = v;
            }
        }
    }
}

}  // namespace

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
    if (bk.n_wtiles > 0)
        hipLaunchKernelGGL(block_state_kernel, dim3(bk.n_wtiles, bk.n_det), dim3(kWave), 0, s,
                           bk.d_wtiles, bk.d_btmpl, bk.d_wa, bk.d_xs, bk.xs_stride, bk.hist_pad,
                           bk.n_det, L, nb, bk.max_chunk / L, bk.d_aL, bk.d_lp, bk.d_state64,
                           bk.n_fpad, bk.d_yt, bk.y_per_det);
    const int ncols = bk.n_det * nb;
    const dim3 grid(bk.n_templates, (ncols + 63) / 64);
    hipLaunchKernelGGL(block_output_kernel, grid, dim3((2 * L / 64) * kWave), 0, s, bk.d_btmpl,
                       bk.d_pa, bk.d_yt, bk.y_per_det, bk.d_xs, bk.xs_stride, bk.hist_pad, bk.n_det,
                       L, nb, n, bk.n_templates, reinterpret_cast<float *>(z));
    return hipGetLastError();
}

}  // namespace spiir
