// Reverse-time adjoint of the SPIIR filter bank, for fitting a_k, b_k to a loss on
// the template outputs (the overlap of Eq. overlap, Section II.B.1, in practice).
//
// With g_t[n] = dL/dRe z_t[n] + i dL/dIm z_t[n] and the per-filter recurrence
// y_k[n] = a_k y_k[n-1] + b_k x[n-d_k] (Eq. zk read per filter), the adjoint state
//     lambda_k[n] = g_t[n] + conj(a_k) lambda_k[n+1]          (lambda_k[N] = 0)
// gives  dL/da_k = sum_n lambda_k[n] conj(y_k[n-1]),  dL/db_k = sum_n lambda_k[n] x[n-d_k]
// (complex gradients as dL/dRe + i dL/dIm).
//
// Work decomposition: one workgroup per FP32-scan slice with one wave per slot,
// one filter per lane.  The waves share the LDS input window of the current
// checkpoint segment.  The forward states are never stored per sample: segments
// are visited last to first from the checkpoint taken by the forward pass; inside a
// segment a forward sweep keeps the state at the start of every level-1 block
// (LDS), each block is re-swept keeping the state at every 16-sample sub-block
// (registers), and each sub-block is recomputed into registers and walked backward.
//
// Segments in parallel (signals of several checkpoint segments): the adjoint is a
// linear recurrence, so inside segment s = [b, e] it splits as
//     lambda[n] = lambda_s[n] + conj(a)^(e+1-n) Lambda_s,   Lambda_s = lambda[e+1],
// lambda_s being the same recurrence started from zero at e.  Every (slice, detector,
// segment) workgroup then walks its segment independently and returns
//     GA_s = sum lambda_s[n] conj(y[n-1]),   EA_s = sum conj(a)^(e+1-n) conj(y[n-1]),
//     GB_s = sum lambda_s[n] x[n-d],         EB_s = sum conj(a)^(e+1-n) x[n-d],
//     L0_s = lambda_s[b],                    W_s  = conj(a)^(e+1-b),
// and a per-filter pass joins them from the last segment down:
//     grad_a += GA_s + Lambda_s EA_s,  grad_b += GB_s + Lambda_s EB_s,
//     Lambda_{s-1} = L0_s + W_s Lambda_s   (Lambda of the last segment = 0).
#include <algorithm>

#include "internal.h"

namespace spiir {
namespace {

// Level-1 block (states in LDS): 128 samples, or 256 for checkpoint strides of 2048 and
// more, where the LDS of 128-sample block states would leave three workgroups per
// compute unit (differentiation workload: backward 1.26 -> 1.13 ms; at a stride of 512
// the longer blocks' extra registers cost more than they save).
__host__ __device__ constexpr int adj_block(int32_t stride) { return stride >= 2048 ? 256 : 128; }
constexpr int kAdjSub = 16;           // level-2 sub-block (states in registers)

struct Cx {
    float r, i;
};

__device__ __forceinline__ Cx step(Cx y, float ar, float ai, float br, float bi, float xv) {
    return Cx{fmaf(ar, y.r, fmaf(-ai, y.i, br * xv)), fmaf(ar, y.i, fmaf(ai, y.r, bi * xv))};
}

// SPLIT = false: one workgroup per slice walks every detector and segment in turn
// and writes the gradients.  SPLIT = true: one workgroup per (slice, segment,
// detector) = (blockIdx.x, blockIdx.y, blockIdx.z) writes its six partial sums to
// `part` ([det][seg][6][lanes]) for join_kernel.
template <bool SPLIT, int BLK>
__global__ __launch_bounds__(512) void backward_kernel(
    const float2 *__restrict__ ca, const float2 *__restrict__ cb, const int32_t *__restrict__ cd,
    const int32_t *__restrict__ perm, const Slice *__restrict__ slices, int64_t lanes_total,
    const float *__restrict__ x, int32_t n, int32_t n_det, int32_t hist_len,
    const float2 *__restrict__ gz, int32_t n_templates, const float2 *__restrict__ ckpt,
    int32_t stride, int32_t n_seg, float2 *__restrict__ grad_a, float2 *__restrict__ grad_b,
    int32_t win_floats, float2 *__restrict__ part) {
    extern __shared__ float smem[];
    float *win = smem;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    constexpr int kSubs = BLK / kAdjSub;
    const int nblk_max = (stride + BLK - 1) / BLK;
    float2 *c1 = reinterpret_cast<float2 *>(smem + win_floats) + (int64_t)wave * nblk_max * kWave;
    const Slice sl = slices[blockIdx.x];
    const bool active = wave < sl.n_slots;
    const int64_t g = (int64_t)(sl.slot_base + (active ? wave : 0)) * kWave + lane;
    float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
    int d = 0;
    if (active) {
        const float2 a = ca[g], b = cb[g];
        ar = a.x; ai = a.y; br = b.x; bi = b.y;
        d = cd[g];
    }
    const int base = hist_len - d;   // window index of x[seg_start - d]
    float gar = 0.f, gai = 0.f, gbr = 0.f, gbi = 0.f;

    const int det_lo = SPLIT ? (int)blockIdx.z : 0, det_hi = SPLIT ? det_lo + 1 : n_det;
    for (int det = det_lo; det < det_hi; ++det) {
        const float *xd = x + (int64_t)det * n;
        const float2 *gt = gz + ((int64_t)det * n_templates + sl.tmpl) * n;
        float lr = 0.f, li = 0.f;   // lambda_k[n+1]
        const int seg_hi = SPLIT ? (int)blockIdx.y : n_seg - 1;
        const int seg_lo = SPLIT ? (int)blockIdx.y : 0;
        for (int seg = seg_hi; seg >= seg_lo; --seg) {
            // SPLIT: lambda restarts from zero at the segment end; w = conj(a)^(e+1-n)
            float wr = 1.f, wi = 0.f, ear = 0.f, eai = 0.f, ebr = 0.f, ebi = 0.f;
            if (SPLIT) {
                lr = 0.f;
                li = 0.f;
                gar = gai = gbr = gbi = 0.f;
            }
            const int s0 = seg * stride;
            const int len = min(stride, n - s0);
            __syncthreads();   // previous window no longer read
            for (int i = threadIdx.x; i < len + hist_len; i += blockDim.x) {
                const int pos = s0 - hist_len + i;
                win[i] = pos >= 0 ? xd[pos] : 0.0f;   // zero history: the signal starts at 0
            }
            __syncthreads();
            if (!active) continue;
            // level 1: states entering each BLK-sample block of the segment
            const float2 y0 = ckpt[((int64_t)det * n_seg + seg) * lanes_total + g];
            Cx y{y0.x, y0.y};
            const int nblk = (len + BLK - 1) / BLK;
            for (int blk = 0; blk < nblk; ++blk) {
                c1[blk * kWave + lane] = make_float2(y.r, y.i);
                const int e = min(BLK, len - blk * BLK);
                const float *xp = win + base + blk * BLK;
                for (int i = 0; i < e; ++i) y = step(y, ar, ai, br, bi, xp[i]);
            }
            for (int blk = nblk - 1; blk >= 0; --blk) {
                const int b0 = blk * BLK;
                const int e = min(BLK, len - b0);
                const int nsub = (e + kAdjSub - 1) / kAdjSub;
                // level 2: states entering each 16-sample sub-block of the block
                Cx c2[kSubs];
                {
                    const float2 cb1 = c1[blk * kWave + lane];
                    Cx yy{cb1.x, cb1.y};
#pragma unroll
                    for (int sb = 0; sb < kSubs; ++sb) {
                        c2[sb] = yy;
                        if (sb < nsub) {
                            const int f = min(kAdjSub, e - sb * kAdjSub);
                            const float *xp = win + base + b0 + sb * kAdjSub;
                            for (int i = 0; i < f; ++i) yy = step(yy, ar, ai, br, bi, xp[i]);
                        }
                    }
                }
#pragma unroll
                for (int sb = kSubs - 1; sb >= 0; --sb) {
                    if (sb >= nsub) continue;
                    const int f = min(kAdjSub, e - sb * kAdjSub);
                    const int q0 = b0 + sb * kAdjSub;   // segment offset of the sub-block
                    const float *xp = win + base + q0;
                    Cx ys[kAdjSub];
                    Cx yy = c2[sb];
#pragma unroll
                    for (int i = 0; i < kAdjSub; ++i) {
                        if (i < f) yy = step(yy, ar, ai, br, bi, xp[i]);
                        ys[i] = yy;
                    }
#pragma unroll
                    for (int i = kAdjSub - 1; i >= 0; --i) {
                        if (i >= f) continue;
                        const float2 gv = gt[s0 + q0 + i];
                        // lambda <- g + conj(a) lambda
                        const float nlr = gv.x + fmaf(ar, lr, ai * li);
                        const float nli = gv.y + fmaf(ar, li, -ai * lr);
                        lr = nlr;
                        li = nli;
                        const Cx yp = i > 0 ? ys[i - 1] : c2[sb];
                        // grad_a += lambda conj(y[n-1]); grad_b += lambda x[n-d]
                        gar = fmaf(lr, yp.r, fmaf(li, yp.i, gar));
                        gai = fmaf(li, yp.r, fmaf(-lr, yp.i, gai));
                        const float xv = xp[i];
                        gbr = fmaf(lr, xv, gbr);
                        gbi = fmaf(li, xv, gbi);
                        if (SPLIT) {
                            // w <- w conj(a); EA += w conj(y[n-1]); EB += w x[n-d]
                            const float nwr = fmaf(wr, ar, wi * ai);
                            const float nwi = fmaf(wi, ar, -wr * ai);
                            wr = nwr;
                            wi = nwi;
                            ear = fmaf(wr, yp.r, fmaf(wi, yp.i, ear));
                            eai = fmaf(wi, yp.r, fmaf(-wr, yp.i, eai));
                            ebr = fmaf(wr, xv, ebr);
                            ebi = fmaf(wi, xv, ebi);
                        }
                    }
                }
            }
            if (SPLIT) {
                float2 *pp = part + ((int64_t)det * n_seg + seg) * 6 * lanes_total + g;
                pp[0 * lanes_total] = make_float2(gar, gai);
                pp[1 * lanes_total] = make_float2(gbr, gbi);
                pp[2 * lanes_total] = make_float2(ear, eai);
                pp[3 * lanes_total] = make_float2(ebr, ebi);
                pp[4 * lanes_total] = make_float2(lr, li);
                pp[5 * lanes_total] = make_float2(wr, wi);
            }
        }
    }
    if (SPLIT) return;
    if (active) {
        const int32_t k = perm[g];
        if (k >= 0) {
            grad_a[k] = make_float2(gar, gai);
            grad_b[k] = make_float2(gbr, gbi);
        }
    }
}

__global__ void set_coeffs_kernel(const int32_t *__restrict__ perm, const float2 *__restrict__ a,
                                  const float2 *__restrict__ b, float2 *__restrict__ ca,
                                  float2 *__restrict__ cb, int64_t lanes) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < lanes;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = perm[i];
        if (k >= 0) {
            ca[i] = a[k];
            cb[i] = b[k];
        }
    }
}

// Joins the segments' partial sums of every filter (see the header): one thread per
// lane of the scan layout, detectors summed, gradients written through perm.
__global__ void join_kernel(const float2 *__restrict__ part, const int32_t *__restrict__ perm,
                            int64_t lanes, int32_t n_det, int32_t n_seg,
                            float2 *__restrict__ grad_a, float2 *__restrict__ grad_b) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < lanes;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = perm[g];
        if (k < 0) continue;
        float gar = 0.f, gai = 0.f, gbr = 0.f, gbi = 0.f;
        for (int det = 0; det < n_det; ++det) {
            float Lr = 0.f, Li = 0.f;   // Lambda of the segment
            for (int seg = n_seg - 1; seg >= 0; --seg) {
                const float2 *pp = part + ((int64_t)det * n_seg + seg) * 6 * lanes + g;
                const float2 ga = pp[0], gb = pp[lanes], ea = pp[2 * lanes], eb = pp[3 * lanes];
                const float2 l0 = pp[4 * lanes], w = pp[5 * lanes];
                gar += ga.x + (Lr * ea.x - Li * ea.y);
                gai += ga.y + (Lr * ea.y + Li * ea.x);
                gbr += gb.x + (Lr * eb.x - Li * eb.y);
                gbi += gb.y + (Lr * eb.y + Li * eb.x);
                const float nr = l0.x + (w.x * Lr - w.y * Li);
                const float ni = l0.y + (w.x * Li + w.y * Lr);
                Lr = nr;
                Li = ni;
            }
        }
        grad_a[k] = make_float2(gar, gai);
        grad_b[k] = make_float2(gbr, gbi);
    }
}

}  // namespace

size_t backward_lds_bytes(int32_t stride, int32_t hist_len, int32_t fpl) {
    const int32_t win_floats = ((stride + hist_len + kSub) + 3) & ~3;
    return (size_t)win_floats * sizeof(float) +
           (size_t)fpl * ((stride + adj_block(stride) - 1) / adj_block(stride)) * kWave *
               sizeof(float2);
}

hipError_t prepare_backward(const Bank &bk) {
    const int lds = (int)backward_lds_bytes(bk.ckpt_stride, bk.hist_len, bk.fpl);
    const bool longb = adj_block(bk.ckpt_stride) == 256;
    hipError_t e = hipFuncSetAttribute(longb ? (const void *)backward_kernel<false, 256>
                                             : (const void *)backward_kernel<false, 128>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(longb ? (const void *)backward_kernel<true, 256>
                                     : (const void *)backward_kernel<true, 128>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

namespace {

template <int BLK>
void launch_backward_blk(const Bank &bk, const float *x, int32_t n, const float2 *gz,
                         const float2 *ckpt, float2 *grad_a, float2 *grad_b, int32_t n_seg,
                         int32_t win_floats, int64_t lanes, size_t lds, hipStream_t s) {
    if (n_seg > 1 && bk.d_bwd_part != nullptr && n_seg <= bk.bwd_max_seg) {
        hipLaunchKernelGGL((backward_kernel<true, BLK>), dim3(bk.n_slices, n_seg, bk.n_det),
                           dim3(kWave * bk.fpl), lds, s, bk.d_a, bk.d_b, bk.d_delay, bk.d_perm,
                           bk.d_slices, lanes, x, n, bk.n_det, bk.hist_len, gz, bk.n_templates, ckpt,
                           bk.ckpt_stride, n_seg, grad_a, grad_b, win_floats, bk.d_bwd_part);
        const int64_t blocks = std::min<int64_t>((lanes + 255) / 256, 8192);
        hipLaunchKernelGGL(join_kernel, dim3((unsigned)blocks), dim3(256), 0, s, bk.d_bwd_part,
                           bk.d_perm, lanes, bk.n_det, n_seg, grad_a, grad_b);
    } else {
        hipLaunchKernelGGL((backward_kernel<false, BLK>), dim3(bk.n_slices), dim3(kWave * bk.fpl),
                           lds, s, bk.d_a, bk.d_b, bk.d_delay, bk.d_perm, bk.d_slices, lanes, x,
                           n, bk.n_det, bk.hist_len, gz, bk.n_templates, ckpt, bk.ckpt_stride,
                           n_seg, grad_a, grad_b, win_floats, nullptr);
    }
}

}  // namespace

hipError_t launch_backward(const Bank &bk, const float *x, int32_t n, const float2 *gz,
                           const float2 *ckpt, float2 *grad_a, float2 *grad_b, hipStream_t s) {
    // every filter sits in exactly one lane of one slice: all gradients are written
    if (n <= 0 || bk.n_slices == 0) return hipSuccess;
    const int32_t n_seg = (n + bk.ckpt_stride - 1) / bk.ckpt_stride;
    const int32_t win_floats = ((bk.ckpt_stride + bk.hist_len + kSub) + 3) & ~3;
    const int64_t lanes = bk.n_slots * kWave;
    const size_t lds = backward_lds_bytes(bk.ckpt_stride, bk.hist_len, bk.fpl);
    if (adj_block(bk.ckpt_stride) == 256)
        launch_backward_blk<256>(bk, x, n, gz, ckpt, grad_a, grad_b, n_seg, win_floats, lanes, lds, s);
    else
        launch_backward_blk<128>(bk, x, n, gz, ckpt, grad_a, grad_b, n_seg, win_floats, lanes, lds, s);
    return hipGetLastError();
}

hipError_t launch_set_coeffs(const Bank &bk, const float2 *a, const float2 *b, hipStream_t s) {
    const int64_t lanes = bk.n_slots * kWave;
    if (lanes == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((lanes + 255) / 256, 4096);
    hipLaunchKernelGGL(set_coeffs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, bk.d_perm, a, b,
                       bk.d_a, bk.d_b, lanes);
    return hipGetLastError();
}

}  // namespace spiir
