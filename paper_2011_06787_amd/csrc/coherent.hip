// Coherent search over sky directions (Section II.C.1, Eq. llr_form; the null
// statistic of the appendix).
//
// For the candidate of detector I (template t, window w) at sample c, a time shift k
// and a sky direction p, detector J contributes v_J = z_J,t[s_J] with
//     s_J = c + tau[p][J] - tau[p][I] + shift[k][(J - I) mod N_d] - shift[k][0]
// (background shifts move the other detectors' series relative to the candidate's
// detector: column r of the shift table is the detector r places after it),
// the coherent SNR^2 is the power of v projected on the signal plane (the first two
// columns of the orthogonal U[p]):  rho_C^2 = sum_{i<2} |sum_J U[p][J][i] v_J|^2, and
// the null SNR^2 is the rest, rho_N^2 = sum_J |v_J|^2 - rho_C^2 (Eq. null_def).  Per
// (candidate, shift) the kernel keeps the direction with the largest rho_C^2 (lowest
// direction on ties).  One workgroup per candidate slot walks the shifts; its threads
// split the directions and meet in a wave-shuffle + LDS arg-max.  A (candidate,
// shift) whose samples leave [0, n) for any direction is marked NaN / -1.
// Per shift the workgroup first copies, for every detector J, the kStage samples of
// z_J centred on the shifted candidate sample into LDS; a direction whose relative
// delay tau[p][J] - tau[p][I] falls inside that window reads LDS, any other reads
// global memory.  A thread keeps the delays and signal-plane columns of its first
// kDirCache directions in registers across the shifts.
#include <cmath>

#include "internal.h"

namespace spiir {
namespace {

constexpr int kCohThreads = 256;
constexpr int kStage = 256;      // staged samples per detector and shift
constexpr int kDirCache = 4;     // directions per thread whose tables stay in registers

struct Best {
    float v;
    int32_t p;
};

__device__ __forceinline__ Best better(Best a, Best b) {
    return (b.v > a.v || (b.v == a.v && b.p < a.p)) ? b : a;
}

template <int ND>
struct Dir {
    int32_t rel[ND];     // tau[p][J] - tau[p][I]
    float u0[ND], u1[ND];
};

template <int ND>
__device__ __forceinline__ Dir<ND> load_dir(const int32_t *__restrict__ tau,
                                            const float *__restrict__ U, int p, int I) {
    Dir<ND> d;
    const int32_t *tp = tau + (int64_t)p * ND;
    const float *Up = U + (int64_t)p * ND * ND;
    const int tI = tp[I];
#pragma unroll
    for (int J = 0; J < ND; ++J) {
        d.rel[J] = tp[J] - tI;
        d.u0[J] = Up[J * ND + 0];
        d.u1[J] = Up[J * ND + 1];
    }
    return d;
}

template <int ND>
__global__ __launch_bounds__(kCohThreads) void coherent_kernel(
    const float2 *__restrict__ z, int32_t n_templates, int32_t n, const int32_t *__restrict__ index,
    int32_t n_win, const float *__restrict__ U, const int32_t *__restrict__ tau, int32_t n_pix,
    const int32_t *__restrict__ shifts, int32_t n_shift, float *__restrict__ snr2,
    int32_t *__restrict__ pix_out, float *__restrict__ null2) {
    __shared__ Best wbest[kCohThreads / kWave];
    __shared__ float wnull[kCohThreads / kWave];
    __shared__ int wbad[kCohThreads / kWave];
    __shared__ float2 stage[ND][kStage];
    const int64_t cand = blockIdx.x;   // (I, t, w)
    const int64_t row = cand / n_win;  // I * T + t
    const int t = (int)(row % n_templates);
    const int I = (int)(row / n_templates);
    const int c = index[cand];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (c < 0) {
        for (int k = threadIdx.x; k < n_shift; k += kCohThreads) {
            snr2[cand * n_shift + k] = __builtin_nanf("");
            null2[cand * n_shift + k] = __builtin_nanf("");
            pix_out[cand * n_shift + k] = -1;
        }
        return;
    }
    const float2 *zt[ND];
#pragma unroll
    for (int J = 0; J < ND; ++J) zt[J] = z + ((int64_t)J * n_templates + t) * n;
    Dir<ND> dc[kDirCache];
#pragma unroll
    for (int i = 0; i < kDirCache; ++i) {
        const int p = threadIdx.x + i * kCohThreads;
        if (p < n_pix) dc[i] = load_dir<ND>(tau, U, p, I);
    }
    for (int k = 0; k < n_shift; ++k) {
        int base[ND];
#pragma unroll
        for (int J = 0; J < ND; ++J) {
            const int r = J >= I ? J - I : J - I + ND;
            base[J] = c + shifts[k * ND + r] - shifts[k * ND];
        }
        for (int e = threadIdx.x; e < ND * kStage; e += kCohThreads) {
            const int J = e / kStage, o = e % kStage;
            const int s = base[J] + o - kStage / 2;
            stage[J][o] = (s >= 0 && s < n) ? zt[J][s] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        Best best{-1.0f, INT32_MAX};
        float best_null = 0.0f;
        int bad = 0;
        auto eval = [&](const Dir<ND> &d, int p) {
            float c0r = 0.f, c0i = 0.f, c1r = 0.f, c1i = 0.f, tot = 0.f;
            bool ok = true;
#pragma unroll
            for (int J = 0; J < ND; ++J) {
                const int s = base[J] + d.rel[J];
                const bool in = s >= 0 && s < n;
                ok = ok && in;
                const int o = d.rel[J] + kStage / 2;   // staged entries are zero outside [0, n)
                const float2 v = (o >= 0 && o < kStage) ? stage[J][o]
                                                        : (in ? zt[J][s] : make_float2(0.f, 0.f));
                c0r = fmaf(d.u0[J], v.x, c0r);
                c0i = fmaf(d.u0[J], v.y, c0i);
                c1r = fmaf(d.u1[J], v.x, c1r);
                c1i = fmaf(d.u1[J], v.y, c1i);
                tot = fmaf(v.x, v.x, fmaf(v.y, v.y, tot));
            }
            if (!ok) bad = 1;
            const float rc = c0r * c0r + c0i * c0i + c1r * c1r + c1i * c1i;
            const Best cur{rc, p};
            const Best nb = better(best, cur);
            if (nb.p == p) best_null = tot - rc;
            best = nb;
        };
#pragma unroll
        for (int i = 0; i < kDirCache; ++i) {
            const int p = threadIdx.x + i * kCohThreads;
            if (p < n_pix) eval(dc[i], p);
        }
        for (int p = threadIdx.x + kDirCache * kCohThreads; p < n_pix; p += kCohThreads)
            eval(load_dir<ND>(tau, U, p, I), p);
        // arg-max over the workgroup (carrying the null power of the winner)
        for (int off = kWave / 2; off >= 1; off >>= 1) {
            const Best o{__shfl_xor(best.v, off), __shfl_xor(best.p, off)};
            const float on = __shfl_xor(best_null, off);
            const int ob = __shfl_xor(bad, off);
            const Best nb = better(best, o);
            if (nb.p != best.p) best_null = on;
            best = nb;
            bad |= ob;
        }
        if (lane == 0) {
            wbest[wave] = best;
            wnull[wave] = best_null;
            wbad[wave] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            Best b = wbest[0];
            float nl = wnull[0];
            int bd = wbad[0];
            for (int w = 1; w < kCohThreads / kWave; ++w) {
                const Best nb = better(b, wbest[w]);
                if (nb.p != b.p) nl = wnull[w];
                b = nb;
                bd |= wbad[w];
            }
            const int64_t o = cand * n_shift + k;
            if (bd || b.p == INT32_MAX) {
                snr2[o] = __builtin_nanf("");
                null2[o] = __builtin_nanf("");
                pix_out[o] = -1;
            } else {
                snr2[o] = b.v;
                null2[o] = nl;
                pix_out[o] = b.p;
            }
        }
        __syncthreads();   // stage and wbest are rewritten by the next shift
    }
}

}  // namespace

hipError_t launch_coherent(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                           const int32_t *index, int32_t n_win, const float *U, const int32_t *tau,
                           int32_t n_pix, const int32_t *shifts, int32_t n_shift, float *snr2,
                           int32_t *pix, float *null2, hipStream_t s) {
    const int64_t cands = (int64_t)n_det * n_templates * n_win;
    if (cands <= 0 || n_shift <= 0) return hipSuccess;
    const dim3 grid((unsigned)cands), block(kCohThreads);
#define SPIIR_COH(ND)                                                                          \
    case ND:                                                                                   \
        hipLaunchKernelGGL(coherent_kernel<ND>, grid, block, 0, s, z, n_templates, n, index,   \
                           n_win, U, tau, n_pix, shifts, n_shift, snr2, pix, null2);            \
        break;
    switch (n_det) {
        SPIIR_COH(2)
        SPIIR_COH(3)
        SPIIR_COH(4)
        SPIIR_COH(5)
        SPIIR_COH(6)
        SPIIR_COH(7)
        SPIIR_COH(8)
    default: return hipErrorInvalidValue;
    }
#undef SPIIR_COH
    return hipGetLastError();
}

}  // namespace spiir
