// Signal-consistency statistic (Section II.C.1).
//
// autocorr: the correlation of a template with itself, R_t[j] = sum_m u_t[m+j]
// conj(u_t[m]) for lags j = 0..nj, where u_t is the template's response to a unit
// impulse (u_t[m] = sum_k b_k a_k^(m-d_k) for m >= d_k).  For every pair of filters
// (k, l) of the template the sum over m is geometric:
//     b_k conj(b_l) / (1 - a_k conj(a_l)) * a_k^e          e = d_l + j - d_k >= 0
//     b_k conj(b_l) / (1 - a_k conj(a_l)) * conj(a_l)^-e   e < 0
// so R_t costs F_t^2 terms per lag, in FP64.  One workgroup per (template, block of
// kLagBlock lags); each thread owns filters k and walks all l; along the lags of the
// block the power is advanced by one multiplication per lag: upward (times a_k) from
// the first lag with e >= 0, downward (times conj(a_l), walking the lags backwards)
// below it.  Per-thread partial sums are reduced with wave shuffles and one LDS pass.
//
// xi2: at a candidate sample c of row (detector, template),
//     xi^2 = sum_{j=-nj..nj} |v[c+j] - v[c] A[j]|^2 / sum_{j=-nj..nj} (2 - 2|A[j]|^2),
// A[j] = R[j] / R[0] (A[-j] = conj(A[j])), v = z sqrt(2 / R[0]) (unit variance per
// quadrature for unit white input).  One wave per candidate, FP64 sums.
#include <cmath>

#include "internal.h"

namespace spiir {
namespace {

constexpr int kLagBlock = 16;
constexpr int kAcThreads = 256;

struct Cd {
    double r, i;
};

__device__ __forceinline__ Cd cmul(Cd a, Cd b) { return Cd{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

__device__ __forceinline__ Cd cpow(Cd a, int e) {   // e >= 0, repeated squaring
    Cd r{1.0, 0.0};
    for (; e > 0; e >>= 1) {
        if (e & 1) r = cmul(r, a);
        a = cmul(a, a);
    }
    return r;
}

__global__ __launch_bounds__(kAcThreads) void autocorr_kernel(const int32_t *__restrict__ offsets,
                                                              const float2 *__restrict__ ca,
                                                              const float2 *__restrict__ cb,
                                                              const int32_t *__restrict__ cd,
                                                              int32_t nj, double2 *__restrict__ R) {
    __shared__ double2 part[kAcThreads / kWave][kLagBlock];
    const int t = blockIdx.x;
    const int j0 = blockIdx.y * kLagBlock;
    const int lo = offsets[t], hi = offsets[t + 1];
    Cd acc[kLagBlock];
#pragma unroll
    for (int s = 0; s < kLagBlock; ++s) acc[s] = Cd{0.0, 0.0};
    for (int k = lo + (int)threadIdx.x; k < hi; k += kAcThreads) {
        const Cd ak{(double)ca[k].x, (double)ca[k].y};
        const Cd bk{(double)cb[k].x, (double)cb[k].y};
        const int dk = cd[k];
        for (int l = lo; l < hi; ++l) {
            const Cd al{(double)ca[l].x, -(double)ca[l].y};   // conj(a_l)
            const Cd bl{(double)cb[l].x, -(double)cb[l].y};   // conj(b_l)
            const Cd num = cmul(bk, bl);
            const Cd den{1.0 - (ak.r * al.r - ak.i * al.i), -(ak.r * al.i + ak.i * al.r)};
            const double den2 = den.r * den.r + den.i * den.i;
            const Cd g{(num.r * den.r + num.i * den.i) / den2, (num.i * den.r - num.r * den.i) / den2};
            const int e0 = cd[l] + j0 - dk;   // exponent at the block's first lag
            // lags s >= sp have e >= 0 (power a_k^e), lags s < sp have e < 0
            const int sp = min(max(-e0, 0), kLagBlock);
            if (sp < kLagBlock) {
                Cd p = cpow(ak, e0 + sp);   // exponent at lag sp (0 when e0 < 0)
#pragma unroll
                for (int s = 0; s < kLagBlock; ++s) {
                    if (s >= sp) {
                        const Cd v = cmul(g, p);
                        acc[s].r += v.r;
                        acc[s].i += v.i;
                        p = cmul(p, ak);
                    }
                }
            }
            if (sp > 0) {
                Cd q = cpow(al, -(e0 + sp - 1));   // conj(a_l)^-e at lag sp-1
#pragma unroll
                for (int s = kLagBlock - 1; s >= 0; --s) {
                    if (s < sp) {
                        const Cd v = cmul(g, q);
                        acc[s].r += v.r;
                        acc[s].i += v.i;
                        q = cmul(q, al);
                    }
                }
            }
        }
    }
    // reduce over the workgroup: shuffles inside each wave, then the waves via LDS
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int s = 0; s < kLagBlock; ++s) {
        double r = acc[s].r, i = acc[s].i;
        for (int off = kWave / 2; off >= 1; off >>= 1) {
            r += __shfl_xor(r, off);
            i += __shfl_xor(i, off);
        }
        if (lane == 0) part[wave][s] = make_double2(r, i);
    }
    __syncthreads();
    if (threadIdx.x < kLagBlock) {
        const int s = threadIdx.x;
        double r = 0.0, i = 0.0;
        for (int w = 0; w < kAcThreads / kWave; ++w) {
            r += part[w][s].x;
            i += part[w][s].y;
        }
        if (j0 + s <= nj) R[(int64_t)t * (nj + 1) + j0 + s] = make_double2(r, i);
    }
}

// xi^2 of the series zr at candidate sample c (c - nj >= 0, c + nj < n checked by the
// caller), returned in every lane of the wave: one wave, lags strided over the lanes,
// FP64 sums reduced with shuffles.
__device__ __forceinline__ double xi2_wave(const float2 *__restrict__ zr, int c,
                                           const double2 *__restrict__ Rt, int nj, int lane) {
    const double r0 = Rt[0].x;
    const double zcr = zr[c].x, zci = zr[c].y;
    double num = 0.0, den = 0.0;
    for (int j = -nj + lane; j <= nj; j += kWave) {
        const double2 rj = Rt[j >= 0 ? j : -j];
        const double Ar = rj.x / r0, Ai = (j >= 0 ? rj.y : -rj.y) / r0;
        const double dr = (double)zr[c + j].x - (zcr * Ar - zci * Ai);
        const double di = (double)zr[c + j].y - (zcr * Ai + zci * Ar);
        num += dr * dr + di * di;
        den += 2.0 - 2.0 * (Ar * Ar + Ai * Ai);
    }
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        num += __shfl_xor(num, off);
        den += __shfl_xor(den, off);
    }
    return num * (2.0 / r0) / den;
}

__global__ __launch_bounds__(kWave) void xi2_kernel(const float2 *__restrict__ z, int32_t n_templates,
                                                    int32_t n, const int32_t *__restrict__ index,
                                                    int32_t n_win, const double2 *__restrict__ R,
                                                    int32_t nj, float *__restrict__ xi2) {
    const int64_t cand = blockIdx.x;   // (row, window)
    const int64_t row = cand / n_win;
    const int t = (int)(row % n_templates);
    const int lane = threadIdx.x;
    const int c = index[cand];
    if (c < 0 || c - nj < 0 || c + nj >= n) {
        if (lane == 0) xi2[cand] = __builtin_nanf("");
        return;
    }
    const double v = xi2_wave(z + row * (int64_t)n, c, R + (int64_t)t * (nj + 1), nj, lane);
    if (lane == 0) xi2[cand] = (float)v;
}

// Detector average xi^2_C at coherent candidates: one workgroup per candidate (detector
// I, template t, window w), wave J evaluates detector J's series at its arrival time
// s_J = c + tau[p][J] - tau[p][I] in the candidate's direction p; the first thread
// averages the n_det values in detector order.
constexpr int kMaxNetDet = 8;

__global__ __launch_bounds__(kWave *kMaxNetDet) void xi2_network_kernel(
    const float2 *__restrict__ z, int32_t n_det, int32_t n_templates, int32_t n,
    const int32_t *__restrict__ index, const int32_t *__restrict__ pix, int32_t n_win,
    const int32_t *__restrict__ tau, int32_t n_pix, const double2 *__restrict__ R, int32_t nj,
    float *__restrict__ xi2_det, float *__restrict__ xi2_c) {
    __shared__ double part[kMaxNetDet];
    const int64_t cand = blockIdx.x;                 // ((I * T) + t) * n_win + w
    const int64_t row = cand / n_win;                // I * T + t
    const int t = (int)(row % n_templates);
    const int I = (int)(row / n_templates);
    const int J = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int c = index[cand];
    const int p = pix[cand];
    bool ok = c >= 0 && p >= 0 && p < n_pix;
    if (ok) {
        const int32_t *tp = tau + (int64_t)p * n_det;
        for (int q = 0; q < n_det; ++q) {
            const int s = c + tp[q] - tp[I];
            ok = ok && s - nj >= 0 && s + nj < n;
        }
    }
    if (!ok) {
        if (lane == 0 && xi2_det != nullptr) xi2_det[cand * n_det + J] = __builtin_nanf("");
        if (threadIdx.x == 0) xi2_c[cand] = __builtin_nanf("");
        return;
    }
    const int s = c + tau[(int64_t)p * n_det + J] - tau[(int64_t)p * n_det + I];
    const float2 *zr = z + ((int64_t)J * n_templates + t) * n;
    const double v = xi2_wave(zr, s, R + (int64_t)t * (nj + 1), nj, lane);
    if (lane == 0) {
        part[J] = v;
        if (xi2_det != nullptr) xi2_det[cand * n_det + J] = (float)v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int q = 0; q < n_det; ++q) sum += part[q];
        xi2_c[cand] = (float)(sum / n_det);
    }
}

}  // namespace

hipError_t launch_autocorr(int32_t n_templates, const int32_t *offsets, const float2 *a,
                           const float2 *b, const int32_t *d, int32_t nj, double2 *R, hipStream_t s) {
    if (n_templates <= 0) return hipSuccess;
    const dim3 grid(n_templates, (nj + 1 + kLagBlock - 1) / kLagBlock);
    hipLaunchKernelGGL(autocorr_kernel, grid, dim3(kAcThreads), 0, s, offsets, a, b, d, nj, R);
    return hipGetLastError();
}

hipError_t launch_xi2(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                      const int32_t *index, int32_t n_win, const double2 *R, int32_t nj, float *xi2,
                      hipStream_t s) {
    const int64_t cands = (int64_t)n_det * n_templates * n_win;
    if (cands <= 0) return hipSuccess;
    hipLaunchKernelGGL(xi2_kernel, dim3((unsigned)cands), dim3(kWave), 0, s, z, n_templates, n, index,
                       n_win, R, nj, xi2);
    return hipGetLastError();
}

}  // namespace spiir

namespace spiir {

hipError_t launch_xi2_network(const float2 *z, int32_t n_det, int32_t n_templates, int32_t n,
                              const int32_t *index, const int32_t *pix, int32_t n_win,
                              const int32_t *tau, int32_t n_pix, const double2 *R, int32_t nj,
                              float *xi2_det, float *xi2_c, hipStream_t s) {
    const int64_t cands = (int64_t)n_det * n_templates * n_win;
    if (cands <= 0) return hipSuccess;
    hipLaunchKernelGGL(xi2_network_kernel, dim3((unsigned)cands), dim3(kWave * n_det), 0, s, z,
                       n_det, n_templates, n, index, pix, n_win, tau, n_pix, R, nj, xi2_det,
                       xi2_c);
    return hipGetLastError();
}

}  // namespace spiir
