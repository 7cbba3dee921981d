// Preparation of the time-blocked split-bf16 form.  The host sorts every
// template's filters by delay and lays out the operand blocks of the two products in
// the order the matrix-core kernels read them (tiles, bands, offsets: integer work on
// the bank's shape); the operand values themselves are computed on the GPU in FP64
// from the coefficients, and every value v is split into bf16 hi = rne(v) and
// lo = rne(v - hi).  The same kernels run again when the coefficients are replaced.
//
// Operand block = 32 rows x 16 K entries, hi then lo (1024 bf16, 2 KiB), rows
// row-major, so that lane l of a wave reads row l%32, entries 8*(l/32) .. +8.
#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace spiir {
namespace {

inline int64_t ceil16(int64_t v) { return (v + 15) / 16 * 16; }

struct Cd {
    double r, i;
};

__device__ __forceinline__ Cd cmul(Cd a, Cd b) { return Cd{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

__device__ __forceinline__ Cd cpow(Cd a, int e) {   // e >= 0, by repeated squaring
    Cd r{1.0, 0.0};
    for (; e > 0; e >>= 1) {
        if (e & 1) r = cmul(r, a);
        a = cmul(a, a);
    }
    return r;
}

__device__ __forceinline__ Cd coeff(const float2 *v, int64_t g) {
    const float2 c = v[g];
    return Cd{(double)c.x, (double)c.y};
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// value v at (row, k) of the operand block starting at blk: hi and lo bf16 halves
__device__ __forceinline__ void put(uint16_t *blk, int row, int k, double v) {
    const uint16_t h = bf16_rne((float)v);
    const double hv = (double)__uint_as_float((uint32_t)h << 16);
    blk[row * 16 + k] = h;
    blk[512 + row * 16 + k] = bf16_rne((float)(v - hv));
}

constexpr int kPadDelay = 1 << 28;   // delay of padding filters: outside every band

// a^L in FP64 and the long-pole flag, per filter in sorted-padded order
__global__ void block_filter_kernel(const float2 *__restrict__ ga, int64_t n_fpad, int32_t L,
                                    double thr2, double2 *__restrict__ aL, int32_t *__restrict__ lp) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_fpad;
         g += (int64_t)gridDim.x * blockDim.x) {
        const Cd a = coeff(ga, g);
        const Cd p = cpow(a, L);
        aL[g] = make_double2(p.r, p.i);
        lp[g] = (a.r * a.r + a.i * a.i > thr2) ? 1 : 0;
    }
}

// Input-to-state operand: block (tile w, K step ks) = rows 2r, 2r+1 (re, im) of the
// tile's filter r, K entry kk = input offset sigma = sigma_lo + 16 ks + kk:
// W'[sigma] = b a^(L-1-i) at i = sigma + d in [0, L), else 0.  One workgroup per block,
// thread (r, kk).
__global__ __launch_bounds__(256) void block_w_kernel(const WTile *__restrict__ tiles,
                                                      const int32_t *__restrict__ wblk,
                                                      const float2 *__restrict__ ga,
                                                      const float2 *__restrict__ gb,
                                                      const int32_t *__restrict__ gd, int32_t L,
                                                      uint16_t *__restrict__ wa) {
    const int64_t blk_id = blockIdx.x;
    const WTile w = tiles[wblk[blk_id]];
    const int ks = (int)(blk_id - w.a_off / 1024);
    const int r = threadIdx.x / 16, kk = threadIdx.x % 16;
    const int64_t g = w.g0 + r;
    const int i = w.sigma_lo + 16 * ks + kk + gd[g];
    Cd v{0.0, 0.0};
    if (i >= 0 && i < L) v = cmul(coeff(gb, g), cpow(coeff(ga, g), L - 1 - i));
    uint16_t *blk = wa + blk_id * 1024;
    put(blk, 2 * r, kk, v.r);
    put(blk, 2 * r + 1, kk, v.i);
}

// Output operand, state part: block (template t, K step ks < nks_p, row tile rt):
// row 2j + c, K entry 2 fi + cc holds [[Re p, -Im p], [Im p, Re p]][c][cc] with
// p = a_fi^(j+1).  grid (T, blocks of the largest template); thread (row, kk).
__global__ __launch_bounds__(512) void block_p_kernel(const BTemplate *__restrict__ tmpls,
                                                      const float2 *__restrict__ ga, int32_t L,
                                                      uint16_t *__restrict__ pa) {
    const int rt_per = 2 * L / 32;
    const BTemplate bt = tmpls[blockIdx.x];
    const int b = blockIdx.y;
    if (b >= bt.nks_p * rt_per) return;
    const int ks = b / rt_per, rt = b % rt_per;
    const int row = threadIdx.x / 16, kk = threadIdx.x % 16;
    const int R = rt * 32 + row, j = R / 2, c = R % 2;
    const int K = ks * 16 + kk, fi = K / 2, cc = K % 2;
    const Cd p = cpow(coeff(ga, bt.g0 + fi), j + 1);
    const double v = c == 0 ? (cc == 0 ? p.r : -p.i) : (cc == 0 ? p.i : p.r);
    put(pa + bt.a_off + (int64_t)b * 1024, row, kk, v);
}

// Output operand, input part: M_t[j][sigma] = sum over the template's filters with
// 0 <= j - sigma - d_k <= j of b_k a_k^(j - sigma - d_k), i.e. d_k in [-sigma, j - sigma]:
// a contiguous run of the delay-sorted filters (found by binary search), summed in
// sorted order in FP64.  Block (template t, K step nks_p + km, row tile rt) holds rows
// 2j (re) and 2j+1 (im) for 16 values of j and K entries sigma - sigma_lo.
// grid (T, blocks of the largest template); thread (j, kk).
__global__ __launch_bounds__(256) void block_m_kernel(const BTemplate *__restrict__ tmpls,
                                                      const float2 *__restrict__ ga,
                                                      const float2 *__restrict__ gb,
                                                      const int32_t *__restrict__ gd, int32_t L,
                                                      uint16_t *__restrict__ pa) {
    const int rt_per = 2 * L / 32;
    const BTemplate bt = tmpls[blockIdx.x];
    const int b = blockIdx.y;
    if (b >= bt.nks_m * rt_per) return;
    const int km = b / rt_per, rt = b % rt_per;
    const int jl = threadIdx.x / 16, kk = threadIdx.x % 16;
    const int j = rt * 16 + jl;
    const int sigma = bt.sigma_lo + km * 16 + kk;
    const int32_t *d = gd + bt.g0;
    // first filter with d >= -sigma, first with d > j - sigma
    auto lower = [&](int v) {
        int lo = 0, hi = bt.fpad;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (d[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int k0 = lower(-sigma), k1 = lower(j - sigma + 1);
    Cd m{0.0, 0.0};
    for (int k = k0; k < k1; ++k) {
        const Cd t = cmul(coeff(gb, bt.g0 + k), cpow(coeff(ga, bt.g0 + k), j - sigma - d[k]));
        m.r += t.r;
        m.i += t.i;
    }
    uint16_t *blk = pa + bt.a_off + ((int64_t)(bt.nks_p + km) * rt_per + rt) * 1024;
    put(blk, 2 * jl, kk, m.r);
    put(blk, 2 * jl + 1, kk, m.i);
}

// coefficients in original filter order -> sorted-padded order (padding keeps 0)
__global__ void block_gather_kernel(const int32_t *__restrict__ perm, const float2 *__restrict__ a,
                                    const float2 *__restrict__ b, int64_t n_fpad,
                                    float2 *__restrict__ ga, float2 *__restrict__ gb) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_fpad;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = perm[g];
        ga[g] = k >= 0 ? a[k] : make_float2(0.0f, 0.0f);
        gb[g] = k >= 0 ? b[k] : make_float2(0.0f, 0.0f);
    }
}

}  // namespace

spiir_status plan_block(Bank &bk, const int32_t *offsets, const float *a, const float *b,
                        const int32_t *delay, hipStream_t s, std::string &err) {
    const int L = bk.block_len;
    const int T = bk.n_templates;
    const int rt_per = 2 * L / 32;
    const int64_t nb_max = bk.max_chunk / L;
    bk.hist_pad = (int32_t)ceil16(bk.hist_len);

    std::vector<BTemplate> tm(T);
    std::vector<std::vector<int32_t>> order(T);   // filters of t sorted by delay
    std::vector<int64_t> tile_base(T + 1, 0);
    std::vector<WTile> tiles;
    int64_t g = 0, yoff = 0, aoff = 0, waoff = 0;
    for (int t = 0; t < T; ++t) {
        const int32_t lo = offsets[t], hi = offsets[t + 1], f = hi - lo;
        auto &ord = order[t];
        ord.resize(f);
        std::iota(ord.begin(), ord.end(), lo);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t p, int32_t q) { return delay[p] < delay[q]; });
        BTemplate &bt = tm[t];
        bt.fpad = (int32_t)ceil16(f);
        bt.g0 = g;
        bt.y_off = yoff;
        bt.a_off = aoff;
        const int32_t dmax = f > 0 ? delay[ord[f - 1]] : 0;
        bt.sigma_lo = f > 0 ? -(int32_t)ceil16(dmax) : 0;
        bt.nks_p = 2 * bt.fpad / 16;
        bt.nks_m = f > 0 ? (L - bt.sigma_lo) / 16 : 0;
        g += bt.fpad;
        yoff += nb_max * 2 * bt.fpad;
        aoff += (int64_t)(bt.nks_p + bt.nks_m) * rt_per * 1024;
        tile_base[t] = (int64_t)tiles.size();
        for (int32_t f0 = 0; f0 < f; f0 += 16) {
            const int32_t f1 = std::min(f, f0 + 16);
            const int32_t dmin = delay[ord[f0]], dmx = delay[ord[f1 - 1]];
            WTile w{};
            w.tmpl = t;
            w.f0 = f0;
            w.sigma_lo = -(int32_t)ceil16(dmx);
            w.nks = (int32_t)((ceil16(L - dmin) - w.sigma_lo) / 16);
            w.a_off = waoff;
            w.g0 = bt.g0 + f0;
            waoff += (int64_t)w.nks * 1024;
            tiles.push_back(w);
        }
    }
    tile_base[T] = (int64_t)tiles.size();
    // widest input band of a group of 4 consecutive tiles (one block_state workgroup)
    int32_t band = 0;
    for (size_t i = 0; i < tiles.size(); i += 4) {
        int32_t lo = 1 << 30, hi = -(1 << 30);
        for (size_t j = i; j < std::min(tiles.size(), i + 4); ++j) {
            lo = std::min(lo, tiles[j].sigma_lo);
            hi = std::max(hi, tiles[j].sigma_lo + 16 * tiles[j].nks);
        }
        band = std::max(band, hi - lo);
    }
    bk.max_wg_band = band;
    bk.n_fpad = g;
    bk.y_per_det = std::max<int64_t>(yoff, 32);
    bk.n_wtiles = (int32_t)tiles.size();
    bk.xs_stride = ceil16(bk.hist_pad + bk.max_chunk + 16);

    // coefficients in sorted-padded order (padding: a = b = 0, delay past every band),
    // the original index of every filter, and the tile of every W' operand block
    std::vector<float2> ga((size_t)std::max<int64_t>(g, 1), make_float2(0.f, 0.f));
    std::vector<float2> gb(ga.size(), make_float2(0.f, 0.f));
    std::vector<int32_t> gd(ga.size(), kPadDelay), perm(ga.size(), -1);
    const double thr2 = bk.long_pole * bk.long_pole;
    int32_t n_lp = 0;
    for (int t = 0; t < T; ++t) {
        const auto &ord = order[t];
        for (size_t fi = 0; fi < ord.size(); ++fi) {
            const int32_t k = ord[fi];
            const int64_t gi = tm[t].g0 + (int64_t)fi;
            ga[gi] = make_float2(a[2 * (int64_t)k], a[2 * (int64_t)k + 1]);
            gb[gi] = make_float2(b[2 * (int64_t)k], b[2 * (int64_t)k + 1]);
            gd[gi] = delay[k];
            perm[gi] = k;
            const double ar = a[2 * (int64_t)k], ai = a[2 * (int64_t)k + 1];
            n_lp += ar * ar + ai * ai > thr2 ? 1 : 0;
        }
    }
    bk.n_long_pole = n_lp;
    std::vector<int32_t> wblk((size_t)std::max<int64_t>(waoff / 1024, 1), 0);
    for (size_t i = 0; i < tiles.size(); ++i)
        for (int32_t ks = 0; ks < tiles[i].nks; ++ks) wblk[(size_t)(tiles[i].a_off / 1024 + ks)] = (int32_t)i;
    bk.n_wblocks = waoff / 1024;
    // every operand block (32 rows x 16 K entries, hi and lo planes) takes part in three
    // 32x32x16 products per 32 columns: 32 x 16 x 2 x 3 flop per column
    bk.block_flop_per_col = (waoff / 1024 + aoff / 1024) * (32 * 16 * 2 * 3);
    int32_t pmax = 0, mmax = 0;
    for (const BTemplate &bt : tm) {
        pmax = std::max(pmax, bt.nks_p * rt_per);
        mmax = std::max(mmax, bt.nks_m * rt_per);
    }
    bk.max_p_blocks = pmax;
    bk.max_m_blocks = mmax;
    int32_t min_k = INT32_MAX;
    for (const BTemplate &bt : tm)
        if (bt.nks_p + bt.nks_m > 0) min_k = std::min(min_k, bt.nks_p + bt.nks_m);
    bk.out_ksplit = block_output_ksplit(bk, min_k == INT32_MAX ? 0 : min_k);
    if (pmax > 65535 || mmax > 65535) {   // the operand kernels put them on grid.y
        err = "block form: a template's output operand has more than 65535 blocks";
        return SPIIR_E_UNSUPPORTED;
    }

    auto alloc = [&](void **ptr, int64_t bytes) -> bool {
        bytes = (std::max<int64_t>(bytes, 16) + 255) & ~int64_t(255);
        if (hipMalloc(ptr, (size_t)bytes) != hipSuccess) {
            (void)hipGetLastError();
            err = "hipMalloc of " + std::to_string(bytes) + " bytes failed (block form)";
            return false;
        }
        bk.allocations.push_back(*ptr);
        bk.device_bytes += bytes;
        return true;
    };
    const int64_t D = bk.n_det;
    if (!alloc((void **)&bk.d_wtiles, (int64_t)std::max<size_t>(tiles.size(), 1) * sizeof(WTile)) ||
        !alloc((void **)&bk.d_btmpl, (int64_t)T * sizeof(BTemplate)) ||
        !alloc((void **)&bk.d_wa, std::max<int64_t>(waoff, 1024) * 2) ||
        !alloc((void **)&bk.d_pa, std::max<int64_t>(aoff, 1024) * 2) ||
        !alloc((void **)&bk.d_aL, (int64_t)ga.size() * sizeof(double2)) ||
        !alloc((void **)&bk.d_lp, (int64_t)ga.size() * 4) ||
        !alloc((void **)&bk.d_perm, (int64_t)perm.size() * 4) ||
        !alloc((void **)&bk.d_ga, (int64_t)ga.size() * sizeof(float2)) ||
        !alloc((void **)&bk.d_gb, (int64_t)gb.size() * sizeof(float2)) ||
        !alloc((void **)&bk.d_gd, (int64_t)gd.size() * 4) ||
        !alloc((void **)&bk.d_wblk, (int64_t)wblk.size() * 4) ||
        !alloc((void **)&bk.d_state64, D * (int64_t)ga.size() * sizeof(double2)) ||
        !alloc((void **)&bk.d_yt, 2 * D * bk.y_per_det * 2) ||
        !alloc((void **)&bk.d_xs, 2 * D * bk.xs_stride * 2) ||
        !alloc((void **)&bk.d_zbuf, D * T * (int64_t)bk.max_chunk * sizeof(float2)) ||
        (bk.out_ksplit > 1 &&
         !alloc((void **)&bk.d_zpart,
                (int64_t)bk.out_ksplit * D * T * (int64_t)bk.max_chunk * sizeof(float2))))
        return SPIIR_E_NOMEM;
    struct Up { void *dst; const void *src; size_t bytes; };
    const Up ups[] = {
        {bk.d_wtiles, tiles.data(), tiles.size() * sizeof(WTile)},
        {bk.d_btmpl, tm.data(), tm.size() * sizeof(BTemplate)},
        {bk.d_perm, perm.data(), perm.size() * 4},
        {bk.d_ga, ga.data(), ga.size() * sizeof(float2)},
        {bk.d_gb, gb.data(), gb.size() * sizeof(float2)},
        {bk.d_gd, gd.data(), gd.size() * 4},
        {bk.d_wblk, wblk.data(), wblk.size() * 4},
    };
    for (const Up &u : ups) {
        if (u.bytes == 0) continue;
        const hipError_t e = hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            err = std::string("hipMemcpyAsync: ") + hipGetErrorString(e);
            return SPIIR_E_HIP;
        }
    }
    hipError_t e = launch_block_operands(bk, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host vectors die at return
    if (e != hipSuccess) {
        err = std::string("block operands: ") + hipGetErrorString(e);
        return SPIIR_E_HIP;
    }
    return SPIIR_OK;
}

hipError_t launch_block_operands(const Bank &bk, hipStream_t s) {
    const int L = bk.block_len;
    const int T = bk.n_templates;
    if (bk.n_fpad == 0) return hipSuccess;
    const unsigned fblocks = (unsigned)std::min<int64_t>((bk.n_fpad + 255) / 256, 4096);
    hipLaunchKernelGGL(block_filter_kernel, dim3(fblocks), dim3(256), 0, s, bk.d_ga, bk.n_fpad, L,
                       bk.long_pole * bk.long_pole, bk.d_aL, bk.d_lp);
    if (bk.n_wblocks > 0)
        hipLaunchKernelGGL(block_w_kernel, dim3((unsigned)bk.n_wblocks), dim3(256), 0, s,
                           bk.d_wtiles, bk.d_wblk, bk.d_ga, bk.d_gb, bk.d_gd, L, bk.d_wa);
    if (bk.max_p_blocks > 0)
        hipLaunchKernelGGL(block_p_kernel, dim3((unsigned)T, (unsigned)bk.max_p_blocks), dim3(512), 0,
                           s, bk.d_btmpl, bk.d_ga, L, bk.d_pa);
    if (bk.max_m_blocks > 0)
        hipLaunchKernelGGL(block_m_kernel, dim3((unsigned)T, (unsigned)bk.max_m_blocks), dim3(256), 0,
                           s, bk.d_btmpl, bk.d_ga, bk.d_gb, bk.d_gd, L, bk.d_pa);
    return hipGetLastError();
}

hipError_t launch_block_set_coeffs(const Bank &bk, const float2 *a, const float2 *b, hipStream_t s) {
    if (bk.n_fpad == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((bk.n_fpad + 255) / 256, 4096);
    hipLaunchKernelGGL(block_gather_kernel, dim3(blocks), dim3(256), 0, s, bk.d_perm, a, b,
                       bk.n_fpad, bk.d_ga, bk.d_gb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_block_operands(bk, s);
}

}  // namespace spiir
