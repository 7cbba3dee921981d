// Host-side preparation of the time-blocked split-bf16 form: sorts every
// template's filters by delay, lays out the operand blocks of the two products
// in the order the matrix-core kernels read them, and fills them in FP64 before
// splitting each value v into bf16 hi = rne(v) and lo = rne(v - hi).
//
// Operand block = 32 rows x 16 K entries, hi then lo (1024 bf16, 2 KiB), rows
// row-major, so that lane l of a wave reads row l%32, entries 8*(l/32) .. +8.
#include <algorithm>
#include <atomic>
#include <complex>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "internal.h"

namespace spiir {
namespace {

using cplx = std::complex<double>;

inline int64_t ceil16(int64_t v) { return (v + 15) / 16 * 16; }

inline uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

inline float bf16_to_float(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

inline void split(double v, uint16_t &hi, uint16_t &lo) {
    hi = bf16_rne((float)v);
    lo = bf16_rne((float)(v - (double)bf16_to_float(hi)));
}

// store one real value at (row, k) of the operand block starting at blk
inline void put(uint16_t *blk, int row, int k, double v) {
    uint16_t h, l;
    split(v, h, l);
    blk[row * 16 + k] = h;
    blk[512 + row * 16 + k] = l;
}

template <typename F>
void parallel_for(int64_t n, F &&fn) {
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(n, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    std::atomic<int64_t> next{0};
    for (int64_t w = 0; w < nt; ++w)
        pool.emplace_back([&]() {
            for (int64_t i; (i = next.fetch_add(1)) < n;) fn(i);
        });
    for (auto &th : pool) th.join();
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

    std::vector<uint16_t> wa((size_t)std::max<int64_t>(waoff, 1024), 0);
    std::vector<uint16_t> pa((size_t)std::max<int64_t>(aoff, 1024), 0);
    std::vector<double2> aL((size_t)std::max<int64_t>(g, 1), make_double2(0.0, 0.0));
    std::vector<int32_t> lp((size_t)std::max<int64_t>(g, 1), 0);
    std::vector<int32_t> perm((size_t)std::max<int64_t>(g, 1), -1);
    const double thr2 = bk.long_pole * bk.long_pole;
    std::atomic<int32_t> n_lp{0};

    parallel_for(T, [&](int64_t t) {
        const BTemplate &bt = tm[t];
        const auto &ord = order[t];
        const int32_t f = (int32_t)ord.size();
        if (f == 0) return;
        std::vector<cplx> pw(L), p(L);
        // output operand: M part accumulated in FP64, [j][sigma - sigma_lo]
        const int ms = L - bt.sigma_lo;
        std::vector<cplx> M((size_t)L * ms, cplx(0.0, 0.0));
        int32_t local_lp = 0;
        for (int32_t fi = 0; fi < f; ++fi) {
            const int32_t k = ord[fi];
            const cplx ak(a[2 * (int64_t)k], a[2 * (int64_t)k + 1]);
            const cplx bkc(b[2 * (int64_t)k], b[2 * (int64_t)k + 1]);
            const int32_t d = delay[k];
            const int64_t gi = bt.g0 + fi;
            perm[gi] = k;
            // powers a^m, m = 0..L
            cplx pwr(1.0, 0.0);
            for (int m = 0; m < L; ++m) {
                pw[m] = bkc * pwr;   // b a^m
                pwr *= ak;
                p[m] = pwr;          // a^(m+1)
            }
            aL[gi] = make_double2(p[L - 1].real(), p[L - 1].imag());
            if (std::norm(ak) > thr2) {
                lp[gi] = 1;
                ++local_lp;
            }
            // state part of the output operand: rows 2j+c, K entries 2fi+c'
            for (int j = 0; j < L; ++j) {
                const int rows[2] = {2 * j, 2 * j + 1};
                const double v[2][2] = {{p[j].real(), -p[j].imag()}, {p[j].imag(), p[j].real()}};
                for (int c = 0; c < 2; ++c)
                    for (int cc = 0; cc < 2; ++cc) {
                        const int kk = 2 * fi + cc;
                        const int row = rows[c];
                        uint16_t *blk = pa.data() + bt.a_off +
                                        ((int64_t)(kk / 16) * rt_per + row / 32) * 1024;
                        put(blk, row % 32, kk % 16, v[c][cc]);
                    }
            }
            // input part: M[j][sigma] += b a^m with sigma = j - m - d
            for (int j = 0; j < L; ++j) {
                cplx *row = M.data() + (size_t)j * ms;
                for (int m = 0; m <= j; ++m) row[j - m - d - bt.sigma_lo] += pw[m];
            }
            // input-to-state operand of the filter's tile: W'[sigma] = b a^(L-1-(sigma+d))
            const WTile &w = tiles[tile_base[t] + fi / 16];
            const int r = fi % 16;
            for (int ks = 0; ks < w.nks; ++ks) {
                uint16_t *blk = wa.data() + w.a_off + (int64_t)ks * 1024;
                for (int kk = 0; kk < 16; ++kk) {
                    const int i = w.sigma_lo + 16 * ks + kk + d;
                    if (i < 0 || i >= L) continue;
                    const cplx v = pw[L - 1 - i];
                    put(blk, 2 * r, kk, v.real());
                    put(blk, 2 * r + 1, kk, v.imag());
                }
            }
        }
        n_lp += local_lp;
        for (int j = 0; j < L; ++j)
            for (int sg = 0; sg < ms; ++sg) {
                const cplx v = M[(size_t)j * ms + sg];
                const int kk = sg;   // K entry within the input part
                for (int c = 0; c < 2; ++c) {
                    const int row = 2 * j + c;
                    uint16_t *blk = pa.data() + bt.a_off +
                                    ((int64_t)(bt.nks_p + kk / 16) * rt_per + row / 32) * 1024;
                    put(blk, row % 32, kk % 16, c == 0 ? v.real() : v.imag());
                }
            }
    });
    bk.n_long_pole = n_lp.load();

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
        !alloc((void **)&bk.d_wa, (int64_t)wa.size() * 2) ||
        !alloc((void **)&bk.d_pa, (int64_t)pa.size() * 2) ||
        !alloc((void **)&bk.d_aL, (int64_t)aL.size() * sizeof(double2)) ||
        !alloc((void **)&bk.d_lp, (int64_t)lp.size() * 4) ||
        !alloc((void **)&bk.d_perm, (int64_t)perm.size() * 4) ||
        !alloc((void **)&bk.d_state64, D * (int64_t)aL.size() * sizeof(double2)) ||
        !alloc((void **)&bk.d_yt, 2 * D * bk.y_per_det * 2) ||
        !alloc((void **)&bk.d_xs, 2 * D * bk.xs_stride * 2) ||
        !alloc((void **)&bk.d_zbuf, D * T * (int64_t)bk.max_chunk * sizeof(float2)))
        return SPIIR_E_NOMEM;
    struct Up { void *dst; const void *src; size_t bytes; };
    const Up ups[] = {
        {bk.d_wtiles, tiles.data(), tiles.size() * sizeof(WTile)},
        {bk.d_btmpl, tm.data(), tm.size() * sizeof(BTemplate)},
        {bk.d_wa, wa.data(), wa.size() * 2},
        {bk.d_pa, pa.data(), pa.size() * 2},
        {bk.d_aL, aL.data(), aL.size() * sizeof(double2)},
        {bk.d_lp, lp.data(), lp.size() * 4},
        {bk.d_perm, perm.data(), perm.size() * 4},
    };
    for (const Up &u : ups) {
        if (u.bytes == 0) continue;
        const hipError_t e = hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            err = std::string("hipMemcpyAsync: ") + hipGetErrorString(e);
            return SPIIR_E_HIP;
        }
    }
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
        return SPIIR_E_HIP;
    }
    return SPIIR_OK;
}

}  // namespace spiir
