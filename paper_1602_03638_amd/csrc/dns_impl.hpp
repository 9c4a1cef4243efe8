// Launchers of the kernel templates for one real type; included by the
// per-precision translation units, which instantiate every supported N.
#pragma once

#include <algorithm>
#include <cmath>

#include <type_traits>

#include "dns_kernels.hpp"
#include "dns_mfma.hpp"
#include "dns_ops.hpp"

namespace dns {

constexpr size_t LDS_LIMIT = 160 * 1024;

template <typename R, int N> struct Impl {
    using C = cx<R>;
    static constexpr int G = N / 8;                // threads per z line
    static constexpr int GX = N / x_elems<R>(N);   // threads per x line
    static constexpr size_t CB = sizeof(C);
    static constexpr int XCOLS = N * (N / 2);
    static constexpr int YE0 = default_y_elems<R>(N);
    static constexpr bool CY0 = default_curl_in_y<R>(N);
    // FP64 lines of 8 complex doubles per thread need more than the 128
    // registers a 1024-thread workgroup leaves each thread: at most 512.
    static constexpr int MAXT = sizeof(R) == 8 ? 512 : 1024;

    // Feasibility of a workgroup shape: at most 1024 threads and the LDS limit.
    // (lines of more than 8 elements per thread need more than the 128
    // registers a 1024-thread workgroup leaves each thread)
    template <int T> static constexpr bool x_ok() {
        return T <= N && GX * T <= (x_elems<R>(N) > 8 ? 512 : 1024) && (size_t)T * N * CB <= LDS_LIMIT;
    }
    // The RHS/RK4 passes hold three lines plus state per thread: in FP64
    // their 1024-thread shapes (128 registers per thread) only spill.
    template <int T, int RS = 0> static constexpr bool xr_ok() {
        return x_ok<T>() && (sizeof(R) == 4 || GX * T <= 512) &&
               (size_t)T * N * CB + 2 * 8 * (size_t)GX * T + (size_t)tw_size(N, RS) * CB <= LDS_LIMIT;
    }
    // XCD-grouped tile order (x_tile): where an x tile's row segment is 32
    // or 64 bytes, from 256^3 up, with both tile counts multiples of 8 times
    // the number of tiles per 128-byte line.
    template <int T> static constexpr bool pair_ok() {
        constexpr int grp = line_group<R, T>();
        return N >= 256 && (T * CB == 64 || T * CB == 32) && (XCOLS / T) % (8 * grp) == 0 &&
               (N / T) % (8 * grp) == 0;
    }
    // the same for the y passes (128-byte y tiles hold one workgroup per CU
    // at 512 and 1024: narrower grouped tiles fit two or three)
    template <int T> static constexpr bool ypair_ok() {
        constexpr int grp = line_group<R, T>();
        return N >= 256 && (T * CB == 64 || T * CB == 32) && (N * ((N / 2) / T)) % (8 * grp) == 0 &&
               (N / T) % (8 * grp) == 0;
    }
    // y shapes with YE elements per thread; CURL: the vorticity-forming
    // inverse pass (twiddles in shared memory)
    template <int T, int YE, bool CURL, int RS = 0> static constexpr bool y_ok() {
        return YE >= 8 && N % YE == 0 && T <= N / 2 && (N / YE) * T <= 1024 &&
               ((size_t)T * N + (y_twiddles_in_lds(YE) || CURL ? (size_t)tw_size(N, RS) : 0)) * CB <= LDS_LIMIT;
    }
    // z shapes: at least 16 threads, and up to 128 threads for small N
    // (ZP: one LDS pad slot after every 2^ZP elements of a line, 0 = none)
    template <int L, int ZP = 3, int RS = 0> static constexpr bool z_ok() {
        return L <= N * N && G * L <= 1024 && G * L >= 16 && L <= (128 / G > 8 ? 128 / G : 8) &&
               (size_t)L * padded_line<N>(ZP) * CB + (size_t)tw_size(N, RS) * CB <= LDS_LIMIT;
    }
    template <int T> static constexpr int x_groups() { return XCOLS / T + N / T; }

    // Default widths: 128-byte row segments, and for small N at least one
    // full 64-lane wave per workgroup.
    static constexpr int want_width(int threads_per_line) {
        const int w = (int)(128 / CB), wave = 64 / threads_per_line;
        return w > wave ? w : (wave > 0 ? wave : 1);
    }
    // Widest power-of-two width <= want whose x stage shape is feasible.
    static constexpr int x_default_width() {
        int best = 4;
        const int want = want_width(N / 8);
        if (xr_ok<4>() && GX * 4 <= MAXT && 4 <= want) best = 4;
        if (xr_ok<8>() && GX * 8 <= MAXT && 8 <= want) best = 8;
        if (N <= 64 && xr_ok<16>() && GX * 16 <= MAXT && 16 <= want) best = 16;
        if (N <= 64 && xr_ok<32>() && GX * 32 <= MAXT && 32 <= want) best = 32;
        if (N > 64 && xr_ok<16>() && GX * 16 <= MAXT && 16 <= want) best = 16;
        return best;
    }
    template <int YE> static constexpr int y_default_width() {
        if (N % YE != 0) return 0;
        int best = 0;
        const int want = want_width(N / 8) > want_width(N / YE) ? want_width(N / 8) : want_width(N / YE);
        if (y_ok<4, YE, false>() && (N / YE) * 4 <= MAXT && 4 <= want) best = 4;
        if (y_ok<8, YE, false>() && (N / YE) * 8 <= MAXT && 8 <= want) best = 8;
        if (y_ok<16, YE, false>() && (N / YE) * 16 <= MAXT && 16 <= want) best = 16;
        if (y_ok<32, YE, false>() && (N / YE) * 32 <= MAXT && 32 <= want) best = 32;
        return best;
    }
    static constexpr int XD = x_default_width();

    // ---- pass launchers ----------------------------------------------------
    template <int T, bool CY, bool PAIR, int RS = 0>
    static void xinv(const void* U, void* W, const void* tw, const Batch& b, hipStream_t s) {
        hipLaunchKernelGGL((k_xinv_curl<R, N, T, CY, PAIR, RS>), dim3(x_groups<T>(), b.members), dim3(GX * T), 0, s,
                           (const C*)U, (C*)W, (const C*)tw, b.sst, b.wst);
    }
    template <int T, int DIR, int NF, int YE, bool PAIR = false, int RS = 0>
    static void ypass(void* W, const void* tw, const Batch& b, hipStream_t s) {
        hipLaunchKernelGGL((k_yline<R, N, T, DIR, NF, YE, PAIR, RS>), dim3(y_tiles<R, N, T>(), b.members),
                           dim3((N / YE) * T), 0, s, (C*)W, (const C*)tw, b.wst);
    }
    template <int DIR, int NF, bool CURL>
    static void ymfma(void* W, const void* tw, const void* roots, const void* tw2, const Batch& b, hipStream_t s) {
        if constexpr (std::is_same_v<R, float> && N >= 64) {
            hipLaunchKernelGGL((k_yline_mfma<N, DIR, NF, CURL>), dim3(MfmaY<N>::TILES, b.members),
                               dim3(MfmaY<N>::NT), 0, s, (C*)W, (const C*)tw, (const C*)roots, (const C*)tw2, b.wst);
        }
    }
    // inverse y pass of a stage with the vorticity combinations formed from
    // the x pass's five outputs
    template <int T, bool PAIR = false, int RS = 0>
    static void yinv_curl(void* W, const void* tw, const Batch& b, hipStream_t s) {
        hipLaunchKernelGGL((k_yinv_curl<R, N, T, PAIR, RS>), dim3(y_tiles<R, N, T>(), b.members), dim3((N / 8) * T), 0,
                           s, (C*)W, (const C*)tw, b.wst);
    }
    template <int L, int ZP = 3, int RS = 0>
    static void zcross(void* W, const void* tw, const Batch& b, hipStream_t s) {
        const R scale = (R)std::ldexp(1.0, -6 * ilog2(N));
        hipLaunchKernelGGL((k_zcross<R, N, L, ZP, RS>), dim3((N * N) / L, b.members), dim3(G * L), 0, s, (C*)W,
                           (const C*)tw, scale, b.wst);
    }
    // stages 3 and 4 (last of a step) have an instance with the fused
    // diagnostics, launched when a.diag is set
    template <int T, bool PAIR, int ST, int RS>
    static void xrhs_st(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                        const Batch& b, hipStream_t s) {
        if (ST >= 3 && a.diag != nullptr)
            hipLaunchKernelGGL((k_xrhs<R, N, T, ST, PAIR, ST >= 3, RS>), dim3(x_groups<T>(), b.members), dim3(GX * T), 0,
                               s, (const C*)W, (C*)U0, (C*)U1, (C*)Us, (const C*)tw, a, b.sst, b.wst);
        else
            hipLaunchKernelGGL((k_xrhs<R, N, T, ST, PAIR, false, RS>), dim3(x_groups<T>(), b.members), dim3(GX * T), 0,
                               s, (const C*)W, (C*)U0, (C*)U1, (C*)Us, (const C*)tw, a, b.sst, b.wst);
    }
    template <int T, bool PAIR, int RS = 0>
    static void xrhs(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                     const Batch& b, hipStream_t s) {
        switch (a.stage) {
            case 0: xrhs_st<T, PAIR, 0, RS>(W, U0, U1, Us, tw, a, b, s); break;
            case 1: xrhs_st<T, PAIR, 1, RS>(W, U0, U1, Us, tw, a, b, s); break;
            case 2: xrhs_st<T, PAIR, 2, RS>(W, U0, U1, Us, tw, a, b, s); break;
            case 3: xrhs_st<T, PAIR, 3, RS>(W, U0, U1, Us, tw, a, b, s); break;
            case 4: xrhs_st<T, PAIR, 4, RS>(W, U0, U1, Us, tw, a, b, s); break;
            default: xrhs_st<T, PAIR, -1, RS>(W, U0, U1, Us, tw, a, b, s); break;
        }
    }

    template <int T, bool CY, bool PAIR, int ST, int RS>
    static void xstage_st(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                          const Batch& b, hipStream_t s) {
        if (ST >= 3 && a.diag != nullptr)
            hipLaunchKernelGGL((k_xstage<R, N, T, ST, CY, PAIR, ST >= 3, RS>), dim3(x_groups<T>(), b.members),
                               dim3(GX * T), 0, s, (C*)W, (C*)U0, (C*)U1, (C*)Us, (const C*)tw, a, b.sst, b.wst);
        else
            hipLaunchKernelGGL((k_xstage<R, N, T, ST, CY, PAIR, false, RS>), dim3(x_groups<T>(), b.members),
                               dim3(GX * T), 0, s, (C*)W, (C*)U0, (C*)U1, (C*)Us, (const C*)tw, a, b.sst, b.wst);
    }
    template <int T, bool CY, bool PAIR, int RS = 0>
    static void xstage(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                       const Batch& b, hipStream_t s) {
        switch (a.stage) {
            case 0: xstage_st<T, CY, PAIR, 0, RS>(W, U0, U1, Us, tw, a, b, s); break;
            case 1: xstage_st<T, CY, PAIR, 1, RS>(W, U0, U1, Us, tw, a, b, s); break;
            case 2: xstage_st<T, CY, PAIR, 2, RS>(W, U0, U1, Us, tw, a, b, s); break;
            case 3: xstage_st<T, CY, PAIR, 3, RS>(W, U0, U1, Us, tw, a, b, s); break;
            default: xstage_st<T, CY, PAIR, 4, RS>(W, U0, U1, Us, tw, a, b, s); break;
        }
    }

    // ---- standalone transforms (fixed shapes) -------------------------------
    template <int T> static constexpr bool xs_ok() { return x_ok<T>() && GX * T <= MAXT; }
    template <int T> static constexpr bool ys_ok() { return y_ok<T, YE0, false>() && (N / YE0) * T <= MAXT; }
    static constexpr int TS = xs_ok<8>() ? 8 : (xs_ok<4>() ? 4 : (xs_ok<2>() ? 2 : 1));
    static constexpr int YS = ys_ok<8>() ? 8 : (ys_ok<4>() ? 4 : (ys_ok<2>() ? 2 : 1));
    static constexpr int LS = N >= 128 ? 4 : 512 / N;
    static void xinv3(const void* U, void* W, const void* tw, hipStream_t s) {
        hipLaunchKernelGGL((k_xplain<R, N, TS, +1, 3>), dim3(x_groups<TS>()), dim3(GX * TS), 0, s,
                           (const C*)U, (C*)W, (const C*)tw);
    }
    static void xfwd3(const void* W, void* U, const void* tw, hipStream_t s) {
        hipLaunchKernelGGL((k_xplain<R, N, TS, -1, 3>), dim3(x_groups<TS>()), dim3(GX * TS), 0, s,
                           (const C*)W, (C*)U, (const C*)tw);
    }
    static void yinv3(void* W, const void* tw, hipStream_t s) { ypass<YS, +1, 3, YE0>(W, tw, Batch{1, 0, 0}, s); }
    static void yfwd3s(void* W, const void* tw, hipStream_t s) { ypass<YS, -1, 3, YE0>(W, tw, Batch{1, 0, 0}, s); }
    static void zr2c(const void* u, void* W, const void* tw, hipStream_t s) {
        hipLaunchKernelGGL((k_zr2c<R, N, LS>), dim3((N * N) / LS), dim3(G * LS), 0, s,
                           (const R*)u, (C*)W, (const C*)tw);
    }
    static void zc2r(const void* W, void* u, const void* tw, hipStream_t s) {
        const R scale = (R)std::ldexp(1.0, -3 * ilog2(N));
        hipLaunchKernelGGL((k_zc2r<R, N, LS>), dim3((N * N) / LS), dim3(G * LS), 0, s,
                           (const C*)W, (R*)u, (const C*)tw, scale);
    }
    static void layout(const void* src, void* dst, bool to_internal, hipStream_t s) {
        const size_t total = (size_t)3 * N * N * (N / 2 + 1);
        const unsigned blocks = (unsigned)((total + 255) / 256);
        if (to_internal)
            hipLaunchKernelGGL((k_layout<R, N, true>), dim3(blocks), dim3(256), 0, s,
                               (const C*)src, (C*)dst, total);
        else
            hipLaunchKernelGGL((k_layout<R, N, false>), dim3(blocks), dim3(256), 0, s,
                               (const C*)src, (C*)dst, total);
    }
    static void diag_partial(const void* U, double* part, hipStream_t s) {
        hipLaunchKernelGGL((k_diag_partial<R, N>), dim3(DIAG_BLOCKS), dim3(256), 0, s, (const C*)U, part);
    }

    static void ic_physical(void* u, int kind, double p0, double p1, double p2, hipStream_t s) {
        const size_t P = (size_t)N * N * N;
        hipLaunchKernelGGL((k_ic_physical<R, N>), dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, (R*)u, kind,
                           p0, p1, p2);
    }
    static void ic_random(void* U, unsigned long long seed, double k0, int mask_lim, hipStream_t s) {
        const size_t M = Lay<R, N>::MODES;
        hipLaunchKernelGGL((k_ic_random<R, N>), dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, (C*)U, seed, k0,
                           mask_lim);
    }
    static void scale(void* U, double factor, hipStream_t s) {
        const size_t T = 3 * Lay<R, N>::FS;
        hipLaunchKernelGGL((k_scale<R, N>), dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, (C*)U, factor);
    }

    // ---- variant tables ------------------------------------------------------
    static int& push(Ops& o, int p, Variant d) {
        int& n = o.nvar[p];
        o.var[p][n] = d;
        return n;
    }
    // x passes of width T with curl placement CY and XCD pairing PAIR
    // (RS: radix plan; plans other than 0 only where they differ from 0)
    template <int T, bool CY, bool PAIR, int RS = 0> static void add_x(Ops& o) {
        if constexpr (T > 16 && N > 64) return;    // wide tiles only for small N
        if constexpr (PAIR && !pair_ok<T>()) return;
        if constexpr (RS != 0 && !radix_plan_new(N, RS)) return;
        if constexpr (x_ok<T>()) {
            int& n = push(o, P_XINV, Variant{T, PAIR, 0, CY, RS, 0});
            o.xinv[n++] = &xinv<T, CY, PAIR, RS>;
        }
        if constexpr (xr_ok<T, RS>()) {
            int& k = push(o, P_XSTAGE, Variant{T, PAIR, 0, CY, RS, 0});
            o.xstage[k] = &xstage<T, CY, PAIR, RS>;
            o.xstage_groups[k++] = x_groups<T>();
        }
    }
    // the RHS pass alone (independent of the curl placement)
    template <int T, bool PAIR, int RS = 0> static void add_xr(Ops& o) {
        if constexpr (T > 16 && N > 64) return;
        if constexpr (PAIR && !pair_ok<T>()) return;
        if constexpr (RS != 0 && !radix_plan_new(N, RS)) return;
        if constexpr (xr_ok<T, RS>()) {
            int& n = push(o, P_XRHS, Variant{T, PAIR, 0, -1, RS, 0});
            o.xrhs[n] = &xrhs<T, PAIR, RS>;
            o.xrhs_groups[n++] = x_groups<T>();
        }
    }
    // inverse y pass forming the vorticity (curl in y, 8 per thread)
    template <int T, bool PAIR = false, int RS = 0> static void add_ycurl(Ops& o) {
        if constexpr (PAIR && !ypair_ok<T>()) return;
        if constexpr (RS != 0 && !radix_plan_new(N, RS)) return;
        if constexpr (T > 0 && y_ok<T, 8, true, RS>()) {
            int& n = push(o, P_YINV6, Variant{T, PAIR, 8, 1, RS, 0});
            o.yinv6[n++] = &yinv_curl<T, PAIR, RS>;
        }
    }
    // inverse y pass of the six fields the x pass wrote (curl in x)
    template <int T, int YE, bool PAIR = false, int RS = 0> static void add_yinv(Ops& o) {
        if constexpr (PAIR && !ypair_ok<T>()) return;
        if constexpr (RS != 0 && !radix_plan_new(N, RS)) return;
        if constexpr (T > 0 && y_ok<T, YE, false, RS>()) {
            int& n = push(o, P_YINV6, Variant{T, PAIR, YE, 0, RS, 0});
            o.yinv6[n++] = &ypass<T, +1, 6, YE, PAIR, RS>;
        }
    }
    template <int T, int YE, bool PAIR = false, int RS = 0> static void add_yfwd(Ops& o) {
        if constexpr (PAIR && !ypair_ok<T>()) return;
        if constexpr (RS != 0 && !radix_plan_new(N, RS)) return;
        if constexpr (T > 0 && y_ok<T, YE, false, RS>()) {
            int& n = push(o, P_YFWD3, Variant{T, PAIR, YE, -1, RS, 0});
            o.yfwd3[n++] = &ypass<T, -1, 3, YE, PAIR, RS>;
        }
    }
    template <int L, int ZP = 3, int RS = 0> static void add_z(Ops& o) {
        if constexpr (RS != 0 && !radix_plan_new(N, RS)) return;
        if constexpr (z_ok<L, ZP, RS>()) {
            int& n = push(o, P_ZCROSS, Variant{L, 0, 0, -1, RS, ZP ? 1 << ZP : 0});
            o.zcross[n++] = &zcross<L, ZP, RS>;
        }
    }
    // The default shape of every pass (as make() picks it) with radix plan RS.
    static constexpr int ZD = (N >= 1024 ? 1 : (N == 256 ? 8 : 4)) > 64 / G ? (N >= 1024 ? 1 : (N == 256 ? 8 : 4))
                                                                              : 64 / G;
    static constexpr int YEF = (std::is_same_v<R, float> && N == 512) ? 16 : YE0;
    template <int RS> static void add_radix_plan(Ops& o) {
        constexpr bool XP = N >= 1024 && pair_ok<XD>();
        add_x<XD, CY0, XP, RS>(o);
        add_xr<XD, XP, RS>(o);
        if constexpr (CY0) add_ycurl<y_default_width<8>(), false, RS>(o);
        else add_yinv<y_default_width<YE0>(), YE0, false, RS>(o);
        add_yfwd<y_default_width<YEF>(), YEF, false, RS>(o);
        add_z<ZD, 3, RS>(o);
    }
    // Radix plan 0 and the standard z-pass pad: the variants a default or
    // reproducible plan is made of.
    static bool reference_shape(int p, const Variant& d) {
        return d.rs == 0 && d.pad == (p == P_ZCROSS ? 8 : 0);
    }
    static int threads_per_line(int p, const Variant& d) {
        if (p == P_YINV6 || p == P_YFWD3) return N / d.ye;
        return p == P_ZCROSS ? G : GX;
    }
    // index of the widest variant of pass p not wider than w whose
    // workgroup has at most MAXT threads and that matches the schedule
    // (curl placement cy, y elements ye, XCD pairing preferred as `pair`);
    // -1 if none
    static int pick(const Ops& o, int p, int w, int cy, int ye, int pair) {
        int best = -1;
        for (int v = 0; v < o.nvar[p]; ++v) {
            const Variant& d = o.var[p][v];
            if (!reference_shape(p, d)) continue;
            if (d.width > w || threads_per_line(p, d) * d.width > MAXT) continue;
            if (d.cy >= 0 && d.cy != cy) continue;
            if (d.ye > 0 && !(p == P_YINV6 && cy == 1) && d.ye != ye) continue;
            if (best < 0) { best = v; continue; }
            const Variant& b = o.var[p][best];
            if (d.width > b.width || (d.width == b.width && d.pair == pair && b.pair != pair)) best = v;
        }
        return best;
    }
    static Ops make() {
        Ops o{};
        o.N = N;
        o.real_size = sizeof(R);
        o.fs = Lay<R, N>::FS;
        o.tw_count = tw_total(N) > 0 ? tw_total(N) : 1;
        for (int r = 0; r < NRS; ++r) o.tw_base[r] = tw_base(N, r);
        if constexpr (CY0) {
            // below 1024: the vorticity in the y pass at every width; the
            // six-field x pass (curl in x) at the default width, with the
            // plain inverse y pass at 8, 16 and 32 elements per thread
            add_x<4, true, false>(o); add_x<8, true, false>(o); add_x<16, true, false>(o); add_x<32, true, false>(o);
            add_x<4, true, true>(o); add_x<8, true, true>(o);
            add_x<XD, false, false>(o);
            add_ycurl<4>(o); add_ycurl<8>(o); add_ycurl<16>(o); add_ycurl<32>(o);
            add_ycurl<4, true>(o); add_ycurl<8, true>(o);
            add_yinv<y_default_width<8>(), 8>(o);
            add_yinv<y_default_width<16>(), 16>(o);
            add_yinv<y_default_width<32>(), 32>(o);
            add_yfwd<4, 8>(o); add_yfwd<8, 8>(o); add_yfwd<16, 8>(o); add_yfwd<32, 8>(o);
            add_yfwd<4, 8, true>(o); add_yfwd<8, 8, true>(o);
            add_yfwd<y_default_width<16>(), 16>(o);
            add_yfwd<y_default_width<32>(), 32>(o);
        } else {
            // 1024: six-field x pass, long y slices
            add_x<4, false, false>(o); add_x<8, false, false>(o); add_x<16, false, false>(o);
            add_x<4, false, true>(o); add_x<8, false, true>(o);
            add_yinv<4, YE0>(o); add_yinv<8, YE0>(o); add_yinv<16, YE0>(o); add_yinv<32, YE0>(o);
            add_yfwd<4, YE0>(o); add_yfwd<8, YE0>(o); add_yfwd<16, YE0>(o); add_yfwd<32, YE0>(o);
            add_yinv<4, YE0, true>(o); add_yinv<8, YE0, true>(o);
            add_yfwd<4, YE0, true>(o); add_yfwd<8, YE0, true>(o);
            // the five-field schedule at the default x width (64-byte rows):
            // the combining y pass holds 8 values per thread, 64-byte rows too
            add_x<XD, true, false>(o); add_x<XD, true, true>(o);
            add_ycurl<XD, false>(o); add_ycurl<XD, true>(o);
        }
        add_xr<4, false>(o); add_xr<8, false>(o); add_xr<16, false>(o); add_xr<32, false>(o);
        add_xr<4, true>(o); add_xr<8, true>(o);
        add_z<1>(o); add_z<2>(o); add_z<4>(o); add_z<8>(o);
        add_z<16>(o); add_z<32>(o); add_z<64>(o); add_z<128>(o);
        // LDS pad of the z pass at its default width: none, every 4 and
        // every 16 elements (bitwise neutral: only shared-memory addresses)
        add_z<ZD, 0>(o); add_z<ZD, 2>(o); add_z<ZD, 4>(o);
        // the other radix plans at the default shapes (not bitwise
        // identical to plan 0: chosen only by a tuning in fastest mode)
        add_radix_plan<1>(o);
        add_radix_plan<2>(o);
        // defaults, the fastest measured on MI355X at 256^3, 512^3 and
        // 1024^3: 128-byte row segments in the x and y passes, four z lines
        // per workgroup (eight for N = 256, one for N = 1024); for small N,
        // at least one full 64-lane wave per workgroup.  At 1024 the x
        // passes (64-byte rows) take the XCD-grouped tile order (stage pass
        // 41.2 -> 38.1 ms FP64, 24.4 -> 22.3 ms FP32); the FP32 forward y
        // pass at 512 holds 16 values per thread (0.638 -> 0.583 ms).
        const int xw = want_width(G), yw = want_width(G);
        const int cy = CY0 ? 1 : 0, pair = N >= 1024 ? 1 : 0;
        const int ye = (std::is_same_v<R, float> && N == 512) ? 16 : YE0;
        o.def[P_XINV] = pick(o, P_XINV, xw, cy, ye, pair);
        o.def[P_XRHS] = pick(o, P_XRHS, xw, cy, ye, pair);
        o.def[P_XSTAGE] = pick(o, P_XSTAGE, xw, cy, ye, pair);
        o.def[P_YINV6] = pick(o, P_YINV6, yw, cy, ye, pair);
        o.def[P_YFWD3] = pick(o, P_YFWD3, yw, cy, ye, pair);
        o.def[P_ZCROSS] = pick(o, P_ZCROSS, std::max(N >= 1024 ? 1 : (N == 256 ? 8 : 4), 64 / G), cy, ye, pair);
        o.xinv3 = &xinv3;
        o.yinv3 = &yinv3;
        o.yfwd3s = &yfwd3s;
        o.xfwd3 = &xfwd3;
        o.zr2c = &zr2c;
        o.zc2r = &zc2r;
        o.layout = &layout;
        o.diag_partial = &diag_partial;
        o.ic_physical = &ic_physical;
        o.ic_random = &ic_random;
        o.scale = &scale;
        if constexpr (std::is_same_v<R, float> && N >= 64) {
            o.ymfma_inv6[0] = &ymfma<+1, 6, false>;
            if constexpr (CY0) o.ymfma_inv6[1] = &ymfma<+1, 6, true>;
            o.ymfma_fwd3 = &ymfma<-1, 3, false>;
        }
        return o;
    }
    static const Ops* table() {
        static const Ops ops = make();
        return &ops;
    }
};

// The table of one (R, N) pair, compiled in a translation unit of its own
// (dns_inst.hip built once per pair) so that the pairs build in parallel.
#if defined(DNS_INST_REAL) && defined(DNS_INST_N)
template <> const Ops* ops_table<DNS_INST_REAL, DNS_INST_N>() { return Impl<DNS_INST_REAL, DNS_INST_N>::table(); }
#endif

}  // namespace dns
