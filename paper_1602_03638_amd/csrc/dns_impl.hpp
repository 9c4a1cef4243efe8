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

    // Feasibility of a workgroup shape: at most 1024 threads and the LDS limit.
    // (lines of more than 8 elements per thread need more than the 128
    // registers a 1024-thread workgroup leaves each thread)
    template <int T> static constexpr bool x_ok() {
        return T <= N && GX * T <= (x_elems<R>(N) > 8 ? 512 : 1024) && (size_t)T * N * CB <= LDS_LIMIT;
    }
    // The RHS/RK4 passes hold three lines plus state per thread: in FP64
    // their 1024-thread shapes (128 registers per thread) only spill.
    template <int T> static constexpr bool xr_ok() {
        return x_ok<T>() && (sizeof(R) == 4 || GX * T <= 512) &&
               (size_t)T * N * CB + 2 * 8 * (size_t)GX * T <= LDS_LIMIT;
    }
    static constexpr int GY = N / y_elems<R>(N);   // threads per y line
    template <int T> static constexpr bool y_ok() {
        return T <= N / 2 && GY * T <= 1024 &&
               ((size_t)T * N + (y_twiddles_in_lds<R>(N) || curl_in_y<R>(N) ? (size_t)tw_size(N) : 0)) * CB <=
                   LDS_LIMIT;
    }
    // z shapes: at least 16 threads, and up to 128 threads for small N
    template <int L> static constexpr bool z_ok() {
        return L <= N * N && G * L <= 1024 && G * L >= 16 && L <= (128 / G > 8 ? 128 / G : 8) &&
               (size_t)L * padded_line<N>(true) * CB + (size_t)tw_size(N) * CB <= LDS_LIMIT;
    }
    template <int T> static constexpr int x_groups() { return XCOLS / T + N / T; }

    // ---- pass launchers ----------------------------------------------------
    template <int T> static void xinv(const void* U, void* W, const void* tw, const Batch& b, hipStream_t s) {
        hipLaunchKernelGGL((k_xinv_curl<R, N, T>), dim3(x_groups<T>(), b.members), dim3(GX * T), 0, s,
                           (const C*)U, (C*)W, (const C*)tw, b.sst, b.wst);
    }
    template <int T, int DIR, int NF> static void ypass(void* W, const void* tw, const Batch& b, hipStream_t s) {
        hipLaunchKernelGGL((k_yline<R, N, T, DIR, NF>), dim3(y_tiles<R, N, T>(), b.members), dim3(GY * T), 0, s,
                           (C*)W, (const C*)tw, b.wst);
    }
    template <int DIR, int NF>
    static void ymfma(void* W, const void* tw, const void* roots, const void* tw2, const Batch& b, hipStream_t s) {
        if constexpr (std::is_same_v<R, float> && N >= 64) {
            hipLaunchKernelGGL((k_yline_mfma<N, DIR, NF>), dim3(MfmaY<N>::TILES, b.members), dim3(MfmaY<N>::NT), 0, s,
                               (C*)W, (const C*)tw, (const C*)roots, (const C*)tw2, b.wst);
        }
    }
    // inverse y pass of a stage: the six fields for the z pass, with the
    // vorticity combinations formed from the x pass's five outputs
    template <int T> static void yinv6(void* W, const void* tw, const Batch& b, hipStream_t s) {
        if constexpr (curl_in_y<R>(N))
            hipLaunchKernelGGL((k_yinv_curl<R, N, T>), dim3(y_tiles<R, N, T>(), b.members), dim3(GY * T), 0, s,
                               (C*)W, (const C*)tw, b.wst);
        else
            ypass<T, +1, 6>(W, tw, b, s);
    }
    template <int T> static void yfwd3(void* W, const void* tw, const Batch& b, hipStream_t s) {
        ypass<T, -1, 3>(W, tw, b, s);
    }
    template <int L> static void zcross(void* W, const void* tw, const Batch& b, hipStream_t s) {
        const R scale = (R)std::ldexp(1.0, -6 * ilog2(N));
        hipLaunchKernelGGL((k_zcross<R, N, L>), dim3((N * N) / L, b.members), dim3(G * L), 0, s, (C*)W,
                           (const C*)tw, scale, b.wst);
    }
    template <int T, int ST>
    static void xrhs_st(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                        const Batch& b, hipStream_t s) {
        hipLaunchKernelGGL((k_xrhs<R, N, T, ST>), dim3(x_groups<T>(), b.members), dim3(GX * T), 0, s,
                           (const C*)W, (C*)U0, (C*)U1, (C*)Us, (const C*)tw, a, b.sst, b.wst);
    }
    template <int T>
    static void xrhs(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                     const Batch& b, hipStream_t s) {
        switch (a.stage) {
            case 0: xrhs_st<T, 0>(W, U0, U1, Us, tw, a, b, s); break;
            case 1: xrhs_st<T, 1>(W, U0, U1, Us, tw, a, b, s); break;
            case 2: xrhs_st<T, 2>(W, U0, U1, Us, tw, a, b, s); break;
            case 3: xrhs_st<T, 3>(W, U0, U1, Us, tw, a, b, s); break;
            case 4: xrhs_st<T, 4>(W, U0, U1, Us, tw, a, b, s); break;
            default: xrhs_st<T, -1>(W, U0, U1, Us, tw, a, b, s); break;
        }
    }

    template <int T, int ST>
    static void xstage_st(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                          const Batch& b, hipStream_t s) {
        hipLaunchKernelGGL((k_xstage<R, N, T, ST>), dim3(x_groups<T>(), b.members), dim3(GX * T), 0, s,
                           (C*)W, (C*)U0, (C*)U1, (C*)Us, (const C*)tw, a, b.sst, b.wst);
    }
    template <int T>
    static void xstage(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                       const Batch& b, hipStream_t s) {
        switch (a.stage) {
            case 0: xstage_st<T, 0>(W, U0, U1, Us, tw, a, b, s); break;
            case 1: xstage_st<T, 1>(W, U0, U1, Us, tw, a, b, s); break;
            case 2: xstage_st<T, 2>(W, U0, U1, Us, tw, a, b, s); break;
            case 3: xstage_st<T, 3>(W, U0, U1, Us, tw, a, b, s); break;
            default: xstage_st<T, 4>(W, U0, U1, Us, tw, a, b, s); break;
        }
    }

    // ---- standalone transforms (fixed shapes) -------------------------------
    // FP64 lines of 8 complex doubles per thread need more than the 128
    // registers a 1024-thread workgroup leaves each thread: at most 512.
    static constexpr int MAXT = sizeof(R) == 8 ? 512 : 1024;
    template <int T> static constexpr bool xs_ok() { return x_ok<T>() && GX * T <= MAXT; }
    template <int T> static constexpr bool ys_ok() { return y_ok<T>() && GY * T <= MAXT; }
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
    static void yinv3(void* W, const void* tw, hipStream_t s) { ypass<YS, +1, 3>(W, tw, Batch{1, 0, 0}, s); }
    static void yfwd3s(void* W, const void* tw, hipStream_t s) { ypass<YS, -1, 3>(W, tw, Batch{1, 0, 0}, s); }
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
    template <int T> static void add_x(Ops& o) {
        if constexpr (T > 16 && N > 64) return;    // wide tiles only for small N
        if constexpr (x_ok<T>()) {
            int& n = o.nvar[P_XINV];
            o.xinv[n] = &xinv<T>;
            o.width[P_XINV][n++] = T;
        }
        if constexpr (xr_ok<T>()) {
            int& n = o.nvar[P_XRHS];
            o.xrhs[n] = &xrhs<T>;
            o.xrhs_groups[n] = x_groups<T>();
            o.width[P_XRHS][n++] = T;
            int& k = o.nvar[P_XSTAGE];
            o.xstage[k] = &xstage<T>;
            o.xstage_groups[k] = x_groups<T>();
            o.width[P_XSTAGE][k++] = T;
        }
    }
    template <int T> static void add_y(Ops& o) {
        if constexpr (y_ok<T>()) {
            int& n = o.nvar[P_YINV6];
            o.yinv6[n] = &yinv6<T>;
            o.yfwd3[n] = &yfwd3<T>;
            o.width[P_YINV6][n] = T;
            o.width[P_YFWD3][n] = T;
            ++n;
            o.nvar[P_YFWD3] = n;
        }
    }
    template <int L> static void add_z(Ops& o) {
        if constexpr (z_ok<L>()) {
            int& n = o.nvar[P_ZCROSS];
            o.zcross[n] = &zcross<L>;
            o.width[P_ZCROSS][n++] = L;
        }
    }
    // index of the widest variant of pass p not wider than w whose
    // workgroup has at most MAXT threads
    static int pick(const Ops& o, int p, int w) {
        const int per_line = (p == P_YINV6 || p == P_YFWD3) ? GY : (p == P_ZCROSS ? G : GX);
        int best = 0;
        for (int v = 0; v < o.nvar[p]; ++v)
            if (o.width[p][v] <= w && per_line * o.width[p][v] <= MAXT) best = v;
        return best;
    }
    static Ops make() {
        Ops o{};
        o.N = N;
        o.real_size = sizeof(R);
        o.fs = Lay<R, N>::FS;
        o.tw_count = tw_size(N) > 0 ? tw_size(N) : 1;
        add_x<4>(o); add_x<8>(o); add_x<16>(o); add_x<32>(o);
        add_y<4>(o); add_y<8>(o); add_y<16>(o); add_y<32>(o);
        add_z<1>(o); add_z<2>(o); add_z<4>(o); add_z<8>(o);
        add_z<16>(o); add_z<32>(o); add_z<64>(o); add_z<128>(o);
        // defaults: 128-byte row segments in the x and y passes, four z lines
        // per workgroup (eight for N = 256, two for N = 1024), the fastest
        // measured on MI355X at 256^3, 512^3 and 1024^3; for small N, at
        // least one full 64-lane wave per workgroup
        const int wave = 64 / G;
        const int xw = std::max((int)(128 / CB), wave), yw = xw;
        o.def[P_XINV] = pick(o, P_XINV, xw);
        o.def[P_XRHS] = pick(o, P_XRHS, xw);
        o.def[P_XSTAGE] = pick(o, P_XSTAGE, xw);
        o.def[P_YINV6] = pick(o, P_YINV6, yw);
        o.def[P_YFWD3] = pick(o, P_YFWD3, yw);
        o.def[P_ZCROSS] = pick(o, P_ZCROSS, std::max(N >= 1024 ? 2 : (N == 256 ? 8 : 4), wave));
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
            o.ymfma_inv6 = &ymfma<+1, 6>;
            o.ymfma_fwd3 = &ymfma<-1, 3>;
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
