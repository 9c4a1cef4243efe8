// Launchers of the kernel templates for one real type; included by the
// per-precision translation units, which instantiate every supported N.
#pragma once

#include <cmath>

#include "dns_kernels.hpp"
#include "dns_ops.hpp"

namespace dns {

template <typename R, int N> struct Impl {
    using K = Cfg<R, N>;
    using C = cx<R>;

    static void xinv(const void* U, void* W, const void* tw, bool curl, hipStream_t s) {
        if (curl)
            hipLaunchKernelGGL((k_xinv<R, N, true>), dim3(K::X_TILES), dim3(K::XTHREADS), 0, s,
                               (const C*)U, (C*)W, (const C*)tw);
        else
            hipLaunchKernelGGL((k_xinv<R, N, false>), dim3(K::X_TILES), dim3(K::XTHREADS), 0, s,
                               (const C*)U, (C*)W, (const C*)tw);
    }
    template <int DIR, int NF>
    static void ypass(void* W, const void* tw, hipStream_t s) {
        hipLaunchKernelGGL((k_yline<R, N, DIR, NF>), dim3(K::Y_TILES), dim3(K::YTHREADS), 0, s,
                           (C*)W, (const C*)tw);
        hipLaunchKernelGGL((k_yline_nyq<R, N, DIR, NF>), dim3(N / K::LY), dim3(K::NYTHREADS), 0, s,
                           (C*)W, (const C*)tw);
    }
    static void yinv6(void* W, const void* tw, hipStream_t s) { ypass<+1, 6>(W, tw, s); }
    static void yinv3(void* W, const void* tw, hipStream_t s) { ypass<+1, 3>(W, tw, s); }
    static void yfwd3(void* W, const void* tw, hipStream_t s) { ypass<-1, 3>(W, tw, s); }
    static void zcross(void* W, const void* tw, hipStream_t s) {
        const R scale = (R)std::ldexp(1.0, -6 * ilog2(N));
        hipLaunchKernelGGL((k_zcross<R, N>), dim3((N * N) / K::LZ), dim3(K::ZTHREADS), 0, s,
                           (C*)W, (const C*)tw, scale);
    }
    static void xrhs(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                     hipStream_t s) {
        hipLaunchKernelGGL((k_xrhs<R, N>), dim3(K::X_TILES), dim3(K::XTHREADS), 0, s,
                           (const C*)W, (C*)U0, (C*)U1, (C*)Us, (const C*)tw, a);
    }
    static void xfwd(const void* W, void* U, const void* tw, hipStream_t s) {
        hipLaunchKernelGGL((k_xfwd<R, N>), dim3(K::X_TILES), dim3(K::XTHREADS), 0, s,
                           (const C*)W, (C*)U, (const C*)tw);
    }
    static void zr2c(const void* u, void* W, const void* tw, hipStream_t s) {
        hipLaunchKernelGGL((k_zr2c<R, N>), dim3((N * N) / K::LZ), dim3(K::ZTHREADS), 0, s,
                           (const R*)u, (C*)W, (const C*)tw);
    }
    static void zc2r(const void* W, void* u, const void* tw, hipStream_t s) {
        const R scale = (R)std::ldexp(1.0, -3 * ilog2(N));
        hipLaunchKernelGGL((k_zc2r<R, N>), dim3((N * N) / K::LZ), dim3(K::ZTHREADS), 0, s,
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

    static const Ops* table() {
        static const Ops ops = {N, sizeof(R), K::X_TILES, tw_size(N) > 0 ? tw_size(N) : 1,
                                &xinv, &yinv6, &zcross, &yfwd3, &xrhs,
                                &yinv3, &xfwd, &zr2c, &zc2r, &layout, &diag_partial};
        return &ops;
    }
};

template <typename R> const Ops* ops_for(int N) {
    switch (N) {
        case 8: return Impl<R, 8>::table();
        case 16: return Impl<R, 16>::table();
        case 32: return Impl<R, 32>::table();
        case 64: return Impl<R, 64>::table();
        case 128: return Impl<R, 128>::table();
        case 256: return Impl<R, 256>::table();
        case 512: return Impl<R, 512>::table();
        case 1024: return Impl<R, 1024>::table();
        default: return nullptr;
    }
}

}  // namespace dns
