// HIP kernels of one time-integration stage of the pseudo-spectral solver
// and of the standalone 3D real transforms (templated on real type R and
// grid size N).
//
// One stage (Sec. 2 eq. NSfinal, Sec. 3.1 computeRHS) runs as five passes
// over HBM-resident half-spectrum fields in the padded internal layout of
// dns_common.hpp:
//   1. k_xinv_curl u_hat -> inverse x FFTs of u_hat and of the kx products
//                  that omega_hat = i k x u_hat needs (5 fields: U, V, W,
//                  F(kx v_hat), F(kx w_hat); at N = 1024 the 6 fields
//                  u, v, w, omega with the combinations formed here)
//   2. k_yinv_curl forms omega_hat from the 5 fields, then the inverse y FFT
//                  of all 6 (in place; the last workgroups take the
//                  kz = N/2 plane); k_yline<+1, 6> at N = 1024
//   3. k_zcross    per (x, y) line: 6 inverse real z FFTs, u x omega in
//                  registers, 3 forward real z FFTs; physical fields never
//                  leave the chip
//   4. k_yline     forward y FFT of the 3 fields
//   5. k_xrhs      forward x FFT, dealias mask, pressure projection,
//                  viscous term and the RK4 (or forward Euler) stage update
//                  (+ diagnostics)
// In the default schedule k_xstage runs pass 5 fused with pass 1 of the next
// stage.  The FP32 y passes can instead run k_yline_mfma (dns_mfma.hpp).
#pragma once

#include "fft_device.hpp"

namespace dns {

__device__ __forceinline__ int kfreq(int i, int n) { return i < n / 2 ? i : i - n; }

// Column c of the x pass: c < N*N/2 is (iy, iz) = (c / (N/2), c % (N/2)) of
// the main block; c >= N*N/2 is iy = c - N*N/2 of the Nyquist plane.  A
// workgroup's columns lie in one of the two blocks (tile widths divide
// both), so the kernels branch once on the block and the row stride is a
// compile-time constant, which lets the compiler see that different rows
// never alias.
template <typename R, int N, bool NYQ> struct XCol {
    using L = Lay<R, N>;
    static constexpr unsigned RS = NYQ ? (unsigned)N : L::XP;   // offset between rows
    unsigned base;   // offset of row 0 in a field
    int ky, kz;
    __device__ __forceinline__ explicit XCol(int c) {
        constexpr int HC = N * (N / 2);
        if constexpr (!NYQ) {
            const int iy = c / (N / 2);
            kz = c % (N / 2);
            ky = kfreq(iy, N);
            base = (unsigned)iy * L::ZP + (unsigned)kz;
        } else {
            const int iy = c - HC;
            base = (unsigned)L::MAIN + (unsigned)iy;
            ky = kfreq(iy, N);
            kz = N / 2;
        }
    }
    __device__ __forceinline__ unsigned at(int row) const { return base + (unsigned)row * RS; }
};

// Element (row g + m G) of field f of the x tile, addressed as a uniform
// base (field + block start + m G rows, kept in scalar registers) plus one
// per-thread 32-bit byte offset (column + g rows, relative to its block)
// shared by every field and row, so that a thread holds one address
// register instead of one per element.  Relative to the block start the
// offset stays below 2^32 bytes for every supported N and precision.
template <typename R, int N, bool NYQ>
struct XAddr {
    using C = cx<R>;
    static constexpr int G = N / x_elems<R>(N);
    static constexpr unsigned RS = XCol<R, N, NYQ>::RS;
    static constexpr size_t BLOCK = NYQ ? Lay<R, N>::MAIN : 0;   // element offset of the block
    unsigned tb;                                                  // byte offset of (column, row g)
    __device__ __forceinline__ XAddr(const XCol<R, N, NYQ>& col, int g)
        : tb(((unsigned)(col.base - BLOCK) + (unsigned)g * RS) * (unsigned)sizeof(C)) {}
    static constexpr bool S = stream_io<R>(N);
    __device__ __forceinline__ GRef<C, S> operator()(C* F, int m) const {
        return {reinterpret_cast<C*>(reinterpret_cast<char*>(F + BLOCK + (size_t)m * G * RS) + tb)};
    }
    __device__ __forceinline__ C operator()(const C* F, int m) const {
        return gload<C, S>(reinterpret_cast<const C*>(reinterpret_cast<const char*>(F + BLOCK + (size_t)m * G * RS) + tb));
    }
};

static_assert((size_t)Lay<double, 1024>::ZP * 1024 + (size_t)(1024 / 8) * Lay<double, 1024>::XP * 16 <
                  (size_t(1) << 32),
              "x-tile byte offsets must fit 32 bits");
static_assert(Lay<double, 1024>::FS < (size_t(1) << 32) && Lay<float, 1024>::FS < (size_t(1) << 32),
              "element offsets within a field must fit 32 bits");

// Number of x-pass workgroups of width T over the main block.
template <int N, int T> constexpr int x_main_tiles() { return (N * (N / 2)) / T; }

// ---------------------------------------------------------------------------
// Pass 1: inverse x transforms for the vorticity omega_hat = i k x u_hat
// (Sec. 3.1 Curl listing):
//   omega_x = i (ky w - kz v), omega_y = i (kz u - kx w), omega_z = i (kx v - ky u).
// ky and kz are constant along an x line, so by linearity only kx v_hat and
// kx w_hat need transforms of their own.  Output fields at W (F = inverse x
// transform), see curl_in_y:
//   curl_in_y:  U, V, W, F(kx v_hat), F(kx w_hat); the inverse y pass
//               (k_yinv_curl) forms the combinations with ky and kz;
//   otherwise:  U, V, W, omega_x = i (ky W - kz V),
//               omega_y = i (kz U - F(kx w_hat)), omega_z = i (F(kx v_hat) - ky U).
// T lines (consecutive columns) per workgroup.  CY selects where the
// vorticity combinations are formed (curl in y: five fields; else six).
// ---------------------------------------------------------------------------
// Inverse x transforms of the velocity held in v[3] (x-spectral), written to
// W as above.  Shared by the first stage's pass and the fused stage pass.
template <typename R, int N, int T, bool NYQ, bool CY, int RS = 0>
__device__ __forceinline__ void xinv_curl_store(cx<R> (&v)[3][x_elems<R>(N)],
                                                cx<R>* __restrict__ W, const XAddr<R, N, NYQ>& A, cx<R>* lt,
                                                const cx<R>* twl, int g, int iky, int ikz) {
    constexpr int E = x_elems<R>(N), G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    if constexpr (!CY) {
        // the six fields u, v, w, omega (combinations formed here)
        const R ky = (R)iky, kz = (R)ikz;
        cx<R> b[E];
        fft_line<R, N, E, +1, true, 0, RS>(v[0], lt, T, twl, g);        // U
#pragma unroll
        for (int m = 0; m < E; ++m) {
            A(W, m) = v[0][m];
            b[m] = cscale<R>(v[1][m], (R)kfreq(g + m * G, N));
        }
        fft_line<R, N, E, +1, true, 0, RS>(b, lt, T, twl, g);           // F(kx v_hat)
#pragma unroll
        for (int m = 0; m < E; ++m) A(W + 5 * FS, m) = cmuli<R>(csub<R>(b[m], cscale<R>(v[0][m], ky)));
        fft_line<R, N, E, +1, true, 0, RS>(v[1], lt, T, twl, g);        // V
#pragma unroll
        for (int m = 0; m < E; ++m) {
            A(W + FS, m) = v[1][m];
            b[m] = cscale<R>(v[2][m], (R)kfreq(g + m * G, N));
        }
        fft_line<R, N, E, +1, true, 0, RS>(b, lt, T, twl, g);           // F(kx w_hat)
#pragma unroll
        for (int m = 0; m < E; ++m) A(W + 4 * FS, m) = cmuli<R>(csub<R>(cscale<R>(v[0][m], kz), b[m]));
        fft_line<R, N, E, +1, true, 0, RS>(v[2], lt, T, twl, g);        // W
#pragma unroll
        for (int m = 0; m < E; ++m) {
            A(W + 2 * FS, m) = v[2][m];
            A(W + 3 * FS, m) = cmuli<R>(csub<R>(cscale<R>(v[2][m], ky), cscale<R>(v[1][m], kz)));
        }
        return;
    }
    // at most three lines live: U is transformed and stored before the
    // first kx product is formed
    cx<R> b[E];
    fft_line<R, N, E, +1, true, 0, RS>(v[0], lt, T, twl, g);            // U
#pragma unroll
    for (int m = 0; m < E; ++m) {
        A(W, m) = v[0][m];
        b[m] = cscale<R>(v[1][m], (R)kfreq(g + m * G, N));
    }
    fft_line<R, N, E, +1, true, 0, RS>(b, lt, T, twl, g);               // F(kx v_hat)
#pragma unroll
    for (int m = 0; m < E; ++m) A(W + 3 * FS, m) = b[m];
    fft_line<R, N, E, +1, true, 0, RS>(v[1], lt, T, twl, g);            // V
#pragma unroll
    for (int m = 0; m < E; ++m) A(W + FS, m) = v[1][m];
#pragma unroll
    for (int m = 0; m < E; ++m) b[m] = cscale<R>(v[2][m], (R)kfreq(g + m * G, N));
    fft_line<R, N, E, +1, true, 0, RS>(b, lt, T, twl, g);               // F(kx w_hat)
#pragma unroll
    for (int m = 0; m < E; ++m) A(W + 4 * FS, m) = b[m];
    fft_line<R, N, E, +1, true, 0, RS>(v[2], lt, T, twl, g);            // W
#pragma unroll
    for (int m = 0; m < E; ++m) A(W + 2 * FS, m) = v[2][m];
}

template <typename R, int N, int T, bool NYQ, bool CY, int RS = 0>
__device__ __forceinline__ void xinv_curl_tile(const cx<R>* __restrict__ U, cx<R>* __restrict__ W,
                                               cx<R>* lds, const cx<R>* twl, int tile) {
    constexpr int E = x_elems<R>(N), G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    const int t = threadIdx.x % T, g = threadIdx.x / T;
    const XCol<R, N, NYQ> col(tile * T + t);
    const XAddr<R, N, NYQ> A(col, g);
    cx<R> v[3][E];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int m = 0; m < E; ++m) v[f][m] = A(U + f * FS, m);
    xinv_curl_store<R, N, T, NYQ, CY, RS>(v, W, A, lds + t, twl, g, col.ky, col.kz);
}

template <typename R, int N, int T, bool CY, bool PAIR, int RS = 0>
__global__ __launch_bounds__(N / x_elems<R>(N) * T)
void k_xinv_curl(const cx<R>* __restrict__ U, cx<R>* __restrict__ W, const cx<R>* __restrict__ tw, size_t sst,
                 size_t wst) {
    U += blockIdx.y * sst;
    W += blockIdx.y * wst;
    __shared__ cx<R> lds[T * N];
    __shared__ cx<R> twl[tw_size(N, RS) > 0 ? tw_size(N, RS) : 1];
    load_twiddles<R, N, RS>(twl, tw);
    const int tile = x_tile<PAIR ? line_group<R, T>() : 1>((int)blockIdx.x, x_main_tiles<N, T>());
    if (tile < x_main_tiles<N, T>()) xinv_curl_tile<R, N, T, false, CY, RS>(U, W, lds, twl, tile);
    else xinv_curl_tile<R, N, T, true, CY, RS>(U, W, lds, twl, tile);
}

// Plain inverse (DIR = +1) or forward (DIR = -1) x transform of NF fields
// from S into D (used by the standalone 3D transforms).
template <typename R, int N, int T, int DIR, int NF, bool NYQ>
__device__ __forceinline__ void xplain_tile(const cx<R>* __restrict__ S, cx<R>* __restrict__ D,
                                            const cx<R>* __restrict__ tw, cx<R>* lds) {
    constexpr int E = x_elems<R>(N), G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    const int t = threadIdx.x % T, g = threadIdx.x / T;
    const XCol<R, N, NYQ> col(blockIdx.x * T + t);
#pragma unroll 1
    for (int f = 0; f < NF; ++f) {
        const cx<R>* src = S + f * FS;
        cx<R>* dst = D + f * FS;
        cx<R> a[E];
#pragma unroll
        for (int m = 0; m < E; ++m) a[m] = src[col.at(g + m * G)];
        fft_line<R, N, E, DIR>(a, lds + t, T, tw, g);
#pragma unroll
        for (int m = 0; m < E; ++m) dst[col.at(g + m * G)] = a[m];
    }
}

template <typename R, int N, int T, int DIR, int NF>
__global__ __launch_bounds__(N / x_elems<R>(N) * T)
void k_xplain(const cx<R>* __restrict__ S, cx<R>* __restrict__ D, const cx<R>* __restrict__ tw) {
    __shared__ cx<R> lds[T * N];
    if ((int)blockIdx.x < x_main_tiles<N, T>()) xplain_tile<R, N, T, DIR, NF, false>(S, D, tw, lds);
    else xplain_tile<R, N, T, DIR, NF, true>(S, D, tw, lds);
}

// ---------------------------------------------------------------------------
// Pass 2/4: y transform (direction DIR) of NF fields, in place.
// Main block: a workgroup takes T consecutive iz of one ix; rows iy are one
// row pitch apart, thread (t, g) holds elements g + m G of line t
// (E = y_elems<R>(N) elements per thread, G = N / E).
// Nyquist plane (kz = N/2, the last N/T workgroups): a workgroup takes T
// consecutive ix, whose lines are contiguous; thread (l, g) holds elements
// g + m G of line l, so consecutive threads read consecutive elements.
// ---------------------------------------------------------------------------
// Tile geometry of the y pass (YE elements per thread): the place of
// element m of this thread's line, the line's place in shared memory, and
// the kz of the line.  Element m of a field F sits at F plus a byte offset
// (shared by every field) of the tile's block blk plus this thread's column
// and row off plus m G rows.  Where a field spans less than 4 GiB the whole
// offset is one 32-bit value per element; above (N = 1024), F + blk is
// formed as a uniform 64-bit base (scalar registers) and only off + m G RS
// sizeof(C), below the plane size, is a 32-bit per-thread offset.
template <typename R, int N, int T, bool NYQ, int YE> struct YTile {
    using L = Lay<R, N>;
    using C = cx<R>;
    static constexpr int E = YE, G = N / E;
    static constexpr int ZT = (N / 2) / T;                 // main tiles per ix
    static constexpr unsigned RS = NYQ ? 1u : L::ZP;      // offset between rows iy
    static constexpr int PS = NYQ ? 1 : T;                 // shared-memory stride of a line
    int g, lo, kz;
    size_t blk;        // element offset of the tile's block (uniform)
    unsigned off;      // byte offset of (line, row g) within the block
    __device__ __forceinline__ explicit YTile(int tile) {
        if constexpr (NYQ) {
            g = threadIdx.x % G;
            const int l = threadIdx.x / G;
            blk = L::MAIN + (size_t)tile * T * N;
            off = ((unsigned)l * N + (unsigned)g) * (unsigned)sizeof(C);
            lo = l * N;
            kz = N / 2;
        } else {
            const int t = threadIdx.x % T;
            g = threadIdx.x / T;
            kz = (tile % ZT) * T + t;
            blk = (size_t)(tile / ZT) * L::XP + (size_t)(tile % ZT) * T;
            off = ((unsigned)t + (unsigned)g * RS) * (unsigned)sizeof(C);
            lo = t;
        }
    }
    static constexpr bool WIDE = L::FS * sizeof(C) >= (size_t(1) << 32);
    __device__ __forceinline__ C* ptr(C* F, int m) const {
        const unsigned step = (unsigned)(G * RS * sizeof(C));
        if constexpr (WIDE)
            return reinterpret_cast<C*>(reinterpret_cast<char*>(F + blk) + (off + (unsigned)m * step));
        else
            return reinterpret_cast<C*>(reinterpret_cast<char*>(F) +
                                        ((unsigned)blk * (unsigned)sizeof(C) + off + (unsigned)m * step));
    }
    // element m of the line in the field starting at F
    template <bool NT = stream_io<R>(N)>
    __device__ __forceinline__ GRef<C, NT> el(C* F, int m) const { return {ptr(F, m)}; }
};
static_assert((size_t)Lay<double, 1024>::XP * sizeof(double2) < (size_t(1) << 32),
              "y-tile byte offsets within a plane must fit 32 bits");

template <typename R, int N, int T, int DIR, int NF, bool NYQ, int YE, int RS = 0>
__device__ __forceinline__ void yline_tile(cx<R>* __restrict__ W, const cx<R>* __restrict__ tw, cx<R>* lds,
                                           int tile) {
    using Y = YTile<R, N, T, NYQ, YE>;
    constexpr int E = Y::E;
    constexpr size_t FS = Lay<R, N>::FS;
    constexpr bool TWL = y_twiddles_in_lds(YE);
    // Streaming (non-temporal) accesses only where the next field's loads
    // are issued ahead (FP64, 8 per thread, 256^3 and 512^3: forward pass
    // 1.211 -> 1.182 ms per 512^3 launch); plain elsewhere: without the
    // prefetch the forward pass measured 1.23 -> 1.44 ms streaming, and the
    // standalone inverse's 64-byte FP32 rows 763 -> 1079 us.
    constexpr bool NT = y_prefetch<R>(N, YE) && stream_io<R>(N);
    const Y y(tile);
    if constexpr (!y_prefetch<R>(N, YE)) {
#pragma unroll 1
        for (int f = 0; f < NF; ++f) {
            cx<R>* F = W + f * FS;
            cx<R> a[E];
#pragma unroll
            for (int m = 0; m < E; ++m) a[m] = y.template el<NT>(F, m);
            fft_line<R, N, E, DIR, TWL, 0, RS>(a, lds + y.lo, Y::PS, tw, y.g);
#pragma unroll
            for (int m = 0; m < E; ++m) y.template el<NT>(F, m) = a[m];
        }
    } else {
        // the next field's values are loaded before this field's transform
        cx<R> a[E], b[E];
#pragma unroll
        for (int m = 0; m < E; ++m) a[m] = y.template el<NT>(W, m);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cx<R>* F = W + f * FS;
            if (f + 1 < NF) {
#pragma unroll
                for (int m = 0; m < E; ++m) b[m] = y.template el<NT>(F + FS, m);
            }
            fft_line<R, N, E, DIR, TWL, 0, RS>(a, lds + y.lo, Y::PS, tw, y.g);
#pragma unroll
            for (int m = 0; m < E; ++m) y.template el<NT>(F, m) = a[m];
            if (f + 1 < NF) {
#pragma unroll
                for (int m = 0; m < E; ++m) a[m] = b[m];
            }
        }
    }
}

// Inverse y transforms of the six fields the z pass needs (u, v, w and
// omega = i k x u_hat, Sec. 3.1 Curl listing), formed from the five the
// x pass writes: U, V, W, F(kx v_hat), F(kx w_hat) (x already inverse
// transformed).  ky varies along the line and kz is the line's, so
//   omega_x = i (ky W - kz V),  omega_y = i (kz U - F(kx w_hat)),
//   omega_z = i (F(kx v_hat) - ky U)
// are combined before the (linear) transform.  Outputs overwrite inputs that
// are no longer needed: omega_z -> field 5, omega_y -> 4, u -> 0,
// omega_x -> 3, v -> 1, w -> 2 (each thread reads and writes only its own
// elements).
template <typename R, int N, int T, bool NYQ, int RS = 0>
__device__ __forceinline__ void yinv_curl_tile(cx<R>* __restrict__ W, const cx<R>* twl, cx<R>* lds, int tile) {
    using Y = YTile<R, N, T, NYQ, 8>;
    constexpr int E = Y::E, G = Y::G;
    constexpr size_t FS = Lay<R, N>::FS;
    constexpr bool TWL = true;          // twiddles from shared memory: three lines live
    const cx<R>* tw = twl;
    const Y y(tile);
    const R kz = (R)y.kz;
    cx<R>* lt = lds + y.lo;
    cx<R> *F1 = W + FS, *F2 = W + 2 * FS, *F3 = W + 3 * FS, *F4 = W + 4 * FS, *F5 = W + 5 * FS;
    cx<R> u[E], a[E], b[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        u[m] = y.el(W, m);
        a[m] = y.el(F3, m);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) a[m] = cmuli<R>(csub<R>(a[m], cscale<R>(u[m], (R)kfreq(y.g + m * G, N))));
    fft_line<R, N, E, +1, TWL, 0, RS>(a, lt, Y::PS, tw, y.g);                    // omega_z
#pragma unroll
    for (int m = 0; m < E; ++m) {
        y.el(F5, m) = a[m];
        a[m] = y.el(F4, m);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) a[m] = cmuli<R>(csub<R>(cscale<R>(u[m], kz), a[m]));
    fft_line<R, N, E, +1, TWL, 0, RS>(a, lt, Y::PS, tw, y.g);                    // omega_y
#pragma unroll
    for (int m = 0; m < E; ++m) {
        y.el(F4, m) = a[m];
        a[m] = y.el(F1, m);
        b[m] = y.el(F2, m);
    }
    fft_line<R, N, E, +1, TWL, 0, RS>(u, lt, Y::PS, tw, y.g);                    // u
#pragma unroll
    for (int m = 0; m < E; ++m) {
        y.el(W, m) = u[m];
        u[m] = cmuli<R>(csub<R>(cscale<R>(b[m], (R)kfreq(y.g + m * G, N)), cscale<R>(a[m], kz)));
    }
    fft_line<R, N, E, +1, TWL, 0, RS>(u, lt, Y::PS, tw, y.g);                    // omega_x
#pragma unroll
    for (int m = 0; m < E; ++m) y.el(F3, m) = u[m];
    fft_line<R, N, E, +1, TWL, 0, RS>(a, lt, Y::PS, tw, y.g);                    // v
#pragma unroll
    for (int m = 0; m < E; ++m) y.el(F1, m) = a[m];
    fft_line<R, N, E, +1, TWL, 0, RS>(b, lt, Y::PS, tw, y.g);                    // w
#pragma unroll
    for (int m = 0; m < E; ++m) y.el(F2, m) = b[m];
}

template <typename R, int N, int T> constexpr int y_main_tiles() { return N * ((N / 2) / T); }
template <typename R, int N, int T> constexpr int y_tiles() { return y_main_tiles<R, N, T>() + N / T; }

// PAIR: the tiles of one 128-byte line (rows shorter than 128 bytes) go to
// workgroups of one XCD, as in the x passes (x_tile).
template <typename R, int N, int T, int DIR, int NF, int YE, bool PAIR = false, int RS = 0>
__global__ __launch_bounds__(N / YE * T)
void k_yline(cx<R>* __restrict__ W, const cx<R>* __restrict__ tw, size_t wst) {
    W += blockIdx.y * wst;
    __shared__ cx<R> lds[T * N];
    constexpr bool TWL = y_twiddles_in_lds(YE);
    __shared__ cx<R> twl[TWL && tw_size(N, RS) > 0 ? tw_size(N, RS) : 1];
    const cx<R>* t = tw;
    if constexpr (TWL) {
        load_twiddles<R, N, RS>(twl, tw);
        t = twl;
    }
    const int b = x_tile<PAIR ? line_group<R, T>() : 1>((int)blockIdx.x, y_main_tiles<R, N, T>());
    if (b < y_main_tiles<R, N, T>()) yline_tile<R, N, T, DIR, NF, false, YE, RS>(W, t, lds, b);
    else yline_tile<R, N, T, DIR, NF, true, YE, RS>(W, t, lds, b - y_main_tiles<R, N, T>());
}

template <typename R, int N, int T, bool PAIR = false, int RS = 0>
__global__ __launch_bounds__(N / 8 * T)
void k_yinv_curl(cx<R>* __restrict__ W, const cx<R>* __restrict__ tw, size_t wst) {
    W += blockIdx.y * wst;
    __shared__ cx<R> lds[T * N];
    __shared__ cx<R> twl[tw_size(N, RS) > 0 ? tw_size(N, RS) : 1];
    load_twiddles<R, N, RS>(twl, tw);
    const int b = x_tile<PAIR ? line_group<R, T>() : 1>((int)blockIdx.x, y_main_tiles<R, N, T>());
    if (b < y_main_tiles<R, N, T>()) yinv_curl_tile<R, N, T, false, RS>(W, twl, lds, b);
    else yinv_curl_tile<R, N, T, true, RS>(W, twl, lds, b - y_main_tiles<R, N, T>());
}

// Load element k (0 <= k < N) of the Hermitian extension of a half-spectrum
// z line: X_k for k <= N/2, conj(X_{N-k}) above; the imaginary parts of
// X_0 and X_{N/2} are dropped (inverse real transform semantics).
template <typename R, int N>
__device__ __forceinline__ cx<R> zline_load(const cx<R>* __restrict__ F, size_t line, int k) {
    using L = Lay<R, N>;
    if (k < N / 2) {
        cx<R> a = F[L::row(line) + k];
        if (k == 0) a.y = R(0);
        return a;
    } else if (k == N / 2) {
        cx<R> a = F[L::MAIN + line];
        a.y = R(0);
        return a;
    } else {
        return cconj<R>(F[L::row(line) + (N - k)]);
    }
}

// Two Hermitian half-spectrum lines X, Y packed as Z = X + i Y: the inverse
// transform of Z is x + i y with x, y the two real inverse transforms.
template <typename R, int N>
__device__ __forceinline__ cx<R> zpair_load(const cx<R>* __restrict__ FX, const cx<R>* __restrict__ FY,
                                             size_t line, int k) {
    const cx<R> x = zline_load<R, N>(FX, line, k);
    const cx<R> y = zline_load<R, N>(FY, line, k);
    return {x.x - y.y, x.y + y.x};
}

// Unpack the forward transform P of p = a + i b (a, b real lines) into the
// half spectra of a and b at wavenumber k (0 <= k <= N/2):
//   A_k = (P_k + conj P_{N-k}) / 2,  B_k = (P_k - conj P_{N-k}) / (2 i).
template <typename R>
__device__ __forceinline__ void zsplit(cx<R> pk, cx<R> pnk, cx<R>& A, cx<R>& B) {
    const R h = R(0.5);
    A = {(pk.x + pnk.x) * h, (pk.y - pnk.y) * h};
    B = {(pk.y + pnk.y) * h, (pnk.x - pk.x) * h};
}

// ---------------------------------------------------------------------------
// Pass 3: per (x, y) line (eq. curl_convection, Sec. 3.4 cross product):
// inverse real z transforms of the six fields (u, v, w, omega) paired into
// three complex transforms, c = (u x omega) / N^6 in registers, forward real
// z transforms of c paired as (c0 + i c1) and (c2 + 0 i).  Writes the half
// spectra of c into fields 0..2 of W (in place: a workgroup owns its lines).
// scale = N^-6 (exact power of two) restores the inverse transforms' 1/N^3.
// ---------------------------------------------------------------------------
template <typename R, int N, int L, int ZP = 3, int RS = 0>
__global__ __launch_bounds__(N / 8 * L)
void k_zcross(cx<R>* __restrict__ W, const cx<R>* __restrict__ tw, R scale, size_t wst) {
    W += blockIdx.y * wst;
    constexpr int E = 8, G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    constexpr int LP = padded_line<N>(ZP);
    constexpr bool SIO = stream_io<R>(N);
    __shared__ cx<R> lds[L * LP];
    __shared__ cx<R> twl[tw_size(N, RS) > 0 ? tw_size(N, RS) : 1];
    const int g = threadIdx.x % G, l = threadIdx.x / G;
    const size_t line = (size_t)blockIdx.x * L + l;
    const size_t zr = Lay<R, N>::row(line);   // start of the line's iz row
    constexpr size_t NQ = Lay<R, N>::MAIN;     // start of the Nyquist plane
    cx<R>* my = lds + l * LP;

    // Each stored coefficient is loaded once (lower half k < N/2 plus the
    // Nyquist value), all six lines before the first transform so that the
    // loads overlap; the upper half of the Hermitian extension,
    // Z_{N-k} = conj X_k + i conj Y_k, is exchanged through shared memory.
    cx<R> xl[3][E / 2], yl[3][E / 2], xn[3], yn[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const cx<R>* FX = W + (2 * p) * FS;
        const cx<R>* FY = W + (2 * p + 1) * FS;
#pragma unroll
        for (int m = 0; m < E / 2; ++m) {
            xl[p][m] = gload<cx<R>, SIO>(FX + zr + g + m * G);
            yl[p][m] = gload<cx<R>, SIO>(FY + zr + g + m * G);
        }
        if (g == 0) {
            xn[p] = gload<cx<R>, SIO>(FX + NQ + line);
            yn[p] = gload<cx<R>, SIO>(FY + NQ + line);
        }
    }
    load_twiddles<R, N, RS>(twl, tw);
    cx<R> z[3][E];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
        for (int m = 0; m < E / 2; ++m) {
            const int k = g + m * G;
            cx<R> X = xl[p][m], Y = yl[p][m];
            if (k == 0) { X.y = R(0); Y.y = R(0); }
            z[p][m] = {X.x - Y.y, X.y + Y.x};
            if (k > 0) my[N - k] = {X.x + Y.y, Y.x - X.y};
        }
        __syncthreads();
#pragma unroll
        for (int m = E / 2; m < E; ++m) {
            const int k = g + m * G;
            z[p][m] = (k == N / 2) ? cx<R>{xn[p].x, yn[p].x} : my[k];
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) fft_line<R, N, E, +1, true, ZP, RS>(z[p], my, 1, twl, g);
    // z[0] = (u, v), z[1] = (w, omega_x), z[2] = (omega_y, omega_z)
    cx<R> P[E], Q[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const R u = z[0][m].x, v = z[0][m].y, w = z[1][m].x;
        const R ox = z[1][m].y, oy = z[2][m].x, oz = z[2][m].y;
        P[m] = {(v * oz - w * oy) * scale, (w * ox - u * oz) * scale};
        Q[m] = {(u * oy - v * ox) * scale, R(0)};
    }
    fft_line<R, N, E, -1, true, ZP, RS>(Q, my, 1, twl, g);
    fft_line<R, N, E, -1, true, ZP, RS>(P, my, 1, twl, g);
    // c2: Q_k is its half spectrum directly
#pragma unroll
    for (int m = 0; m < E / 2; ++m) gstore<cx<R>, SIO>(W + 2 * FS + zr + g + m * G, Q[m]);
    if (g == 0) gstore<cx<R>, SIO>(W + 2 * FS + NQ + line, Q[E / 2]);
    // c0, c1: unpack P through LDS (needs P_{N-k})
#pragma unroll
    for (int m = 0; m < E; ++m) my[g + m * G] = P[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E / 2; ++m) {
        const int k = g + m * G;
        cx<R> A, B;
        zsplit<R>(my[k], my[(N - k) & (N - 1)], A, B);
        gstore<cx<R>, SIO>(W + zr + k, A);
        gstore<cx<R>, SIO>(W + FS + zr + k, B);
    }
    if (g == 0) {
        cx<R> A, B;
        zsplit<R>(my[N / 2], my[N / 2], A, B);
        gstore<cx<R>, SIO>(W + NQ + line, A);
        gstore<cx<R>, SIO>(W + FS + NQ + line, B);
    }
}

// Forward real z transforms of three physical fields u (3, N, N, N) into the
// half spectra of fields 0..2 of W (first step of the forward 3D transform).
template <typename R, int N, int L>
__global__ __launch_bounds__(N / 8 * L)
void k_zr2c(const R* __restrict__ u, cx<R>* __restrict__ W, const cx<R>* __restrict__ tw) {
    constexpr int E = 8, G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    constexpr size_t PS = (size_t)N * N * N;
    constexpr int LP = padded_line<N>(3);
    __shared__ cx<R> lds[L * LP];
    const int g = threadIdx.x % G, l = threadIdx.x / G;
    const size_t line = (size_t)blockIdx.x * L + l;
    const size_t zr = Lay<R, N>::row(line);   // start of the line's iz row
    constexpr size_t NQ = Lay<R, N>::MAIN;     // start of the Nyquist plane
    cx<R>* my = lds + l * LP;
    cx<R> P[E], Q[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const size_t o = line * N + g + m * G;
        P[m] = {u[o], u[PS + o]};
        Q[m] = {u[2 * PS + o], R(0)};
    }
    fft_line<R, N, E, -1, false, 3>(Q, my, 1, tw, g);
    fft_line<R, N, E, -1, false, 3>(P, my, 1, tw, g);
#pragma unroll
    for (int m = 0; m < E / 2; ++m) W[2 * FS + zr + g + m * G] = Q[m];
    if (g == 0) W[2 * FS + NQ + line] = Q[E / 2];
#pragma unroll
    for (int m = 0; m < E; ++m) my[g + m * G] = P[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E / 2; ++m) {
        const int k = g + m * G;
        cx<R> A, B;
        zsplit<R>(my[k], my[(N - k) & (N - 1)], A, B);
        W[0 * FS + zr + k] = A;
        W[1 * FS + zr + k] = B;
    }
    if (g == 0) {
        cx<R> A, B;
        zsplit<R>(my[N / 2], my[N / 2], A, B);
        W[0 * FS + NQ + line] = A;
        W[1 * FS + NQ + line] = B;
    }
}

// Inverse real z transforms of fields 0..2 of W into physical u (3, N, N, N),
// scaled by `scale` (N^-3 for the normalised inverse).
template <typename R, int N, int L>
__global__ __launch_bounds__(N / 8 * L)
void k_zc2r(const cx<R>* __restrict__ W, R* __restrict__ u, const cx<R>* __restrict__ tw, R scale) {
    constexpr int E = 8, G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    constexpr size_t PS = (size_t)N * N * N;
    constexpr int LP = padded_line<N>(3);
    __shared__ cx<R> lds[L * LP];
    const int g = threadIdx.x % G, l = threadIdx.x / G;
    const size_t line = (size_t)blockIdx.x * L + l;
    cx<R>* my = lds + l * LP;
    cx<R> a[E], b[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        a[m] = zpair_load<R, N>(W, W + FS, line, g + m * G);
        b[m] = zline_load<R, N>(W + 2 * FS, line, g + m * G);
    }
    fft_line<R, N, E, +1, false, 3>(a, my, 1, tw, g);
    fft_line<R, N, E, +1, false, 3>(b, my, 1, tw, g);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const size_t o = line * N + g + m * G;
        u[o] = a[m].x * scale;
        u[PS + o] = a[m].y * scale;
        u[2 * PS + o] = b[m].x * scale;
    }
}

// ---------------------------------------------------------------------------
// Pass 5: forward x transform of N_hat = F(u x omega) (fields 0..2 of W),
// then per mode (Sec. 3.1 computeRHS; eqs. mod_pressure, NSfinal):
//   N_hat *= dealias;  P_hat = k . N_hat / |k|^2 (0 at k = 0);
//   N_hat -= k P_hat;  R = N_hat - nu |k|^2 u_s
// and one stage of the classic RK4 scheme of the Appendix solver,
//   u_s1 = u0 + dt/2 k1,  u_s2 = u0 + dt/2 k2,  u_s3 = u0 + dt k3,
//   u_new = u0 + dt/6 (k1 + 2 k2 + 2 k3 + k4),
// with the final sum regrouped so that the state moves 36 fields per step
// instead of 48: dt k1 = 2 (u_s1 - u0), dt k2 = 2 (u_s2 - u0) and
// dt k3 = u_s3 - u0 give
//   u_new = S + u_s3 / 3 + dt/6 k4,   S = (u_s1 + 2 u_s2 - u0) / 3,
// and S is formed at stage 1, where u_s1, u_s2 and u0 are all at hand.
// Arrays: U0 = u0, Us = the current stage velocity, U1 = S.
//   stage 0:  Us = U0 + cb R                                   (u_s = U0)
//   stage 1:  v = U0 + cb R,  U1 = (Us + 2 v - U0) / 3,  Us = v  (u_s = Us)
//   stage 2:  Us = U0 + cb R                                   (u_s = Us)
//   stage 3:  U0 = (U1 + Us / 3) + ca R                        (u_s = Us)
//   stage -1: U1 = R (right-hand side only; u_s = U0)
// with cb = b_s dt (b = 1/2, 1/2, 1) and ca = dt/6.  Stage 4 is the whole
// forward Euler step of the Sec. 3.1 main loop, u_hat += R dt:
//   stage 4:  U0 = U0 + ca R, ca = dt                          (u_s = U0)
// At the last stage of a step (3, or 4 for Euler), in the kernel instance
// with diagnostics (DIAG; launched when diag != nullptr), each workgroup also
// writes partial sums
// of w |u_hat|^2 and w |k x u_hat|^2 of the new state (w = 1 on the kz = 0
// and kz = N/2 planes, 2 elsewhere) to diag[2 blockIdx], diag[2 blockIdx + 1].
// ---------------------------------------------------------------------------
// The mask / projection / viscous / RK4 update of one x tile, shared by the
// RHS pass and the fused stage pass.  nh holds the x-transformed N_hat on
// entry; on return it holds the input of the next stage (Us for stages 0..2,
// the new U0 for stage 3, R for stage -1), which the fused pass transforms
// on without reading it back.

// Dealias mask and projection of mode (kx, ky, kz): n -= k (k . n) / |k|^2.
template <typename R>
__device__ __forceinline__ void project_mode(cx<R>& n0, cx<R>& n1, cx<R>& n2, int kx, int ky, int kz, bool keep) {
    if (!keep) {
        n0 = {R(0), R(0)}; n1 = n0; n2 = n0;
    }
    const int k2 = kx * kx + ky * ky + kz * kz;
    const R fx = (R)kx, fy = (R)ky, fz = (R)kz;
    const R inv = k2 > 0 ? R(1) / (R)k2 : R(0);
    // P_hat = sum_i N_i k_i / |k|^2
    const cx<R> P = {(n0.x * fx + n1.x * fy + n2.x * fz) * inv, (n0.y * fx + n1.y * fy + n2.y * fz) * inv};
    n0 = csub<R>(n0, cscale<R>(P, fx));
    n1 = csub<R>(n1, cscale<R>(P, fy));
    n2 = csub<R>(n2, cscale<R>(P, fz));
}

// S = (u_s1 + 2 v - u0) / 3 (stage 1) and the new state (U1 + u_s3 / 3) + ca R
// (stage 3), written once so that both forms of the update round alike.
// The thirds are correctly rounded divisions, not products with a rounded
// 1/3: these scale whole state values every step, and 1/3 rounded to FP32
// (+3.0e-8 relative) would add that bias to the state each step (an energy
// drift of 6e-8 per step, measured in a 20000-step 512^3 FP32 run).
template <typename R> __device__ __forceinline__ cx<R> cthird(cx<R> a) { return {a.x / R(3), a.y / R(3)}; }
template <typename R> __device__ __forceinline__ cx<R> rk_partial_sum(cx<R> us1, cx<R> v, cx<R> u0) {
    return cthird<R>(csub<R>(cadd<R>(us1, cscale<R>(v, R(2))), u0));
}
template <typename R> __device__ __forceinline__ cx<R> rk_final(cx<R> s, cx<R> us3, cx<R> r, R ca) {
    return cadd<R>(cadd<R>(s, cthird<R>(us3)), cscale<R>(r, ca));
}

// Partial sums of w |v|^2 and w |k x v|^2 of one mode of the new state.
template <typename R, int N>
__device__ __forceinline__ void diag_mode(cx<R> v0, cx<R> v1, cx<R> v2, int kx, int ky, int kz, double& e_acc,
                                          double& w_acc) {
    const double wgt = (kz == 0 || kz == N / 2) ? 1.0 : 2.0;
    const double x0 = v0.x, y0 = v0.y, x1 = v1.x, y1 = v1.y, x2 = v2.x, y2 = v2.y;
    e_acc += wgt * (x0 * x0 + y0 * y0 + x1 * x1 + y1 * y1 + x2 * x2 + y2 * y2);
    const double dx = kx, dy = ky, dz = kz;
    const double cxr = dy * x2 - dz * x1, cxi = dy * y2 - dz * y1;
    const double cyr = dz * x0 - dx * x2, cyi = dz * y0 - dx * y2;
    const double czr = dx * x1 - dy * x0, czi = dx * y1 - dy * y0;
    w_acc += wgt * (cxr * cxr + cxi * cxi + cyr * cyr + cyi * cyi + czr * czr + czi * czi);
}

// Per-element form of the update: each element's state values are loaded,
// combined and stored before the next element's; a compiler memory barrier
// between elements keeps the loads from being batched.  Fewer registers than
// the batched form, for 1024-thread shapes whose register budget is 128 per
// thread.
template <typename R, int N, int E, int STAGE, bool NYQ, bool DIAG>
__device__ __forceinline__ void rk_apply_elementwise(cx<R> (&nh)[3][E], const XCol<R, N, NYQ>& col, int g,
                                                     cx<R>* __restrict__ U0, cx<R>* __restrict__ U1,
                                                     cx<R>* __restrict__ Us, const StageArgs& sa,
                                                     double& e_acc, double& w_acc) {
    constexpr int G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    const int ky = col.ky, kz = col.kz;
    const int lim = sa.mask_lim;
    const bool keep_yz = (3 * abs(ky) < lim) && (3 * abs(kz) < lim);
    const R nu = (R)sa.nu, ca = (R)sa.ca, cb = (R)sa.cb;
    const XAddr<R, N, NYQ> A(col, g);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int kx = kfreq(g + m * G, N);
        const bool keep = keep_yz && (3 * abs(kx) < lim);
        cx<R> n[3] = {nh[0][m], nh[1][m], nh[2][m]};
        project_mode<R>(n[0], n[1], n[2], kx, ky, kz, keep);
        const R visc = nu * (R)(kx * kx + ky * ky + kz * kz);
        const cx<R>* ps = (STAGE <= 0 || STAGE == 4) ? U0 : Us;
        cx<R> us[3], other[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            us[f] = A(ps + f * FS, m);
            if constexpr (STAGE == 1 || STAGE == 2) other[f] = A(U0 + f * FS, m);
            if constexpr (STAGE == 3) other[f] = A(U1 + f * FS, m);
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const cx<R> r = csub<R>(n[f], cscale<R>(us[f], visc));
            cx<R> v;
            if constexpr (STAGE < 0) {
                v = r;
                A(U1 + f * FS, m) = v;
            } else if constexpr (STAGE == 0) {
                v = cadd<R>(us[f], cscale<R>(r, cb));
                A(Us + f * FS, m) = v;
            } else if constexpr (STAGE == 1) {
                v = cadd<R>(other[f], cscale<R>(r, cb));
                A(U1 + f * FS, m) = rk_partial_sum<R>(us[f], v, other[f]);
                A(Us + f * FS, m) = v;
            } else if constexpr (STAGE == 2) {
                v = cadd<R>(other[f], cscale<R>(r, cb));
                A(Us + f * FS, m) = v;
            } else if constexpr (STAGE == 3) {
                v = rk_final<R>(other[f], us[f], r, ca);
                A(U0 + f * FS, m) = v;
            } else {
                v = cadd<R>(us[f], cscale<R>(r, ca));
                A(U0 + f * FS, m) = v;
            }
            nh[f][m] = v;
        }
        if constexpr (STAGE >= 3 && DIAG) diag_mode<R, N>(nh[0][m], nh[1][m], nh[2][m], kx, ky, kz, e_acc, w_acc);
        asm volatile("" ::: "memory");
    }
}

// Batched form: after the projection the three fields are independent, so
// the state is streamed one field at a time with all of a thread's elements
// of that field (u_s and, from stage 1 on, the second array) in flight at
// once; a compiler memory barrier after each field keeps the next field's
// loads from being hoisted into the same batch (which would exhaust the
// registers).
template <typename R, int N, int E, int STAGE, bool NYQ, bool DIAG>
__device__ __forceinline__ void rk_apply_batched(cx<R> (&nh)[3][E], const XCol<R, N, NYQ>& col, int g,
                                               cx<R>* __restrict__ U0, cx<R>* __restrict__ U1,
                                               cx<R>* __restrict__ Us, const StageArgs& sa, double& e_acc,
                                               double& w_acc) {
    constexpr int G = N / E;
    constexpr size_t FS = Lay<R, N>::FS;
    const int ky = col.ky, kz = col.kz;
    const int lim = sa.mask_lim;
    const bool keep_yz = (3 * abs(ky) < lim) && (3 * abs(kz) < lim);
    const R nu = (R)sa.nu, ca = (R)sa.ca, cb = (R)sa.cb;
    const XAddr<R, N, NYQ> A(col, g);

#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int kx = kfreq(g + m * G, N);
        const bool keep = keep_yz && (3 * abs(kx) < lim);
        project_mode<R>(nh[0][m], nh[1][m], nh[2][m], kx, ky, kz, keep);
    }
    const cx<R>* ps = (STAGE <= 0 || STAGE == 4) ? U0 : Us;  // u_s
    const cx<R>* po = (STAGE == 3) ? U1 : U0;                // second array of stages 1..3
    constexpr bool TWO = STAGE >= 1 && STAGE <= 3;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        cx<R> us[E], o[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            us[m] = A(ps + f * FS, m);
            if constexpr (TWO) o[m] = A(po + f * FS, m);
        }
#pragma unroll
        for (int m = 0; m < E; ++m) {
            // R = N_hat - nu |k|^2 u_s (the factor recomputed per field from
            // integers: cheaper than holding E values across the loads)
            const int kx = kfreq(g + m * G, N);
            const R visc = nu * (R)(kx * kx + ky * ky + kz * kz);
            const cx<R> r = csub<R>(nh[f][m], cscale<R>(us[m], visc));
            cx<R> v;
            if constexpr (STAGE < 0) {
                v = r;
                A(U1 + f * FS, m) = v;
            } else if constexpr (STAGE == 0) {
                v = cadd<R>(us[m], cscale<R>(r, cb));
                A(Us + f * FS, m) = v;
            } else if constexpr (STAGE == 1) {
                v = cadd<R>(o[m], cscale<R>(r, cb));
                A(U1 + f * FS, m) = rk_partial_sum<R>(us[m], v, o[m]);
                A(Us + f * FS, m) = v;
            } else if constexpr (STAGE == 2) {
                v = cadd<R>(o[m], cscale<R>(r, cb));
                A(Us + f * FS, m) = v;
            } else if constexpr (STAGE == 3) {
                v = rk_final<R>(o[m], us[m], r, ca);
                A(U0 + f * FS, m) = v;
            } else {
                v = cadd<R>(us[m], cscale<R>(r, ca));
                A(U0 + f * FS, m) = v;
            }
            nh[f][m] = v;
        }
        asm volatile("" ::: "memory");
    }
    if constexpr (STAGE >= 3 && DIAG) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            diag_mode<R, N>(nh[0][m], nh[1][m], nh[2][m], kfreq(g + m * G, N), ky, kz, e_acc, w_acc);
    }
}

// Register budget decides between the two forms of the update: the
// batched one keeps more loads in flight, the per-element one fits the
// 128-register budget of 1024-thread workgroups.  DIAG: the last stage of a
// step also accumulates the diagnostic partial sums (a kernel instance of
// its own, so that steps without diagnostics carry none of that code).
template <typename R, int N, int E, int STAGE, bool NYQ, int NT, bool DIAG>
__device__ __forceinline__ void rk_apply_stage(cx<R> (&nh)[3][E], const XCol<R, N, NYQ>& col, int g,
                                               cx<R>* __restrict__ U0, cx<R>* __restrict__ U1,
                                               cx<R>* __restrict__ Us, const StageArgs& sa, double& e_acc,
                                               double& w_acc) {
    if constexpr (NT > 512)
        rk_apply_elementwise<R, N, E, STAGE, NYQ, DIAG>(nh, col, g, U0, U1, Us, sa, e_acc, w_acc);
    else
        rk_apply_batched<R, N, E, STAGE, NYQ, DIAG>(nh, col, g, U0, U1, Us, sa, e_acc, w_acc);
}

// Fixed-order tree reduction of the two diagnostic partial sums over a
// workgroup of NT threads; thread 0 writes them to diag[2 slot + {0, 1}]
// (slot = the tile, so that the partials do not depend on which workgroup
// took which tile).
template <int NT>
__device__ __forceinline__ void diag_reduce(double (&red)[2][NT], double e_acc, double w_acc, double* diag,
                                            int slot) {
    red[0][threadIdx.x] = e_acc;
    red[1][threadIdx.x] = w_acc;
    __syncthreads();
#pragma unroll 1
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        diag[2 * slot] = red[0][0];
        diag[2 * slot + 1] = red[1][0];
    }
}

template <typename R, int N, int T, int STAGE, bool NYQ, bool DIAG, int RS = 0>
__device__ __forceinline__ void xrhs_tile(const cx<R>* __restrict__ W, cx<R>* __restrict__ U0, cx<R>* __restrict__ U1,
                                          cx<R>* __restrict__ Us, const StageArgs& sa, cx<R>* lds, const cx<R>* twl,
                                          double (&red)[2][DIAG ? N / x_elems<R>(N) * T : 1], int tile) {
    constexpr int E = x_elems<R>(N), G = N / E;
    constexpr int NT = G * T;
    constexpr size_t FS = Lay<R, N>::FS;
    const int t = threadIdx.x % T, g = threadIdx.x / T;
    const XCol<R, N, NYQ> col(tile * T + t);
    cx<R> nh[3][E];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int m = 0; m < E; ++m) nh[f][m] = XAddr<R, N, NYQ>(col, g)(W + f * FS, m);
#pragma unroll
    for (int f = 0; f < 3; ++f) fft_line<R, N, E, -1, true, 0, RS>(nh[f], lds + t, T, twl, g);
    double e_acc = 0.0, w_acc = 0.0;
    rk_apply_stage<R, N, E, STAGE, NYQ, NT, DIAG>(nh, col, g, U0, U1, Us, sa, e_acc, w_acc);
    if constexpr (STAGE >= 3 && DIAG) diag_reduce<NT>(red, e_acc, w_acc, sa.diag, tile);
}

// The RK stage is a template parameter: one kernel per stage gives each
// its own straight-line code and register allocation.
template <typename R, int N, int T, int STAGE, bool PAIR, bool DIAG, int RS = 0>
__global__ __launch_bounds__(N / x_elems<R>(N) * T)
void k_xrhs(const cx<R>* __restrict__ W, cx<R>* __restrict__ U0, cx<R>* __restrict__ U1,
            cx<R>* __restrict__ Us, const cx<R>* __restrict__ tw, StageArgs sa, size_t sst, size_t wst) {
    W += blockIdx.y * wst;
    U0 += blockIdx.y * sst;
    U1 += blockIdx.y * sst;
    Us += blockIdx.y * sst;
    if (sa.diag) sa.diag += 2 * (size_t)gridDim.x * blockIdx.y;
    __shared__ cx<R> lds[T * N];
    __shared__ double red[2][DIAG ? N / x_elems<R>(N) * T : 1];
    __shared__ cx<R> twl[tw_size(N, RS) > 0 ? tw_size(N, RS) : 1];
    load_twiddles<R, N, RS>(twl, tw);
    const int tile = x_tile<PAIR ? line_group<R, T>() : 1>((int)blockIdx.x, x_main_tiles<N, T>());
    if (tile < x_main_tiles<N, T>())
        xrhs_tile<R, N, T, STAGE, false, DIAG, RS>(W, U0, U1, Us, sa, lds, twl, red, tile);
    else
        xrhs_tile<R, N, T, STAGE, true, DIAG, RS>(W, U0, U1, Us, sa, lds, twl, red, tile);
}

// ---------------------------------------------------------------------------
// Pass 5 fused with pass 1 of the next stage: after the RK4 update of stage
// s the tile's next-stage velocity (Us for s < 3, the new U0 for s = 3) is
// still in registers, so its five inverse x transforms (xinv_curl_store,
// as in k_xinv_curl, hence the same bits) are formed right away and the next
// stage does not read it back from memory.  W fields 0..2 are read (N_hat)
// before fields 0..4 are written; a workgroup owns its columns, so this is
// safe in place.
// ---------------------------------------------------------------------------
template <typename R, int N, int T, int STAGE, bool NYQ, bool CY, bool DIAG, int RS = 0>
__device__ __forceinline__ void xstage_tile(cx<R>* __restrict__ W, cx<R>* __restrict__ U0, cx<R>* __restrict__ U1,
                                            cx<R>* __restrict__ Us, const StageArgs& sa, cx<R>* lds,
                                            const cx<R>* twl, double (&red)[2][DIAG ? N / x_elems<R>(N) * T : 1],
                                            int tile) {
    constexpr int E = x_elems<R>(N), G = N / E;
    constexpr int NT = G * T;
    constexpr size_t FS = Lay<R, N>::FS;
    const int t = threadIdx.x % T, g = threadIdx.x / T;
    const XCol<R, N, NYQ> col(tile * T + t);
    const XAddr<R, N, NYQ> A(col, g);

    cx<R> u[3][E];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int m = 0; m < E; ++m) u[f][m] = A(W + f * FS, m);
    cx<R>* lt = lds + t;
#pragma unroll
    for (int f = 0; f < 3; ++f) fft_line<R, N, E, -1, true, 0, RS>(u[f], lt, T, twl, g);
    double e_acc = 0.0, w_acc = 0.0;
    rk_apply_stage<R, N, E, STAGE, NYQ, NT, DIAG>(u, col, g, U0, U1, Us, sa, e_acc, w_acc);
    if constexpr (STAGE >= 3 && DIAG) diag_reduce<NT>(red, e_acc, w_acc, sa.diag, tile);

    // inverse x transforms for the next stage's velocity and vorticity
    xinv_curl_store<R, N, T, NYQ, CY, RS>(u, W, A, lt, twl, g, col.ky, col.kz);
}

template <typename R, int N, int T, int STAGE, bool CY, bool PAIR, bool DIAG, int RS = 0>
__global__ __launch_bounds__(N / x_elems<R>(N) * T)
void k_xstage(cx<R>* __restrict__ W, cx<R>* __restrict__ U0, cx<R>* __restrict__ U1,
              cx<R>* __restrict__ Us, const cx<R>* __restrict__ tw, StageArgs sa, size_t sst, size_t wst) {
    W += blockIdx.y * wst;
    U0 += blockIdx.y * sst;
    U1 += blockIdx.y * sst;
    Us += blockIdx.y * sst;
    if (sa.diag) sa.diag += 2 * (size_t)gridDim.x * blockIdx.y;
    __shared__ cx<R> lds[T * N];
    __shared__ double red[2][DIAG ? N / x_elems<R>(N) * T : 1];
    __shared__ cx<R> twl[tw_size(N, RS) > 0 ? tw_size(N, RS) : 1];
    load_twiddles<R, N, RS>(twl, tw);
    const int tile = x_tile<PAIR ? line_group<R, T>() : 1>((int)blockIdx.x, x_main_tiles<N, T>());
    if (tile < x_main_tiles<N, T>())
        xstage_tile<R, N, T, STAGE, false, CY, DIAG, RS>(W, U0, U1, Us, sa, lds, twl, red, tile);
    else
        xstage_tile<R, N, T, STAGE, true, CY, DIAG, RS>(W, U0, U1, Us, sa, lds, twl, red, tile);
}

// ---------------------------------------------------------------------------
// Layout conversion between the external (3, N, N, N/2+1) array and the
// internal split-Nyquist layout (one thread per complex value).
// ---------------------------------------------------------------------------
template <typename R, int N, bool TO_INTERNAL>
__global__ __launch_bounds__(256)
void k_layout(const cx<R>* __restrict__ src, cx<R>* __restrict__ dst, size_t total) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    constexpr size_t M = N / 2 + 1;
    constexpr size_t FS = Lay<R, N>::FS;
    const size_t c = i / ((size_t)N * N * M);
    const size_t r = i - c * (size_t)N * N * M;
    const size_t iz = r % M;
    const size_t ixy = r / M;            // ix * N + iy
    const size_t in = c * FS + (iz < N / 2 ? Lay<R, N>::row(ixy) + iz : Lay<R, N>::MAIN + ixy);
    if (TO_INTERNAL) dst[in] = src[i];
    else dst[i] = src[in];
}

// ---------------------------------------------------------------------------
// Diagnostics of a state U: per-workgroup partial sums of w |u_hat|^2 and
// w |k x u_hat|^2 over a fixed grid-stride assignment of modes, then one
// workgroup sums the partials in fixed order: E = S_E / (2 N^6),
// Omega = S_W / (2 N^6).  Deterministic for a given N and grid.
// ---------------------------------------------------------------------------
template <typename R, int N>
__global__ __launch_bounds__(256)
void k_diag_partial(const cx<R>* __restrict__ U, double* __restrict__ part) {
    constexpr size_t FS = Lay<R, N>::FS;
    __shared__ double red[2 * 4];
    double e_acc = 0.0, w_acc = 0.0;
    for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < Lay<R, N>::MODES; j += (size_t)DIAG_BLOCKS * 256) {
        int ix, iy, iz;
        size_t i;
        Lay<R, N>::mode(j, ix, iy, iz, i);
        const double kx = kfreq(ix, N), ky = kfreq(iy, N), kz = iz;
        const double wgt = (iz == 0 || iz == N / 2) ? 1.0 : 2.0;
        const cx<R> a = U[i], b = U[FS + i], c = U[2 * FS + i];
        const double x0 = a.x, y0 = a.y, x1 = b.x, y1 = b.y, x2 = c.x, y2 = c.y;
        e_acc += wgt * (x0 * x0 + y0 * y0 + x1 * x1 + y1 * y1 + x2 * x2 + y2 * y2);
        const double cxr = ky * x2 - kz * x1, cxi = ky * y2 - kz * y1;
        const double cyr = kz * x0 - kx * x2, cyi = kz * y0 - kx * y2;
        const double czr = kx * x1 - ky * x0, czi = kx * y1 - ky * y0;
        w_acc += wgt * (cxr * cxr + cxi * cxi + cyr * cyr + cyi * cyi + czr * czr + czi * czi);
    }
    for (int off = 32; off > 0; off >>= 1) {
        e_acc += __shfl_down(e_acc, off, 64);
        w_acc += __shfl_down(w_acc, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { red[2 * wave] = e_acc; red[2 * wave + 1] = w_acc; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double se = 0.0, sw = 0.0;
        for (int i = 0; i < 4; ++i) { se += red[2 * i]; sw += red[2 * i + 1]; }
        part[2 * blockIdx.x] = se;
        part[2 * blockIdx.x + 1] = sw;
    }
}

// ---------------------------------------------------------------------------
// Initial conditions.
// ---------------------------------------------------------------------------
enum IcKind { IC_TAYLOR_GREEN = 0, IC_TAYLOR_GREEN_2D = 1, IC_ABC = 2, IC_SHEAR = 3 };

// Analytic velocity on the mesh x_i = 2 pi i / N (Sec. 2, eq. realmesh),
// written as a (3, N, N, N) real array; sin and cos of 2 pi i / N are taken
// as sinpi/cospi of 2 i / N, so the angle is exact.
//   Taylor-Green (Sec. 4.2, Appendix): (sin x cos y cos z, -cos x sin y cos z, 0)
//   planar Taylor-Green: (sin x cos y, -cos x sin y, 0)
//   ABC: (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x)
//   shear: (amp sin(k z), 0, 0)
template <typename R, int N>
__global__ __launch_bounds__(256) void k_ic_physical(R* __restrict__ u, int kind, double p0, double p1, double p2) {
    constexpr size_t P = (size_t)N * N * N;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    const int ix = (int)(i / ((size_t)N * N)), iy = (int)((i / N) % N), iz = (int)(i % N);
    const double tx = 2.0 * ix / N, ty = 2.0 * iy / N, tz = 2.0 * iz / N;
    double a = 0.0, b = 0.0, c = 0.0;
    if (kind == IC_TAYLOR_GREEN) {
        a = sinpi(tx) * cospi(ty) * cospi(tz);
        b = -cospi(tx) * sinpi(ty) * cospi(tz);
    } else if (kind == IC_TAYLOR_GREEN_2D) {
        a = sinpi(tx) * cospi(ty);
        b = -cospi(tx) * sinpi(ty);
    } else if (kind == IC_ABC) {
        a = p0 * sinpi(tz) + p2 * cospi(ty);
        b = p1 * sinpi(tx) + p0 * cospi(tz);
        c = p2 * sinpi(ty) + p1 * cospi(tx);
    } else {
        // sin(k z) with the integer k reduced modulo N: sinpi(2 (k iz mod N) / N)
        const long kk = (long)p0;
        const long r = ((kk % N) * iz % N + N) % N;
        a = p1 * sinpi(2.0 * r / N);
    }
    u[i] = (R)a;
    u[P + i] = (R)b;
    u[2 * P + i] = (R)c;
}

// SplitMix64 (Steele, Lea & Flood 2014): output function for counter x.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double unit53(unsigned long long z) {
    return ((double)(z >> 11) + 1.0) * 0x1.0p-53;   // (0, 1]
}

// Random solenoidal spectrum, one thread per stored mode (internal layout):
// complex Gaussian components from SplitMix64 counters (key = seed << 40 xor
// the mode's flat index in the external (3, N, N, N/2+1) order; uniforms from
// counters 2 key and 2 key + 1) via Box-Muller, projected onto k-perpendicular,
// amplitude sqrt(E(|k|) / (4 pi |k|^2)) N^3 with E(k) = k^4 exp(-2 (k/k0)^2),
// zero at k = 0 and outside the dealias mask.  On the kz = 0 and kz = N/2
// planes a mode whose mirror (-kx, -ky) comes first in (iy, ix) order takes
// the conjugate of the mirror's value (recomputed from the mirror's own
// counters); a self-mirrored mode keeps its real part.  The energy is
// normalised afterwards by the host.
template <typename R, int N>
__global__ __launch_bounds__(256) void k_ic_random(cx<R>* __restrict__ U, unsigned long long seed, double k0,
                                                   int mask_lim) {
    constexpr size_t FS = Lay<R, N>::FS;
    const size_t j = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= Lay<R, N>::MODES) return;
    int ix, iy, iz;
    size_t i;
    Lay<R, N>::mode(j, ix, iy, iz, i);
    int sx = ix, sy = iy;
    bool conj = false, real_only = false;
    if (iz == 0 || iz == N / 2) {
        const int mx = (N - ix) % N, my = (N - iy) % N;
        if (mx == ix && my == iy) real_only = true;
        else if (my < iy || (my == iy && mx < ix)) { sx = mx; sy = my; conj = true; }
    }
    const int kx = kfreq(sx, N), ky = kfreq(sy, N), kz = iz;
    const long k2 = (long)kx * kx + (long)ky * ky + (long)kz * kz;
    const bool keep = (3 * abs(kx) < mask_lim) && (3 * abs(ky) < mask_lim) && (3 * abs(kz) < mask_lim) && k2 > 0;
    double gr[3], gi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const unsigned long long idx =
            (((unsigned long long)c * N + sx) * N + sy) * (unsigned long long)(N / 2 + 1) + (unsigned long long)iz;
        const unsigned long long key = (seed << 40) ^ idx;
        const double u1 = unit53(splitmix64(key * 2ull));
        const double u2 = unit53(splitmix64(key * 2ull + 1ull));
        const double rad = sqrt(-2.0 * log(u1));
        const double h = 0.70710678118654752440;
        gr[c] = rad * cos(2.0 * M_PI * u2) * h;
        gi[c] = rad * sin(2.0 * M_PI * u2) * h;
    }
    double vr[3] = {0.0, 0.0, 0.0}, vi[3] = {0.0, 0.0, 0.0};
    if (keep) {
        const double fk[3] = {(double)kx, (double)ky, (double)kz};
        const double inv = 1.0 / (double)k2;
        const double pr = (fk[0] * gr[0] + fk[1] * gr[1] + fk[2] * gr[2]) * inv;
        const double pi_ = (fk[0] * gi[0] + fk[1] * gi[1] + fk[2] * gi[2]) * inv;
        const double kmag = sqrt((double)k2);
        const double spec = kmag * kmag * kmag * kmag * exp(-2.0 * (kmag / k0) * (kmag / k0));
        const double amp = sqrt(spec / (4.0 * M_PI * kmag * kmag)) * ((double)N * N * N);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vr[c] = (gr[c] - fk[c] * pr) * amp;
            vi[c] = (gi[c] - fk[c] * pi_) * amp;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double im = conj ? -vi[c] : vi[c];
        if (real_only) im = 0.0;
        U[c * FS + i] = {(R)vr[c], (R)im};
    }
}

// Multiply the three fields at U by s (energy normalisation).
template <typename R, int N>
__global__ __launch_bounds__(256) void k_scale(cx<R>* __restrict__ U, double s) {
    constexpr size_t TOT = 3 * Lay<R, N>::FS;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= TOT) return;
    const cx<R> a = U[i];
    U[i] = {(R)(a.x * s), (R)(a.y * s)};
}

}  // namespace dns
