// Shared compile-time configuration of the HIP pseudo-spectral solver:
// complex vector types, the radix plan of every FFT length, launch shapes
// and the internal field layout.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace dns {

template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename R> using cx = typename cvec<R>::type;

constexpr int ilog2(int n) { int m = 0; while ((1 << m) < n) ++m; return m; }

// ---------------------------------------------------------------------------
// Radix plan of a length-N Stockham FFT: radix-8 stages while three or more
// factors of two remain, then one radix-4 or radix-2 stage.
// ---------------------------------------------------------------------------
constexpr int num_stages(int N) { return ilog2(N) / 3 + (ilog2(N) % 3 ? 1 : 0); }
constexpr int radix_at(int N, int s) {
    return s < ilog2(N) / 3 ? 8 : (ilog2(N) % 3 == 1 ? 2 : 4);
}
// Length of the sub-transforms already formed before stage s.
constexpr int span_at(int N, int s) {
    int L = 1;
    for (int i = 0; i < s; ++i) L *= radix_at(N, i);
    return L;
}
// Offset of stage s in the twiddle table; stage s stores
// span_at(N,s) * (radix_at(N,s) - 1) factors (stage 0 stores none).
constexpr int tw_offset(int N, int s) {
    int off = 0;
    for (int i = 1; i < s; ++i) off += span_at(N, i) * (radix_at(N, i) - 1);
    return off;
}
constexpr int tw_size(int N) { return tw_offset(N, num_stages(N)); }

// ---------------------------------------------------------------------------
// Internal layout of one half-spectrum field of an N^3 grid:
//   main block [ix][iy][iz] for iz in [0, N/2)  (pitch N/2, power-of-two rows)
//   Nyquist plane [ix][iy] for iz = N/2, stored after the main block.
// The same layout holds partially transformed data: after the inverse x pass
// ix is the physical x index, after the inverse y pass iy is physical y.
// ---------------------------------------------------------------------------
constexpr size_t main_size(int N) { return (size_t)N * N * (N / 2); }
constexpr size_t field_size(int N) { return main_size(N) + (size_t)N * N; }

// ---------------------------------------------------------------------------
// Launch shapes.  Every FFT line of length N is held by G = N/E threads, E
// elements each (thread g holds elements g, g+G, ..., g+(E-1)G).
//   TX: lines per workgroup of the x pass (consecutive columns, stride-N^2/2
//       rows), TY: same for the y pass (consecutive iz of one ix),
//   LZ: contiguous lines per workgroup (z pass, Nyquist-plane y lines).
// Column groups span 64 bytes (4 complex doubles / 8 complex floats) and
// are widened so that a workgroup is at least one 64-wide wavefront.
// ---------------------------------------------------------------------------
template <typename R, int N> struct Cfg {
    static constexpr int E = 8;
    static constexpr int G = N / E;
    static constexpr int TB = sizeof(R) == 8 ? 4 : 8;
    static constexpr int TW = (64 / G > TB) ? 64 / G : TB;
    static constexpr int TX = TW < N ? TW : N;
    static constexpr int TY = TW < N / 2 ? TW : N / 2;
    static constexpr int LZ0 = (256 / G) > 1 ? 256 / G : 1;
    static constexpr int LZ = LZ0 < N * N ? LZ0 : N * N;
    static constexpr int LY = LZ0 < N ? LZ0 : N;
    static constexpr int XTHREADS = G * TX;
    static constexpr int YTHREADS = G * TY;
    static constexpr int ZTHREADS = G * LZ;
    static constexpr int NYTHREADS = G * LY;
    static constexpr int X_TILES = (N * (N / 2)) / TX + N / TX;
    static constexpr int Y_TILES = N * ((N / 2) / TY);
    static_assert(N >= 8 && (N & (N - 1)) == 0, "N must be a power of two >= 8");
};

// Workgroups of the standalone diagnostic reduction (fixed, so the summation
// order and hence the result are reproducible).
constexpr int DIAG_BLOCKS = 1024;

// Independent simulations of one size batched into one launch: member m of a
// launch is blockIdx.y = m, its state fields start sst complex values after
// member m-1's and its work fields wst after.  A single simulation is
// {1, 0, 0}.
struct Batch {
    int members;
    size_t sst;
    size_t wst;
};

// Per-stage coefficients of one RK4 stage of the fused x-forward kernel.
struct StageArgs {
    double nu;       // viscosity
    double ca;       // a_s * dt (weight of this stage in the accumulated update)
    double cb;       // b_s * dt (offset of the next stage), unused in the last stage
    int stage;       // 0..3, or -1: write the right-hand side only
    int mask_lim;    // keep a mode iff 3|k_i| < mask_lim on every axis (N or N+2)
    double* diag;    // per-workgroup (E, Omega) partial sums, or nullptr
};

}  // namespace dns
