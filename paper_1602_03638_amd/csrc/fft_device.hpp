// Register/LDS Stockham FFT of one line held by a group of threads.
//
// A line x[0..N) is distributed over G = N/E threads: thread g holds
// v[m] = x[g + m G], m = 0..E-1.  Each radix-R stage (sub-transform span L
// before the stage) computes, for every butterfly b in [0, N/R):
//     j = b mod L,   in_r = x[b + r N/R] * w^(j r),  w = exp(-+ 2 pi i/(L R)),
//     out_m = sum_r in_r exp(-+ 2 pi i r m / R),
//     y[(b - j) R + j + m L] = out_m                  (Stockham autosort)
// Thread g owns butterflies b = g + q G, q < E/R, whose inputs are exactly
// its own v[q + r E/R].  Outputs go through LDS between stages; after the
// last stage (L R = N) the outputs land in the thread's own registers in the
// same natural distribution, so no LDS pass is needed at either end.
// DIR = -1: forward transform exp(-i ...); DIR = +1: inverse (unnormalised).
#pragma once

#include "dns_common.hpp"

namespace dns {

template <typename R> __device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R> __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R> __device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.x * s, a.y * s}; }
template <typename R> __device__ __forceinline__ cx<R> cconj(cx<R> a) { return {a.x, -a.y}; }
// i * a
template <typename R> __device__ __forceinline__ cx<R> cmuli(cx<R> a) { return {-a.y, a.x}; }

// a * exp(DIR * i pi / 2): -i a for the forward direction, +i a for the inverse
template <typename R, int DIR> __device__ __forceinline__ cx<R> rot4(cx<R> a) {
    if constexpr (DIR < 0) return {a.y, -a.x};
    else return {-a.y, a.x};
}
// a * exp(DIR * i pi / 4)
template <typename R, int DIR> __device__ __forceinline__ cx<R> rot8(cx<R> a) {
    const R h = R(0.70710678118654752440084436210484903928);
    if constexpr (DIR < 0) return {(a.x + a.y) * h, (a.y - a.x) * h};
    else return {(a.x - a.y) * h, (a.x + a.y) * h};
}
// a * exp(DIR * 3 i pi / 4)
template <typename R, int DIR> __device__ __forceinline__ cx<R> rot8_3(cx<R> a) {
    const R h = R(0.70710678118654752440084436210484903928);
    if constexpr (DIR < 0) return {(a.y - a.x) * h, -(a.x + a.y) * h};
    else return {-(a.x + a.y) * h, (a.x - a.y) * h};
}

// In-place DFTs of length 2, 4, 8 with natural-order output.
template <typename R, int DIR> __device__ __forceinline__ void dft2(cx<R>* x) {
    cx<R> a = x[0];
    x[0] = cadd<R>(a, x[1]);
    x[1] = csub<R>(a, x[1]);
}
template <typename R, int DIR> __device__ __forceinline__ void dft4(cx<R>& x0, cx<R>& x1, cx<R>& x2, cx<R>& x3) {
    cx<R> a0 = cadd<R>(x0, x2), a1 = csub<R>(x0, x2);
    cx<R> a2 = cadd<R>(x1, x3), a3 = rot4<R, DIR>(csub<R>(x1, x3));
    x0 = cadd<R>(a0, a2);
    x2 = csub<R>(a0, a2);
    x1 = cadd<R>(a1, a3);
    x3 = csub<R>(a1, a3);
}
template <typename R, int DIR> __device__ __forceinline__ void dft4(cx<R>* x) { dft4<R, DIR>(x[0], x[1], x[2], x[3]); }
template <typename R, int DIR> __device__ __forceinline__ void dft8(cx<R>* x) {
    // even/odd split: e = DFT4(x0,x2,x4,x6), o = DFT4(x1,x3,x5,x7)
    cx<R> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    cx<R> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4<R, DIR>(e0, e1, e2, e3);
    dft4<R, DIR>(o0, o1, o2, o3);
    o1 = rot8<R, DIR>(o1);
    o2 = rot4<R, DIR>(o2);
    o3 = rot8_3<R, DIR>(o3);
    x[0] = cadd<R>(e0, o0); x[4] = csub<R>(e0, o0);
    x[1] = cadd<R>(e1, o1); x[5] = csub<R>(e1, o1);
    x[2] = cadd<R>(e2, o2); x[6] = csub<R>(e2, o2);
    x[3] = cadd<R>(e3, o3); x[7] = csub<R>(e3, o3);
}
template <typename R, int RAD, int DIR> __device__ __forceinline__ void dft_small(cx<R>* x) {
    if constexpr (RAD == 2) dft2<R, DIR>(x);
    else if constexpr (RAD == 4) dft4<R, DIR>(x);
    else dft8<R, DIR>(x);
}

// One Stockham stage S of the length-N line FFT (see the file comment).
// lds + p * ps addresses element p of this thread's line in shared memory.
// TWL: the twiddle table lives in shared memory and is re-read at every
// stage (keeps it out of registers, which matters where a kernel holds
// several lines per thread); otherwise it is read from global memory and
// the compiler may keep it in registers across transforms.
// PAD: element p of a contiguous line (ps = 1) is stored at p + (p >> PAD)
// (one unused slot after every 2^PAD elements; 0 = none), so that the
// strided Stockham writes spread over the LDS banks.
// RS: the radix plan (radix_at).
template <int N> constexpr int padded_line(int pad) { return pad ? N + (N >> pad) : N; }
template <int PAD> __device__ __forceinline__ int lds_index(int p) { return PAD ? p + (p >> PAD) : p; }

template <typename R, int N, int E, int DIR, int S, bool TWL = false, int PAD = 0, int RS = 0>
struct FftStage {
    static __device__ __forceinline__ void run(cx<R> (&v)[E], cx<R>* lds, int ps,
                                               const cx<R>* __restrict__ tw, int g) {
        constexpr int G = N / E;
        constexpr int RAD = radix_at(N, S, RS);
        constexpr int L = span_at(N, S, RS);
        constexpr int Q = E / RAD;
        constexpr bool LAST = (S == num_stages(N, RS) - 1);
        static_assert(E % RAD == 0, "radix must divide the per-thread element count");
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int b = g + q * G;
            const int j = b & (L - 1);
            cx<R> x[RAD];
#pragma unroll
            for (int r = 0; r < RAD; ++r) x[r] = v[q + r * Q];
            if constexpr (L > 1) {
                if constexpr (TWL) asm volatile("" ::: "memory");
                const cx<R>* w = tw + tw_offset(N, S, RS) + j * (RAD - 1);
#pragma unroll
                for (int r = 1; r < RAD; ++r)
                    x[r] = (DIR < 0) ? cmul<R>(x[r], w[r - 1]) : cmulc<R>(x[r], w[r - 1]);
            }
            dft_small<R, RAD, DIR>(x);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < RAD; ++r) v[q + r * Q] = x[r];
            } else {
                const int p0 = (b - j) * RAD + j;
#pragma unroll
                for (int r = 0; r < RAD; ++r) lds[lds_index<PAD>(p0 + r * L) * ps] = x[r];
            }
        }
        if constexpr (!LAST) {
            __syncthreads();
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds[lds_index<PAD>(g + m * G) * ps];
            __syncthreads();
            FftStage<R, N, E, DIR, S + 1, TWL, PAD, RS>::run(v, lds, ps, tw, g);
        }
    }
};

// Transform the line held in v (natural distribution in, natural out) with
// radix plan RS, whose twiddle table tw is.
// Every thread of the workgroup must call this (it contains barriers).
template <typename R, int N, int E, int DIR, bool TWL = false, int PAD = 0, int RS = 0>
__device__ __forceinline__ void fft_line(cx<R> (&v)[E], cx<R>* lds, int ps,
                                         const cx<R>* __restrict__ tw, int g) {
    FftStage<R, N, E, DIR, 0, TWL, PAD, RS>::run(v, lds, ps, tw, g);
}

// Copy the twiddle table of plan RS into shared memory (all threads of the
// workgroup call this; ends with a barrier).
template <typename R, int N, int RS = 0>
__device__ __forceinline__ void load_twiddles(cx<R>* twl, const cx<R>* __restrict__ tw) {
    for (int i = threadIdx.x; i < tw_size(N, RS); i += blockDim.x) twl[i] = tw[i];
    __syncthreads();
}

}  // namespace dns
