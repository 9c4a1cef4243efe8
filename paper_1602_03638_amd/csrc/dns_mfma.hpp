// y pass of FP32 contexts with one radix-16 DFT stage on FP16 matrix cores
// (v_mfma_f32_16x16x16f16), selected by dns_opts.mfma_dft.
//
// Each length-N line (N = 16 N2) is split four-step: with n = N2 n1 + n2 and
// k = k1 + 16 k2,
//   A[k1][n2] = sum_{n1} F16[k1][n1] x[N2 n1 + n2]       (16-point DFT, MFMA)
//   A[k1][n2] *= w_N^(n2 k1)                              (twiddle, FP32)
//   X[k1 + 16 k2] = sum_{n2} A[k1][n2] w_N2^(n2 k2)       (Stockham, FP32)
// with w_L = exp(-+ 2 pi i / L).  A workgroup takes 16 consecutive columns
// (lines) of one ix; the MFMA's 16 output columns are these 16 lines at one
// n2, its 16 rows the 16 values of k1, its reduction runs over n1.
//
// Precision: the tile of one field is scaled by the power of two that puts
// its largest magnitude in [2^13, 2^14), each operand is split into FP16
// high and low parts (v = vh + vl, vl = fp16(v - vh)), and the products
// Fl xh + Fh xl + Fh xh are accumulated in FP32 (the Fl xl term, 2^-22
// relative, is dropped).  The remaining stages run in FP32 as in the plain
// y pass.  Lines of the kz = N/2 plane take the plain FP32 y transform.
// Where the y pass forms the vorticity combinations (the plan's curl
// placement), the inverse pass of a stage (CURL) forms those of k_yinv_curl
// as it stages each output's tile, in the same field order.
#pragma once

#include "dns_kernels.hpp"

namespace dns {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int MFMA_T = 16;                  // lines per workgroup
constexpr int MFMA_LP = MFMA_T + 1;         // LDS row pitch (complex), skewed against bank conflicts

template <int N> struct MfmaY {
    static constexpr int NT = N >= 256 ? 512 : 256;         // threads per workgroup
    static constexpr int WAVES = NT / 64;
    static constexpr int N2 = N / 16;
    static constexpr int E2 = N2 < 8 ? N2 : 8;              // elements per thread, sub-transforms
    static constexpr int G2 = N2 / E2;                      // threads per sub-transform
    static constexpr int ROUNDS = 16 * MFMA_T * G2 / NT;    // rounds of sub-transforms per field
    static constexpr int RPT = NT / MFMA_T;                 // rows per pass of the tile load
    static constexpr int YE = default_y_elems<float>(N);     // elements per thread, plain y transform
    static constexpr int GY = N / YE;                        // threads per line, plain y transform
    static constexpr int TN = NT / GY;                      // Nyquist-plane lines per workgroup
    static constexpr int MAIN_TILES = N * ((N / 2) / MFMA_T);
    static constexpr int TILES = MAIN_TILES + N / TN;
    static constexpr int LDS = (N * MFMA_LP > TN * N) ? N * MFMA_LP : TN * N;
    static_assert(N >= 64 && N2 % WAVES == 0 && ROUNDS >= 1 && ROUNDS * NT == 16 * MFMA_T * G2,
                  "sizes of the MFMA y pass");
    static_assert(NT % GY == 0 && TN <= N && TN * GY == NT, "Nyquist-plane tiling");
    static_assert((N / RPT) % 16 == 0 || N / RPT < 16, "tile load batches");
};

// FP16 high and low parts of v (v = hi + lo up to the rounding of lo).
__device__ __forceinline__ void split_half(float v, _Float16& hi, _Float16& lo) {
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

// Step 1 of the matrix-core y pass: stage one output field's tile in shared
// memory (row iy, column t) and return this thread's largest magnitude.
// KIND 0 stages field P as it is; KIND 3, 4, 5 form the vorticity
// combinations of k_yinv_curl from fields P and Q (ky per row, kz per column):
//   5: i (P - ky Q), P = F(kx v_hat), Q = U
//   4: i (kz P - Q), P = U, Q = F(kx w_hat)
//   3: i (ky P - kz Q), P = W, Q = V
// A thread's rows are loaded in batches of up to 16 loads in flight;
// STREAM selects streaming (non-temporal) loads.
template <int N, int KIND, bool STREAM>
__device__ __forceinline__ float stage_tile(const cx<float>* __restrict__ P, const cx<float>* __restrict__ Q,
                                            cx<float>* xs, unsigned base, int th, int t, float kz) {
    using L = Lay<float, N>;
    constexpr int RPT = MfmaY<N>::RPT;
    constexpr int BMAX = KIND == 0 ? 16 : 8;   // rows in flight (two loads each when combining)
    constexpr int ROWS = N / RPT, B = ROWS < BMAX ? ROWS : BMAX;
    float amax = 0.f;
#pragma unroll 1
    for (int c0 = 0; c0 < ROWS; c0 += B) {
        cx<float> v[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int r = th / MFMA_T + RPT * (c0 + j);
            const unsigned at = base + (unsigned)r * L::ZP + (unsigned)t;
            const float ky = (float)kfreq(r, N);
            const cx<float> p = gload<cx<float>, STREAM>(field_el<float, N>(P, at));
            if constexpr (KIND == 0) {
                v[j] = p;
            } else {
                const cx<float> q = gload<cx<float>, STREAM>(field_el<float, N>(Q, at));
                if constexpr (KIND == 5) v[j] = cmuli<float>(csub<float>(p, cscale<float>(q, ky)));
                else if constexpr (KIND == 4) v[j] = cmuli<float>(csub<float>(cscale<float>(p, kz), q));
                else v[j] = cmuli<float>(csub<float>(cscale<float>(p, ky), cscale<float>(q, kz)));
            }
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            amax = fmaxf(amax, fmaxf(fabsf(v[j].x), fabsf(v[j].y)));
            xs[(th / MFMA_T + RPT * (c0 + j)) * MFMA_LP + t] = v[j];
        }
    }
    return amax;
}

template <int N, int DIR, int NF, bool CURL>
__device__ __forceinline__ void ymfma_tile(cx<float>* __restrict__ W, const cx<float>* __restrict__ roots,
                                           const cx<float>* tw2l, cx<float>* xs, float* red, int tile) {
    using L = Lay<float, N>;
    using M = MfmaY<N>;
    constexpr int N2 = M::N2, E2 = M::E2, G2 = M::G2;
    constexpr size_t FS = L::FS;
    constexpr int ZT = (N / 2) / MFMA_T;
    constexpr int NT = M::NT, WAVES = M::WAVES, RPT = M::RPT;
    const int th = threadIdx.x, lane = th & 63, wave = th >> 6;
    const int t = th % MFMA_T;
    constexpr bool STREAM = DIR > 0 && stream_io<float>(N);   // as k_yline
    const unsigned base = (unsigned)(tile / ZT) * L::XP + (unsigned)((tile % ZT) * MFMA_T);

    // A operand: F16[k1 = lane % 16][n1 = 4 (lane / 16) + j], hi/lo parts,
    // and the negated imaginary parts (they enter the real output with a
    // minus sign)
    half4_t fhr, flr, fhi, fli, nfhi, nfli;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k1 = lane % 16, n1 = 4 * (lane / 16) + j;
        const cx<float> w = roots[((N / 16) * n1 * k1) % N];
        const float wr = w.x, wi = DIR < 0 ? w.y : -w.y;
        _Float16 h, l;
        split_half(wr, h, l);
        fhr[j] = h;
        flr[j] = l;
        split_half(wi, h, l);
        fhi[j] = h;
        fli[j] = l;
        nfhi[j] = -h;
        nfli[j] = -l;
    }

    const float kz = (float)((tile % ZT) * MFMA_T + t);
#pragma unroll 1
    for (int i = 0; i < NF; ++i) {
        // CURL: outputs 5, 4, 0, 3, 1, 2 overwrite only inputs no longer
        // needed (as in k_yinv_curl)
        const int f = CURL ? (i == 0 ? 5 : i == 1 ? 4 : i == 2 ? 0 : i == 3 ? 3 : i == 4 ? 1 : 2) : i;
        cx<float>* F = W + f * FS;
        // 1. tile -> LDS (row iy, column t), and the largest magnitude
        float amax;
        if constexpr (CURL) {
            switch (f) {
                case 5: amax = stage_tile<N, 5, STREAM>(W + 3 * FS, W, xs, base, th, t, kz); break;
                case 4: amax = stage_tile<N, 4, STREAM>(W, W + 4 * FS, xs, base, th, t, kz); break;
                case 3: amax = stage_tile<N, 3, STREAM>(W + 2 * FS, W + FS, xs, base, th, t, kz); break;
                default: amax = stage_tile<N, 0, STREAM>(F, F, xs, base, th, t, kz); break;
            }
        } else {
            amax = stage_tile<N, 0, STREAM>(F, F, xs, base, th, t, kz);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        if (lane == 0) red[wave] = amax;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < WAVES; ++w) amax = fmaxf(amax, red[w]);
        int e = 0;
        (void)frexpf(amax, &e);
        const float scale = amax > 0.f ? ldexpf(1.f, 14 - e) : 1.f;
        const float unscale = amax > 0.f ? ldexpf(1.f, e - 14) : 1.f;

        // 2. 16-point DFTs over n1 on the matrix cores, one n2 per block;
        // every lane writes back exactly the four slots it read
#pragma unroll 1
        for (int n2 = wave; n2 < N2; n2 += WAVES) {
            const int q = lane / 16;
            half4_t bhr, blr, bhi, bli;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const cx<float> v = xs[(N2 * (4 * q + j) + n2) * MFMA_LP + t];
                _Float16 h, l;
                split_half(v.x * scale, h, l);
                bhr[j] = h;
                blr[j] = l;
                split_half(v.y * scale, h, l);
                bhi[j] = h;
                bli[j] = l;
            }
            // re = Fr xr - Fi xi, im = Fr xi + Fi xr; small products first
            float4_t dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
            dr = __builtin_amdgcn_mfma_f32_16x16x16f16(flr, bhr, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f32_16x16x16f16(fhr, blr, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f32_16x16x16f16(nfli, bhi, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f32_16x16x16f16(nfhi, bli, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f32_16x16x16f16(fhr, bhr, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f32_16x16x16f16(nfhi, bhi, dr, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x16f16(flr, bhi, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x16f16(fhr, bli, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x16f16(fli, bhr, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x16f16(fhi, blr, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x16f16(fhr, bhi, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x16f16(fhi, bhr, di, 0, 0, 0);
            // D[k1 = 4 q + i][t]: twiddle w_N^(n2 k1), undo the scale
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k1 = 4 * q + i;
                const cx<float> w = roots[(n2 * k1) % N];
                const cx<float> a = {dr[i] * unscale, di[i] * unscale};
                xs[(N2 * k1 + n2) * MFMA_LP + t] = (DIR < 0) ? cmul<float>(a, w) : cmulc<float>(a, w);
            }
        }
        __syncthreads();

        // 3. N2-point transforms over n2 of every (line t, k1), in FP32;
        // outputs X[k1 + 16 k2] go straight to memory
        const int rest = th / MFMA_T, g2 = rest % G2;
#pragma unroll 1
        for (int rho = 0; rho < M::ROUNDS; ++rho) {
            const int k1 = rho * (NT / MFMA_T / G2) + rest / G2;
            cx<float>* sub = xs + (N2 * k1) * MFMA_LP + t;
            cx<float> v[E2];
#pragma unroll
            for (int m = 0; m < E2; ++m) v[m] = sub[(g2 + m * G2) * MFMA_LP];
            __syncthreads();   // the transform's first exchange overwrites these slots
            fft_line<float, N2, E2, DIR, true>(v, sub, MFMA_LP, tw2l, g2);
#pragma unroll
            for (int m = 0; m < E2; ++m)
                gstore<cx<float>, STREAM>(
                    field_el<float, N>(F, base + (unsigned)(k1 + 16 * (g2 + m * G2)) * L::ZP + (unsigned)t), v[m]);
            __syncthreads();
        }
    }
}

template <int N, int DIR, int NF, bool CURL>
__global__ __launch_bounds__(MfmaY<N>::NT)
void k_yline_mfma(cx<float>* __restrict__ W, const cx<float>* __restrict__ tw, const cx<float>* __restrict__ roots,
                  const cx<float>* __restrict__ tw2, size_t wst) {
    using M = MfmaY<N>;
    W += blockIdx.y * wst;
    __shared__ cx<float> xs[M::LDS];
    __shared__ cx<float> tw2l[tw_size(M::N2) > 0 ? tw_size(M::N2) : 1];
    __shared__ float red[M::WAVES];
    constexpr bool TWL = y_twiddles_in_lds(M::YE);
    __shared__ cx<float> twl[TWL ? tw_size(N) : 1];
    // CURL: the inverse pass of a stage forms the vorticity (five input fields)
    static_assert(!CURL || (DIR > 0 && NF == 6 && M::YE == 8), "vorticity in the y pass: inverse, 6 fields, 8 per thread");
    const int b = blockIdx.x;
    if (b < M::MAIN_TILES) {
        load_twiddles<float, M::N2>(tw2l, tw2);
        ymfma_tile<N, DIR, NF, CURL>(W, roots, tw2l, xs, red, b);
    } else {
        const cx<float>* t = tw;
        if constexpr (TWL) {
            load_twiddles<float, N>(twl, tw);
            t = twl;
        }
        if constexpr (CURL) yinv_curl_tile<float, N, M::TN, true>(W, t, xs, b - M::MAIN_TILES);
        else yline_tile<float, N, M::TN, DIR, NF, true, M::YE>(W, t, xs, b - M::MAIN_TILES);
    }
}

}  // namespace dns
