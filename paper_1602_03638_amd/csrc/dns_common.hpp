// Shared compile-time configuration of the HIP pseudo-spectral solver:
// complex vector types, the radix plan of every FFT length, launch shapes
// and the internal field layout.
#pragma once

#include <type_traits>

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
// Radix plans of a length-N Stockham FFT (N = 2^l), selected by RS:
//   RS = 0: radix-8 stages while three or more factors of two remain, then
//           one radix-4 or radix-2 stage (the reference plan: every default
//           kernel uses it);
//   RS = 1: the radix-4 or radix-2 stage first, then radix-8 stages;
//   RS = 2: radix-4 stages, the last one radix 8 where l is odd.
// The plans compute the same DFT with different rounding, so a plan with
// RS != 0 is chosen only where the caller accepts results that are not
// bitwise identical to the reference plan's.
// ---------------------------------------------------------------------------
constexpr int NRS = 3;
constexpr int num_stages(int N, int RS = 0) {
    const int l = ilog2(N);
    if (RS == 2) return (l % 2) ? (l - 3) / 2 + 1 : l / 2;
    return l / 3 + (l % 3 ? 1 : 0);
}
constexpr int radix_at(int N, int s, int RS = 0) {
    const int l = ilog2(N), rem = l % 3;
    if (RS == 1) return (rem != 0 && s == 0) ? (rem == 1 ? 2 : 4) : 8;
    if (RS == 2) return s < ((l % 2) ? (l - 3) / 2 : l / 2) ? 4 : 8;
    return s < l / 3 ? 8 : (rem == 1 ? 2 : 4);
}
// Length of the sub-transforms already formed before stage s.
constexpr int span_at(int N, int s, int RS = 0) {
    int L = 1;
    for (int i = 0; i < s; ++i) L *= radix_at(N, i, RS);
    return L;
}
// Offset of stage s in the twiddle table of plan RS; stage s stores
// span_at(N,s) * (radix_at(N,s) - 1) factors (stage 0 stores none).
constexpr int tw_offset(int N, int s, int RS = 0) {
    int off = 0;
    for (int i = 1; i < s; ++i) off += span_at(N, i, RS) * (radix_at(N, i, RS) - 1);
    return off;
}
constexpr int tw_size(int N, int RS = 0) { return tw_offset(N, num_stages(N, RS), RS); }
// The tables of all plans are stored one after the other (plan 0 first).
constexpr int tw_base(int N, int RS) {
    int off = 0;
    for (int r = 0; r < RS; ++r) off += tw_size(N, r);
    return off;
}
constexpr int tw_total(int N) { return tw_base(N, NRS); }
constexpr int tw_size_max(int N) {
    int m = 0;
    for (int r = 0; r < NRS; ++r) m = tw_size(N, r) > m ? tw_size(N, r) : m;
    return m;
}
// Plan RS differs from every plan with a smaller index (else it adds nothing).
constexpr bool radix_plan_new(int N, int RS) {
    for (int r = 0; r < RS; ++r) {
        bool same = num_stages(N, r) == num_stages(N, RS);
        for (int s = 0; same && s < num_stages(N, RS); ++s) same = radix_at(N, s, r) == radix_at(N, s, RS);
        if (same) return false;
    }
    return true;
}
constexpr bool radix_plan_valid(int N, int RS) {
    int p = 1;
    for (int s = 0; s < num_stages(N, RS); ++s) {
        const int r = radix_at(N, s, RS);
        if (r != 2 && r != 4 && r != 8) return false;
        p *= r;
    }
    return p == N;
}
static_assert(radix_plan_valid(8, 0) && radix_plan_valid(16, 1) && radix_plan_valid(32, 2) &&
                  radix_plan_valid(512, 2) && radix_plan_valid(1024, 1) && radix_plan_valid(1024, 2) &&
                  radix_plan_valid(128, 2) && radix_plan_valid(256, 1),
              "radix plans multiply to N");

// ---------------------------------------------------------------------------
// Internal layout of one half-spectrum field of an N^3 grid (complex values
// of type cx<R>):
//   main block, iz in [0, N/2):  element (ix, iy, iz) at ix * XP + iy * ZP + iz
//   Nyquist plane, iz = N/2:     element (ix, iy) at MAIN + ix * N + iy
// Every iz row and every ix plane ends in a 128-byte gap (PAD values that no
// kernel reads or writes): with power-of-two pitches the rows of an x or y
// tile would all fall on the same few HBM channels; a 128-byte skew spreads
// them (measured on MI355X: 4.3 -> 5.0 TB/s for x tiles, 4.6 -> 5.1 TB/s for
// y tiles, contiguous z lines within 4%).
// The same layout holds partially transformed data: after the inverse x pass
// ix is the physical x index, after the inverse y pass iy is physical y.
// ---------------------------------------------------------------------------
template <typename R, int N> struct Lay {
    static constexpr unsigned PAD = 128 / (2 * sizeof(R));
    static constexpr unsigned ZP = N / 2 + PAD;            // pitch of the iz rows
    static constexpr unsigned XP = N * ZP + PAD;           // pitch of the ix planes
    static constexpr size_t MAIN = (size_t)N * XP;         // start of the Nyquist plane
    static constexpr size_t FS = MAIN + (size_t)N * N;     // complex values per field
    // logical modes per field (main block, then Nyquist plane)
    static constexpr size_t MODES = (size_t)N * N * (N / 2) + (size_t)N * N;
    __host__ __device__ static constexpr size_t at(int ix, int iy, int iz) {
        return (size_t)ix * XP + (size_t)iy * ZP + (size_t)iz;
    }
    // start of the iz row of z line `line` = ix * N + iy
    __host__ __device__ static constexpr size_t row(size_t line) { return (line / N) * XP + (line % N) * ZP; }
    // indices and address of logical mode j (main block in (ix, iy, iz)
    // order, then the Nyquist plane in (ix, iy) order)
    __host__ __device__ static void mode(size_t j, int& ix, int& iy, int& iz, size_t& addr) {
        constexpr size_t MM = (size_t)N * N * (N / 2);
        if (j < MM) {
            iz = (int)(j % (N / 2));
            iy = (int)((j / (N / 2)) % N);
            ix = (int)(j / ((size_t)N * (N / 2)));
            addr = at(ix, iy, iz);
        } else {
            const size_t r = j - MM;
            iz = N / 2;
            iy = (int)(r % N);
            ix = (int)(r / N);
            addr = MAIN + r;
        }
    }
};

// Global-memory access of one complex value, streaming (non-temporal) or
// plain.  The stage passes read and write every value once; where that pays
// (stream_io), their loads and stores are non-temporal.
template <typename T, bool NT> __device__ __forceinline__ T gload(const T* p) {
    if constexpr (NT) {
        using S = decltype(p->x);
        using V = S __attribute__((ext_vector_type(2)));
        const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
        return T{v.x, v.y};
    } else {
        return *p;
    }
}
template <typename T, bool NT> __device__ __forceinline__ void gstore(T* p, T a) {
    if constexpr (NT) {
        using S = decltype(p->x);
        using V = S __attribute__((ext_vector_type(2)));
        const V v = {a.x, a.y};
        __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
    } else {
        *p = a;
    }
}
// Reference to one complex value in global memory: reads through gload,
// assignments through gstore.
template <typename T, bool NT> struct GRef {
    T* p;
    __device__ __forceinline__ operator T() const { return gload<T, NT>(p); }
    __device__ __forceinline__ const GRef& operator=(const T& a) const { gstore<T, NT>(p, a); return *this; }
};

// Sizes whose stage passes use streaming accesses (measured on MI355X, same
// build otherwise).  512^3: step 37.1 -> 35.8 ms (FP64), 19.0 -> 18.35 ms
// (FP32); 256^3: 4.79 -> 4.40 ms (FP64), 2.43 -> 2.25 ms (FP32).  The plain
// y-line kernel (forward y pass, standalone inverse) keeps plain accesses:
// streaming loads measured 1.23 -> 1.44 ms per forward launch at 512^3 FP64.
// 1024^3: the x passes lost 18-22% (their 64-byte rows are read in halves by
// neighbouring workgroups, which plain loads share through L2) and the y
// passes up to 10%.  32^3 to 128^3 (the ensemble): the batched step lost 12%;
// all fields of a 128^3 simulation (about 130 MB in FP32) fit in the 256 MB
// last-level cache between passes.
template <typename R> constexpr bool stream_io(int N) { return N == 256 || N == 512; }

// Element `at` (element offset) of the field starting at F.  Where a field
// spans less than 4 GiB the byte offset is formed in 32 bits, so a uniform
// field base plus one 32-bit per-thread register addresses it (no 64-bit
// address per element); larger fields index in 64 bits.
template <typename R, int N, typename P> __device__ __forceinline__ P* field_el(P* F, unsigned at) {
    using B = std::conditional_t<std::is_const_v<P>, const char, char>;
    if constexpr (Lay<R, N>::FS * sizeof(cx<R>) < (size_t(1) << 32))
        return reinterpret_cast<P*>(reinterpret_cast<B*>(F) + (size_t)(at * (unsigned)sizeof(cx<R>)));
    else
        return F + at;
}

// Elements per thread of the y-pass line transforms (a plan choice, see
// dns_impl.hpp; every choice runs the same butterflies with the same
// twiddles, so the results are bitwise identical).  Default: lines of 1024
// take 16 (FP64) or 32 (FP32) complex values per thread, so that a workgroup
// of 128-byte row segments (8 FP64 or 16 FP32 columns) has 512 threads, each
// holding one 256-byte line slice; shorter lines take 8.
template <typename R> constexpr int default_y_elems(int N) { return N >= 1024 ? (sizeof(R) == 8 ? 16 : 32) : 8; }
// With more than 8 elements per thread the y pass reads its twiddles from
// shared memory at every stage (kept in registers they would crowd out the
// line).
constexpr bool y_twiddles_in_lds(int E) { return E > 8; }

// The plain y pass loads the next field's values before the current
// field's transform (one more line held per thread) where registers are free
// to do so: FP64 with 8 values per thread below 1024, whose 512-thread
// workgroups hold one per CU at any register count up to 256 (512^3 forward
// y pass 1.245 -> 1.206 ms).  FP32 shapes at 128-byte rows are 1024-thread
// workgroups with 128 registers per thread; 1024-point lines need more
// registers for the transform itself.  (The vorticity-forming inverse y pass
// measured slower with its loads moved earlier: 2.235 -> 2.265 ms.)
template <typename R> constexpr bool y_prefetch(int N, int E) { return sizeof(R) == 8 && E == 8 && N < 1024; }

// Where the vorticity combinations i (ky w - kz v), i (kz u - kx w),
// i (kx v - ky u) are formed (a plan choice, bitwise neutral: the same
// operations in another kernel).  With 8 elements per y-line thread the
// inverse y pass can form them as it loads (the x pass writes U, V, W,
// F(kx v_hat) and F(kx w_hat): five fields instead of six, 8 of 180 fields
// per step less); with longer y slices three live lines per thread would
// spill, so there the x pass writes the six fields u, v, w, omega and the y
// pass transforms them as they are.  Default: in the y pass below 1024.
template <typename R> constexpr bool default_curl_in_y(int N) { return default_y_elems<R>(N) == 8; }

// Elements per thread of the x-pass line transforms.  8 for every size: the
// fused stage kernel holds three lines per thread, and 16 per thread (which
// would fit 128-byte FP32 rows of 1024-lines into fewer threads) spilled and
// measured slower at 1024^3 (24.7 vs 22.1 ms per launch on MI355X).
template <typename R> constexpr int x_elems(int) { return 8; }

// Tile handled by workgroup b of an x pass.  Workgroups are dispatched to
// the 8 XCDs in turn (workgroup b to XCD b mod 8), each with its own L2.
// Where an x tile's row segments are shorter than 128 bytes, GRP
// consecutive tiles share every 128-byte line; with GRP > 1 they go to
// workgroups b, b + 8, ..., b + 8 (GRP - 1) of one XCD, which start together
// and share its L2, instead of to GRP XCDs that each fetch the whole line.
// Tiles are permuted within the main block and within the Nyquist-plane
// block separately (both counts multiples of 8 GRP).
template <int GRP> __device__ __forceinline__ int x_tile(int b, int main_tiles) {
    if constexpr (GRP == 1) {
        return b;
    } else {
        const int base = b < main_tiles ? 0 : main_tiles;
        const int r = b - base, xcd = r & 7, k = r >> 3;
        return base + GRP * (8 * (k / GRP) + xcd) + (k % GRP);
    }
}
// Tiles of width T (columns of type R) sharing one 128-byte line.
template <typename R, int T> constexpr int line_group() {
    return (T <= 0 || T * 2 * (int)sizeof(R) >= 128) ? 1 : 128 / (T * 2 * (int)sizeof(R));
}

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
    double ca;       // dt / 6, the weight of R in the last stage's update
    double cb;       // b_s * dt (offset of the next stage), unused in the last stage
    int stage;       // 0..3, or -1: write the right-hand side only
    int mask_lim;    // keep a mode iff 3|k_i| < mask_lim on every axis (N or N+2)
    double* diag;    // per-workgroup (E, Omega) partial sums, or nullptr
};

}  // namespace dns
