// Host-side launch table of the kernels for one (real type, N) pair, with
// the variants the autotuner chooses between.  The variants of radix plan 0
// run the same per-line arithmetic, so they give bitwise identical results;
// they differ in how many lines share a workgroup (width), in the order in
// which workgroups take tiles (XCD pairing), in how many elements a y-pass
// thread holds, in which kernel forms the vorticity combinations, and in the
// shared-memory padding of the z pass.  Variants of another radix plan
// compute the same transforms with other rounding.
#pragma once

#include "dns_common.hpp"

namespace dns {

constexpr int MAXV = 24;   // variants per pass

// Descriptor of one variant of a pass.
struct Variant {
    int width;   // lines (columns) per workgroup
    int pair;    // 1: x tiles sharing 128-byte lines go to one XCD (x passes); else 0
    int ye;      // y passes: complex values per thread (8, 16, 32); 0 for other passes
    int cy;      // 1: vorticity formed in the inverse y pass (five x-pass fields), 0: in the
                 // x pass (six fields); -1 for passes that do not depend on it
    int rs;      // radix plan of the line transforms (radix_at; 0 = the reference plan)
    int pad;     // z pass: one shared-memory pad slot after every `pad` elements of a
                 // line (0 = none; 8 by default); 0 for other passes
};

// The kernels of a stage: the inverse x pass with the curl (first stage
// only when fused), the inverse y pass, the fused z pass, the forward y
// pass, and either the RHS pass (unfused schedule) or the RHS pass fused
// with the next stage's inverse x pass.
enum Pass { P_XINV = 0, P_YINV6, P_ZCROSS, P_YFWD3, P_XRHS, P_XSTAGE, P_COUNT };

using XinvFn = void (*)(const void* U, void* W, const void* tw, const Batch& b, hipStream_t s);
using YFn = void (*)(void* W, const void* tw, const Batch& b, hipStream_t s);
using ZFn = void (*)(void* W, const void* tw, const Batch& b, hipStream_t s);
using XrhsFn = void (*)(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a,
                        const Batch& b, hipStream_t s);
// y pass with the radix-16 stage on FP16 matrix cores: roots = w_N^j
// (j < N), tw2 = twiddle table of the N/16-point transforms
using YMfmaFn = void (*)(void* W, const void* tw, const void* roots, const void* tw2, const Batch& b,
                         hipStream_t s);

struct Ops {
    int N;
    size_t real_size;      // bytes of one real value
    size_t fs;             // complex values of one field in the internal layout
    int tw_count;          // complex entries of the twiddle tables (all radix plans)
    int tw_base[NRS];      // first entry of radix plan r's table
    // variants of the passes of one RK4 stage; var[p][v] describes variant v
    // of pass p
    int nvar[P_COUNT];
    Variant var[P_COUNT][MAXV];
    int def[P_COUNT];      // default variant (before tuning)
    XinvFn xinv[MAXV];
    YFn yinv6[MAXV];
    ZFn zcross[MAXV];
    YFn yfwd3[MAXV];
    XrhsFn xrhs[MAXV];
    XrhsFn xstage[MAXV];
    int xrhs_groups[MAXV]; // workgroups of each xrhs variant (= fused diagnostic partials)
    int xstage_groups[MAXV];
    // y passes with the matrix-core DFT stage (FP32, N >= 64; else nullptr);
    // the inverse one per curl placement ([0]: six input fields, [1]: five)
    YMfmaFn ymfma_inv6[2];
    YMfmaFn ymfma_fwd3;
    // standalone transforms and utilities (default shapes)
    void (*xinv3)(const void* U, void* W, const void* tw, hipStream_t s);
    void (*yinv3)(void* W, const void* tw, hipStream_t s);
    void (*yfwd3s)(void* W, const void* tw, hipStream_t s);   // single simulation
    void (*xfwd3)(const void* W, void* U, const void* tw, hipStream_t s);
    void (*zr2c)(const void* u, void* W, const void* tw, hipStream_t s);
    void (*zc2r)(const void* W, void* u, const void* tw, hipStream_t s);
    void (*layout)(const void* src, void* dst, bool to_internal, hipStream_t s);
    void (*diag_partial)(const void* U, double* part, hipStream_t s);
    void (*ic_physical)(void* u, int kind, double p0, double p1, double p2, hipStream_t s);
    void (*ic_random)(void* U, unsigned long long seed, double k0, int mask_lim, hipStream_t s);
    void (*scale)(void* U, double factor, hipStream_t s);
};

// Launch table of one (real type, N) pair; defined for N = 8, 16, ..., 1024.
template <typename R, int N> const Ops* ops_table();

// Launch table of a size N (nullptr for an unsupported N).
const Ops* ops_f64(int N);
const Ops* ops_f32(int N);

// Twiddle table of the length-N transform with radix plan rs (forward
// direction), long-double accurate, rounded to double.
void make_twiddles(int N, double* re_im, int rs = 0);

void launch_diag_final(const double* part, int nparts, double inv_norm, double* out,
                       double* hist, int* count, int cap, hipStream_t s);

}  // namespace dns
