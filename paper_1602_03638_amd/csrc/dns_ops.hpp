// Host-side launch table of the kernels for one (real type, N) pair.
#pragma once

#include "dns_common.hpp"

namespace dns {

struct Ops {
    int N;
    size_t real_size;      // bytes of one real value
    int x_tiles;           // workgroups of an x pass (= fused diagnostic partials)
    int tw_count;          // complex entries of the twiddle table
    // one RK4 stage
    void (*xinv)(const void* U, void* W, const void* tw, bool curl, hipStream_t s);
    void (*yinv6)(void* W, const void* tw, hipStream_t s);
    void (*zcross)(void* W, const void* tw, hipStream_t s);
    void (*yfwd3)(void* W, const void* tw, hipStream_t s);
    void (*xrhs)(const void* W, void* U0, void* U1, void* Us, const void* tw, const StageArgs& a, hipStream_t s);
    // standalone transforms and utilities
    void (*yinv3)(void* W, const void* tw, hipStream_t s);
    void (*xfwd)(const void* W, void* U, const void* tw, hipStream_t s);
    void (*zr2c)(const void* u, void* W, const void* tw, hipStream_t s);
    void (*zc2r)(const void* W, void* u, const void* tw, hipStream_t s);
    void (*layout)(const void* src, void* dst, bool to_internal, hipStream_t s);
    void (*diag_partial)(const void* U, double* part, hipStream_t s);
};

const Ops* ops_f64(int N);
const Ops* ops_f32(int N);

// Twiddle table of the length-N plan (forward direction), long-double
// accurate, rounded to double.
void make_twiddles(int N, double* re_im);

void launch_diag_final(const double* part, int nparts, double inv_norm, double* out,
                       double* hist, int* count, int cap, hipStream_t s);

}  // namespace dns
