// C ABI of the MI355X pseudo-spectral RK4 library (declared in dns.h):
// context lifetime, stream ordering, the RK4 step schedule, graph replay,
// transforms, diagnostics and profiling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dns.h"
#include "dns_ops.hpp"

namespace dns {

// ---------------------------------------------------------------------------
// Twiddle factors exp(-2 pi i m / n), m reduced modulo n before the angle is
// formed, evaluated in long double and exact at the multiples of pi/4 where
// the value is 0, +-1 or +-sqrt(1/2) per component.
// ---------------------------------------------------------------------------
static void unit_root(long m, long n, double* re, double* im) {
    m %= n;
    if (m < 0) m += n;
    if ((4 * m) % n == 0) {
        const long q = (4 * m) / n;   // quarter turns
        const double c[4] = {1.0, 0.0, -1.0, 0.0}, s[4] = {0.0, -1.0, 0.0, 1.0};
        *re = c[q];
        *im = s[q];
        return;
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double ang = 2.0L * pi * (long double)m / (long double)n;
    *re = (double)cosl(ang);
    *im = (double)(-sinl(ang));
}

void make_twiddles(int N, double* out) {
    const int ns = num_stages(N);
    for (int s = 1; s < ns; ++s) {
        const int L = span_at(N, s), Rr = radix_at(N, s);
        double* w = out + 2 * tw_offset(N, s);
        for (int j = 0; j < L; ++j)
            for (int r = 1; r < Rr; ++r) {
                const int idx = j * (Rr - 1) + (r - 1);
                unit_root((long)j * r, (long)L * Rr, &w[2 * idx], &w[2 * idx + 1]);
            }
    }
}

__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ part, int nparts, double inv_norm,
                                                    double* __restrict__ out, double* __restrict__ hist,
                                                    int* __restrict__ count, int cap) {
    __shared__ double red[2][256];
    double e = 0.0, w = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) {
        e += part[2 * i];
        w += part[2 * i + 1];
    }
    red[0][threadIdx.x] = e;
    red[1][threadIdx.x] = w;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double E = red[0][0] * inv_norm, W = red[1][0] * inv_norm;
        out[0] = E;
        out[1] = W;
        if (hist != nullptr) {
            const int c = *count;
            if (c < cap) {
                hist[2 * c] = E;
                hist[2 * c + 1] = W;
            }
            *count = c + 1;
        }
    }
}

void launch_diag_final(const double* part, int nparts, double inv_norm, double* out, double* hist, int* count,
                       int cap, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, part, nparts, inv_norm, out, hist, count, cap);
}

}  // namespace dns

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct dns_ctx {
    int N = 0, dtype = 0;
    double nu = 0, dt = 0;
    dns_opts opts{};
    int mask_lim = 0;
    hipStream_t user = nullptr;     // caller's stream (ordering reference)
    hipStream_t s = nullptr;        // library stream (graph capture needs a non-null stream)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipEvent_t ev_prof[2] = {nullptr, nullptr};
    const dns::Ops* ops = nullptr;
    int sel[dns::P_COUNT] = {0, 0, 0, 0, 0, 0};   // chosen variant of each pass
    bool w_ready = false;           // W holds the inverse-x/curl fields of U0 (fused schedule)
    size_t cbytes = 0;              // bytes of one complex value
    size_t fbytes = 0;              // bytes of one half-spectrum field
    char* state = nullptr;          // U0 | U1 | Us, three fields each
    char* work = nullptr;           // W: six fields
    void* tw = nullptr;
    double* part = nullptr;         // diagnostic partials
    int npart_cap = 0;
    double* dout = nullptr;         // [E, Omega] of the last reduction
    double* hist = nullptr;         // [cap][2]
    int* hist_count = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // step without / with diagnostics
    bool has_state = false;
    long long steps = 0;
    std::string err;

    char* U0() const { return state; }
    char* U1() const { return state + 3 * fbytes; }
    char* Us() const { return state + 6 * fbytes; }
};

namespace {

int fail(dns_t* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_check(dns_t* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return DNS_OK;
    return fail(c, DNS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define DNS_TRY(ctx, call) \
    do { int _r = hip_check((ctx), (call), #call); if (_r != DNS_OK) return _r; } while (0)

int launched(dns_t* c, const char* what) { return hip_check(c, hipGetLastError(), what); }

bool valid_n(int N) { return N >= 8 && N <= 1024 && (N & (N - 1)) == 0; }

// Make the library stream wait for work already enqueued on the caller's
// stream, and the caller's stream wait for what the library enqueues.
int enter(dns_t* c) {
    DNS_TRY(c, hipEventRecord(c->ev_in, c->user));
    DNS_TRY(c, hipStreamWaitEvent(c->s, c->ev_in, 0));
    return DNS_OK;
}
int leave(dns_t* c) {
    DNS_TRY(c, hipEventRecord(c->ev_out, c->s));
    DNS_TRY(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
    return DNS_OK;
}

const double RK4_A[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
const double RK4_B[3] = {0.5, 0.5, 1.0};

dns::StageArgs stage_args(const dns_t* c, int stage, double* diag) {
    dns::StageArgs a;
    a.nu = c->nu;
    a.ca = stage >= 0 ? RK4_A[stage] * c->dt : 0.0;
    a.cb = (stage >= 0 && stage < 3) ? RK4_B[stage] * c->dt : 0.0;
    a.stage = stage;
    a.mask_lim = c->mask_lim;
    a.diag = diag;
    return a;
}

double inv_norm(int N) { return 1.0 / (2.0 * std::pow((double)N, 6)); }

// Enqueue one RHS evaluation of stage `stage` on stream s (Sec. 3.1
// computeRHS): the five passes of dns_kernels.hpp.
void launch_pass(dns_t* c, int pass, int variant, int stage, double* diag, hipStream_t s) {
    const dns::Ops* o = c->ops;
    switch (pass) {
        case dns::P_XINV: o->xinv[variant](stage <= 0 ? c->U0() : c->Us(), c->work, c->tw, s); break;
        case dns::P_YINV6: o->yinv6[variant](c->work, c->tw, s); break;
        case dns::P_ZCROSS: o->zcross[variant](c->work, c->tw, s); break;
        case dns::P_YFWD3: o->yfwd3[variant](c->work, c->tw, s); break;
        case dns::P_XRHS: {
            const dns::StageArgs a = stage_args(c, stage, diag);
            o->xrhs[variant](c->work, c->U0(), c->U1(), c->Us(), c->tw, a, s);
            break;
        }
        default: {
            const dns::StageArgs a = stage_args(c, stage, diag);
            o->xstage[variant](c->work, c->U0(), c->U1(), c->Us(), c->tw, a, s);
        }
    }
}

// Unfused stage: inverse x (+curl), inverse y, z, forward y, RHS + RK4.
void enqueue_stage(dns_t* c, int stage, bool with_diag, hipStream_t s) {
    for (int p = dns::P_XINV; p <= dns::P_XRHS; ++p)
        launch_pass(c, p, c->sel[p], stage, (p == dns::P_XRHS && stage == 3 && with_diag) ? c->part : nullptr, s);
}

int diag_groups(const dns_t* c) {
    return c->opts.fuse ? c->ops->xstage_groups[c->sel[dns::P_XSTAGE]] : c->ops->xrhs_groups[c->sel[dns::P_XRHS]];
}

// One RK4 step.  Fused schedule: W already holds the inverse-x/curl fields
// of U0 (prepared by the previous step's last kernel or by one k_xinv_curl
// launch), and each stage ends with the RHS pass fused with the next
// stage's inverse x pass, so a step is 16 kernels.  Unfused: 20 kernels.
void enqueue_step(dns_t* c, bool with_diag, hipStream_t s) {
    if (c->opts.fuse) {
        for (int st = 0; st < 4; ++st) {
            for (int p = dns::P_YINV6; p <= dns::P_YFWD3; ++p) launch_pass(c, p, c->sel[p], st, nullptr, s);
            launch_pass(c, dns::P_XSTAGE, c->sel[dns::P_XSTAGE], st, (st == 3 && with_diag) ? c->part : nullptr, s);
        }
    } else {
        for (int st = 0; st < 4; ++st) enqueue_stage(c, st, with_diag, s);
    }
    if (with_diag)
        dns::launch_diag_final(c->part, diag_groups(c), inv_norm(c->N), c->dout, c->hist, c->hist_count,
                               c->opts.history_cap, s);
}

int build_graph(dns_t* c, int which) {
    if (c->gexec[which]) return DNS_OK;
    hipGraph_t g = nullptr;
    DNS_TRY(c, hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
    enqueue_step(c, which == 1, c->s);
    hipError_t le = hipGetLastError();
    hipError_t ee = hipStreamEndCapture(c->s, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_check(c, le, "kernel launch during capture");
    }
    DNS_TRY(c, ee);
    hipError_t ie = hipGraphInstantiate(&c->gexec[which], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return hip_check(c, ie, "hipGraphInstantiate");
}

int reduce_state(dns_t* c, const void* U, double* E, double* W) {
    c->ops->diag_partial(U, c->part, c->s);
    int r = launched(c, "diag_partial");
    if (r) return r;
    dns::launch_diag_final(c->part, dns::DIAG_BLOCKS, inv_norm(c->N), c->dout, nullptr, nullptr, 0, c->s);
    r = launched(c, "diag_final");
    if (r) return r;
    double h[2];
    DNS_TRY(c, hipMemcpyAsync(h, c->dout, sizeof(h), hipMemcpyDeviceToHost, c->s));
    DNS_TRY(c, hipStreamSynchronize(c->s));
    if (E) *E = h[0];
    if (W) *W = h[1];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return fail(c, DNS_E_NONFINITE, "diagnostic is not finite");
    return DNS_OK;
}

void release(dns_t* c) {
    for (auto& g : c->gexec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    if (c->state) (void)hipFree(c->state);
    if (c->work) (void)hipFree(c->work);
    if (c->tw) (void)hipFree(c->tw);
    if (c->part) (void)hipFree(c->part);
    if (c->dout) (void)hipFree(c->dout);
    if (c->hist) (void)hipFree(c->hist);
    if (c->hist_count) (void)hipFree(c->hist_count);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    for (auto& e : c->ev_prof)
        if (e) (void)hipEventDestroy(e);
    if (c->s) (void)hipStreamDestroy(c->s);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void dns_default_opts(dns_opts* o) {
    if (!o) return;
    o->dealias = DNS_DEALIAS_TEXT;
    o->diag_every = 0;
    o->history_cap = 4096;
    o->use_graph = 1;
    o->autotune = 0;
    o->fuse = 1;
}

size_t dns_state_bytes(int N, int dtype) {
    if (!valid_n(N) || (dtype != DNS_FP64 && dtype != DNS_FP32)) return 0;
    const size_t rs = dtype == DNS_FP64 ? 8 : 4;
    return 15 * dns::field_size(N) * 2 * rs + (size_t)dns::tw_size(N) * 2 * rs;
}

int dns_create(int N, double nu, double dt, int dtype, dns_t** out) {
    return dns_create_ex(N, nu, dt, dtype, nullptr, nullptr, out);
}

int dns_create_ex(int N, double nu, double dt, int dtype, const dns_opts* opts, void* stream, dns_t** out) {
    if (!out) return DNS_E_INVAL;
    *out = nullptr;
    if (!valid_n(N) || !(nu >= 0.0) || !std::isfinite(nu) || !(dt > 0.0) || !std::isfinite(dt) ||
        (dtype != DNS_FP64 && dtype != DNS_FP32))
        return DNS_E_INVAL;
    dns_opts o;
    dns_default_opts(&o);
    if (opts) o = *opts;
    if ((o.dealias != DNS_DEALIAS_TEXT && o.dealias != DNS_DEALIAS_APPENDIX) || o.diag_every < 0 ||
        o.history_cap < 0 || (o.fuse != 0 && o.fuse != 1))
        return DNS_E_INVAL;

    dns_t* c = new (std::nothrow) dns_ctx();
    if (!c) return DNS_E_NOMEM;
    c->N = N;
    c->nu = nu;
    c->dt = dt;
    c->dtype = dtype;
    c->opts = o;
    c->mask_lim = (o.dealias == DNS_DEALIAS_TEXT) ? N : N + 2;
    c->user = (hipStream_t)stream;
    c->ops = dtype == DNS_FP64 ? dns::ops_f64(N) : dns::ops_f32(N);
    const size_t rs = c->ops->real_size;
    c->cbytes = 2 * rs;
    c->fbytes = dns::field_size(N) * c->cbytes;

    auto bail = [&](int code, const char* what, hipError_t e) {
        std::fprintf(stderr, "dns_create: %s: %s\n", what, hipGetErrorString(e));
        release(c);
        delete c;
        return code;
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking)) != hipSuccess)
        return bail(DNS_E_HIP, "hipStreamCreate", e);
    if ((e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreate(&c->ev_prof[0])) != hipSuccess || (e = hipEventCreate(&c->ev_prof[1])) != hipSuccess)
        return bail(DNS_E_HIP, "hipEventCreate", e);
    if ((e = hipMalloc((void**)&c->state, 9 * c->fbytes)) != hipSuccess) return bail(DNS_E_NOMEM, "hipMalloc(state)", e);
    if ((e = hipMalloc((void**)&c->work, 6 * c->fbytes)) != hipSuccess) return bail(DNS_E_NOMEM, "hipMalloc(work)", e);
    c->npart_cap = dns::DIAG_BLOCKS;
    for (int v = 0; v < c->ops->nvar[dns::P_XRHS]; ++v)
        if (c->ops->xrhs_groups[v] > c->npart_cap) c->npart_cap = c->ops->xrhs_groups[v];
    for (int p = 0; p < dns::P_COUNT; ++p) c->sel[p] = c->ops->def[p];
    if ((e = hipMalloc((void**)&c->part, 2 * sizeof(double) * c->npart_cap)) != hipSuccess ||
        (e = hipMalloc((void**)&c->dout, 2 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&c->hist, 2 * sizeof(double) * (o.history_cap > 0 ? o.history_cap : 1))) != hipSuccess ||
        (e = hipMalloc((void**)&c->hist_count, sizeof(int))) != hipSuccess)
        return bail(DNS_E_NOMEM, "hipMalloc(diagnostics)", e);

    // twiddles: long-double accurate, rounded to the context's precision
    const int ntw = c->ops->tw_count;
    std::vector<double> twd(2 * (size_t)ntw, 0.0);
    dns::make_twiddles(N, twd.data());
    if ((e = hipMalloc(&c->tw, (size_t)ntw * c->cbytes)) != hipSuccess) return bail(DNS_E_NOMEM, "hipMalloc(tw)", e);
    if (dtype == DNS_FP64) {
        e = hipMemcpy(c->tw, twd.data(), (size_t)ntw * c->cbytes, hipMemcpyHostToDevice);
    } else {
        std::vector<float> twf(twd.size());
        for (size_t i = 0; i < twd.size(); ++i) twf[i] = (float)twd[i];
        e = hipMemcpy(c->tw, twf.data(), (size_t)ntw * c->cbytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return bail(DNS_E_HIP, "hipMemcpy(tw)", e);
    if ((e = hipMemset(c->state, 0, 9 * c->fbytes)) != hipSuccess ||
        (e = hipMemset(c->hist_count, 0, sizeof(int))) != hipSuccess)
        return bail(DNS_E_HIP, "hipMemset", e);
    if (o.autotune) {
        const int r = dns_autotune(c, 3);
        if (r != DNS_OK) {
            release(c);
            delete c;
            return r;
        }
    }
    *out = c;
    return DNS_OK;
}

int dns_destroy(dns_t* c) {
    if (!c) return DNS_OK;
    if (c->s) (void)hipStreamSynchronize(c->s);
    release(c);
    delete c;
    return DNS_OK;
}

static int reset_counters(dns_t* c) {
    c->steps = 0;
    c->has_state = true;
    DNS_TRY(c, hipMemsetAsync(c->hist_count, 0, sizeof(int), c->s));
    return DNS_OK;
}

int dns_set_velocity(dns_t* c, const void* u) {
    if (!c || !u) return fail(c, DNS_E_INVAL, "null argument");
    int r = enter(c);
    if (r) return r;
    c->w_ready = false;
    c->ops->zr2c(u, c->work, c->tw, c->s);
    c->ops->yfwd3[c->sel[dns::P_YFWD3]](c->work, c->tw, c->s);
    c->ops->xfwd3(c->work, c->U0(), c->tw, c->s);
    if ((r = launched(c, "set_velocity"))) return r;
    if ((r = reset_counters(c))) return r;
    return leave(c);
}

int dns_set_spectral(dns_t* c, const void* uh) {
    if (!c || !uh) return fail(c, DNS_E_INVAL, "null argument");
    int r = enter(c);
    if (r) return r;
    c->w_ready = false;
    c->ops->layout(uh, c->U0(), true, c->s);
    if ((r = launched(c, "set_spectral"))) return r;
    if ((r = reset_counters(c))) return r;
    return leave(c);
}

int dns_get_spectral(dns_t* c, void* uh) {
    if (!c || !uh) return fail(c, DNS_E_INVAL, "null argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    int r = enter(c);
    if (r) return r;
    c->ops->layout(c->U0(), uh, false, c->s);
    if ((r = launched(c, "get_spectral"))) return r;
    return leave(c);
}

int dns_get_velocity(dns_t* c, void* u) {
    if (!c || !u) return fail(c, DNS_E_INVAL, "null argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    int r = enter(c);
    if (r) return r;
    c->w_ready = false;
    c->ops->xinv3(c->U0(), c->work, c->tw, c->s);
    c->ops->yinv3(c->work, c->tw, c->s);
    c->ops->zc2r(c->work, u, c->tw, c->s);
    if ((r = launched(c, "get_velocity"))) return r;
    return leave(c);
}

int dns_forward(dns_t* c, const void* u, void* uh) {
    if (!c || !u || !uh) return fail(c, DNS_E_INVAL, "null argument");
    int r = enter(c);
    if (r) return r;
    c->w_ready = false;
    c->ops->zr2c(u, c->work, c->tw, c->s);
    c->ops->yfwd3[c->sel[dns::P_YFWD3]](c->work, c->tw, c->s);
    c->ops->xfwd3(c->work, c->Us(), c->tw, c->s);
    c->ops->layout(c->Us(), uh, false, c->s);
    if ((r = launched(c, "forward"))) return r;
    return leave(c);
}

int dns_inverse(dns_t* c, const void* uh, void* u) {
    if (!c || !u || !uh) return fail(c, DNS_E_INVAL, "null argument");
    int r = enter(c);
    if (r) return r;
    c->w_ready = false;
    c->ops->layout(uh, c->Us(), true, c->s);
    c->ops->xinv3(c->Us(), c->work, c->tw, c->s);
    c->ops->yinv3(c->work, c->tw, c->s);
    c->ops->zc2r(c->work, u, c->tw, c->s);
    if ((r = launched(c, "inverse"))) return r;
    return leave(c);
}

int dns_step(dns_t* c, int nsteps) {
    if (!c || nsteps < 0) return fail(c, DNS_E_INVAL, "bad argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    if (nsteps == 0) return DNS_OK;
    int r = enter(c);
    if (r) return r;
    if (c->opts.fuse && !c->w_ready) {
        launch_pass(c, dns::P_XINV, c->sel[dns::P_XINV], 0, nullptr, c->s);
        if ((r = launched(c, "xinv_curl"))) return r;
    }
    for (int i = 0; i < nsteps; ++i) {
        const long long n = c->steps + 1;
        const bool diag = c->opts.diag_every > 0 && (n % c->opts.diag_every) == 0;
        if (c->opts.use_graph) {
            if ((r = build_graph(c, diag ? 1 : 0))) return r;
            DNS_TRY(c, hipGraphLaunch(c->gexec[diag ? 1 : 0], c->s));
        } else {
            enqueue_step(c, diag, c->s);
            if ((r = launched(c, "step"))) return r;
        }
        c->steps = n;
    }
    c->w_ready = c->opts.fuse != 0;
    return leave(c);
}

int dns_rhs(dns_t* c, void* out) {
    if (!c || !out) return fail(c, DNS_E_INVAL, "null argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    int r = enter(c);
    if (r) return r;
    c->w_ready = false;
    enqueue_stage(c, -1, false, c->s);
    c->ops->layout(c->U1(), out, false, c->s);
    if ((r = launched(c, "rhs"))) return r;
    return leave(c);
}

int dns_diagnostics(dns_t* c, double* E, double* W) {
    if (!c) return DNS_E_INVAL;
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    int r = enter(c);
    if (r) return r;
    r = reduce_state(c, c->U0(), E, W);
    int r2 = leave(c);
    return r ? r : r2;
}

int dns_energy(dns_t* c, double* E) {
    if (!c || !E) return fail(c, DNS_E_INVAL, "null argument");
    return dns_diagnostics(c, E, nullptr);
}

int dns_enstrophy(dns_t* c, double* W) {
    if (!c || !W) return fail(c, DNS_E_INVAL, "null argument");
    return dns_diagnostics(c, nullptr, W);
}

int dns_history(dns_t* c, double* E, double* W, int max, int* count) {
    if (!c || !count || max < 0 || (max > 0 && (!E || !W))) return fail(c, DNS_E_INVAL, "bad argument");
    DNS_TRY(c, hipStreamSynchronize(c->s));
    int n = 0;
    DNS_TRY(c, hipMemcpy(&n, c->hist_count, sizeof(int), hipMemcpyDeviceToHost));
    *count = n;
    const int avail = n < c->opts.history_cap ? n : c->opts.history_cap;
    const int m = avail < max ? avail : max;
    if (m > 0) {
        std::vector<double> h(2 * (size_t)m);
        DNS_TRY(c, hipMemcpy(h.data(), c->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int i = 0; i < m; ++i) {
            E[i] = h[2 * i];
            W[i] = h[2 * i + 1];
        }
    }
    return DNS_OK;
}

int dns_steps_taken(const dns_t* c, long long* steps) {
    if (!c || !steps) return DNS_E_INVAL;
    *steps = c->steps;
    return DNS_OK;
}

int dns_synchronize(dns_t* c) {
    if (!c) return DNS_E_INVAL;
    DNS_TRY(c, hipStreamSynchronize(c->s));
    return DNS_OK;
}

static const char* kPassNames[dns::P_COUNT] = {"xinv_curl", "yinv6", "zcross", "yfwd3", "xrhs_rk4", "xstage"};

int dns_profile_step(dns_t* c, int nsteps, float* ms, const char** names, int max, int* count) {
    if (!c || !ms || !count || nsteps <= 0 || max < 0) return fail(c, DNS_E_INVAL, "bad argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    int r = enter(c);
    if (r) return r;
    double acc[dns::P_COUNT] = {0, 0, 0, 0, 0, 0};
    int launches[dns::P_COUNT] = {0, 0, 0, 0, 0, 0};
    auto timed = [&](int k, int st) -> int {
        DNS_TRY(c, hipEventRecord(c->ev_prof[0], c->s));
        launch_pass(c, k, c->sel[k], st, nullptr, c->s);
        int rr = launched(c, kPassNames[k]);
        if (rr) return rr;
        DNS_TRY(c, hipEventRecord(c->ev_prof[1], c->s));
        DNS_TRY(c, hipEventSynchronize(c->ev_prof[1]));
        float t = 0.f;
        DNS_TRY(c, hipEventElapsedTime(&t, c->ev_prof[0], c->ev_prof[1]));
        acc[k] += t;
        launches[k] += 1;
        return DNS_OK;
    };
    for (int n = 0; n < nsteps; ++n) {
        if (c->opts.fuse) {
            if (!c->w_ready && (r = timed(dns::P_XINV, 0))) return r;
            for (int st = 0; st < 4; ++st) {
                for (int k = dns::P_YINV6; k <= dns::P_YFWD3; ++k)
                    if ((r = timed(k, st))) return r;
                if ((r = timed(dns::P_XSTAGE, st))) return r;
            }
            c->w_ready = true;
        } else {
            for (int st = 0; st < 4; ++st)
                for (int k = dns::P_XINV; k <= dns::P_XRHS; ++k)
                    if ((r = timed(k, st))) return r;
        }
        c->steps += 1;
    }
    const int m = max < dns::P_COUNT ? max : dns::P_COUNT;
    for (int k = 0; k < m; ++k) {
        ms[k] = launches[k] ? (float)(acc[k] / launches[k]) : 0.f;
        if (names) names[k] = kPassNames[k];
    }
    *count = m;
    return leave(c);
}

// Time every tile-shape variant of every pass on the context's buffers and
// keep the fastest.  The RHS pass is timed in its stage-1 form, which reads
// U0 but writes only U1 and Us, so the current state is preserved.
int dns_autotune(dns_t* c, int reps) {
    if (!c || reps < 0) return fail(c, DNS_E_INVAL, "bad argument");
    if (reps == 0) reps = 3;
    int r = enter(c);
    if (r) return r;
    for (auto& g : c->gexec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    for (int p = 0; p < dns::P_COUNT; ++p) {
        float best = 1e30f;
        int bestv = c->sel[p];
        for (int v = 0; v < c->ops->nvar[p]; ++v) {
            launch_pass(c, p, v, 1, nullptr, c->s);                  // warm-up
            DNS_TRY(c, hipEventRecord(c->ev_prof[0], c->s));
            for (int i = 0; i < reps; ++i) launch_pass(c, p, v, 1, nullptr, c->s);
            if ((r = launched(c, kPassNames[p]))) return r;
            DNS_TRY(c, hipEventRecord(c->ev_prof[1], c->s));
            DNS_TRY(c, hipEventSynchronize(c->ev_prof[1]));
            float t = 0.f;
            DNS_TRY(c, hipEventElapsedTime(&t, c->ev_prof[0], c->ev_prof[1]));
            if (t < best) { best = t; bestv = v; }
        }
        c->sel[p] = bestv;
    }
    c->w_ready = false;
    return leave(c);
}

int dns_get_plan(const dns_t* c, int* widths, int max, int* count) {
    if (!c || !count || max < 0 || (max > 0 && !widths)) return DNS_E_INVAL;
    const int m = max < dns::P_COUNT ? max : dns::P_COUNT;
    for (int p = 0; p < m; ++p) widths[p] = c->ops->width[p][c->sel[p]];
    *count = dns::P_COUNT;
    return DNS_OK;
}

int dns_set_plan(dns_t* c, const int* widths, int n) {
    if (!c || !widths || n != dns::P_COUNT) return fail(c, DNS_E_INVAL, "bad argument");
    int sel[dns::P_COUNT];
    for (int p = 0; p < dns::P_COUNT; ++p) {
        sel[p] = -1;
        for (int v = 0; v < c->ops->nvar[p]; ++v)
            if (c->ops->width[p][v] == widths[p]) sel[p] = v;
        if (sel[p] < 0) return fail(c, DNS_E_INVAL, "no variant of that width for this N and dtype");
    }
    DNS_TRY(c, hipStreamSynchronize(c->s));
    for (auto& g : c->gexec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    for (int p = 0; p < dns::P_COUNT; ++p) c->sel[p] = sel[p];
    c->w_ready = false;
    return DNS_OK;
}

int dns_plan_variants(const dns_t* c, int pass, int* widths, int max, int* count) {
    if (!c || !count || pass < 0 || pass >= dns::P_COUNT || max < 0 || (max > 0 && !widths)) return DNS_E_INVAL;
    const int n = c->ops->nvar[pass];
    for (int v = 0; v < n && v < max; ++v) widths[v] = c->ops->width[pass][v];
    *count = n;
    return DNS_OK;
}

const char* dns_strerror(int s) {
    switch (s) {
        case DNS_OK: return "ok";
        case DNS_E_INVAL: return "invalid argument";
        case DNS_E_NOMEM: return "device allocation failed";
        case DNS_E_HIP: return "HIP runtime error";
        case DNS_E_STATE: return "invalid state (no velocity set)";
        case DNS_E_NONFINITE: return "non-finite diagnostic";
        case DNS_E_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* dns_last_error(const dns_t* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
