// C ABI of the MI355X pseudo-spectral RK4 library (declared in dns.h):
// context lifetime, stream ordering, the RK4 step schedule, graph replay,
// transforms, diagnostics and profiling.
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "dns.h"
#include "dns_ops.hpp"

namespace dns {

// ---------------------------------------------------------------------------
// Twiddle factors exp(-2 pi i m / n), m reduced modulo n before the angle is
// formed, evaluated in long double and exact at the multiples of pi/4 where
// the value is 0, +-1 or +-sqrt(1/2) per component.
// ---------------------------------------------------------------------------
void unit_root(long m, long n, double* re, double* im) {
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

void make_twiddles(int N, double* out, int rs) {
    const int ns = num_stages(N, rs);
    for (int s = 1; s < ns; ++s) {
        const int L = span_at(N, s, rs), Rr = radix_at(N, s, rs);
        double* w = out + 2 * tw_offset(N, s, rs);
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

// Copy of nrows rows of row_bytes bytes (a multiple of 16), row r at byte
// offset r * pitch in both buffers; one 16-byte vector per thread, so the
// row_bytes / 16 threads of a row issue one row_bytes request.
__global__ __launch_bounds__(256) void k_copy_rows(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   size_t nrows, unsigned row_vecs, size_t pitch_vecs) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t r = i / row_vecs;
    if (r >= nrows) return;
    const size_t at = r * pitch_vecs + (i - r * row_vecs);
    dst[at] = src[at];
}

}  // namespace dns

// ---------------------------------------------------------------------------
// Context.  A context holds `members` independent simulations of one size,
// precision, viscosity and time step (1 for dns_create); the stage kernels
// advance all members in one launch (grid y = member).
// ---------------------------------------------------------------------------
struct dns_ctx {
    int N = 0, dtype = 0;
    double nu = 0, dt = 0;
    dns_opts opts{};
    int mask_lim = 0;
    int members = 1;
    hipStream_t user = nullptr;     // caller's stream (ordering reference)
    hipStream_t s = nullptr;        // library stream (graph capture needs a non-null stream)
    bool own_stream = true;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipEvent_t ev_prof[2] = {nullptr, nullptr};
    const dns::Ops* ops = nullptr;
    int sel[dns::P_COUNT] = {0, 0, 0, 0, 0, 0};   // chosen variant of each pass
    bool w_ready = false;           // W holds the inverse-x/curl fields of U0 (fused schedule)
    size_t fs = 0;                  // complex values per half-spectrum field
    size_t cbytes = 0;              // bytes of one complex value
    size_t fbytes = 0;              // bytes of one half-spectrum field
    char* mem = nullptr;            // one device block holding every buffer below
    bool own_mem = true;            // false: the block is the caller's workspace
    char* state = nullptr;          // per member: U0 | U1 | Us, three fields each
    char* work = nullptr;           // per member: W, six fields
    void* tw = nullptr;
    void* mfma_tw = nullptr;        // w_N^j (j < N), then the N/16-point twiddle table (mfma_dft)
    double* part = nullptr;         // diagnostic partials, npart_cap pairs per member
    int npart_cap = 0;
    double* dout = nullptr;         // [member][E, Omega] of the last reduction
    double* hist = nullptr;         // [member][cap][2]
    int* hist_count = nullptr;      // [member]
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // step without / with diagnostics
    bool has_state = false;
    bool inject_fault = false;      // DNS_FAULT_INJECT=launch at creation: launch checks fail
    long long steps = 0;
    std::string err;

    char* U0(int m = 0) const { return state + (size_t)m * 9 * fbytes; }
    char* U1(int m = 0) const { return U0(m) + 3 * fbytes; }
    char* Us(int m = 0) const { return U0(m) + 6 * fbytes; }
    char* W(int m = 0) const { return work + (size_t)m * 6 * fbytes; }
    dns::Batch batch() const { return dns::Batch{members, 9 * fs, 6 * fs}; }
    int hist_cap() const { return opts.history_cap > 0 ? opts.history_cap : 1; }
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

// Status of the kernels just enqueued.  With DNS_FAULT_INJECT=launch in the
// environment when the context was created, every check reports DNS_E_HIP
// (after consuming the real status), so that callers can test their error
// handling without a device fault.
int launched(dns_t* c, const char* what) {
    const int r = hip_check(c, hipGetLastError(), what);
    if (r == DNS_OK && c && c->inject_fault) return fail(c, DNS_E_HIP, std::string(what) + ": injected launch failure");
    return r;
}

bool valid_n(int N) { return N >= 8 && N <= 1024 && (N & (N - 1)) == 0; }

// Make the library stream wait for work already enqueued on the caller's
// stream, and the caller's stream wait for what the library enqueues.
int enter(dns_t* c) {
    if (c->user == c->s) return DNS_OK;
    DNS_TRY(c, hipEventRecord(c->ev_in, c->user));
    DNS_TRY(c, hipStreamWaitEvent(c->s, c->ev_in, 0));
    return DNS_OK;
}
int leave(dns_t* c) {
    if (c->user == c->s) return DNS_OK;
    DNS_TRY(c, hipEventRecord(c->ev_out, c->s));
    DNS_TRY(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
    return DNS_OK;
}

// Classic RK4 (Appendix solver): stage offsets b and final weights a; the
// stage kernels use b_s dt and a_3 dt (the other weights enter through the
// regrouped final sum, see the stage update in dns_kernels.hpp).
const double RK4_A[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
const double RK4_B[3] = {0.5, 0.5, 1.0};

dns::StageArgs stage_args(const dns_t* c, int stage, double* diag) {
    dns::StageArgs a;
    a.nu = c->nu;
    a.ca = stage == 3 ? RK4_A[3] * c->dt : (stage == 4 ? c->dt : 0.0);
    a.cb = (stage >= 0 && stage < 3) ? RK4_B[stage] * c->dt : 0.0;
    a.stage = stage;
    a.mask_lim = c->mask_lim;
    a.diag = diag;
    return a;
}

double inv_norm(int N) { return 1.0 / (2.0 * std::pow((double)N, 6)); }

// Stages of one time step: the four RK4 stages 0..3 (Appendix solver), or
// the single forward Euler stage 4 (Sec. 3.1 main loop).
int step_stages(const dns_t* c) { return c->opts.integrator == DNS_EULER ? 1 : 4; }
int stage_id(const dns_t* c, int i) { return c->opts.integrator == DNS_EULER ? 4 : i; }
int last_stage(const dns_t* c) { return stage_id(c, step_stages(c) - 1); }

int diag_groups(const dns_t* c) {
    return c->opts.fuse ? c->ops->xstage_groups[c->sel[dns::P_XSTAGE]] : c->ops->xrhs_groups[c->sel[dns::P_XRHS]];
}

// The N/16-point twiddle table that follows the N unit roots in mfma_tw.
const void* mfma_tw2(const dns_t* c) { return (const char*)c->mfma_tw + (size_t)c->N * c->cbytes; }

// Curl placement of the context's plan: 1 = the inverse y pass forms the
// vorticity from the x pass's five fields, 0 = the x pass writes six.
int plan_cy(const dns_t* c) { return c->ops->var[dns::P_XSTAGE][c->sel[dns::P_XSTAGE]].cy; }

// Twiddle table of radix plan rs in the context's table.
const void* tw_of(const dns_t* c, int rs) { return (const char*)c->tw + (size_t)c->ops->tw_base[rs] * c->cbytes; }

// Launch one pass of stage `stage` for all members (member < 0, one batched
// launch) or for one member only.  diag: fused diagnostic partials of
// member 0; member m's sit 2 * groups * m doubles further.
void launch_pass(dns_t* c, int pass, int variant, int stage, double* diag, hipStream_t s, int member = -1) {
    const dns::Ops* o = c->ops;
    const void* tw = tw_of(c, o->var[pass][variant].rs);
    const int m = member < 0 ? 0 : member;
    const dns::Batch b = member < 0 ? c->batch() : dns::Batch{1, 0, 0};
    double* dg = diag ? diag + (size_t)2 * diag_groups(c) * m : nullptr;
    switch (pass) {
        case dns::P_XINV: {
            // the stage's velocity: U0 at RK4 stage 0, for the RHS alone and
            // for the Euler step; the stage velocity Us at RK4 stages 1..3
            const bool from_u0 = stage <= 0 || stage == 4;
            o->xinv[variant](from_u0 ? c->U0(m) : c->Us(m), c->W(m), tw, b, s);
            break;
        }
        case dns::P_YINV6:
            if (c->opts.mfma_dft)
                o->ymfma_inv6[plan_cy(c)](c->W(m), c->tw, c->mfma_tw, mfma_tw2(c), b, s);
            else
                o->yinv6[variant](c->W(m), tw, b, s);
            break;
        case dns::P_ZCROSS: o->zcross[variant](c->W(m), tw, b, s); break;
        case dns::P_YFWD3:
            if (c->opts.mfma_dft)
                o->ymfma_fwd3(c->W(m), c->tw, c->mfma_tw, mfma_tw2(c), b, s);
            else
                o->yfwd3[variant](c->W(m), tw, b, s);
            break;
        case dns::P_XRHS: {
            const dns::StageArgs a = stage_args(c, stage, dg);
            o->xrhs[variant](c->W(m), c->U0(m), c->U1(m), c->Us(m), tw, a, b, s);
            break;
        }
        default: {
            const dns::StageArgs a = stage_args(c, stage, dg);
            o->xstage[variant](c->W(m), c->U0(m), c->U1(m), c->Us(m), tw, a, b, s);
        }
    }
}

// Unfused stage: inverse x (+curl), inverse y, z, forward y, RHS + RK4.
void enqueue_stage(dns_t* c, int stage, bool with_diag, hipStream_t s, int member = -1) {
    for (int p = dns::P_XINV; p <= dns::P_XRHS; ++p)
        launch_pass(c, p, c->sel[p], stage, (p == dns::P_XRHS && stage == last_stage(c) && with_diag) ? c->part : nullptr, s,
                    member);
}

void enqueue_diag_final(dns_t* c, hipStream_t s, int member) {
    const int groups = diag_groups(c);
    const int m0 = member < 0 ? 0 : member, m1 = member < 0 ? c->members : member + 1;
    for (int m = m0; m < m1; ++m)
        dns::launch_diag_final(c->part + (size_t)2 * groups * m, groups, inv_norm(c->N), c->dout + 2 * m,
                               c->hist + (size_t)2 * c->hist_cap() * m, c->hist_count + m, c->opts.history_cap, s);
}

// One RK4 step.  Fused schedule: W already holds the inverse-x/curl fields
// of U0 (prepared by the previous step's last kernel or by one k_xinv_curl
// launch), and each stage ends with the RHS pass fused with the next
// stage's inverse x pass, so a step is 16 kernels.  Unfused: 20 kernels.
void enqueue_step(dns_t* c, bool with_diag, hipStream_t s, int member = -1) {
    if (c->opts.fuse) {
        for (int i = 0; i < step_stages(c); ++i) {
            const int st = stage_id(c, i);
            for (int p = dns::P_YINV6; p <= dns::P_YFWD3; ++p) launch_pass(c, p, c->sel[p], st, nullptr, s, member);
            launch_pass(c, dns::P_XSTAGE, c->sel[dns::P_XSTAGE], st,
                        (st == last_stage(c) && with_diag) ? c->part : nullptr, s, member);
        }
    } else {
        for (int i = 0; i < step_stages(c); ++i) enqueue_stage(c, stage_id(c, i), with_diag, s, member);
    }
    if (with_diag) enqueue_diag_final(c, s, member);
}

void drop_graphs(dns_t* c) {
    for (auto& g : c->gexec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
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

// The curl/inverse-x fields of U0 that the fused schedule starts from.
int prepare_w(dns_t* c) {
    if (!c->opts.fuse || c->w_ready) return DNS_OK;
    launch_pass(c, dns::P_XINV, c->sel[dns::P_XINV], 0, nullptr, c->s);
    return launched(c, "xinv_curl");
}

// Energy and enstrophy of member m's U0 (synchronous, fixed order).
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
    drop_graphs(c);
    if (c->mem && c->own_mem) (void)hipFree(c->mem);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    for (auto& e : c->ev_prof)
        if (e) (void)hipEventDestroy(e);
    if (c->s && c->own_stream) (void)hipStreamDestroy(c->s);
}

// Process-wide cache of autotuned plans, keyed by (device identity, N,
// dtype, simulations per launch, tuning mode).  A plan is stored as the
// descriptor (width, XCD grouping, y elements, curl placement, radix plan,
// z-pass pad) of the chosen variant of every pass, so that a plan read back
// from a file written by another build is used only where those variants
// still exist.  dns_autotune stores its
// result; a context created with opts.autotune takes a cached plan instead
// of timing again.  With DNS_PLAN_CACHE set to a file path, the cache is
// read from that file on first use and written back after every autotune;
// dns_plan_cache_save / dns_plan_cache_load do the same explicitly.
using PlanKey = std::tuple<std::string, int, int, int, int>;
using Plan = std::array<dns::Variant, dns::P_COUNT>;
std::mutex g_plan_mu;
std::map<PlanKey, Plan> g_plans;
bool g_plan_env_loaded = false;

// "arch|name|compute units" of the current device ('"' and '|' removed).
std::string device_identity() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "device" + std::to_string(dev);
    std::string id = std::string(p.gcnArchName) + "|" + p.name + "|" + std::to_string(p.multiProcessorCount);
    for (char& ch : id)
        if (ch == '"' || ch == '\\' || ch < 32) ch = ' ';
    return id;
}

PlanKey plan_key(const dns_t* c, int mode) { return PlanKey{device_identity(), c->N, c->dtype, c->members, mode}; }

// Cache file: valid JSON, one plan per line.
int plan_cache_write(const char* path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return DNS_E_INVAL;
    std::fprintf(f, "{\"format\": \"dns-plan-cache-2\", \"plans\": [\n");
    size_t i = 0;
    for (const auto& kv : g_plans) {
        std::fprintf(f,
                     "{\"device\": \"%s\", \"N\": %d, \"dtype\": %d, \"members\": %d, \"mode\": %d, "
                     "\"variants\": [",
                     std::get<0>(kv.first).c_str(), std::get<1>(kv.first), std::get<2>(kv.first),
                     std::get<3>(kv.first), std::get<4>(kv.first));
        for (int p = 0; p < dns::P_COUNT; ++p) {
            const dns::Variant& v = kv.second[p];
            std::fprintf(f, "%s[%d, %d, %d, %d, %d, %d]", p ? ", " : "", v.width, v.pair, v.ye, v.cy, v.rs, v.pad);
        }
        std::fprintf(f, "]}%s\n", ++i < g_plans.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) return DNS_E_INVAL;
    return DNS_OK;
}

// Read the plans of a cache file into the cache; the number read, or -1.
int plan_cache_read(const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    int n = 0;
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
        const char* d = std::strstr(line, "{\"device\": \"");
        if (!d) continue;
        d += 12;
        const char* q = std::strchr(d, '"');
        if (!q) continue;
        const std::string dev(d, q);
        constexpr int NV = 4 + 6 * dns::P_COUNT;   // N, dtype, members, mode, 6 per variant
        long v[NV];
        int k = 0;
        for (const char* t = q + 1; *t && k < (int)(sizeof v / sizeof v[0]);) {
            if (*t == '-' || (*t >= '0' && *t <= '9')) {
                char* end = nullptr;
                v[k++] = std::strtol(t, &end, 10);
                t = end;
            } else {
                ++t;
            }
        }
        if (k != NV || (v[3] != DNS_TUNE_REPRODUCIBLE && v[3] != DNS_TUNE_FASTEST)) continue;
        Plan p;
        for (int i = 0; i < dns::P_COUNT; ++i) {
            const long* d = v + 4 + 6 * i;
            p[i] = dns::Variant{(int)d[0], (int)d[1], (int)d[2], (int)d[3], (int)d[4], (int)d[5]};
        }
        g_plans[PlanKey{dev, (int)v[0], (int)v[1], (int)v[2], (int)v[3]}] = p;
        ++n;
    }
    std::fclose(f);
    return n;
}

// Load DNS_PLAN_CACHE once (caller holds g_plan_mu).
void plan_env_load() {
    if (g_plan_env_loaded) return;
    g_plan_env_loaded = true;
    const char* path = std::getenv("DNS_PLAN_CACHE");
    if (path && *path) (void)plan_cache_read(path);
}

bool plan_consistent(const dns_t* c, const int* sel);

void store_plan(const dns_t* c, int mode) {
    Plan p;
    for (int k = 0; k < dns::P_COUNT; ++k) p[k] = c->ops->var[k][c->sel[k]];
    const PlanKey key = plan_key(c, mode);
    std::lock_guard<std::mutex> lock(g_plan_mu);
    plan_env_load();
    g_plans[key] = p;
    const char* path = std::getenv("DNS_PLAN_CACHE");
    if (path && *path) (void)plan_cache_write(path);
}

bool same_variant(const dns::Variant& a, const dns::Variant& b) {
    return a.width == b.width && a.pair == b.pair && a.ye == b.ye && a.cy == b.cy && a.rs == b.rs && a.pad == b.pad;
}

bool load_plan(dns_t* c, int mode) {
    const PlanKey key = plan_key(c, mode);
    std::lock_guard<std::mutex> lock(g_plan_mu);
    plan_env_load();
    auto it = g_plans.find(key);
    if (it == g_plans.end()) return false;
    int sel[dns::P_COUNT];
    for (int k = 0; k < dns::P_COUNT; ++k) {
        sel[k] = -1;
        const dns::Variant& want = it->second[k];
        for (int v = 0; v < c->ops->nvar[k]; ++v) {
            const dns::Variant& d = c->ops->var[k][v];
            if (same_variant(d, want)) sel[k] = v;
        }
        if (sel[k] < 0) return false;   // a variant of another build
    }
    if (!plan_consistent(c, sel)) return false;
    for (int k = 0; k < dns::P_COUNT; ++k) c->sel[k] = sel[k];
    return true;
}

// Tuned plan for a new context (opts.autotune 1: reproducible, 2: fastest):
// from the cache, else timed (and cached).
int tune_new(dns_t* c) {
    const int mode = c->opts.autotune == 2 ? DNS_TUNE_FASTEST : DNS_TUNE_REPRODUCIBLE;
    if (load_plan(c, mode)) return DNS_OK;
    return dns_autotune_ex(c, 3, mode);
}

// Variants a reproducible plan is made of: radix plan 0 and the standard
// z-pass pad (their results are bitwise those of the default plan).
bool reference_shape(int p, const dns::Variant& d) { return d.rs == 0 && d.pad == (p == dns::P_ZCROSS ? 8 : 0); }

// A plan is consistent when the passes whose fields depend on the curl
// placement (inverse x, inverse y, fused stage) agree on it, and, with the
// matrix-core option, that y kernel exists for it.
bool plan_consistent(const dns_t* c, const int* sel) {
    const dns::Ops& o = *c->ops;
    const int a = o.var[dns::P_XINV][sel[dns::P_XINV]].cy;
    const int b = o.var[dns::P_YINV6][sel[dns::P_YINV6]].cy;
    const int d = o.var[dns::P_XSTAGE][sel[dns::P_XSTAGE]].cy;
    if (a != b || b != d) return false;
    return !c->opts.mfma_dft || o.ymfma_inv6[a] != nullptr;
}

// Variant of pass p that matches the schedule (curl placement cy, y elements
// ye for the y passes, XCD pairing pair where a paired variant exists), of
// width w if there is one, else the widest narrower, else the narrowest
// wider; -1 if no variant matches the schedule.
int find_variant(const dns::Ops& o, int p, int w, int cy, int ye, int pair) {
    int best = -1;
    auto rank = [&](const dns::Variant& d) {   // larger is better
        const int wr = d.width == w ? 3 * 4096 : (d.width < w ? 2 * 4096 + d.width : 4096 - d.width);
        return 2 * wr + (d.pair == pair ? 1 : 0);
    };
    for (int v = 0; v < o.nvar[p]; ++v) {
        const dns::Variant& d = o.var[p][v];
        if (!reference_shape(p, d)) continue;
        if (d.cy >= 0 && d.cy != cy) continue;
        if (d.ye > 0 && d.ye != ye && !(p == dns::P_YINV6 && cy == 1)) continue;
        if (best < 0 || rank(d) > rank(o.var[p][best])) best = v;
    }
    return best;
}

// Select, for every pass, the variant of the current width that runs the
// schedule (y_elems 0, curl_in_y -1 and xcd_pair -1 keep the defaults).
int apply_schedule(dns_t* c, int y_elems, int curl_in_y, int xcd_pair) {
    const dns::Ops& o = *c->ops;
    const int cy = curl_in_y >= 0 ? curl_in_y : o.var[dns::P_XSTAGE][o.def[dns::P_XSTAGE]].cy;
    const int ye = y_elems > 0 ? y_elems : o.var[dns::P_YFWD3][o.def[dns::P_YFWD3]].ye;
    const int pair = xcd_pair >= 0 ? xcd_pair : o.var[dns::P_XSTAGE][o.def[dns::P_XSTAGE]].pair;
    int sel[dns::P_COUNT];
    for (int p = 0; p < dns::P_COUNT; ++p) {
        sel[p] = find_variant(o, p, o.var[p][c->sel[p]].width, cy, ye, pair);
        if (sel[p] < 0) return fail(c, DNS_E_UNSUPPORTED, "schedule not provided for this N and dtype");
    }
    if (pair == 1) {
        bool any = false;
        for (int p : {dns::P_XINV, dns::P_XRHS, dns::P_XSTAGE}) any = any || o.var[p][sel[p]].pair == 1;
        if (!any) return fail(c, DNS_E_UNSUPPORTED, "no XCD-paired x pass for this N and dtype");
    }
    if (!plan_consistent(c, sel)) return fail(c, DNS_E_UNSUPPORTED, "schedule not provided with these options");
    for (int p = 0; p < dns::P_COUNT; ++p) c->sel[p] = sel[p];
    return DNS_OK;
}

int check_args(int N, double nu, double dt, int dtype, const dns_opts& o) {
    if (!valid_n(N) || !(nu >= 0.0) || !std::isfinite(nu) || !(dt > 0.0) || !std::isfinite(dt) ||
        (dtype != DNS_FP64 && dtype != DNS_FP32))
        return DNS_E_INVAL;
    if ((o.dealias != DNS_DEALIAS_TEXT && o.dealias != DNS_DEALIAS_APPENDIX) || o.diag_every < 0 ||
        o.history_cap < 0 || (o.fuse != 0 && o.fuse != 1) ||
        (o.integrator != DNS_RK4 && o.integrator != DNS_EULER) || (o.mfma_dft != 0 && o.mfma_dft != 1))
        return DNS_E_INVAL;
    if (o.mfma_dft && (dtype != DNS_FP32 || N < 64)) return DNS_E_UNSUPPORTED;
    if ((o.y_elems != 0 && o.y_elems != 8 && o.y_elems != 16 && o.y_elems != 32) || o.curl_in_y < -1 ||
        o.curl_in_y > 1 || o.xcd_pair < -1 || o.xcd_pair > 1 || o.autotune < 0 || o.autotune > 2)
        return DNS_E_INVAL;
    return DNS_OK;
}

// Byte offsets of a context's device buffers inside its one memory block,
// each 256-byte aligned.
struct Carve {
    size_t state, work, part, dout, hist, hist_count, tw, mfma_tw, total;
    int npart_cap;
};

Carve carve(const dns::Ops* ops, int N, const dns_opts& o, int members) {
    Carve k{};
    const size_t cb = 2 * ops->real_size, fb = ops->fs * cb;
    k.npart_cap = dns::DIAG_BLOCKS;
    for (int v = 0; v < ops->nvar[dns::P_XRHS]; ++v)
        if (ops->xrhs_groups[v] > k.npart_cap) k.npart_cap = ops->xrhs_groups[v];
    for (int v = 0; v < ops->nvar[dns::P_XSTAGE]; ++v)
        if (ops->xstage_groups[v] > k.npart_cap) k.npart_cap = ops->xstage_groups[v];
    const size_t hist_cap = o.history_cap > 0 ? (size_t)o.history_cap : 1;
    const int ntw2 = dns::tw_size(N / 16);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    k.state = take((size_t)members * 9 * fb);
    k.work = take((size_t)members * 6 * fb);
    k.part = take(2 * sizeof(double) * (size_t)k.npart_cap * members);
    k.dout = take(2 * sizeof(double) * (size_t)members);
    k.hist = take(2 * sizeof(double) * hist_cap * members);
    k.hist_count = take(sizeof(int) * (size_t)members);
    k.tw = take((size_t)ops->tw_count * cb);
    k.mfma_tw = o.mfma_dft ? take(((size_t)N + (size_t)(ntw2 > 0 ? ntw2 : 1)) * cb) : 0;
    k.total = off;
    return k;
}

// Create a context of `members` simulations.  lib_stream: when non-null the
// context enqueues on that stream (owned by an ensemble) instead of its own.
// workspace: when non-null, a caller-owned device block of `ws_bytes` bytes
// (256-byte aligned, at least carve().total) that holds every device buffer;
// otherwise the library allocates the block.
int create_ctx(int N, double nu, double dt, int dtype, const dns_opts& o, hipStream_t user, int members,
               hipStream_t lib_stream, dns_t** out, void* workspace = nullptr, size_t ws_bytes = 0) {
    *out = nullptr;
    dns_t* c = new (std::nothrow) dns_ctx();
    if (!c) return DNS_E_NOMEM;
    c->N = N;
    c->nu = nu;
    c->dt = dt;
    c->dtype = dtype;
    c->opts = o;
    c->members = members;
    c->mask_lim = (o.dealias == DNS_DEALIAS_TEXT) ? N : N + 2;
    c->user = user;
    const char* fi = std::getenv("DNS_FAULT_INJECT");
    c->inject_fault = fi != nullptr && std::strcmp(fi, "launch") == 0;
    c->ops = dtype == DNS_FP64 ? dns::ops_f64(N) : dns::ops_f32(N);
    const size_t rs = c->ops->real_size;
    c->fs = c->ops->fs;
    c->cbytes = 2 * rs;
    c->fbytes = c->fs * c->cbytes;

    auto bail = [&](int code, const char* what, hipError_t e) {
        std::fprintf(stderr, "dns_create: %s: %s\n", what, hipGetErrorString(e));
        release(c);
        delete c;
        return code;
    };
    hipError_t e;
    if (lib_stream) {
        c->s = lib_stream;
        c->own_stream = false;
    } else if ((e = hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking)) != hipSuccess) {
        return bail(DNS_E_HIP, "hipStreamCreate", e);
    }
    if ((e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreate(&c->ev_prof[0])) != hipSuccess || (e = hipEventCreate(&c->ev_prof[1])) != hipSuccess)
        return bail(DNS_E_HIP, "hipEventCreate", e);
    const Carve k = carve(c->ops, N, o, members);
    if (workspace) {
        c->mem = (char*)workspace;
        c->own_mem = false;
    } else if ((e = hipMalloc((void**)&c->mem, k.total)) != hipSuccess) {
        return bail(DNS_E_NOMEM, "hipMalloc", e);
    }
    (void)ws_bytes;   // checked by the caller against carve().total
    c->state = c->mem + k.state;
    c->work = c->mem + k.work;
    c->part = (double*)(c->mem + k.part);
    c->dout = (double*)(c->mem + k.dout);
    c->hist = (double*)(c->mem + k.hist);
    c->hist_count = (int*)(c->mem + k.hist_count);
    c->tw = c->mem + k.tw;
    c->mfma_tw = o.mfma_dft ? (void*)(c->mem + k.mfma_tw) : nullptr;
    c->npart_cap = k.npart_cap;
    for (int p = 0; p < dns::P_COUNT; ++p) {
        c->sel[p] = c->ops->def[p];
        if (c->sel[p] < 0 || c->sel[p] >= c->ops->nvar[p]) {
            std::fprintf(stderr, "dns_create: no default variant of pass %d for N = %d\n", p, N);
            release(c);
            delete c;
            return DNS_E_UNSUPPORTED;
        }
    }
    if (o.y_elems != 0 || o.curl_in_y >= 0 || o.xcd_pair >= 0 || o.mfma_dft) {
        const int r = apply_schedule(c, o.y_elems, o.curl_in_y, o.xcd_pair);
        if (r != DNS_OK) {
            std::fprintf(stderr, "dns_create: %s\n", c->err.c_str());
            release(c);
            delete c;
            return r;
        }
    }

    // twiddles: long-double accurate, rounded to the context's precision
    const int ntw = c->ops->tw_count;
    std::vector<double> twd(2 * (size_t)ntw, 0.0);
    for (int r = 0; r < dns::NRS; ++r) dns::make_twiddles(N, twd.data() + 2 * (size_t)c->ops->tw_base[r], r);
    if (dtype == DNS_FP64) {
        e = hipMemcpy(c->tw, twd.data(), (size_t)ntw * c->cbytes, hipMemcpyHostToDevice);
    } else {
        std::vector<float> twf(twd.size());
        for (size_t i = 0; i < twd.size(); ++i) twf[i] = (float)twd[i];
        e = hipMemcpy(c->tw, twf.data(), (size_t)ntw * c->cbytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return bail(DNS_E_HIP, "hipMemcpy(tw)", e);
    if (o.mfma_dft) {
        // FP32 only (checked by the caller): the unit roots w_N^j and the
        // twiddle table of the N/16-point transforms, long-double accurate
        const int n2 = N / 16, ntw2 = dns::tw_size(n2);
        std::vector<double> roots(2 * (size_t)N + 2 * (size_t)(ntw2 > 0 ? ntw2 : 1), 0.0);
        for (int j = 0; j < N; ++j) dns::unit_root(j, N, &roots[2 * j], &roots[2 * j + 1]);
        if (ntw2 > 0) dns::make_twiddles(n2, roots.data() + 2 * (size_t)N);
        std::vector<float> rf(roots.size());
        for (size_t i = 0; i < roots.size(); ++i) rf[i] = (float)roots[i];
        if ((e = hipMemcpy(c->mfma_tw, rf.data(), rf.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
            return bail(DNS_E_HIP, "hipMemcpy(mfma_tw)", e);
    }
    if ((e = hipMemset(c->state, 0, (size_t)members * 9 * c->fbytes)) != hipSuccess ||
        (e = hipMemset(c->hist_count, 0, sizeof(int) * (size_t)members)) != hipSuccess)
        return bail(DNS_E_HIP, "hipMemset", e);
    *out = c;
    return DNS_OK;
}

int reset_counters(dns_t* c) {
    c->steps = 0;
    c->has_state = true;
    DNS_TRY(c, hipMemsetAsync(c->hist_count, 0, sizeof(int) * (size_t)c->members, c->s));
    return DNS_OK;
}

// ---- per-member operations (shared by the single-simulation API and the
// ensemble API); the caller brackets them with enter/leave -----------------
int set_velocity_m(dns_t* c, int m, const void* u) {
    c->w_ready = false;
    c->ops->zr2c(u, c->W(m), c->tw, c->s);
    c->ops->yfwd3[c->sel[dns::P_YFWD3]](c->W(m), tw_of(c, c->ops->var[dns::P_YFWD3][c->sel[dns::P_YFWD3]].rs),
                                        dns::Batch{1, 0, 0}, c->s);
    c->ops->xfwd3(c->W(m), c->U0(m), c->tw, c->s);
    return launched(c, "set_velocity");
}

int init_velocity_m(dns_t* c, int m, int kind, const double* p) {
    c->w_ready = false;
    // the physical field is written into work fields 3..5 (3 N^3 reals fit in
    // three half-spectrum fields), then transformed as dns_set_velocity does
    void* phys = c->W(m) + 3 * c->fbytes;
    c->ops->ic_physical(phys, kind, p[0], p[1], p[2], c->s);
    int r = launched(c, "ic_physical");
    if (r) return r;
    return set_velocity_m(c, m, phys);
}

int init_random_m(dns_t* c, int m, unsigned long long seed, double k0, double energy) {
    c->w_ready = false;
    c->ops->ic_random(c->U0(m), seed, k0, c->mask_lim, c->s);
    int r = launched(c, "init_random");
    if (r) return r;
    double E = 0.0;
    if ((r = reduce_state(c, c->U0(m), &E, nullptr))) return r;
    if (!(E > 0.0)) return fail(c, DNS_E_NONFINITE, "random field has no energy (mask empty?)");
    c->ops->scale(c->U0(m), std::sqrt(energy / E), c->s);
    return launched(c, "scale");
}

int set_spectral_m(dns_t* c, int m, const void* uh) {
    c->w_ready = false;
    c->ops->layout(uh, c->U0(m), true, c->s);
    return launched(c, "set_spectral");
}

int get_spectral_m(dns_t* c, int m, void* uh) {
    c->ops->layout(c->U0(m), uh, false, c->s);
    return launched(c, "get_spectral");
}

int get_velocity_m(dns_t* c, int m, void* u) {
    c->w_ready = false;
    c->ops->xinv3(c->U0(m), c->W(m), c->tw, c->s);
    c->ops->yinv3(c->W(m), c->tw, c->s);
    c->ops->zc2r(c->W(m), u, c->tw, c->s);
    return launched(c, "get_velocity");
}

// Advance all members nsteps steps as replayed graphs (use_graph) or
// launch by launch; per_member launches every member's kernels separately.
int step_all(dns_t* c, int nsteps, bool per_member) {
    int r = DNS_OK;
    if (c->opts.fuse && !c->w_ready) {
        if (per_member) {
            for (int m = 0; m < c->members; ++m)
                launch_pass(c, dns::P_XINV, c->sel[dns::P_XINV], 0, nullptr, c->s, m);
            if ((r = launched(c, "xinv_curl"))) return r;
        } else if ((r = prepare_w(c))) {
            return r;
        }
    }
    for (int i = 0; i < nsteps; ++i) {
        const long long n = c->steps + 1;
        const bool diag = c->opts.diag_every > 0 && (n % c->opts.diag_every) == 0;
        if (per_member) {
            for (int m = 0; m < c->members; ++m) enqueue_step(c, diag, c->s, m);
            if ((r = launched(c, "step"))) return r;
        } else if (c->opts.use_graph) {
            if ((r = build_graph(c, diag ? 1 : 0))) return r;
            DNS_TRY(c, hipGraphLaunch(c->gexec[diag ? 1 : 0], c->s));
        } else {
            enqueue_step(c, diag, c->s);
            if ((r = launched(c, "step"))) return r;
        }
        c->steps = n;
    }
    c->w_ready = c->opts.fuse != 0;
    return DNS_OK;
}

int history_m(dns_t* c, int m, double* E, double* W, int max, int* count) {
    DNS_TRY(c, hipStreamSynchronize(c->s));
    int n = 0;
    DNS_TRY(c, hipMemcpy(&n, c->hist_count + m, sizeof(int), hipMemcpyDeviceToHost));
    *count = n;
    const int avail = n < c->opts.history_cap ? n : c->opts.history_cap;
    const int k = avail < max ? avail : max;
    if (k > 0) {
        std::vector<double> h(2 * (size_t)k);
        DNS_TRY(c, hipMemcpy(h.data(), c->hist + (size_t)2 * c->hist_cap() * m, h.size() * sizeof(double),
                             hipMemcpyDeviceToHost));
        for (int i = 0; i < k; ++i) {
            E[i] = h[2 * i];
            W[i] = h[2 * i + 1];
        }
    }
    return DNS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context-free right-hand side (dns_rhs_noalloc): every device buffer it
// needs beyond the caller's input and output lives in one file-scope array,
// so a call allocates nothing.  Layout of the array (all offsets 256-byte
// aligned): U0 (3 fields, the input in the internal layout), U1 (3 fields,
// the right-hand side), W (6 work fields), each field of the largest grid
// served (N = 64, FP64); then one twiddle-table slot per (precision, N).
// ---------------------------------------------------------------------------
namespace {
constexpr int NA_MAX_N = 64;
constexpr size_t NA_FIELD = (dns::Lay<double, NA_MAX_N>::FS * sizeof(double2) + 255) / 256 * 256;
constexpr size_t NA_TW_SLOT = 4096;   // bytes per twiddle table (64-point FP64: 896)
constexpr int NA_SIZES = 4;           // N = 8, 16, 32, 64
constexpr size_t NA_TW = 12 * NA_FIELD;
constexpr size_t NA_BYTES = NA_TW + 2 * NA_SIZES * NA_TW_SLOT;
static_assert((size_t)dns::tw_size(NA_MAX_N) * sizeof(double2) <= NA_TW_SLOT, "twiddle slot");
constexpr int NA_MAX_DEV = 64;

thread_local std::string g_free_err;   // message of the last failed context-free call

int free_fail(int code, const std::string& msg) {
    g_free_err = msg;
    return code;
}

size_t na_tw_offset(int dtype, int N) { return NA_TW + (size_t)(dtype * NA_SIZES + (dns::ilog2(N) - 3)) * NA_TW_SLOT; }
}  // namespace

// The scratch array: one copy per GPU, held until the process ends.  Host
// code never uses this name as an address (on the host it is only a
// stand-in); it uses the device address na_base() obtained for the current
// device.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
std::mutex g_na_mu;
char* g_na_base[NA_MAX_DEV] = {};

// Device address of the scratch array on the current device.  The first
// call on a device (under g_na_mu, with that device current) looks the
// address up and uploads the twiddle tables of every served (precision, N),
// long-double accurate as for a context, with a synchronous copy.
int na_base(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return free_fail(DNS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= NA_MAX_DEV) return free_fail(DNS_E_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (g_na_base[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return free_fail(DNS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        double tw[2 * NA_TW_SLOT / sizeof(double2) * 2];
        float twf[2 * NA_TW_SLOT / sizeof(double2) * 2];
        for (int n = 8; n <= NA_MAX_N; n *= 2) {
            const int cnt = dns::tw_size(n);
            if (cnt == 0) continue;
            dns::make_twiddles(n, tw);
            for (int i = 0; i < 2 * cnt; ++i) twf[i] = (float)tw[i];
            char* base = (char*)p;
            if ((e = hipMemcpy(base + na_tw_offset(DNS_FP64, n), tw, (size_t)cnt * sizeof(double2),
                               hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(base + na_tw_offset(DNS_FP32, n), twf, (size_t)cnt * sizeof(float2),
                               hipMemcpyHostToDevice)) != hipSuccess)
                return free_fail(DNS_E_HIP, std::string("twiddle upload: ") + hipGetErrorString(e));
        }
        g_na_base[dev] = (char*)p;
    }
    *out = g_na_base[dev];
    return DNS_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI: single simulation
// ---------------------------------------------------------------------------
extern "C" {

int dns_rhs_noalloc(int N, int dtype, double nu, int dealias, const void* uhat_dev, void* rhs_dev, void* stream) {
    if (!uhat_dev || !rhs_dev) return free_fail(DNS_E_INVAL, "null argument");
    if (!valid_n(N) || (dtype != DNS_FP64 && dtype != DNS_FP32) || !(nu >= 0.0) || !std::isfinite(nu) ||
        (dealias != DNS_DEALIAS_TEXT && dealias != DNS_DEALIAS_APPENDIX))
        return free_fail(DNS_E_INVAL, "bad argument");
    if (N > NA_MAX_N) return free_fail(DNS_E_INVAL, "dns_rhs_noalloc serves N <= 64 (its fixed scratch size)");
    char* base = nullptr;
    int r = na_base(&base);
    if (r != DNS_OK) return r;
    const dns::Ops* o = dtype == DNS_FP64 ? dns::ops_f64(N) : dns::ops_f32(N);
    const size_t fb = o->fs * 2 * o->real_size;   // the kernels address the fields at this stride
    char* U0 = base;
    char* U1 = base + 3 * NA_FIELD;
    char* W = base + 6 * NA_FIELD;
    if (3 * fb > 3 * NA_FIELD) return free_fail(DNS_E_UNSUPPORTED, "field larger than its scratch slot");
    const void* tw = base + na_tw_offset(dtype, N);
    hipStream_t s = (hipStream_t)stream;
    const dns::Batch b{1, 0, 0};
    dns::StageArgs a;
    a.nu = nu;
    a.ca = 0.0;
    a.cb = 0.0;
    a.stage = -1;                     // right-hand side only: U1 = R
    a.mask_lim = dealias == DNS_DEALIAS_TEXT ? N : N + 2;
    a.diag = nullptr;
    // the unfused stage of dns_rhs, default variants: inverse x (+curl),
    // inverse y, z pass, forward y, forward x + RHS
    o->layout(uhat_dev, U0, true, s);
    o->xinv[o->def[dns::P_XINV]](U0, W, tw, b, s);
    o->yinv6[o->def[dns::P_YINV6]](W, tw, b, s);
    o->zcross[o->def[dns::P_ZCROSS]](W, tw, b, s);
    o->yfwd3[o->def[dns::P_YFWD3]](W, tw, b, s);
    o->xrhs[o->def[dns::P_XRHS]](W, U0, U1, U1, tw, a, b, s);
    o->layout(U1, rhs_dev, false, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return free_fail(DNS_E_HIP, std::string("dns_rhs_noalloc launch: ") + hipGetErrorString(e));
    return DNS_OK;
}


void dns_default_opts(dns_opts* o) {
    if (!o) return;
    o->dealias = DNS_DEALIAS_TEXT;
    o->diag_every = 0;
    o->history_cap = 4096;
    o->use_graph = 1;
    o->autotune = 0;
    o->fuse = 1;
    o->integrator = DNS_RK4;
    o->mfma_dft = 0;
    o->y_elems = 0;
    o->curl_in_y = -1;
    o->xcd_pair = -1;
}

size_t dns_state_bytes(int N, int dtype) {
    dns_opts o;
    dns_default_opts(&o);
    return dns_workspace_bytes(N, dtype, &o);
}

size_t dns_workspace_bytes(int N, int dtype, const dns_opts* opts) {
    if (!valid_n(N) || (dtype != DNS_FP64 && dtype != DNS_FP32)) return 0;
    dns_opts o;
    dns_default_opts(&o);
    if (opts) o = *opts;
    if (check_args(N, 1.0, 1.0, dtype, o) != DNS_OK) return 0;
    const dns::Ops* ops = dtype == DNS_FP64 ? dns::ops_f64(N) : dns::ops_f32(N);
    return carve(ops, N, o, 1).total;
}

int dns_create(int N, double nu, double dt, int dtype, dns_t** out) {
    return dns_create_ex(N, nu, dt, dtype, nullptr, nullptr, out);
}

int dns_create_ws(int N, double nu, double dt, int dtype, const dns_opts* opts, void* workspace, size_t bytes,
                  void* stream, dns_t** out) {
    if (!out || !workspace) return DNS_E_INVAL;
    *out = nullptr;
    dns_opts o;
    dns_default_opts(&o);
    if (opts) o = *opts;
    int r = check_args(N, nu, dt, dtype, o);
    if (r) return r;
    if (((uintptr_t)workspace & 255) != 0 || bytes < dns_workspace_bytes(N, dtype, &o)) return DNS_E_INVAL;
    dns_t* c = nullptr;
    if ((r = create_ctx(N, nu, dt, dtype, o, (hipStream_t)stream, 1, nullptr, &c, workspace, bytes))) return r;
    if (o.autotune && (r = tune_new(c)) != DNS_OK) {
        release(c);
        delete c;
        return r;
    }
    *out = c;
    return DNS_OK;
}

int dns_create_ex(int N, double nu, double dt, int dtype, const dns_opts* opts, void* stream, dns_t** out) {
    if (!out) return DNS_E_INVAL;
    *out = nullptr;
    dns_opts o;
    dns_default_opts(&o);
    if (opts) o = *opts;
    int r = check_args(N, nu, dt, dtype, o);
    if (r) return r;
    dns_t* c = nullptr;
    if ((r = create_ctx(N, nu, dt, dtype, o, (hipStream_t)stream, 1, nullptr, &c))) return r;
    if (o.autotune && (r = tune_new(c)) != DNS_OK) {
        release(c);
        delete c;
        return r;
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

int dns_set_velocity(dns_t* c, const void* u) {
    if (!c || !u) return fail(c, DNS_E_INVAL, "null argument");
    int r = enter(c);
    if (r || (r = set_velocity_m(c, 0, u)) || (r = reset_counters(c))) return r;
    return leave(c);
}

int dns_init_velocity(dns_t* c, int kind, const double* params, int nparams) {
    if (!c || kind < DNS_IC_TAYLOR_GREEN || kind > DNS_IC_SHEAR || nparams < 0 || (nparams > 0 && !params))
        return fail(c, DNS_E_INVAL, "bad argument");
    double p[3] = {1.0, 1.0, 1.0};
    for (int i = 0; i < nparams && i < 3; ++i) p[i] = params[i];
    int r = enter(c);
    if (r || (r = init_velocity_m(c, 0, kind, p)) || (r = reset_counters(c))) return r;
    return leave(c);
}

int dns_init_random(dns_t* c, unsigned long long seed, double k0, double energy) {
    if (!c || !(k0 > 0.0) || !(energy > 0.0) || !std::isfinite(k0) || !std::isfinite(energy))
        return fail(c, DNS_E_INVAL, "bad argument");
    int r = enter(c);
    if (r || (r = init_random_m(c, 0, seed, k0, energy)) || (r = reset_counters(c))) return r;
    return leave(c);
}

int dns_set_spectral(dns_t* c, const void* uh) {
    if (!c || !uh) return fail(c, DNS_E_INVAL, "null argument");
    int r = enter(c);
    if (r || (r = set_spectral_m(c, 0, uh)) || (r = reset_counters(c))) return r;
    return leave(c);
}

int dns_get_spectral(dns_t* c, void* uh) {
    if (!c || !uh) return fail(c, DNS_E_INVAL, "null argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    int r = enter(c);
    if (r || (r = get_spectral_m(c, 0, uh))) return r;
    return leave(c);
}

int dns_get_velocity(dns_t* c, void* u) {
    if (!c || !u) return fail(c, DNS_E_INVAL, "null argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    int r = enter(c);
    if (r || (r = get_velocity_m(c, 0, u))) return r;
    return leave(c);
}

int dns_forward(dns_t* c, const void* u, void* uh) {
    if (!c || !u || !uh) return fail(c, DNS_E_INVAL, "null argument");
    int r = enter(c);
    if (r) return r;
    c->w_ready = false;
    c->ops->zr2c(u, c->W(), c->tw, c->s);
    c->ops->yfwd3[c->sel[dns::P_YFWD3]](c->W(), tw_of(c, c->ops->var[dns::P_YFWD3][c->sel[dns::P_YFWD3]].rs),
                                        dns::Batch{1, 0, 0}, c->s);
    c->ops->xfwd3(c->W(), c->Us(), c->tw, c->s);
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
    c->ops->xinv3(c->Us(), c->W(), c->tw, c->s);
    c->ops->yinv3(c->W(), c->tw, c->s);
    c->ops->zc2r(c->W(), u, c->tw, c->s);
    if ((r = launched(c, "inverse"))) return r;
    return leave(c);
}

int dns_step(dns_t* c, int nsteps) {
    if (!c || nsteps < 0) return fail(c, DNS_E_INVAL, "bad argument");
    if (!c->has_state) return fail(c, DNS_E_STATE, "no velocity set");
    if (nsteps == 0) return DNS_OK;
    int r = enter(c);
    if (r || (r = step_all(c, nsteps, false))) return r;
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
    return history_m(c, 0, E, W, max, count);
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
            for (int i = 0; i < step_stages(c); ++i) {
                for (int k = dns::P_YINV6; k <= dns::P_YFWD3; ++k)
                    if ((r = timed(k, stage_id(c, i)))) return r;
                if ((r = timed(dns::P_XSTAGE, stage_id(c, i)))) return r;
            }
            c->w_ready = true;
        } else {
            for (int i = 0; i < step_stages(c); ++i)
                for (int k = dns::P_XINV; k <= dns::P_XRHS; ++k)
                    if ((r = timed(k, stage_id(c, i)))) return r;
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

// Time every variant of every pass on the context's buffers and keep the
// fastest plan.  The RHS passes are timed in their stage-1 form, which reads
// U0 but writes only U1, Us and W, so the current state is preserved.  The
// passes whose fields depend on the curl placement are chosen together: for
// each placement the fastest variants of the inverse x, inverse y and stage
// passes are summed with the weights of one step, and the cheaper placement
// wins; the other passes take their fastest variant.
int dns_autotune(dns_t* c, int reps) { return dns_autotune_ex(c, reps, DNS_TUNE_REPRODUCIBLE); }

int dns_autotune_ex(dns_t* c, int reps, int mode) {
    if (!c || reps < 0 || (mode != DNS_TUNE_REPRODUCIBLE && mode != DNS_TUNE_FASTEST))
        return fail(c, DNS_E_INVAL, "bad argument");
    if (reps == 0) reps = 3;
    int r = enter(c);
    if (r) return r;
    drop_graphs(c);
    const dns::Ops& o = *c->ops;
    std::vector<std::vector<float>> t(dns::P_COUNT);
    // reproducible mode: radix plan 0 only (every such plan gives the
    // default plan's bits)
    auto allowed = [&](int p, int v) { return mode == DNS_TUNE_FASTEST || o.var[p][v].rs == 0; };
    for (int p = 0; p < dns::P_COUNT; ++p) {
        t[p].assign(o.nvar[p], 1e30f);
        for (int v = 0; v < o.nvar[p]; ++v) {
            if (!allowed(p, v)) continue;
            launch_pass(c, p, v, 1, nullptr, c->s);                  // warm-up
            DNS_TRY(c, hipEventRecord(c->ev_prof[0], c->s));
            for (int i = 0; i < reps; ++i) launch_pass(c, p, v, 1, nullptr, c->s);
            if ((r = launched(c, kPassNames[p]))) return r;
            DNS_TRY(c, hipEventRecord(c->ev_prof[1], c->s));
            DNS_TRY(c, hipEventSynchronize(c->ev_prof[1]));
            float ms = 0.f;
            DNS_TRY(c, hipEventElapsedTime(&ms, c->ev_prof[0], c->ev_prof[1]));
            t[p][v] = ms;
        }
    }
    // fastest variant of pass p usable with curl placement cy (-1: any)
    auto fastest = [&](int p, int cy) {
        int best = -1;
        for (int v = 0; v < o.nvar[p]; ++v) {
            const int vc = o.var[p][v].cy;
            if (!allowed(p, v) || (cy >= 0 && vc >= 0 && vc != cy)) continue;
            if (best < 0 || t[p][v] < t[p][best]) best = v;
        }
        return best;
    };
    int best_cy = plan_cy(c);
    float best_cost = 1e30f;
    for (int cy = 0; cy <= 1; ++cy) {
        const int vx = fastest(dns::P_XINV, cy), vy = fastest(dns::P_YINV6, cy), vs = fastest(dns::P_XSTAGE, cy);
        if (vx < 0 || vy < 0 || vs < 0 || o.var[dns::P_XINV][vx].cy != cy || o.var[dns::P_YINV6][vy].cy != cy ||
            o.var[dns::P_XSTAGE][vs].cy != cy)
            continue;
        if (c->opts.mfma_dft && !o.ymfma_inv6[cy]) continue;
        const float cost = c->opts.fuse ? 4.f * (t[dns::P_YINV6][vy] + t[dns::P_XSTAGE][vs])
                                        : 4.f * (t[dns::P_YINV6][vy] + t[dns::P_XINV][vx]);
        if (cost < best_cost) { best_cost = cost; best_cy = cy; }
    }
    int sel[dns::P_COUNT];
    for (int p = 0; p < dns::P_COUNT; ++p) {
        const int cy = (p == dns::P_XINV || p == dns::P_YINV6 || p == dns::P_XSTAGE) ? best_cy : -1;
        sel[p] = fastest(p, cy);
    }
    if (plan_consistent(c, sel))
        for (int p = 0; p < dns::P_COUNT; ++p) c->sel[p] = sel[p];
    c->w_ready = false;
    store_plan(c, mode);
    return leave(c);
}

int dns_copy_rows(const void* src, void* dst, size_t nrows, int row_bytes, size_t pitch, void* stream) {
    if (!src || !dst || row_bytes <= 0 || row_bytes % 16 != 0 || pitch < (size_t)row_bytes || pitch % 16 != 0)
        return DNS_E_INVAL;
    if (nrows == 0) return DNS_OK;
    const unsigned vecs = (unsigned)(row_bytes / 16);
    const size_t threads = nrows * vecs;
    const size_t blocks = (threads + 255) / 256;
    if (blocks > 0x7fffffffu) return DNS_E_INVAL;
    hipLaunchKernelGGL(dns::k_copy_rows, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const uint4*)src, (uint4*)dst, nrows, vecs, pitch / 16);
    return hipGetLastError() == hipSuccess ? DNS_OK : DNS_E_HIP;
}

int dns_plan_cache_entries(void) {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    plan_env_load();
    return (int)g_plans.size();
}

int dns_plan_cache_save(const char* path) {
    if (!path || !*path) return DNS_E_INVAL;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    plan_env_load();
    return plan_cache_write(path);
}

int dns_plan_cache_load(const char* path) {
    if (!path || !*path) return DNS_E_INVAL;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    plan_env_load();
    const int n = plan_cache_read(path);
    return n < 0 ? DNS_E_INVAL : n;
}

int dns_plan_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plan_env_loaded = true;   // a cleared cache is not refilled from DNS_PLAN_CACHE
    g_plans.clear();
    return DNS_OK;
}

int dns_get_plan(const dns_t* c, int* widths, int max, int* count) {
    if (!c || !count || max < 0 || (max > 0 && !widths)) return DNS_E_INVAL;
    const int m = max < dns::P_COUNT ? max : dns::P_COUNT;
    for (int p = 0; p < m; ++p) widths[p] = c->ops->var[p][c->sel[p]].width;
    *count = dns::P_COUNT;
    return DNS_OK;
}

// Install plan `sel` (variant indices): waits for the stream and drops the
// captured graphs, whose kernels it changes.
int install_plan(dns_t* c, const int* sel) {
    DNS_TRY(c, hipStreamSynchronize(c->s));
    drop_graphs(c);
    for (int p = 0; p < dns::P_COUNT; ++p) c->sel[p] = sel[p];
    c->w_ready = false;
    return DNS_OK;
}

int dns_set_plan(dns_t* c, const int* widths, int n) {
    if (!c || !widths || n != dns::P_COUNT) return fail(c, DNS_E_INVAL, "bad argument");
    const dns::Ops& o = *c->ops;
    const int cy = plan_cy(c);
    int sel[dns::P_COUNT];
    for (int p = 0; p < dns::P_COUNT; ++p) {
        // the variant of that width with the current schedule
        const dns::Variant& cur = o.var[p][c->sel[p]];
        sel[p] = -1;
        // (same radix plan and pad as the current variant where there is one)
        auto rank = [&](const dns::Variant& d) {
            return 2 * (d.rs == cur.rs && d.pad == cur.pad ? 1 : 0) + (d.pair == cur.pair ? 1 : 0);
        };
        for (int v = 0; v < o.nvar[p]; ++v) {
            const dns::Variant& d = o.var[p][v];
            if (d.width != widths[p] || (d.cy >= 0 && d.cy != cy) || (d.ye > 0 && d.ye != cur.ye)) continue;
            if (!reference_shape(p, d) && !(d.rs == cur.rs && d.pad == cur.pad)) continue;
            if (sel[p] < 0 || rank(d) > rank(o.var[p][sel[p]])) sel[p] = v;
        }
        if (sel[p] < 0) return fail(c, DNS_E_INVAL, "no variant of that width for this N, dtype and schedule");
    }
    return install_plan(c, sel);
}

int dns_plan_variants(const dns_t* c, int pass, int* widths, int max, int* count) {
    if (!c || !count || pass < 0 || pass >= dns::P_COUNT || max < 0 || (max > 0 && !widths)) return DNS_E_INVAL;
    // distinct widths of the variants that run the current schedule
    const dns::Ops& o = *c->ops;
    const int cy = plan_cy(c);
    const dns::Variant& cur = o.var[pass][c->sel[pass]];
    int n = 0;
    for (int v = 0; v < o.nvar[pass]; ++v) {
        const dns::Variant& d = o.var[pass][v];
        if ((d.cy >= 0 && d.cy != cy) || (d.ye > 0 && d.ye != cur.ye)) continue;
        if (!reference_shape(pass, d) && !(d.rs == cur.rs && d.pad == cur.pad)) continue;
        bool seen = false;
        for (int u = 0; u < v; ++u) {
            const dns::Variant& e = o.var[pass][u];
            seen = seen || (e.width == d.width && (e.cy < 0 || e.cy == cy) && (e.ye <= 0 || e.ye == cur.ye) &&
                            (reference_shape(pass, e) || (e.rs == cur.rs && e.pad == cur.pad)));
        }
        if (seen) continue;
        if (n < max) widths[n] = d.width;
        ++n;
    }
    *count = n;
    return DNS_OK;
}

int dns_plan_variants_ex(const dns_t* c, int pass, dns_variant* out, int max, int* count) {
    if (!c || !count || pass < 0 || pass >= dns::P_COUNT || max < 0 || (max > 0 && !out)) return DNS_E_INVAL;
    const dns::Ops& o = *c->ops;
    for (int v = 0; v < o.nvar[pass] && v < max; ++v) {
        out[v].width = o.var[pass][v].width;
        out[v].xcd_pair = o.var[pass][v].pair;
        out[v].y_elems = o.var[pass][v].ye;
        out[v].curl_in_y = o.var[pass][v].cy;
        out[v].radix = o.var[pass][v].rs;
        out[v].lds_pad = o.var[pass][v].pad;
    }
    *count = o.nvar[pass];
    return DNS_OK;
}

int dns_get_plan_ex(const dns_t* c, int* variants, int max, int* count) {
    if (!c || !count || max < 0 || (max > 0 && !variants)) return DNS_E_INVAL;
    for (int p = 0; p < dns::P_COUNT && p < max; ++p) variants[p] = c->sel[p];
    *count = dns::P_COUNT;
    return DNS_OK;
}

int dns_set_plan_ex(dns_t* c, const int* variants, int n) {
    if (!c || !variants || n != dns::P_COUNT) return fail(c, DNS_E_INVAL, "bad argument");
    for (int p = 0; p < dns::P_COUNT; ++p)
        if (variants[p] < 0 || variants[p] >= c->ops->nvar[p]) return fail(c, DNS_E_INVAL, "variant index out of range");
    if (!plan_consistent(c, variants))
        return fail(c, DNS_E_INVAL, "inverse x, inverse y and stage passes disagree on the curl placement");
    return install_plan(c, variants);
}

int dns_set_schedule(dns_t* c, int y_elems, int curl_in_y, int xcd_pair) {
    if (!c || (y_elems != 0 && y_elems != 8 && y_elems != 16 && y_elems != 32) || curl_in_y < -1 ||
        curl_in_y > 1 || xcd_pair < -1 || xcd_pair > 1)
        return fail(c, DNS_E_INVAL, "bad argument");
    int keep[dns::P_COUNT];
    for (int p = 0; p < dns::P_COUNT; ++p) keep[p] = c->sel[p];
    int r = apply_schedule(c, y_elems, curl_in_y, xcd_pair);
    if (r != DNS_OK) return r;
    int sel[dns::P_COUNT];
    for (int p = 0; p < dns::P_COUNT; ++p) {
        sel[p] = c->sel[p];
        c->sel[p] = keep[p];
    }
    return install_plan(c, sel);
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

const char* dns_last_error(const dns_t* c) { return c ? c->err.c_str() : g_free_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// C ABI: ensembles of independent simulations
// ---------------------------------------------------------------------------
struct dns_ens {
    hipStream_t user = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<dns_t*> cls;              // one context per (N, nu, dt) class
    std::vector<int> cls_of, idx_of;      // member i -> (class, index in class)
    std::vector<char> ready;              // member i has a velocity field
    hipGraphExec_t gexec = nullptr;       // one step of every class
    // DNS_ENS_ONE_GRAPH: graphs of whole multi-step calls, by step count
    std::vector<std::pair<int, hipGraphExec_t>> multi;
    std::string err;
};

namespace {

int ens_fail(dns_ens_t* e, int code, const std::string& msg) {
    if (e) e->err = msg;
    return code;
}

int ens_enter(dns_ens_t* e) {
    if (hipEventRecord(e->ev_in, e->user) != hipSuccess || hipStreamWaitEvent(e->s, e->ev_in, 0) != hipSuccess)
        return ens_fail(e, DNS_E_HIP, "stream ordering");
    return DNS_OK;
}

int ens_leave(dns_ens_t* e) {
    if (hipEventRecord(e->ev_out, e->s) != hipSuccess || hipStreamWaitEvent(e->user, e->ev_out, 0) != hipSuccess)
        return ens_fail(e, DNS_E_HIP, "stream ordering");
    return DNS_OK;
}

int ens_cls_error(dns_ens_t* e, dns_t* c, int r) {
    if (r != DNS_OK && c) e->err = c->err;
    return r;
}

void ens_release(dns_ens_t* e) {
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    for (auto& m : e->multi) (void)hipGraphExecDestroy(m.second);
    e->multi.clear();
    for (dns_t* c : e->cls) {
        release(c);
        delete c;
    }
    e->cls.clear();
    if (e->ev_in) (void)hipEventDestroy(e->ev_in);
    if (e->ev_out) (void)hipEventDestroy(e->ev_out);
    if (e->s) (void)hipStreamDestroy(e->s);
}

bool ens_member(const dns_ens_t* e, int i) { return e && i >= 0 && i < (int)e->cls_of.size(); }

}  // namespace

extern "C" {

int dns_ens_create(int count, const int* N, const double* nu, const double* dt, int dtype, const dns_opts* opts,
                   void* stream, dns_ens_t** out) {
    if (!out) return DNS_E_INVAL;
    *out = nullptr;
    if (count <= 0 || !N || !nu || !dt) return DNS_E_INVAL;
    dns_opts o;
    dns_default_opts(&o);
    if (opts) o = *opts;
    for (int i = 0; i < count; ++i) {
        const int r = check_args(N[i], nu[i], dt[i], dtype, o);
        if (r) return r;
    }
    dns_ens_t* e = new (std::nothrow) dns_ens();
    if (!e) return DNS_E_NOMEM;
    e->user = (hipStream_t)stream;
    if (hipStreamCreateWithFlags(&e->s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming) != hipSuccess) {
        ens_release(e);
        delete e;
        return DNS_E_HIP;
    }
    // group members by (N, nu, dt), in order of first appearance
    std::vector<int> key_n;
    std::vector<double> key_nu, key_dt;
    std::vector<int> cnt;
    e->cls_of.resize(count);
    e->idx_of.resize(count);
    e->ready.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        int k = -1;
        for (size_t j = 0; j < key_n.size(); ++j)
            if (key_n[j] == N[i] && key_nu[j] == nu[i] && key_dt[j] == dt[i]) k = (int)j;
        if (k < 0) {
            k = (int)key_n.size();
            key_n.push_back(N[i]);
            key_nu.push_back(nu[i]);
            key_dt.push_back(dt[i]);
            cnt.push_back(0);
        }
        e->cls_of[i] = k;
        e->idx_of[i] = cnt[k]++;
    }
    for (size_t k = 0; k < key_n.size(); ++k) {
        dns_t* c = nullptr;
        int r = create_ctx(key_n[k], key_nu[k], key_dt[k], dtype, o, e->s, cnt[k], e->s, &c);
        if (r) {
            ens_release(e);
            delete e;
            return r;
        }
        e->cls.push_back(c);
        // tile shapes timed on the batched launches of this class
        if (o.autotune && (r = tune_new(c)) != DNS_OK) {
            ens_release(e);
            delete e;
            return r;
        }
    }
    *out = e;
    return DNS_OK;
}

int dns_ens_destroy(dns_ens_t* e) {
    if (!e) return DNS_OK;
    if (e->s) (void)hipStreamSynchronize(e->s);
    ens_release(e);
    delete e;
    return DNS_OK;
}

int dns_ens_size(const dns_ens_t* e, int* count, int* classes) {
    if (!e || !count) return DNS_E_INVAL;
    *count = (int)e->cls_of.size();
    if (classes) *classes = (int)e->cls.size();
    return DNS_OK;
}

int dns_ens_set_spectral(dns_ens_t* e, int i, const void* uh) {
    if (!ens_member(e, i) || !uh) return ens_fail(e, DNS_E_INVAL, "bad argument");
    dns_t* c = e->cls[e->cls_of[i]];
    int r = ens_enter(e);
    if (r || (r = ens_cls_error(e, c, set_spectral_m(c, e->idx_of[i], uh))) || (r = reset_counters(c))) return r;
    e->ready[i] = 1;
    return ens_leave(e);
}

int dns_ens_set_velocity(dns_ens_t* e, int i, const void* u) {
    if (!ens_member(e, i) || !u) return ens_fail(e, DNS_E_INVAL, "bad argument");
    dns_t* c = e->cls[e->cls_of[i]];
    int r = ens_enter(e);
    if (r || (r = ens_cls_error(e, c, set_velocity_m(c, e->idx_of[i], u))) || (r = reset_counters(c))) return r;
    e->ready[i] = 1;
    return ens_leave(e);
}

int dns_ens_init_random(dns_ens_t* e, int i, unsigned long long seed, double k0, double energy) {
    if (!ens_member(e, i) || !(k0 > 0.0) || !(energy > 0.0)) return ens_fail(e, DNS_E_INVAL, "bad argument");
    dns_t* c = e->cls[e->cls_of[i]];
    int r = ens_enter(e);
    if (r || (r = ens_cls_error(e, c, init_random_m(c, e->idx_of[i], seed, k0, energy))) ||
        (r = reset_counters(c)))
        return r;
    e->ready[i] = 1;
    return ens_leave(e);
}

int dns_ens_get_spectral(dns_ens_t* e, int i, void* uh) {
    if (!ens_member(e, i) || !uh) return ens_fail(e, DNS_E_INVAL, "bad argument");
    dns_t* c = e->cls[e->cls_of[i]];
    if (!e->ready[i]) return ens_fail(e, DNS_E_STATE, "no velocity set");
    int r = ens_enter(e);
    if (r || (r = ens_cls_error(e, c, get_spectral_m(c, e->idx_of[i], uh)))) return r;
    return ens_leave(e);
}

// Capture `steps` steps of every class (in class order) into one graph.
int ens_capture(dns_ens_t* e, int steps, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(e->s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return ens_fail(e, DNS_E_HIP, "hipStreamBeginCapture");
    for (int i = 0; i < steps; ++i)
        for (dns_t* c : e->cls) enqueue_step(c, false, e->s);
    hipError_t le = hipGetLastError();
    hipError_t ee = hipStreamEndCapture(e->s, &g);
    if (le != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return ens_fail(e, DNS_E_HIP, "ensemble graph capture");
    }
    hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return ens_fail(e, DNS_E_HIP, "hipGraphInstantiate");
    return DNS_OK;
}

int dns_ens_step(dns_ens_t* e, int nsteps, int mode) {
    if (!e || nsteps < 0 || (mode != DNS_ENS_BATCHED && mode != DNS_ENS_PER_SIM && mode != DNS_ENS_ONE_GRAPH))
        return ens_fail(e, DNS_E_INVAL, "bad argument");
    for (char ok : e->ready)
        if (!ok) return ens_fail(e, DNS_E_STATE, "a member has no velocity set");
    if (nsteps == 0) return DNS_OK;
    int r = ens_enter(e);
    if (r) return r;
    bool diag = false;
    for (dns_t* c : e->cls) diag = diag || c->opts.diag_every > 0;
    if (mode == DNS_ENS_PER_SIM || diag || !e->cls[0]->opts.use_graph) {
        // every class advanced by its own batched launches, or every member
        // by its own launches (the unbatched baseline)
        for (dns_t* c : e->cls)
            if ((r = ens_cls_error(e, c, step_all(c, nsteps, mode == DNS_ENS_PER_SIM)))) return r;
        return ens_leave(e);
    }
    for (dns_t* c : e->cls)
        if ((r = ens_cls_error(e, c, prepare_w(c)))) return r;
    if (mode == DNS_ENS_ONE_GRAPH) {
        // all nsteps steps of every class in one captured graph (one launch);
        // graphs are kept per step count (the four most recent)
        hipGraphExec_t g = nullptr;
        for (auto& m : e->multi)
            if (m.first == nsteps) g = m.second;
        if (!g) {
            if ((r = ens_capture(e, nsteps, &g))) return r;
            if (e->multi.size() >= 4) {
                (void)hipGraphExecDestroy(e->multi.front().second);
                e->multi.erase(e->multi.begin());
            }
            e->multi.emplace_back(nsteps, g);
        }
        if (hipGraphLaunch(g, e->s) != hipSuccess) return ens_fail(e, DNS_E_HIP, "hipGraphLaunch");
    } else {
        // batched: one captured graph advances every class by one step
        if (!e->gexec && (r = ens_capture(e, 1, &e->gexec))) return r;
        for (int i = 0; i < nsteps; ++i)
            if (hipGraphLaunch(e->gexec, e->s) != hipSuccess) return ens_fail(e, DNS_E_HIP, "hipGraphLaunch");
    }
    for (dns_t* c : e->cls) {
        c->steps += nsteps;
        c->w_ready = c->opts.fuse != 0;
    }
    return ens_leave(e);
}

int dns_ens_diagnostics(dns_ens_t* e, double* E, double* W) {
    if (!e || (!E && !W)) return ens_fail(e, DNS_E_INVAL, "bad argument");
    int r = ens_enter(e);
    if (r) return r;
    int status = DNS_OK;
    for (size_t i = 0; i < e->cls_of.size(); ++i) {
        dns_t* c = e->cls[e->cls_of[i]];
        if (!e->ready[i]) return ens_fail(e, DNS_E_STATE, "a member has no velocity set");
        double a = 0.0, b = 0.0;
        r = reduce_state(c, c->U0(e->idx_of[i]), &a, &b);
        if (r == DNS_E_NONFINITE) status = r;
        else if (r) return ens_cls_error(e, c, r);
        if (E) E[i] = a;
        if (W) W[i] = b;
    }
    r = ens_leave(e);
    return status ? status : r;
}

int dns_ens_synchronize(dns_ens_t* e) {
    if (!e) return DNS_E_INVAL;
    if (hipStreamSynchronize(e->s) != hipSuccess) return ens_fail(e, DNS_E_HIP, "hipStreamSynchronize");
    return DNS_OK;
}

const char* dns_ens_last_error(const dns_ens_t* e) { return e ? e->err.c_str() : ""; }

}  // extern "C"
