/*
 * dns.h - C ABI of the MI355X pseudo-spectral Navier-Stokes RK4 library.
 *
 * The library advances the incompressible Navier-Stokes equations in
 * rotational form in the triply periodic box [0, 2 pi)^3 with the Fourier-
 * Galerkin pseudo-spectral method of Mortensen & Langtangen, "High
 * performance Python for direct numerical simulations of turbulent flows"
 * (arXiv:1602.03638):
 *
 *   d u_hat/dt = N_hat - nu |k|^2 u_hat - k (k . N_hat) / |k|^2,
 *   N_hat = dealias * F(u x omega),  omega = F^-1(i k x u_hat)
 *
 * (Sec. 2, eqs. NSfinal and curl_convection; Sec. 3.1 computeRHS listing),
 * integrated with classic RK4 (Appendix solver) or forward Euler (Sec. 3.1
 * main loop).  All compute runs in HIP kernels for gfx950; there is no CPU
 * fallback.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - N is the number of mesh points per axis, a power of two with
 *   8 <= N <= 1024 (Sec. 3.1 requires N = 2^M).
 * - Physical arrays: (3, N, N, N) real, C order, index [c][i][j][k] for the
 *   point (x_i, y_j, z_k) = 2 pi (i, j, k) / N (Sec. 2, eq. realmesh).
 * - Spectral arrays: (3, N, N, N/2+1) complex interleaved (re, im), C order,
 *   index [c][ix][iy][iz] with kx = ix for ix < N/2 else ix - N (same for
 *   ky) and kz = iz, so iz = N/2 is kz = +N/2 (Sec. 3.1 storage order).
 *   Values are the unnormalised forward transform
 *   u_hat(k) = sum_x u(x) exp(-i k.x) (Sec. 2, eq. iffteq), i.e. what
 *   numpy.fft.rfftn(u, axes=(1,2,3)) returns.
 * - The real type is the context's dtype: double for DNS_FP64, float for
 *   DNS_FP32 (complex = two of them).  Energy and enstrophy are always
 *   accumulated and returned in double.
 * - Every data pointer is a DEVICE pointer owned by the caller; the library
 *   copies from it on set and writes into it on get, and never frees it.
 * - Calls are ordered on the context's stream (the stream given at creation,
 *   or the null stream): dns_step and the set/get calls are asynchronous
 *   with respect to the host; dns_energy, dns_enstrophy, dns_diagnostics,
 *   dns_history and dns_synchronize wait for the stream.
 * - Every function returns a dns_status; no C++ exception crosses the ABI.
 *   After a failure dns_last_error(ctx) holds a message.  A context is not
 *   thread-safe; distinct contexts are independent.
 */
#ifndef DNS_H
#define DNS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dns_status {
    DNS_OK = 0,
    DNS_E_INVAL = -1,        /* bad argument (N, nu, dt, dtype, NULL pointer, size) */
    DNS_E_NOMEM = -2,        /* device allocation failed */
    DNS_E_HIP = -3,          /* a HIP runtime call or kernel launch failed */
    DNS_E_STATE = -4,        /* call not valid in the context's state (no velocity set) */
    DNS_E_NONFINITE = -5,    /* a diagnostic came out NaN or Inf */
    DNS_E_UNSUPPORTED = -6   /* valid request the library does not provide */
} dns_status;

typedef enum dns_dtype { DNS_FP64 = 0, DNS_FP32 = 1 } dns_dtype;

/* Dealiasing constant (Sec. 3.1 listing: kmax = N/3; Appendix: kmax =
 * 2/3 (N/2+1)).  A mode is kept iff 3|k_i| < N (TEXT) or 3|k_i| < N + 2
 * (APPENDIX) on all three axes. */
typedef enum dns_dealias { DNS_DEALIAS_TEXT = 0, DNS_DEALIAS_APPENDIX = 1 } dns_dealias;

/* Time integrator: classic RK4 (Appendix solver; default) or forward Euler,
 * u_hat += RHS(u_hat) dt (the main loop of the Sec. 3.1 listing). */
typedef enum dns_integrator { DNS_RK4 = 0, DNS_EULER = 1 } dns_integrator;

typedef struct dns_opts {
    int dealias;      /* dns_dealias; default DNS_DEALIAS_TEXT */
    int diag_every;   /* record E and Omega after every k-th step into the
                         history buffer (0 = never); default 0 */
    int history_cap;  /* capacity of the history buffer in steps; default 4096 */
    int use_graph;    /* 1 = replay each RK4 step as one captured HIP graph
                         (default), 0 = launch kernels one by one */
    int autotune;     /* 1 = tune the plan at creation in reproducible mode
                         (dns_autotune), 2 = in fastest mode
                         (dns_autotune_ex, DNS_TUNE_FASTEST); default 0 */
    int fuse;         /* 1 = fuse each stage's RHS/RK4 pass with the next
                         stage's inverse x pass (16 kernels per step, default);
                         0 = unfused schedule (20 kernels per step).  Both give
                         bitwise identical results. */
    int integrator;   /* dns_integrator; default DNS_RK4.  A forward Euler
                         step is one stage (4 kernels fused, 5 unfused). */
    int mfma_dft;     /* 1 = the y passes of the step take one radix-16 DFT
                         stage on FP16 matrix cores with high/low split
                         operands and FP32 accumulation (four-step split
                         N = 16 (N/16); the rest in FP32).  FP32 contexts with
                         N >= 64 only (DNS_E_UNSUPPORTED otherwise); results
                         differ from the plain FP32 path at the 1e-6 level.
                         Default 0. */
    /* Schedule of the step (see dns_set_schedule; every choice gives
     * bitwise identical results).  0 / -1 / -1 = the defaults for N. */
    int y_elems;      /* complex values per thread in the y passes: 8, 16, 32
                         (0 = default: 8 below 1024, 16 in the FP32 forward
                         y pass at 512; 16 FP64, 32 FP32 at 1024) */
    int curl_in_y;    /* 1 = the inverse y pass forms the vorticity from five
                         x-pass fields, 0 = the x pass writes all six fields;
                         -1 = default (1 below 1024, 0 at 1024) */
    int xcd_pair;     /* 1 = x passes whose row segments are shorter than
                         128 bytes hand the tiles of each 128-byte line to
                         one XCD; 0 = not; -1 = default (1 at 1024) */
} dns_opts;

typedef struct dns_ctx dns_t;

/* Fill *opts with the defaults listed above. */
void dns_default_opts(dns_opts* opts);

/* Create a solver for N^3 points, viscosity nu >= 0, time step dt > 0 and
 * dtype DNS_FP64 or DNS_FP32 (Sec. 3.1: float is a placeholder for single
 * or double precision).  The library allocates its device state in one
 * block of dns_workspace_bytes (15 half-spectrum fields of N*N*(N/2+1)
 * complex values in a padded layout, diagnostic buffers and O(N) tables) on
 * the current HIP device.  stream: a hipStream_t cast to void*, or NULL for
 * the null stream.  opts may be NULL.  On success *out owns the context.
 * DNS_E_INVAL for invalid arguments or options, DNS_E_UNSUPPORTED for an
 * option this dtype or N does not provide, DNS_E_NOMEM if the allocation
 * fails. */
int dns_create(int N, double nu, double dt, int dtype, dns_t** out);
int dns_create_ex(int N, double nu, double dt, int dtype, const dns_opts* opts,
                  void* stream, dns_t** out);

/* Wait for the context's stream, then release every allocation of ctx
 * (device state, graphs, stream); NULL is a no-op.  Does not free caller
 * memory (a workspace given to dns_create_ws). */
int dns_destroy(dns_t* ctx);

/* Bytes of device memory a context of this size holds with the default
 * options (the same as dns_workspace_bytes(N, dtype, NULL)). */
size_t dns_state_bytes(int N, int dtype);

/* Bytes of the device workspace a context with these options needs (opts
 * may be NULL for the defaults); 0 for invalid arguments.  The workspace
 * holds the 15 half-spectrum fields (padded layout), the diagnostic and
 * history buffers and the twiddle tables. */
size_t dns_workspace_bytes(int N, int dtype, const dns_opts* opts);

/* As dns_create_ex, with every device buffer of the context placed in the
 * caller's workspace (e.g. memory from PyTorch's allocator) instead of
 * library allocations: workspace is a device pointer aligned to 256 bytes,
 * bytes >= dns_workspace_bytes(N, dtype, opts) (DNS_E_INVAL otherwise).  The
 * caller owns the workspace, must keep it alive until dns_destroy and must
 * not touch it meanwhile; dns_destroy never frees it. */
int dns_create_ws(int N, double nu, double dt, int dtype, const dns_opts* opts, void* workspace, size_t bytes,
                  void* stream, dns_t** out);

/* u_hat = F(u) for the physical (3, N, N, N) real field u_dev: real
 * transform along z, then complex along y, then x (Sec. 2, eq. fft);
 * unnormalised.  No masking or projection is applied (the Appendix solver
 * transforms its initial condition as given).  Resets the step counter and
 * the history. */
int dns_set_velocity(dns_t* ctx, const void* u_dev);

/* Analytic initial velocity generated on the device and transformed as by
 * dns_set_velocity (kinds below; params may be NULL for the defaults):
 *   DNS_IC_TAYLOR_GREEN     (sin x cos y cos z, -cos x sin y cos z, 0)
 *                           (Sec. 4.2 and the Appendix solver)
 *   DNS_IC_TAYLOR_GREEN_2D  (sin x cos y, -cos x sin y, 0)
 *   DNS_IC_ABC              (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x),
 *                           params {A, B, C}, default 1, 1, 1
 *   DNS_IC_SHEAR            (amp sin(k z), 0, 0), params {k, amp}, default 1, 1
 * Angles are 2 pi i / N evaluated as sinpi/cospi of 2 i / N.  Uses the work
 * space; resets the step counter and the history. */
enum { DNS_IC_TAYLOR_GREEN = 0, DNS_IC_TAYLOR_GREEN_2D = 1, DNS_IC_ABC = 2, DNS_IC_SHEAR = 3 };
int dns_init_velocity(dns_t* ctx, int kind, const double* params, int nparams);

/* Seeded random solenoidal initial spectrum (not from the paper: a synthetic
 * workload).  Per stored mode and component, two uniforms in (0, 1] come
 * from SplitMix64 (Steele, Lea & Flood 2014) of counters 2 key and 2 key + 1,
 * key = (seed << 40) xor ((c N + ix) N + iy)(N/2 + 1) + iz; Box-Muller gives
 * a complex Gaussian g with E|g|^2 = 1; g is projected to k . g = 0 and
 * scaled by sqrt(E(|k|) / (4 pi |k|^2)) N^3, E(k) = k^4 exp(-2 (k/k0)^2); k = 0
 * and modes outside the dealias mask are zero; the kz = 0 and kz = N/2 planes
 * are made Hermitian (a mode whose mirror comes first in (iy, ix) order takes
 * the conjugate of the mirror's value; self-mirrored modes are real); the
 * field is then scaled to mean kinetic energy `energy`.  Synchronous. */
int dns_init_random(dns_t* ctx, unsigned long long seed, double k0, double energy);

/* Load u_hat from a (3, N, N, N/2+1) complex array. */
int dns_set_spectral(dns_t* ctx, const void* uhat_dev);

/* Copy the current u_hat into a (3, N, N, N/2+1) complex array. */
int dns_get_spectral(dns_t* ctx, void* uhat_dev);

/* u = F^-1(u_hat) into a (3, N, N, N) real array: complex inverse along x,
 * then y, then the inverse real transform along z, with 1/N^3 (Sec. 2,
 * eq. ifft); the imaginary parts of the kz = 0 and kz = N/2 coefficients do
 * not enter (numpy irfftn semantics). */
int dns_get_velocity(dns_t* ctx, void* u_dev);

/* Advance nsteps >= 0 time steps of the context's integrator: classic RK4
 * (Appendix solver: a = 1/6, 1/3, 1/3, 1/6; b = 1/2, 1/2, 1), or forward
 * Euler (u_hat += RHS dt).  Each stage evaluates eq. NSfinal: inverse
 * transforms of u_hat and omega_hat = i k x u_hat, u x omega in physical
 * space, forward transform, dealias mask, pressure projection and viscous
 * term.  Asynchronous; each step is replayed as one captured HIP graph
 * unless opts.use_graph = 0.  DNS_E_STATE before a velocity is set. */
int dns_step(dns_t* ctx, int nsteps);

/* One evaluation of the right-hand side of eq. NSfinal at the current
 * state, written as a (3, N, N, N/2+1) complex array; the state is not
 * changed.  For verification of a single stage. */
int dns_rhs(dns_t* ctx, void* rhs_dev);

/* dns_rhs without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the right-hand side of eq. NSfinal of the
 * (3, N, N, N/2+1) spectrum uhat_dev, written to rhs_dev (same layout and
 * dtype), for viscosity nu and the dealias rule `dealias`, enqueued on
 * `stream` (a hipStream_t cast to void*, NULL = null stream); asynchronous.
 * Same kernels and default plan as dns_rhs, hence the same bits.
 *
 * Allocates nothing: its work space (input and output in the internal
 * layout and six work fields, 32.4 MB) is one array that the library holds
 * on every GPU it runs on until the process ends, so N is limited to
 * N <= 64 (DNS_E_INVAL beyond; the message is in dns_last_error(NULL)).
 * Every call on a GPU uses that GPU's one array: calls that overlap in time
 * on one GPU (different streams or threads) race and must be ordered by the
 * caller.  Nothing in the array needs to start at zero (every value read is
 * written earlier in the same call).  The first call on each device looks
 * up the array's address and uploads the twiddle tables with a synchronous
 * copy; make it before capturing a graph.  DNS_E_INVAL for invalid
 * arguments, DNS_E_HIP if a launch fails. */
int dns_rhs_noalloc(int N, int dtype, double nu, int dealias, const void* uhat_dev, void* rhs_dev, void* stream);

/* E = mean over the mesh of |u|^2 / 2 (the Appendix's final energy) and
 * Omega = mean of |omega|^2 / 2, evaluated from the spectrum by Parseval
 * with FP64 accumulation in a fixed order.  Synchronous.  DNS_E_NONFINITE
 * if the value is NaN or Inf (the value is still written). */
int dns_energy(dns_t* ctx, double* E);
int dns_enstrophy(dns_t* ctx, double* Omega);
int dns_diagnostics(dns_t* ctx, double* E, double* Omega);

/* Copy up to max recorded (E, Omega) pairs (one per diag_every steps since
 * the last set) into host arrays E and Omega; *count receives the number
 * recorded.  Synchronous. */
int dns_history(dns_t* ctx, double* E, double* Omega, int max, int* count);

/* Number of time steps taken since the last set call. */
int dns_steps_taken(const dns_t* ctx, long long* steps);

/* Wait until all work the context enqueued has finished. */
int dns_synchronize(dns_t* ctx);

/* Time each kernel of one time step: runs nsteps steps with kernels launched
 * one by one on the context's stream, bracketed by HIP events, and writes
 * the mean duration in milliseconds of each of the step's kernels (in
 * launch order) into ms[0..*count-1] (at most max entries) and their names
 * (static strings) into names when non-NULL.  Advances the state. */
int dns_profile_step(dns_t* ctx, int nsteps, float* ms, const char** names, int max, int* count);

/* Standalone 3D transforms on caller buffers, using the context's plan and
 * work space (the state is not changed): forward real-to-complex
 * (3, N, N, N) -> (3, N, N, N/2+1) and inverse complex-to-real. */
int dns_forward(dns_t* ctx, const void* u_dev, void* uhat_dev);
int dns_inverse(dns_t* ctx, const void* uhat_dev, void* u_dev);

/* Execution plan.  Each of the six kernels (index order: inverse x pass
 * with curl, inverse y pass, fused z pass, forward y pass, forward x pass
 * with the RHS and RK4 update, and the latter fused with the next stage's
 * inverse x pass) has several variants.  Most differ only in how many FFT
 * lines share a workgroup (the "width") and in the schedule choices below;
 * they perform the same arithmetic per line, so results are bitwise
 * identical whichever is chosen.  The variants with another radix plan
 * (dns_variant.radix != 0) compute the same transforms with other rounding.
 *
 * dns_autotune times every variant of radix plan 0 on the context's own
 * buffers (reps launches each, 0 = 3) and keeps the fastest, so the tuned
 * plan gives the default plan's bits (reproducible mode); the velocity state
 * is preserved.  dns_autotune_ex with mode DNS_TUNE_FASTEST also times the
 * variants of the other radix plans and may choose them (results then agree
 * with the default plan to rounding, not bitwise); DNS_TUNE_REPRODUCIBLE is
 * dns_autotune.  dns_get_plan writes the chosen widths (6 entries);
 * dns_set_plan selects variants by width, keeping the current schedule and,
 * where such a variant exists, the current radix plan and pad (else plan 0
 * and the default pad); DNS_E_INVAL if a width does not exist for this N and
 * dtype.  dns_plan_variants lists the widths available for one kernel (pass
 * index 0..5) with the current schedule.  With opts.mfma_dft the y passes run the
 * matrix-core kernel, which has a single shape; their widths then only
 * matter for a later context without the option.
 *
 * Tuned plans are cached for the life of the process, keyed by (device
 * identity: architecture, name and compute units; N, dtype, simulations per
 * launch, tuning mode), each as the descriptors of its variants (see
 * dns_variant below): dns_autotune(_ex) stores its choice, and a context or
 * ensemble created with opts.autotune = 1 (2) takes the cached plan of the
 * reproducible (fastest) mode when one exists instead of timing again.
 * dns_plan_cache_entries returns the number of cached plans;
 * dns_plan_cache_clear empties the cache.  Persistence across processes:
 * dns_plan_cache_save writes the cache to a file (JSON, one plan per line),
 * dns_plan_cache_load adds a file's plans to the cache and returns how many
 * it read (DNS_E_INVAL if the file cannot be read); with the environment
 * variable DNS_PLAN_CACHE set to a path, the cache is loaded from it on
 * first use and saved to it after every autotune.  A stored plan whose
 * variants this build does not have is ignored.  All thread-safe. */
#define DNS_TUNE_REPRODUCIBLE 0
#define DNS_TUNE_FASTEST 1
int dns_autotune(dns_t* ctx, int reps);
int dns_autotune_ex(dns_t* ctx, int reps, int mode);
int dns_get_plan(const dns_t* ctx, int* widths, int max, int* count);
int dns_set_plan(dns_t* ctx, const int* widths, int n);
int dns_plan_variants(const dns_t* ctx, int pass, int* widths, int max, int* count);
int dns_plan_cache_entries(void);
int dns_plan_cache_clear(void);
int dns_plan_cache_save(const char* path);
int dns_plan_cache_load(const char* path);

/* Schedule of a step.  Besides the width, a pass variant fixes four choices
 * that change where work is done, never the arithmetic (results stay
 * bitwise identical):
 *  - y_elems: complex values per thread in the y passes (8, 16 or 32): the
 *    forward y pass, and the inverse one where the x pass forms the
 *    vorticity (the combining inverse y pass always holds 8);
 *  - curl_in_y: where the vorticity i k x u_hat of the Curl listing (Sec. 3.1)
 *    is combined.  Its components with ky and kz commute with the x
 *    transform, so the inverse x pass need transform only u_hat and the kx
 *    products; 1 = the inverse y pass combines them from the x pass's five
 *    fields, 0 = the x pass writes all six;
 *  - xcd_pair: the device dispatches workgroup b to XCD b mod 8, each XCD
 *    with its own L2.  Where an x- or y-pass tile's row segments are
 *    shorter than 128 bytes (32 or 64; N >= 256), 1 = the two or four tiles
 *    of each 128-byte line go to workgroups b, b + 8, ... (one XCD), 0 = to
 *    consecutive workgroups;
 *  - lds_pad (z pass only, else 0): a line's element p sits in shared
 *    memory at p + p / lds_pad (one unused slot after every lds_pad
 *    elements; 0 = no padding; default 8), which spreads the strided
 *    Stockham exchanges over the banks.
 * and one that changes the rounding:
 *  - radix: the radix plan of the line transforms (Stockham stages with
 *    N = 2^l): 0 = radix-8 stages, then one radix-4 or radix-2 stage (the
 *    default plan); 1 = that radix-4 or radix-2 stage first; 2 = radix-4
 *    stages, the last one radix 8 where l is odd.  Plans 1 and 2 exist, at
 *    the default shape of each pass, only for the N where they differ from
 *    the plans before them; only dns_autotune_ex in fastest mode or an
 *    explicit dns_set_plan_ex chooses them.
 * dns_set_schedule selects, for every pass, the variant of radix plan 0 and
 * the default pad of the current width (else the nearest width) that runs
 * the given schedule; y_elems 0, curl_in_y -1 and xcd_pair -1 take the
 * defaults for N.  DNS_E_INVAL for an
 * invalid value, DNS_E_UNSUPPORTED for a schedule this N and dtype (or the
 * matrix-core option) do not provide.  Waits for the stream.
 *
 * dns_plan_variants_ex lists every variant of one pass (index order of
 * dns_get_plan) with its descriptor (y_elems 0 for passes other than the y
 * passes; curl_in_y -1 for passes that do not depend on it; radix and
 * lds_pad as above).
 * dns_get_plan_ex / dns_set_plan_ex read and install a plan as one variant
 * index per pass; DNS_E_INVAL if an index is out of range or the inverse x,
 * inverse y and stage passes disagree on curl_in_y. */
typedef struct dns_variant {
    int width;
    int xcd_pair;
    int y_elems;
    int curl_in_y;
    int radix;
    int lds_pad;
} dns_variant;
int dns_set_schedule(dns_t* ctx, int y_elems, int curl_in_y, int xcd_pair);
int dns_plan_variants_ex(const dns_t* ctx, int pass, dns_variant* out, int max, int* count);
int dns_get_plan_ex(const dns_t* ctx, int* variants, int max, int* count);
int dns_set_plan_ex(dns_t* ctx, const int* variants, int n);

/* Measurement helper (not part of the method): copy nrows rows of
 * row_bytes bytes (a multiple of 16) from src to dst, row r at byte offset
 * r * pitch in both device buffers, each row read and written as one
 * row_bytes request (16 bytes per thread), enqueued on `stream`.  A copy of
 * known bytes with the row length of a pass's tiles calibrates the
 * hardware's HBM byte counters for that request size.  DNS_E_INVAL for a
 * row length that is not a positive multiple of 16 or a pitch shorter than
 * the row. */
int dns_copy_rows(const void* src, void* dst, size_t nrows, int row_bytes, size_t pitch, void* stream);

/* dns_strerror: a static description of a status code.  dns_last_error:
 * the message of the context's last failure ("" if none); with NULL, the
 * message of the calling thread's last failed context-free call.
 *
 * Testing error paths: with the environment variable DNS_FAULT_INJECT set to
 * "launch" when a context is created, every launch check of that context
 * reports DNS_E_HIP ("injected launch failure") after the kernels have been
 * enqueued normally; no device fault is involved. */
const char* dns_strerror(int status);
const char* dns_last_error(const dns_t* ctx);

/* ---------------------------------------------------------------------------
 * Ensembles of independent simulations (possibly of different N).
 *
 * Members with equal (N, nu, dt) form a class whose state lives in one
 * allocation; every stage kernel advances all members of a class in one
 * launch (one workgroup row per member).  Member i is addressed by its index
 * in the arrays given at creation.  Same conventions, ownership and
 * ordering rules as the single-simulation calls; opts applies to all
 * members.
 * ------------------------------------------------------------------------- */
typedef struct dns_ens dns_ens_t;
enum {
    DNS_ENS_BATCHED = 0,   /* one captured graph per step covering every class,
                              replayed once per step */
    DNS_ENS_PER_SIM = 1,   /* every member's kernels launched separately (baseline) */
    DNS_ENS_ONE_GRAPH = 2  /* all nsteps steps of every class captured into one
                              graph and launched once (captured on the first
                              call with that nsteps; the four most recent step
                              counts are kept) */
};
int dns_ens_create(int count, const int* N, const double* nu, const double* dt, int dtype,
                   const dns_opts* opts, void* stream, dns_ens_t** out);
int dns_ens_destroy(dns_ens_t* ens);
int dns_ens_size(const dns_ens_t* ens, int* count, int* classes);
int dns_ens_set_velocity(dns_ens_t* ens, int i, const void* u_dev);
int dns_ens_set_spectral(dns_ens_t* ens, int i, const void* uhat_dev);
int dns_ens_init_random(dns_ens_t* ens, int i, unsigned long long seed, double k0, double energy);
int dns_ens_get_spectral(dns_ens_t* ens, int i, void* uhat_dev);
/* Advance every member nsteps time steps; mode DNS_ENS_BATCHED,
 * DNS_ENS_PER_SIM or DNS_ENS_ONE_GRAPH (bitwise identical results).  With
 * per-step diagnostics (opts.diag_every) or opts.use_graph = 0 the batched
 * modes launch kernel by kernel. */
int dns_ens_step(dns_ens_t* ens, int nsteps, int mode);
/* E[i], Omega[i] for every member (either pointer may be NULL). Synchronous. */
int dns_ens_diagnostics(dns_ens_t* ens, double* E, double* Omega);
int dns_ens_synchronize(dns_ens_t* ens);
const char* dns_ens_last_error(const dns_ens_t* ens);

#ifdef __cplusplus
}
#endif

#endif /* DNS_H */
