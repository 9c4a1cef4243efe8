"""Benchmark: ms per RK4 step of the Taylor-Green vortex at 512^3 on one
MI355X, FP64 (headline) and FP32, through the C ABI of libdns.so.

Prints ONE JSON line.  Inputs are resident in HBM before the timed region;
the timed region is K graph-replayed RK4 steps bracketed by device
synchronisation.  The roofline object reports the dominant kernel's
algorithmic HBM bytes per launch over its mean duration (HIP events on the
library's stream), against the 8 TB/s HBM peak.  The cpu_baseline object
times the CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per RK4 step at 512^3 (FP64 vs FP32) + HBM GB/s; ensemble steps/s"
HBM_PEAK_GBPS = 8000.0
N_DEFAULT, NU, DT = 512, 1.0 / 1600, 1e-3

# Algorithmic HBM traffic of each kernel, in half-spectrum fields
# C = N^2 (N/2+1) complex values (read + write).  The RK4 state moves 36C per
# step (stage 0: read U0, write Us; stage 1: read Us, U0, write Us, U1;
# stage 2: read Us, U0, write Us; stage 3: read Us, U1, write U0), and the
# forward x pass reads N_hat (3C) at every stage, so xrhs_rk4 averages
# (36 + 12) / 4 = 12C; xstage adds the inverse-x fields it writes for the
# next stage.  Below N = 1024 the inverse y pass forms the vorticity from
# five x-pass fields (U, V, W, F(kx v), F(kx w)): xinv_curl 3C + 5C,
# yinv6 5C + 6C, xstage 12C + 5C, fused step 4 * (11 + 9 + 6 + 17) C = 172 C.
# Where the x pass writes all six (the default at N = 1024, or a plan with
# the vorticity formed in the x pass): 9C, 12C, 18C and 180 C per step.
# Unfused (either): 4 * (9 + 27) C + 48 C = 192 C.
def curl_in_y(N, cy=None):
    """True where the inverse y pass combines the vorticity: the plan's
    choice cy when given, else the default (N < 1024)."""
    return bool(cy) if cy is not None else N < 1024


def fields_per_launch(N, cy=None):
    x = 5.0 if curl_in_y(N, cy) else 6.0
    return {"xinv_curl": 3.0 + x, "yinv6": x + 6.0, "zcross": 9.0, "yfwd3": 6.0, "xrhs_rk4": 48.0 / 4,
            "xstage": 48.0 / 4 + x}


def fields_per_step(N, cy=None):
    f = fields_per_launch(N, cy)
    return 4 * (f["yinv6"] + f["zcross"] + f["yfwd3"] + f["xstage"])


def kernel_source_hash():
    """SHA-256 of the HIP sources with // comments and blank lines removed, so
    that counter summaries stay valid across comment-only edits."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_1602_03638_amd", "csrc", "*"))):
        with open(path) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(N, dtype, kernel, cy=None):
    """HBM bytes per launch of `kernel` (averaged over its RK stages) from the
    committed rocprofv3 counter summary, calibrated against a plain copy;
    None when no summary exists for this size or the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_tg{N}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    real = "double" if dtype == "f64" else "float"
    name = {"xstage": "k_xstage", "xrhs_rk4": "k_xrhs", "xinv_curl": "k_xinv_curl", "zcross": "k_zcross",
            "yinv6": "k_yinv_curl" if curl_in_y(N, cy) else "k_yline", "yfwd3": "k_yline"}[kernel]

    def args(k):   # template arguments after <real, N, width
        return [a.strip() for a in k[k.index("<") + 1:k.rindex(">")].split(",")][3:]
    vals = [v["traffic_bytes_calibrated"] for k, v in rec["kernels"].items()
            if k.startswith(f"{name}<{real}, {N},")
            and (kernel != "yinv6" or curl_in_y(N, cy) or args(k)[:2] == ["1", "6"])
            and (kernel != "yfwd3" or args(k)[:2] == ["-1", "3"])]
    return sum(vals) / len(vals) if vals else None


def oracle_tg_error(N, n, E, W):
    """Relative energy and enstrophy errors after n steps of the Re = 1600
    Taylor-Green run against the CPU oracle's values, stored by
    tests/golden/make_tg_reference.py from a 64^3 oracle run (the low-mode
    content of this run is resolution independent over its first 100 steps,
    so the values hold for any N >= 64); None beyond the stored steps."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "tg_re1600_n64.npz")
    if N < 64 or not os.path.exists(path):
        return None
    g = np.load(path)
    if n >= len(g["energy"]):
        return None
    E0, W0 = float(g["energy"][n]), float(g["enstrophy"][n])
    return {"step": n, "rel_energy": abs(E - E0) / E0, "rel_enstrophy": abs(W - W0) / W0,
            "reference": "CPU oracle (FP64 plain DFT), tests/golden/tg_re1600_n64.npz"}


def progress(msg):
    """One line per finished leg on stderr (long runs show that they move)."""
    print(msg, file=sys.stderr, flush=True)


def field_bytes(N, dtype):
    return N * N * (N // 2 + 1) * (16 if dtype == "f64" else 8)


ERROR_STEP = 50   # the Taylor-Green 512^3 case is stated after 50 steps


def tg_velocity_error(s, n):
    """Relative L2 (Hermitian-weighted, equal to the physical-space relative
    L2 by Parseval) of the context's velocity after n steps of the Re = 1600
    Taylor-Green run against the oracle's stored run: its coefficients
    u_hat / N^3 of every mode with |k_i| <= kmax, and zero outside that box
    (where the oracle's field holds a fraction outside_rel_l2 of the norm,
    stored with it).  None when the run is not stored at step n."""
    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", "tg_re1600_n64.npz")
    g = np.load(path)
    if f"modes_{n}" not in g.files:
        return None
    N = s.N
    ref = g[f"modes_{n}"]
    kxy, kz = g["kxy"], g["kz"]
    uh = s.get_spectral()
    ix = torch.as_tensor(np.where(kxy < 0, kxy + N, kxy), device="cuda")
    iz = torch.as_tensor(kz, device="cuda")
    sel = (slice(None), ix[:, None, None], ix[None, :, None], iz[None, None, :])
    box = uh[sel].cpu().numpy().astype(np.complex128) / float(N) ** 3
    uh[sel] = 0
    w = torch.full((N // 2 + 1,), 2.0, dtype=torch.float64, device="cuda")
    w[0] = w[-1] = 1.0
    out2 = float((uh.abs().double() ** 2 * w).sum().item()) / float(N) ** 6
    del uh
    torch.cuda.empty_cache()
    wb = np.where(kz == 0, 1.0, 2.0)
    num = np.sum(wb * np.abs(box - ref) ** 2) + out2
    den = np.sum(wb * np.abs(ref) ** 2)
    return {"velocity_rel_l2": float(np.sqrt(num / den)),
            "velocity_rel_l2_outside_box": float(np.sqrt(out2 / den)),
            "box_kmax": int(g["kmax"]), "oracle_outside_rel_l2": float(g[f"outside_rel_l2_{n}"])}


def run_gpu(N, dtype, steps, warmup, prof_steps, error_step=ERROR_STEP):
    """Time `steps` RK4 steps of the Taylor-Green field after `warmup`, then
    continue (untimed) to step `error_step` and state the errors against the
    CPU oracle there; mean kernel times from `prof_steps` profiled steps."""
    import torch
    import workloads
    from paper_1602_03638_amd import Solver

    u0 = torch.from_numpy(workloads.taylor_green(N)).to(torch.float64 if dtype == "f64" else torch.float32)
    u0 = u0.cuda().contiguous()
    s = Solver(N, NU, DT, dtype=dtype)
    s.set_velocity(u0)
    del u0
    cy = s.schedule()["xstage"]["curl_in_y"]
    s.step(warmup)
    s.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.synchronize()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    progress(f"taylor_green {N}^3 {dtype}: {ms:.3f} ms/step")
    done = warmup + steps
    if done < error_step:
        s.step(error_step - done)
        done = error_step
    E, W = s.diagnostics()
    err = oracle_tg_error(N, done, E, W) if error_step > 0 else None
    if err is not None:
        v = tg_velocity_error(s, done)
        if v is not None:
            err.update(v)
    kern = s.profile_step(prof_steps) if prof_steps > 0 else {}
    s.close()
    torch.cuda.empty_cache()
    C = field_bytes(N, dtype)
    out = {"ms_per_step": ms, "model_GBps": fields_per_step(N, cy) * C / (ms * 1e-3) / 1e9,
           "energy": E, "enstrophy": W, "error_vs_oracle": err, "kernels_ms": kern, "curl_in_y": cy}
    if kern:
        achieved = {k: fields_per_launch(N, cy)[k] * C / (v * 1e-3) / 1e9 for k, v in kern.items()}
        out["kernels_GBps"] = achieved
    return out


# Ensemble workload: 64 members at 32^3, 16 at 64^3 and 4 at 128^3, FP32,
# seeded random isotropic fields (member j: seed 1000 + j, k0 = 4, E = 0.5).
ENSEMBLE = [(32, 64), (64, 16), (128, 4)]
ENS_NU, ENS_DT = 0.01, 0.005


def run_ensemble(steps, warmup, per_sim_steps, autotune=True):
    """Ensemble steps per second: batched kernels (each advances every member
    of one size) replayed as one captured graph per step, all `steps` steps
    captured into one graph launched once, and per-simulation launches of
    the same kernels (the baseline)."""
    import torch
    from paper_1602_03638_amd import Ensemble

    Ns = [N for N, count in ENSEMBLE for _ in range(count)]
    ens = Ensemble(Ns, [ENS_NU] * len(Ns), [ENS_DT] * len(Ns), dtype="f32", autotune=autotune)
    for j in range(len(Ns)):
        ens.init_random(j, 1000 + j, k0=4.0, energy=0.5)

    def timed(n, mode):
        kw = {"batched": mode != "per_sim", "one_graph": mode == "one_graph"}
        ens.step(n if mode == "one_graph" else warmup, **kw)   # one_graph: captures the n-step graph
        ens.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.step(n, **kw)
        ens.synchronize()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    ms_b = timed(steps, "batched")
    ms_o = timed(steps, "one_graph")
    ms_p = timed(per_sim_steps, "per_sim")
    E, _ = ens.diagnostics()
    ens.close()
    traffic = sum(count * fields_per_step(N) * field_bytes(N, "f32") for N, count in ENSEMBLE)

    def rec(n, ms):
        return {"steps": n, "ms_per_step": round(ms, 4), "ens_steps_per_s": round(1e3 / ms, 1),
                "sim_steps_per_s": round(len(Ns) * 1e3 / ms, 1), "model_GBps": round(traffic / (ms * 1e-3) / 1e9, 1)}
    return {"workload": "+".join(f"{count}x{N}^3" for N, count in ENSEMBLE) + " f32 random isotropic",
            "members": len(Ns), "nu": ENS_NU, "dt": ENS_DT, "autotuned_plans": autotune,
            "one_graph": rec(steps, ms_o), "batched": rec(steps, ms_b), "per_sim": rec(per_sim_steps, ms_p),
            "speedup": round(ms_p / ms_o, 2), "speedup_per_step_replay": round(ms_p / ms_b, 2),
            "energy_mean": sum(E) / len(E)}


# Random isotropic field at 1024^3 (seed 1, k0 = 4, E = 0.5): FP32 path
# timed, FP64 path as its reference (the CPU oracle cannot hold 1024^3).
ISO_N, ISO_NU, ISO_DT, ISO_STEPS, ISO_SEED = 1024, 1e-3, 5e-4, 20, 1


def run_isotropic(N=ISO_N, steps=ISO_STEPS, warmup=2):
    """ms per RK4 step of the random isotropic field in FP32 (plain Stockham
    y passes, and with the radix-16 stage of the y passes on FP16 matrix
    cores) and in FP64, and each FP32 run's errors against the FP64 path
    after `steps` steps (relative energy and enstrophy differences, relative
    L2 of the spectral velocity).  All start from the same FP64-generated
    spectrum (FP32 takes it rounded), so the differences are the FP32
    arithmetic alone.  Mean kernel times come from one extra profiled step."""
    import torch
    from paper_1602_03638_amd import Solver

    def run(dtype, uh0, **kw):
        s = Solver(N, ISO_NU, ISO_DT, dtype=dtype, **kw)
        s.set_spectral(uh0.to(s.complex).contiguous())
        s.step(warmup)
        s.synchronize()
        s.set_spectral(uh0.to(s.complex).contiguous())   # timed run from the initial field
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.synchronize()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        E, W = s.diagnostics()
        out = s.get_spectral()
        s.set_spectral(uh0.to(s.complex).contiguous())
        kern = {k: round(v, 3) for k, v in s.profile_step(1).items()}
        s.close()
        progress(f"random_isotropic {N}^3 {dtype}{' mfma_dft' if kw else ''}: {ms:.3f} ms/step")
        return ms, E, W, out, kern

    s = Solver(N, ISO_NU, ISO_DT, dtype="f64")
    s.init_random(ISO_SEED, k0=4.0, energy=0.5)
    E0, W0 = s.diagnostics()
    uh0 = s.get_spectral()
    s.close()
    torch.cuda.empty_cache()
    ms32, E32, W32, u32, k32 = run("f32", uh0)
    u32 = u32.cpu()
    torch.cuda.empty_cache()
    msm, Em, Wm, um, km = run("f32", uh0, mfma_dft=True)
    um = um.cpu()
    torch.cuda.empty_cache()
    ms64, E64, W64, u64, k64 = run("f64", uh0)
    del uh0
    torch.cuda.empty_cache()
    norm64 = torch.linalg.vector_norm(u64)

    def errors(E, W, u):
        d = u.to(u64.device).to(torch.complex128) - u64
        out = {"rel_energy": abs(E - E64) / E64, "rel_enstrophy": abs(W - W64) / W64,
               "rel_l2_spectral_velocity": float(torch.linalg.vector_norm(d) / norm64)}
        del d
        return out

    err32, errm = errors(E32, W32, u32), errors(Em, Wm, um)
    del u64, u32, um
    torch.cuda.empty_cache()
    C = field_bytes(N, "f32")
    return {"workload": f"random_isotropic_{N}_rk4", "N": N, "nu": ISO_NU, "dt": ISO_DT, "steps": steps,
            "seed": ISO_SEED, "k0": 4.0, "E0": E0, "Omega0": W0,
            "fp32": {"ms_per_step": round(ms32, 3), "model_GBps": round(fields_per_step(N) * C / (ms32 * 1e-3) / 1e9, 1),
                     "energy": E32, "enstrophy": W32, "kernels_ms": k32},
            "fp32_mfma_dft": {"ms_per_step": round(msm, 3),
                              "model_GBps": round(fields_per_step(N) * C / (msm * 1e-3) / 1e9, 1),
                              "energy": Em, "enstrophy": Wm, "kernels_ms": km,
                              "y_stage": "radix-16 DFT on FP16 matrix cores (hi/lo split, FP32 accumulation)"},
            "fp64": {"ms_per_step": round(ms64, 3),
                     "model_GBps": round(fields_per_step(N) * 2 * C / (ms64 * 1e-3) / 1e9, 1),
                     "energy": E64, "enstrophy": W64, "kernels_ms": k64},
            "fp32_vs_fp64": err32, "fp32_mfma_dft_vs_fp64": errm}


# The paper's FFT benchmark (Sec. 4.3): one forward and one inverse 3D real
# transform, fastest of 10, here of a 3-component field held in HBM.
FFT_SIZES = (128, 256, 512, 1024)


def run_fft(sizes=FFT_SIZES, dtypes=("f32", "f64"), reps=10):
    """Time dns_set_velocity (z r2c, y, x: physical -> internal spectrum) plus
    dns_get_velocity (x, y, z c2r) of a random 3-component field: fastest
    and mean of `reps` pairs (torch events on the caller's stream, which the
    library's stream is ordered with).  Algorithmic traffic of one pair:
    forward 3R + 15C (z pass reads 3 real fields, writes 3 spectra; y in
    place; x out of place), inverse the same, R = N^3 reals, C = N^2 (N/2+1)
    complex values."""
    import torch
    from paper_1602_03638_amd import Solver
    out = []
    for dtype in dtypes:
        for N in sizes:
            real = torch.float64 if dtype == "f64" else torch.float32
            g = torch.Generator(device="cuda").manual_seed(N)
            u = torch.randn((3, N, N, N), generator=g, dtype=real, device="cuda")
            v = torch.empty_like(u)
            torch.cuda.empty_cache()
            s = Solver(N, NU, DT, dtype=dtype)
            for _ in range(2):
                s.set_velocity(u)
                s.get_velocity(v)
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                s.set_velocity(u)
                s.get_velocity(v)
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            err = float(torch.linalg.vector_norm(v - u) / torch.linalg.vector_norm(u))
            s.close()
            del u, v
            torch.cuda.empty_cache()
            S = 8 if dtype == "f64" else 4
            nbytes = 2 * (3 * N ** 3 * S + 15 * field_bytes(N, dtype))
            best = min(times)
            out.append({"N": N, "dtype": dtype, "ms_pair_best": round(best, 4),
                        "ms_pair_mean": round(sum(times) / len(times), 4),
                        "ms_pair_per_component": round(best / 3, 4),
                        "GBps_best": round(nbytes / (best * 1e-3) / 1e9, 1),
                        "roundtrip_rel_l2": err})
    return {"workload": "forward + inverse 3D real FFT of a 3-component random field, fastest of "
                        f"{reps}", "results": out}


def run_tg_long(N, dtype, steps, out_path, chunk=1000):
    """The paper's Taylor-Green verification run (Sec. 4.2: Re = 1600,
    nu = 1/1600, dt = 1e-3, t = 0 -> 20): energy and enstrophy after every
    step, written as JSON to out_path; progress every `chunk` steps.  The
    energy budget residual (E_{n+1} - E_n)/dt + nu (Omega_n + Omega_{n+1}) is
    reported alongside (the semi-discrete system has dE/dt = -2 nu Omega)."""
    import torch
    import workloads
    from paper_1602_03638_amd import Solver

    u0 = torch.from_numpy(workloads.taylor_green(N)).to(torch.float64 if dtype == "f64" else torch.float32)
    s = Solver(N, NU, DT, dtype=dtype, diag_every=1, history_cap=steps)
    s.set_velocity(u0.cuda().contiguous())
    del u0
    E0, W0 = s.diagnostics()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        s.step(n)
        s.synchronize()
        done += n
        print(f"tg-long N={N} {dtype}: {done}/{steps} steps, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    wall = time.perf_counter() - t0
    E, W = s.history()
    s.close()
    E, W = [E0] + list(E), [W0] + list(W)
    res = [abs((E[n + 1] - E[n]) / DT + NU * (W[n] + W[n + 1])) / (NU * (W[n] + W[n + 1])) for n in range(len(E) - 1)]
    rec = {"workload": f"taylor_green_{N}_rk4_re1600", "N": N, "dtype": dtype, "nu": NU, "dt": DT, "steps": steps,
           "ms_per_step": wall * 1e3 / steps, "energy": E, "enstrophy": W, "max_rel_budget_residual": max(res)}
    with open(out_path, "w") as f:
        json.dump(rec, f)
    peak = max(range(len(W)), key=lambda i: W[i])
    return {"N": N, "dtype": dtype, "steps": steps, "ms_per_step": round(rec["ms_per_step"], 3),
            "E_final": E[-1], "enstrophy_peak": W[peak], "t_enstrophy_peak": peak * DT,
            "max_rel_budget_residual": max(res)}


def host_info():
    """The host's CPU model and core counts (from /proc/cpuinfo and the
    scheduler affinity), and the threads the oracle's BLAS uses."""
    model, cores = None, set()
    try:
        phys = core = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [threads])
    except Exception:
        pass
    return {"cpu_model": model, "host_physical_cores": len(cores) or None, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "blas_threads": threads}


def cpu_baseline(N_metric, sizes=((128, 3), (256, 1))):
    """Time the CPU oracle's full RK4 step (oracle.spectral.rk4_step: four
    right-hand sides, each nine plain-DFT 3D transforms plus the elementwise
    curl, cross product, mask, projection and viscous term) on the host, on
    the Taylor-Green field of the benchmark: the median of the steps run at
    each size.  The metric's size is reached from the largest size timed by
    the growth factor measured between the two sizes (the DFT-matrix
    transforms cost N^4)."""
    import statistics

    import workloads
    from oracle import spectral

    times = {}
    for N, nsteps in sizes:
        s = spectral.Solver(N, NU, DT).set_velocity(workloads.taylor_green(N))
        t = []
        for _ in range(nsteps):
            t0 = time.perf_counter()
            s.step(1)
            t.append(time.perf_counter() - t0)
        times[N] = statistics.median(t)
        del s
    (n0, _), (n1, _) = sizes[0], sizes[-1]
    growth = times[n1] / times[n0]
    per_doubling = growth ** (1.0 / max(1, (n1 // n0).bit_length() - 1))
    steps_to_metric = max(0, (N_metric // n1).bit_length() - 1)
    ms = times[n1] * per_doubling ** steps_to_metric * 1e3
    h = host_info()
    return {"value": ms, "unit": "ms/step", "cores": h["blas_threads"], "kind": "oracle_step",
            "sample": f"full oracle RK4 steps of the Taylor-Green field: median of {sizes[0][1]} at {n0}^3 "
                      f"({times[n0]:.2f} s), {sizes[-1][1]} at {n1}^3 ({times[n1]:.2f} s); {N_metric}^3 value = "
                      f"the {n1}^3 step x {per_doubling:.1f} per doubling of N (measured {n0}->{n1})",
            "measured_s_per_step": {str(k): v for k, v in times.items()}, "growth_per_doubling": per_doubling,
            **h}


def gpu_clocks():
    """Current and enabled clock levels reported by rocm-smi (text lines), or
    None when rocm-smi is not available."""
    import shutil
    import subprocess
    exe = shutil.which("rocm-smi") or "/opt/rocm/bin/rocm-smi"
    if not os.path.exists(exe):
        return None
    try:
        r = subprocess.run([exe, "--showclocks"], capture_output=True, text=True, timeout=30)
    except Exception:
        return None
    lines = [ln.strip() for ln in r.stdout.splitlines() if "clock level" in ln.lower() or "Mhz" in ln]
    return lines[:12] or None


def sweep(N, dtype, reps=2):
    """Time every variant of every pass (HIP events, mean over the launches
    of `reps` profiled steps) with the other passes at the default plan, and
    the autotuner's choice in its reproducible and fastest modes (with the
    step time of each plan); fused and unfused schedules."""
    import torch
    import workloads
    from paper_1602_03638_amd import Solver

    u0 = torch.from_numpy(workloads.taylor_green(N)).to(torch.float64 if dtype == "f64" else torch.float32)
    u0 = u0.cuda().contiguous()
    out = {"N": N, "dtype": dtype, "passes": {}}
    for fuse in (True, False):
        s = Solver(N, NU, DT, dtype=dtype, fuse=fuse).set_velocity(u0)
        base = s.plan_ex()
        var = s.plan_variants_ex()
        out["default_schedule"] = s.schedule()
        mine = ("yinv6", "zcross", "yfwd3", "xstage") if fuse else ("xinv_curl", "xrhs_rk4")
        for p in mine:
            res = []
            for v, d in enumerate(var[p]):
                s.set_plan_ex(s.plan_with(p, v, base))
                s.profile_step(1)            # warm (rebuilds the fused work space)
                res.append(dict(d, ms=round(s.profile_step(reps)[p], 4)))
            out["passes"][p] = res
            progress(f"sweep {N}^3 {dtype} {p}: {len(res)} variants")
        s.set_plan_ex(base)
        key = "fused" if fuse else "unfused"
        for mode, tag in (("reproducible", ""), ("fastest", "fastest_")):
            s.autotune(mode=mode)
            out[f"autotuned_{tag}{key}"] = s.schedule()
            s.profile_step(1)
            out[f"autotuned_{tag}ms_{key}"] = {k: round(v, 4) for k, v in s.profile_step(reps).items()}
            s.step(1)
            s.synchronize()
            t0 = time.perf_counter()
            s.step(10)
            s.synchronize()
            out[f"autotuned_{tag}step_ms_{key}"] = round((time.perf_counter() - t0) * 100.0, 4)
            s.set_plan_ex(base)
        s.close()
    print(json.dumps(out), flush=True)
    return 0


def calibrate_copy(gib, row_bytes=0, pitch=0, reps=5):
    """A copy of known size for calibrating the per-kernel HBM byte counters:
    row_bytes = 0 is a plain device copy (torch), else dns_copy_rows with rows
    of row_bytes bytes (one request each) every `pitch` bytes (default: the
    row length, i.e. contiguous).  Prints the bytes read and written."""
    import ctypes

    import torch
    from paper_1602_03638_amd import load_library
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    if row_bytes <= 0:
        def run():
            dst.copy_(src)
        moved = n * 8
        desc = "plain device copy"
    else:
        pitch = pitch or row_bytes
        nrows = (n * 8) // pitch
        lib = load_library()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

        def run():
            st = lib.dns_copy_rows(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nrows,
                                   int(row_bytes), int(pitch), stream)
            if st != 0:
                raise RuntimeError(f"dns_copy_rows: status {st}")
        moved = nrows * row_bytes
        desc = f"dns_copy_rows: {nrows} rows of {row_bytes} B, pitch {pitch} B"
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    print(json.dumps({"copy": desc, "copy_bytes_read": moved, "copy_bytes_written": moved, "launches": reps + 1,
                      "ms": ms, "GBps_read_plus_write": 2 * moved / (ms * 1e-3) / 1e9}), flush=True)
    return 0


# ---------------------------------------------------------------------------
# Summaries of rocprofv3 output (kernel trace statistics and HBM counters),
# written under profiles/ with the command that made them.
# ---------------------------------------------------------------------------
def kernel_short_name(name):
    """'void dns::k_x<double, 512, 8>(...)' -> 'k_x<double, 512, 8>'."""
    name = name.strip().strip('"')
    if name.startswith("void "):
        name = name[5:]
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return name[:cut].replace("dns::", "").strip()


def algorithmic_bytes(short):
    """Algorithmic HBM bytes (read + write) of one launch of a stage kernel,
    from its template arguments (see the traffic model at the top of this
    file); None for other kernels."""
    import re
    m = re.match(r"(k_\w+)<(.*)>$", short)
    if not m:
        return None
    kind, args = m.group(1), [a.strip() for a in m.group(2).split(",")]
    if kind == "k_yline_mfma":
        N, DIR, NF = int(args[0]), int(args[1]), int(args[2])
        return 2 * NF * field_bytes(N, "f32")
    if len(args) < 2 or args[0] not in ("double", "float"):
        return None
    dt = "f64" if args[0] == "double" else "f32"
    N = int(args[1])
    C = field_bytes(N, dt)
    state = {0: 6, 1: 12, 2: 9, 3: 9, 4: 6, -1: 6}
    if kind == "k_xinv_curl":
        return (3 + (5 if args[3] == "true" else 6)) * C
    if kind == "k_yinv_curl":
        return 11 * C
    if kind == "k_yline":
        return 2 * int(args[4]) * C
    if kind == "k_zcross":
        return 9 * C
    if kind == "k_xrhs":
        return (3 + state[int(args[3])]) * C
    if kind == "k_xstage":
        return (3 + state[int(args[3])] + (5 if args[4] == "true" else 6)) * C
    return None


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits


def summarize_trace(stats_dir, out_md, command, title):
    """Kernel trace statistics (rocprofv3 --kernel-trace --stats) as a table
    of calls and durations per kernel instance, with the algorithmic bytes
    and bandwidth at the mean duration for the stage kernels."""
    rows = []
    for path in _find(stats_dir, "kernel_stats.csv"):
        rows += _csv_rows(path)
    lines = [f"# {title}", "", "Command (repository root, on the MI355X machine):", "", "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | alg. bytes / launch (GB) | GB/s at avg |",
             "|---|---|---|---|---|---|---|"]
    recs = []
    for r in rows:
        name = kernel_short_name(r["Name"])
        avg = float(r["AverageNs"]) / 1e3
        alg = algorithmic_bytes(name)
        recs.append((float(r["TotalDurationNs"]), name, int(r["Calls"]), avg, float(r["MinNs"]) / 1e3,
                     float(r["MaxNs"]) / 1e3, alg))
    for _, name, calls, avg, mn, mx, alg in sorted(recs, reverse=True):
        a = f"{alg / 1e9:.3f}" if alg else ""
        bw = f"{alg / (avg * 1e-6) / 1e9:.0f}" if alg else ""
        lines.append(f"| `{name}` | {calls} | {avg:.1f} | {mn:.1f} | {mx:.1f} | {a} | {bw} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return 0


def _counter_means(d, counter):
    """Mean value of `counter` per kernel instance over its dispatches."""
    acc = {}
    for path in _find(d, "counter_collection.csv"):
        for r in _csv_rows(path):
            if r.get("Counter_Name") != counter:
                continue
            name = kernel_short_name(r["Kernel_Name"])
            v = float(r["Counter_Value"])
            s, n = acc.get(name, (0.0, 0))
            acc[name] = (s + v, n + 1)
    return {k: (s / n, n) for k, (s, n) in acc.items()}


def summarize_counters(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, cal_bytes, N, out_json, out_md,
                       commands, title):
    """HBM traffic per dispatch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs
    (KiB per dispatch), each scaled by the factor that maps the same counter
    of a copy of known size (cal_bytes read and written, dns_copy_rows or a
    device copy) to its bytes.  Keyed by the hash of the kernel sources
    (comments removed) at the time of summarising."""
    fetch, write = _counter_means(fetch_dir, "FETCH_SIZE"), _counter_means(write_dir, "WRITE_SIZE")
    cf, cw = _counter_means(cal_fetch_dir, "FETCH_SIZE"), _counter_means(cal_write_dir, "WRITE_SIZE")
    def copy_kernel(c):   # the copy itself, not the fill that made its source
        named = {k: v for k, v in c.items() if "copy" in k.lower()}
        return max((named or c).items(), key=lambda kv: kv[1][0])
    copy_f, copy_w = copy_kernel(cf), copy_kernel(cw)
    ff = cal_bytes / (copy_f[1][0] * 1024.0)
    fw = cal_bytes / (copy_w[1][0] * 1024.0)
    kernels = {}
    for name in sorted(set(fetch) | set(write)):
        fk = fetch.get(name, (0.0, 0))[0]
        wk = write.get(name, (0.0, 0))[0]
        kernels[name] = {"fetch_kib_raw": fk, "write_kib_raw": wk, "fetch_factor": ff, "write_factor": fw,
                         "traffic_bytes_calibrated": fk * 1024.0 * ff + wk * 1024.0 * fw,
                         "dispatches": max(fetch.get(name, (0, 0))[1], write.get(name, (0, 0))[1]),
                         "alg_bytes": algorithmic_bytes(name)}
    rec = {"source_sha256": kernel_source_hash(), "N": N, "calibration": {
        "kernel_fetch": copy_f[0], "kernel_write": copy_w[0], "bytes_each_way": cal_bytes,
        "fetch_factor": ff, "write_factor": fw}, "commands": commands, "kernels": kernels}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# {title}", "", "Commands (repository root, on the MI355X machine), one counter per run:", "", "```"]
    lines += commands + ["```", "",
                         f"Calibration: `{copy_f[0]}` moving {cal_bytes} bytes each way reads FETCH_SIZE "
                         f"{copy_f[1][0]:.0f} KiB (factor {ff:.3f}) and WRITE_SIZE {copy_w[1][0]:.0f} KiB "
                         f"(factor {fw:.3f}).", "",
                         "| kernel | dispatches | FETCH_SIZE KiB (raw, mean) | WRITE_SIZE KiB (mean) | "
                         "traffic GB (calibrated) | alg. GB | traffic / alg. |", "|---|---|---|---|---|---|---|"]
    for name, v in sorted(kernels.items(), key=lambda kv: -kv[1]["traffic_bytes_calibrated"]):
        alg = v["alg_bytes"]
        ratio = f"{v['traffic_bytes_calibrated'] / alg:.3f}" if alg else ""
        a_gb = f"{alg / 1e9:.3f}" if alg else ""
        lines.append(f"| `{name}` | {v['dispatches']} | {v['fetch_kib_raw']:.0f} | {v['write_kib_raw']:.0f} | "
                     f"{v['traffic_bytes_calibrated'] / 1e9:.3f} | {a_gb} | {ratio} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return 0


def summarize_tg_long(out_md, ref_path, f32_path, coarse_path):
    """Table of the Taylor-Green Re = 1600 runs to t = 20 (bench.py --tg-long
    output files): E, Omega and the dissipation 2 nu Omega of the reference
    run at chosen times, the FP32 run's and the coarser grid's relative
    differences, the enstrophy peaks, step times and the largest relative
    energy-budget residuals."""
    runs = []
    for path in (ref_path, f32_path, coarse_path):
        with open(path) as f:
            runs.append(json.load(f))
    ref, f32, coarse = runs
    commands = [f"python -u bench.py --tg-long {r['N']} {r['dtype']} {r['steps']} --tg-long-out {path}"
                for r, path in zip(runs, (ref_path, f32_path, coarse_path))]
    commands.append(f"python bench.py --summarize-tg-long {out_md} {ref_path} {f32_path} {coarse_path}")

    def at(r, t):
        n = int(round(t / r["dt"]))
        return r["energy"][n], r["enstrophy"][n]

    def peak(r):
        W = r["enstrophy"]
        i = max(range(len(W)), key=lambda k: W[k])
        return i * r["dt"], W[i]

    def name(r):
        return f"{r['N']}^3 {'FP64' if r['dtype'] == 'f64' else 'FP32'}"
    lines = ["# Taylor-Green vortex, Re = 1600, t = 0 -> 20 (20 000 RK4 steps, E and Omega every step)", "",
             "Commands (repository root, on the MI355X machine):", "", "```"] + commands + ["```", "",
             f"nu = {ref['nu']}, dt = {ref['dt']}, N/3 dealias, Taylor-Green initial field.", "",
             "| run | ms/step | E(t = 20) | enstrophy peak | at t | max relative budget residual |",
             "|---|---|---|---|---|---|"]
    for r in runs:
        tp, wp = peak(r)
        lines.append(f"| {name(r)} | {r['ms_per_step']:.3f} | {r['energy'][-1]:.9f} | {wp:.5f} | {tp:.3f} | "
                     f"{r['max_rel_budget_residual']:.2e} |")
    lines += ["", "Budget residual per step: |(E_{n+1} - E_n)/dt + nu (Omega_n + Omega_{n+1})| / "
              "(nu (Omega_n + Omega_{n+1})) (the semi-discrete system has dE/dt = -2 nu Omega).", "",
              f"| t | E ({name(ref)}) | Omega | 2 nu Omega | E rel. diff. {name(f32)} | E rel. diff. {name(coarse)} | "
              f"Omega rel. diff. {name(coarse)} |", "|---|---|---|---|---|---|---|"]
    for t in (0, 2, 4, 6, 8, 9, 10, 12, 16, 20):
        e, w = at(ref, t)
        e32, _ = at(f32, t)
        ec, wc = at(coarse, t)
        lines.append(f"| {t} | {e:.6f} | {w:.5f} | {2 * ref['nu'] * w:.6f} | {abs(e32 - e) / e:.1e} | "
                     f"{abs(ec - e) / e:.1e} | {abs(wc - w) / w:.1e} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=N_DEFAULT)
    ap.add_argument("--prof-steps", type=int, default=2)
    ap.add_argument("--error-step", type=int, default=ERROR_STEP,
                    help="step at which the errors against the oracle are stated (0: none)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-only", action="store_true")
    ap.add_argument("--no-isotropic", action="store_true", help="skip the 1024^3 random isotropic leg")
    ap.add_argument("--isotropic-only", action="store_true")
    ap.add_argument("--iso-steps", type=int, default=ISO_STEPS, help="timed steps of the 1024^3 leg")
    ap.add_argument("--no-fft", action="store_true", help="skip the FFT-only leg")
    ap.add_argument("--tg-long", nargs=3, metavar=("N", "DTYPE", "STEPS"),
                    help="only run the long Taylor-Green Re=1600 case (history to --tg-long-out)")
    ap.add_argument("--tg-long-out", default="tg_long.json")
    ap.add_argument("--fft-only", action="store_true")
    ap.add_argument("--ens-steps", type=int, default=100)
    ap.add_argument("--ens-per-sim-steps", type=int, default=20)
    ap.add_argument("--ens-default-tiles", action="store_true", help="ensemble without the tile autotuner")
    ap.add_argument("--sweep", action="store_true", help="only time every kernel variant at --N")
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="only time a copy of this many GiB (counter calibration)")
    ap.add_argument("--copy-row-bytes", type=int, default=0,
                    help="with --calibrate-copy: rows of this many bytes (0 = plain device copy)")
    ap.add_argument("--copy-pitch", type=int, default=0, help="with --copy-row-bytes: bytes from row to row")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("STATS_DIR", "OUT_MD", "COMMAND", "TITLE"),
                    help="write a kernel-trace summary from rocprofv3 --stats output")
    ap.add_argument("--summarize-counters", nargs=10,
                    metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR", "CAL_BYTES", "N", "OUT_JSON",
                             "OUT_MD", "COMMANDS_FILE", "TITLE"),
                    help="write an HBM-traffic summary from rocprofv3 FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--summarize-tg-long", nargs=4, metavar=("OUT_MD", "REF_JSON", "F32_JSON", "COARSE_JSON"),
                    help="write the table of three --tg-long runs (reference, FP32, coarser grid)")
    a = ap.parse_args(argv)
    if a.summarize_tg_long:
        return summarize_tg_long(*a.summarize_tg_long)
    if a.summarize_trace:
        d, out, cmd, title = a.summarize_trace
        return summarize_trace(d, out, cmd, title)
    if a.summarize_counters:
        fd, wd, cfd, cwd, cb, n, oj, om, cmds, title = a.summarize_counters
        with open(cmds) as f:
            commands = [ln.rstrip() for ln in f if ln.strip()]
        return summarize_counters(fd, wd, cfd, cwd, int(cb), int(n), oj, om, commands, title)
    if a.calibrate_copy > 0:
        return calibrate_copy(a.calibrate_copy, a.copy_row_bytes, a.copy_pitch)
    if a.sweep:
        for dt in ("f64", "f32"):
            sweep(a.N, dt)
        return 0
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(sharding the slab decomposition over several GPUs is designed, not built)", file=sys.stderr)
        return 2

    if a.tg_long:
        N, dtype, steps = int(a.tg_long[0]), a.tg_long[1], int(a.tg_long[2])
        print(json.dumps({"tg_long": run_tg_long(N, dtype, steps, a.tg_long_out)}), flush=True)
        return 0
    if a.fft_only:
        print(json.dumps({"fft": run_fft()}), flush=True)
        return 0
    if a.isotropic_only:
        print(json.dumps({"random_isotropic": run_isotropic(steps=a.iso_steps)}), flush=True)
        return 0
    if a.ensemble_only:
        ens = run_ensemble(a.ens_steps, a.warmup, a.ens_per_sim_steps, not a.ens_default_tiles)
        print(json.dumps({"ensemble": ens}), flush=True)
        return 0
    if a.no_fp64:
        f32 = run_gpu(a.N, "f32", a.steps, a.warmup, a.prof_steps, a.error_step)
        print(json.dumps({"fp32": f32, "N": a.N, "steps": a.steps}), flush=True)
        return 0
    clocks_before = gpu_clocks()
    f64 = run_gpu(a.N, "f64", a.steps, a.warmup, a.prof_steps, a.error_step)
    f32 = None if a.no_fp32 else run_gpu(a.N, "f32", a.steps, a.warmup, a.prof_steps, a.error_step)
    clocks_after = gpu_clocks()

    roof = None
    if f64["kernels_ms"]:
        dom = max(f64["kernels_ms"], key=f64["kernels_ms"].get)
        C = field_bytes(a.N, "f64")
        ach = f64["kernels_GBps"][dom]
        tr = measured_traffic(a.N, "f64", dom, f64["curl_in_y"])
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                "traffic": None if tr is None else round(tr / 1e9, 3), "traffic_unit": "GB per launch",
                "bytes_per_launch": fields_per_launch(a.N, f64["curl_in_y"])[dom] * C,
                "mean_launch_ms": f64["kernels_ms"][dom]}
    ens = None if a.no_ensemble else run_ensemble(a.ens_steps, a.warmup, a.ens_per_sim_steps, not a.ens_default_tiles)
    iso = None if a.no_isotropic else run_isotropic(steps=a.iso_steps)
    fft = None if a.no_fft else run_fft()
    cpu = None if a.no_cpu_baseline else cpu_baseline(a.N)
    line_clocks = {"before": clocks_before, "after": clocks_after}
    line = {
        "metric": METRIC, "value": round(f64["ms_per_step"], 4), "unit": "ms/step",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(f64["ms_per_step"], 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"taylor_green_{a.N}_rk4", "N": a.N, "nu": NU, "dt": DT,
                   "dealias": "2/3 rule, kmax = N/3", "parallelism": "single_gpu"},
        "model_GBps": round(f64["model_GBps"], 1),
        "model_frac_of_hbm_peak": round(f64["model_GBps"] / HBM_PEAK_GBPS, 4),
        "energy": f64["energy"], "enstrophy": f64["enstrophy"],
        "error_vs_oracle": f64["error_vs_oracle"],
        "kernels_ms": f64["kernels_ms"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "gpu_clocks": line_clocks,
    }
    if f32 is not None:
        line["fp32"] = {"ms_per_step": round(f32["ms_per_step"], 4), "model_GBps": round(f32["model_GBps"], 1),
                        "energy": f32["energy"], "enstrophy": f32["enstrophy"],
                        "rel_energy_diff_vs_fp64": abs(f32["energy"] - f64["energy"]) / f64["energy"],
                        "error_vs_oracle": f32["error_vs_oracle"],
                        "kernels_ms": f32["kernels_ms"]}
    if ens is not None:
        line["ensemble"] = ens
    if iso is not None:
        line["random_isotropic"] = iso
    if fft is not None:
        line["fft"] = fft
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
