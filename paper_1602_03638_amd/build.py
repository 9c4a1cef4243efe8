"""Build libdns.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python -m paper_1602_03638_amd.build [--jobs J] [--debug]
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdns.so")
# (object name, source, extra defines): the C ABI, the size dispatch, and the
# kernels of each (precision, N) pair compiled from dns_inst.hip
SIZES = (8, 16, 32, 64, 128, 256, 512, 1024)
UNITS = [("dns_api", "dns_api.hip", []), ("dns_tables", "dns_tables.hip", [])] + [
    (f"dns_inst_{tag}_{n}", "dns_inst.hip", [f"-DDNS_INST_REAL={real}", f"-DDNS_INST_N={n}"])
    for n in reversed(SIZES) for tag, real in (("f64", "double"), ("f32", "float"))]
ARCH = "gfx950"


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def common_flags(debug=False):
    return [
        f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
        "-O1" if debug else "-O3",
        # packed FP32 instructions are disabled in all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # no multiply-add contraction: the same expression compiles to the same
        # rounding in every kernel that inlines it, so fused and unfused
        # schedules and all tile shapes give bitwise identical results
        "-ffp-contract=off",
        "-I", INCLUDE, "-I", CSRC,
        "-Wno-unused-result",
    ]


def compile_one(unit, debug):
    name, src, defines = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc()] + common_flags(debug) + defines + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {name} ({src}) failed:\n{res.stderr[-6000:]}")
    return obj


def default_jobs():
    return max(1, min(8, os.cpu_count() or 1))


def build(jobs=None, debug=False, verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs or default_jobs()) as ex:
        objs = list(ex.map(lambda u: compile_one(u, debug), UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libdns.so failed:\n{res.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args(argv)
    build(a.jobs, a.debug)


if __name__ == "__main__":
    sys.exit(main())
