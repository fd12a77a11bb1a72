"""Builds the HIP library ``_lib/liblsh.so`` for gfx950 with hipcc.

Translation units compile in parallel (one hipcc per unit), then link into one
shared library.  ``python -m paper_1411_0330_amd.build`` rebuilds it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "liblsh.so")
OBJDIR = os.path.join(ROOT, "_build", "obj")

ARCH = "gfx950"
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
         # keep packed FP32 instructions out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", CSRC, "-I", INCLUDE]

# roctx ranges (rocprofiler-sdk) for profiler timelines
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]

UNITS = [
    ("k_x.hip", "k_x_f32.o", ["-DLSH_X_TYPE=float", "-DLSH_X_PART=0"]),
    ("k_x.hip", "k_x_f64.o", ["-DLSH_X_TYPE=double", "-DLSH_X_PART=0"]),
    ("k_x.hip", "k_xi2_f32.o", ["-DLSH_X_TYPE=float", "-DLSH_X_PART=2"]),
    ("k_x.hip", "k_xi2_f64.o", ["-DLSH_X_TYPE=double", "-DLSH_X_PART=2"]),
    ("k_x.hip", "k_xi3_f32.o", ["-DLSH_X_TYPE=float", "-DLSH_X_PART=3"]),
    ("k_x.hip", "k_xi3_f64.o", ["-DLSH_X_TYPE=double", "-DLSH_X_PART=3"]),
    ("k_x.hip", "k_xi6_f32.o", ["-DLSH_X_TYPE=float", "-DLSH_X_PART=6"]),
    ("k_x.hip", "k_xi6_f64.o", ["-DLSH_X_TYPE=double", "-DLSH_X_PART=6"]),
    ("k_xc.hip", "k_xc_f32.o", ["-DLSH_XC_TYPE=float"]),
    ("k_xc.hip", "k_xc_f64.o", ["-DLSH_XC_TYPE=double"]),
    ("k_y.hip", "k_y_f32.o", ["-DLSH_Y_TYPE=float"]),
    ("k_y.hip", "k_y_f64.o", ["-DLSH_Y_TYPE=double"]),
    ("k_z.hip", "k_z_f32.o", ["-DLSH_Z_TYPE=float"]),
    ("k_z.hip", "k_z_f64.o", ["-DLSH_Z_TYPE=double"]),
    ("k_z.hip", "k_zs_f32.o", ["-DLSH_Z_TYPE=float", "-DLSH_Z_STORED"]),
    ("k_z.hip", "k_zs_f64.o", ["-DLSH_Z_TYPE=double", "-DLSH_Z_STORED"]),
    ("k_tiny.hip", "k_tiny_f32.o", ["-DLSH_TINY_TYPE=float"]),
    ("k_tiny.hip", "k_tiny_f64.o", ["-DLSH_TINY_TYPE=double"]),
    ("runtime.hip", "runtime.o", []),
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(unit):
    src, obj, extra = unit
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", os.path.join(OBJDIR, obj)]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {extra}:\n{proc.stderr[-6000:]}")
    return obj


def build(verbose: bool = True, jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_consts.py")], check=True)
    jobs = jobs or min(len(UNITS), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, u) for u in UNITS]
        for f in cf.as_completed(futs):
            obj = f.result()
            if verbose:
                print(f"[build] compiled {obj}", flush=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC",
           *[os.path.join(OBJDIR, u[1]) for u in UNITS], *LINK, "-o", tmp]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"link failed:\n{proc.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] wrote {LIB}", flush=True)
    return LIB


SAN_DIR = os.path.join(ROOT, "_build", "hostsan")


def sanitizer_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime (preloaded into the
    process that loads the host-sanitizer build)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = shutil.which("amdclang") or "/opt/rocm/llvm/bin/clang"
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return out.stdout.strip()


def build_host_sanitized() -> str:
    """Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the
    library: runtime.hip (every host line of the C ABI, the solvers' control
    flow, the scheduler) compiled with both sanitizers on its host pass only,
    linked with the device units of the last build().  Device code is
    unchanged (GPU sanitizers are not used).  Returns the library path."""
    objs = [os.path.join(OBJDIR, u[1]) for u in UNITS if u[0] != "runtime.hip"]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"device units not built (run build() first): {missing[:3]}")
    os.makedirs(SAN_DIR, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    obj = os.path.join(SAN_DIR, "runtime_san.o")
    flags = [f if f != "-O3" else "-O1" for f in FLAGS]
    proc = subprocess.run([hipcc(), *flags, *san, "-c", os.path.join(CSRC, "runtime.hip"), "-o", obj],
                          capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"sanitized compile failed:\n{proc.stderr[-4000:]}")
    lib = os.path.join(SAN_DIR, "liblsh_hostsan.so")
    proc = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *san[:4], "-shared-libsan",
                           *objs, obj, *LINK, "-o", lib], capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{proc.stderr[-4000:]}")
    return lib


if __name__ == "__main__":
    build()
