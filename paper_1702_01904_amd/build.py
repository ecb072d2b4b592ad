"""Compile libprism.so (HIP kernels for gfx950 + host plan) in-tree.

Usage: ``python -m paper_1702_01904_amd.build`` or ``build()`` from Python.
Objects go to ``_build/`` at the repository root; the shared library is
written next to this file, where the binding loads it from.

``build_sanitized()`` links the same device objects with the host sources
(plan, serving layer) built with AddressSanitizer and UndefinedBehavior-
Sanitizer into ``_build/san/libprism_san.so``, for the CPU-side ABI tests
(run with the ASan runtime preloaded and PRISM_LIBRARY naming that file).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libprism.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INC}", f"-I{SRC}", "-Wall", "-Wno-unused-function"]
# device code: gfx950 only, packed FP32 instructions disabled; the sign of
# zero carries no meaning in these kernels, so x + 0 may fold (pruned FFTs)
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-signed-zeros"]

SOURCES = ["slice_kernels.hip", "probe_kernels.hip", "probe16_kernels.hip", "scratch.hip",
           "plan.cpp", "server.cpp"]


def _cmd(src, obj):
    if src.endswith(".hip"):
        return [HIPCC, "-x", "hip", *DEVICE, *COMMON, "-c", os.path.join(SRC, src), "-o", obj]
    # host-only C++ against the HIP runtime API (no device code in these files)
    return [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON, "-c",
            os.path.join(SRC, src), "-o", obj]


HOST_SOURCES = ["plan.cpp", "server.cpp"]
SAN_DIR = os.path.join(OUT_DIR, "san")
SAN_LIB = os.path.join(SAN_DIR, "libprism_san.so")
# host code only: each sanitizer flag applies to the host compilation
SAN_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime():
    """Path of the ASan runtime of the HIP toolchain (to preload), or None."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_sanitized(verbose=False):
    """Host sources with ASan + UBSan, linked with the device objects of
    build() (run build() first). Returns the library path."""
    os.makedirs(SAN_DIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        if src in HOST_SOURCES:
            obj = os.path.join(SAN_DIR, os.path.splitext(src)[0] + ".o")
            cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-std=c++17",
                   "-fPIC", f"-I{INC}", f"-I{SRC}", *SAN_FLAGS, "-c", os.path.join(SRC, src),
                   "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
            if res.returncode != 0:
                raise RuntimeError(f"sanitized build of {src} failed:\n" +
                                   res.stdout.decode(errors="replace"))
        else:
            obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
            if not os.path.exists(obj):
                raise RuntimeError(f"{obj} missing: run build() first")
        objs.append(obj)
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", SAN_LIB, *objs]
    res = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if res.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + res.stdout.decode(errors="replace"))
    return SAN_LIB


def build(verbose=False):
    """Compile every source (always) and link libprism.so; raises on failure."""
    os.makedirs(OUT_DIR, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = _cmd(src, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errors = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        if pr.returncode != 0:
            errors.append(f"--- {src} ---\n{text}")
        elif verbose and text.strip():
            print(text)
    if errors:
        raise RuntimeError("libprism build failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if res.returncode != 0:
        raise RuntimeError("libprism link failed:\n" + res.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
