"""Build libkgrape.so (HIP for gfx950) in-tree.

    python -m paper_2010_03598_amd.build

compiles csrc/*.hip and csrc/*.cpp with hipcc into paper_2010_03598_amd/libkgrape.so.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libkgrape.so")

ARCH = os.environ.get("KG_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # packed FP32 instructions stay off: hipcc would otherwise form them from float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP toolchain (ROCm) is required to build libkgrape")
    return path


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the sanitizer
# build: every flag applies to the host compilation only (device code is built
# as usual); a UB finding aborts like an address error.
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address",
                  "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined"]
SANITIZED_LIB = os.path.join(PKG, "_build", "asan", "libkgrape.so")


def build(verbose: bool = False, sanitized: bool = False) -> str:
    """Compile every source for gfx950 and link libkgrape.so; returns its path.
    With `sanitized`, the host code is instrumented (SANITIZE_FLAGS) and the
    library goes to SANITIZED_LIB; it needs the clang AddressSanitizer runtime
    preloaded (asan_runtime())."""
    objs = []
    procs = []
    objdir = os.path.join(PKG, "_build", "asan" if sanitized else "")
    os.makedirs(objdir, exist_ok=True)
    flags = HIP_FLAGS + (SANITIZE_FLAGS if sanitized else [])
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc(), *flags, f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{text}")
        if verbose and text.strip():
            print(text)
    lib = SANITIZED_LIB if sanitized else LIB
    tmp = lib + ".tmp"
    link_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-shared-libasan"] if sanitized else []
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_san, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, lib)
    return lib


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that a process loading the sanitizer
    build must preload."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = found[0] if found else ""
    if not path:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitized="--sanitized" in sys.argv))
