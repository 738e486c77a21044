"""Build the gfx950 shared library libdmdmi.so in-tree with hipcc.

Every HIP source is compiled for gfx950 only (no other targets, no host
fallback) and linked into one C-ABI library next to this file.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libdmdmi.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["gemm.hip", "recon.hip", "small.hip", "eig.hip", "adjoint.hip", "edit.hip", "rollout.hip", "upsample.hip",
           "optdmd.hip", "modelio.hip", "api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # packed FP32 instructions are disabled for every kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{INCLUDE}", f"-I{CSRC}", "-Wno-unused-result",
    ]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
    cmd = [hipcc(), *_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 6) -> str:
    """Compile every source for gfx950 and link libdmdmi.so; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


# A build of the same sources whose host code carries AddressSanitizer and
# UndefinedBehaviorSanitizer (each sanitizer flag applies to the host pass only), for the
# ABI's argument checks, carving and host orchestration run on the CPU.  It is rebuilt only
# when a source or header is newer than the library.
SAN_DIR = os.path.join(OBJDIR, "san")
SAN_OUT = os.path.join(SAN_DIR, "libdmdmi_san.so")
_SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_sanitized(verbose: bool = False, jobs: int = 6) -> str:
    """Compile every source with ASan + UBSan on the host pass into a separate library; returns its path."""
    os.makedirs(SAN_DIR, exist_ok=True)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    if os.path.exists(SAN_OUT) and os.path.getmtime(SAN_OUT) > max(os.path.getmtime(d) for d in deps):
        return SAN_OUT

    def one(src: str) -> str:
        obj = os.path.join(SAN_DIR, src.replace(".hip", ".o"))
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
               *_SAN_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-Wno-unused-result", "-c", os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized host compile failed on {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = SAN_OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *_SAN_FLAGS, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_OUT)
    return SAN_OUT


def asan_runtime() -> str:
    """Path of the compiler's shared ASan runtime (preloaded into a Python that loads SAN_OUT)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/lib/llvm/bin/clang"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("ASan runtime not found")
    return path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
