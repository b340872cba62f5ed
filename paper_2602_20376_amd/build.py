"""Builds liblrqo.so (all HIP sources, gfx950) in the package directory.

    python -m paper_2602_20376_amd.build [--jobs N] [--sanitize]

Each source is compiled to an object under _build/ in parallel, then linked.
Packed FP32 instructions are disabled for every device compilation
(-target-feature -packed-fp32-ops).

--sanitize builds a second copy, _build_san/liblrqo.so, whose host code is
instrumented with AddressSanitizer and UndefinedBehaviorSanitizer (every
sanitizer flag goes to the host pass only; device code is unchanged).  It is
for host-side checks on the CPU, with the clang ASan runtime preloaded.
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liblrqo.so")
BUILD_SAN = os.path.join(ROOT, "_build_san")
LIB_SAN = os.path.join(BUILD_SAN, "liblrqo.so")
SOURCES = ["lrqo_runtime.hip", "select.hip", "sampled.hip", "sampled_probe.hip", "api_sampled.hip", "exact.hip",
           "batched.hip", "proposal.hip", "graph.hip", "sort.hip", "rank1.hip", "lanczos.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # MFMA accumulators in ordinary VGPRs: in-place accumulation, no
          # accumulator-register copies inside the scoring loops
          "-mllvm", "-amdgpu-mfma-vgpr-form",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
          "-I", os.path.join(ROOT, "include")]


# host pass only: -Xarch_host before every flag
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """The clang ASan runtime that a sanitized build expects to be preloaded."""
    out = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    if out and os.path.exists(out):
        return out
    base = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "llvm", "lib", "clang")
    for root, _dirs, files in os.walk(base):
        if "libclang_rt.asan-x86_64.so" in files:
            return os.path.join(root, "libclang_rt.asan-x86_64.so")
    raise RuntimeError("clang ASan runtime not found")


def compile_one(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, *(SANITIZE if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 8, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    os.makedirs(BUILD_SAN if sanitize else BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda src: compile_one(src, sanitize), SOURCES))
    tmp = out + f".tmp{os.getpid()}"
    link_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-shared-libsan"] if sanitize else []
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *link_san, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--sanitize", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.sanitize))
