"""Build libwsfft.so (HIP, gfx950) in-tree.

    python -m paper_2209_15040_amd.build [--incremental] [--jobs N]

Every ``csrc/*.hip`` translation unit is compiled with hipcc for gfx950 into
``_build/`` and linked into ``libwsfft.so`` next to this file.  Without
``--incremental`` every unit is recompiled.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwsfft.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CXXFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]


def _headers_mtime() -> float:
    hs = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(CSRC, "*.inc"))
    hs += glob.glob(os.path.join(ROOT, "include", "*.h"))
    return max(os.path.getmtime(h) for h in hs)


# Per-file additions.  persist.hip: its single-lane ticket atomics are claimed
# one tile ahead; the wave-reduction rewrite of uniform atomics would wait for
# each result at once and undo that.
EXTRA_FLAGS = {
    "persist.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"],
}


def _compile(src: str, incremental: bool, hdr_mtime: float) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t >= os.path.getmtime(src) and t >= hdr_mtime:
            return obj
    cmd = [HIPCC, *CXXFLAGS, *EXTRA_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so
    noise = ("packed-fp32-ops", "is not a recognized feature for this target", "(ignoring feature)")
    err = "\n".join(l for l in r.stderr.splitlines() if not any(n in l for n in noise))
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    os.replace(obj + ".tmp", obj)
    return obj


def build(incremental: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    hdr = _headers_mtime()
    jobs = jobs or min(16, max(1, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental, hdr), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


# Host-side sanitizer build for the CPU tests of the C-ABI: the units with host
# logic (argument checks, plans, schedules, the batch and pointwise entry
# points) recompiled with AddressSanitizer and UndefinedBehaviorSanitizer on
# their host code only, linked with the kernel units of the regular build.
# Run its users with the ASan runtime preloaded (asan_runtime()).
SANITIZED_UNITS = ["wsfft_api.hip", "persist.hip", "pointwise.hip"]
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SANITIZED_LIB = os.path.join(BUILD, "libwsfft_hostsan.so")


def asan_runtime() -> str:
    pat = os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "llvm", "lib", "clang", "*", "lib", "linux",
                       "libclang_rt.asan-x86_64.so")
    found = sorted(glob.glob(pat))
    return found[-1] if found else ""


def build_host_sanitized() -> str:
    """Builds SANITIZED_LIB from the kernel objects of a previous build; returns
    its path, or "" when those objects are missing."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = []
    for src in srcs:
        name = os.path.basename(src)
        if name in SANITIZED_UNITS:
            obj = os.path.join(BUILD, name + ".hostsan.o")
            cmd = [HIPCC, *CXXFLAGS, *EXTRA_FLAGS.get(name, []), *HOST_SANITIZE, "-g", "-c", src, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
            objs.append(obj)
        else:
            obj = os.path.join(BUILD, name + ".o")
            if not os.path.exists(obj):
                return ""
            objs.append(obj)
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *HOST_SANITIZE, "-shared-libsan",
           "-o", SANITIZED_LIB + ".tmp", *objs]
    subprocess.check_call(cmd)
    os.replace(SANITIZED_LIB + ".tmp", SANITIZED_LIB)
    return SANITIZED_LIB


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--host-sanitized", action="store_true",
                    help="also build the host-sanitized library for the CPU tests")
    a = ap.parse_args()
    print(build(a.incremental, a.jobs))
    if a.host_sanitized:
        print(build_host_sanitized())


if __name__ == "__main__":
    main()
