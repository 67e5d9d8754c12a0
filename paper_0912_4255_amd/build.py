"""Build librsfstat.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_0912_4255_amd.build [--jobs N] [--sanitize]

--sanitize builds a second copy, _build/san/librsfstat.so, whose host code
(argument checks, planning, launch set-up) carries AddressSanitizer and
UndefinedBehaviorSanitizer; device code is built as usual.  It is loaded
with the clang ASan runtime preloaded (see san_runtime()).
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librsfstat.so")

SOURCES = ["rsf_abi.cpp", "rsf_rtc.cpp", "rsf_resample.hip", "rsf_fft.hip", "rsf_point.hip", "rsf_topk.hip", "rsf_sft.hip",
           "rsf_semico.hip", "rsf_hetdec.hip"]
# the headers a first-pass row plan compiled at run time is built from (their
# hash is recorded in the library, which compiles only from matching ones)
ROW_HEADERS = ["rsf_pass_a.h", "rsf_device.h", "rsf_spill.h", "rsf_params.h"]

ARCH = os.environ.get("RSF_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def row_src_hash():
    """FNV-1a (64 bit) over the run-time row-plan headers, in ROW_HEADERS order."""
    h = 1469598103934665603
    for name in ROW_HEADERS:
        with open(os.path.join(CSRC, name), "rb") as f:
            for b in f.read():
                h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


# host-only sanitizers: every -fsanitize= sits right after -Xarch_host
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]
SAN_BUILD = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_BUILD, "librsfstat.so")


def san_runtime():
    """Path of the clang ASan runtime matching hipcc's host compiler (it also
    carries the UBSan handlers), or None."""
    import glob
    for pat in ("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so",
                "/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"):
        hits = sorted(glob.glob(pat))
        if hits:
            return hits[-1]
    return None


def _compile(src, sanitize=False):
    out = SAN_BUILD if sanitize else BUILD
    obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
    defs = [f"-DRSF_ROW_SRC_HASH={row_src_hash():#x}ull", f'-DRSF_OFFLOAD_ARCH="{ARCH}"']
    cmd = [hipcc(), *FLAGS, *defs, *(SAN_FLAGS if sanitize else []), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs=None, verbose=False, sanitize=False):
    out = SAN_BUILD if sanitize else BUILD
    lib = SAN_LIB if sanitize else LIB
    os.makedirs(out, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), srcs))
    tmp = lib + ".tmp"
    # the sanitized library leaves the runtime's symbols to the preloaded ASan runtime
    link_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-shared-libsan"] if sanitize else []
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_san, *objs, "-lhiprtc", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--sanitize", action="store_true", help="host ASan + UBSan copy under _build/san/")
    a = ap.parse_args(argv)
    build(a.jobs, verbose=True, sanitize=a.sanitize)


if __name__ == "__main__":
    sys.exit(main())
