"""Build libidg.so in-tree: HIP kernels and C ABI for gfx950, planner with g++.

    python -m paper_1909_07226_amd.build [--sanitize]

Compiles every time it is called.  Packed FP32 instructions are disabled for
all device code (``-Xclang -target-feature -Xclang -packed-fp32-ops``).  The
planner is compiled without floating-point contraction so that its integer
output is decided by exactly the float64 operations its rule states.

``--sanitize`` builds ``_build_san/libidg_san.so`` instead: the host code of
the planner, the taper and the C ABI (argument checks, plans, scratch and
work-list set-up) under AddressSanitizer and UndefinedBehaviorSanitizer with
clang; the kernel objects (device code and their launchers) are those of the
last plain build.  It serves host tests that make no device call; the
library is loaded with clang's ASan runtime preloaded and ``IDG_LIBRARY``
pointing at it (``sanitizer_env()``).
"""

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libidg.so")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"build step failed ({res.returncode}): {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return res


BUILD_SAN = os.path.join(PKG, "_build_san")
LIB_SAN = os.path.join(BUILD_SAN, "libidg_san.so")
# host code only: every sanitizer flag on a hipcc line goes after -Xarch_host
SAN_HOST = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def _clang():
    for cand in (os.environ.get("IDG_CLANGXX"), "/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("clang++ not found (the sanitizer build needs ROCm's clang)")


def asan_runtime():
    """Path of clang's shared AddressSanitizer runtime (preloaded by sanitizer_env())."""
    res = subprocess.run([_clang(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang's shared ASan runtime was not found")
    return path


def sanitizer_env(base=None):
    """Environment for a process that loads libidg_san.so."""
    env = dict(os.environ if base is None else base)
    env["LD_PRELOAD"] = asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["IDG_LIBRARY"] = LIB_SAN
    return env


def build_sanitized(verbose=False):
    """Host code under ASan + UBSan, device code left out (see the module docstring)."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc, clang = _hipcc(), _clang()
    os.makedirs(BUILD_SAN, exist_ok=True)
    xhost = [f for flag in SAN_HOST for f in ("-Xarch_host", flag)]
    hip_flags = [f for f in HIP_FLAGS if f != "-O3"] + ["-O1", "--offload-host-only"] + xhost
    host_flags = [f for f in CXX_FLAGS if f != "-O2"] + ["-O1"] + SAN_HOST
    kernel_objs = [os.path.join(BUILD, src.replace(".", "_") + ".o") for src in ("kernels.hip", "image.hip", "calib.hip")]
    missing = [o for o in kernel_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"sanitizer build: run the plain build first ({', '.join(missing)} missing)")
    api = os.path.join(BUILD_SAN, "api_cpp.o")
    jobs = [([hipcc, "-x", "hip", *hip_flags, "-c", os.path.join(CSRC, "api.cpp"), "-o", api], api)]
    for src in ("plan.cpp", "taper.cpp"):
        obj = os.path.join(BUILD_SAN, src.replace(".", "_") + ".o")
        jobs.append(([clang, *host_flags, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda j: _run(j[0], verbose), jobs))
    tmp = LIB_SAN + ".tmp"
    # the sanitizer runtime is not linked into the library: the loading process preloads it
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *kernel_objs, *[j[1] for j in jobs], "-o", tmp],
         verbose)
    os.replace(tmp, LIB_SAN)
    return LIB_SAN


def build(verbose=False):
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, lang in (("kernels.hip", "hip"), ("image.hip", "hip"), ("calib.hip", "hip"), ("api.cpp", "hip")):
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        _run([hipcc, "-x", lang, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in ("plan.cpp", "taper.cpp"):
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        _run([os.environ.get("CXX", "g++"), *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-q" not in sys.argv))
    else:
        print(build(verbose="-q" not in sys.argv))
