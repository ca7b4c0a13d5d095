"""Build libhankel.so for gfx950 with hipcc (in-tree, no JIT cache).

python -m paper_1810_01478_amd.build [--jobs N]
"""
import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhankel.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["k_factor.hip", "k_upd_valu.hip", "k_upd_mfma.hip", "k_kara.hip", "k_upd_toep.hip", "k_solve.hip", "k_eig.hip", "k_adjoint.hip",
           "hl_noalloc.hip",
           "hl_api.cpp", "hl_batch.cpp"]

# packed-fp32 instructions are kept off in every device compilation
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-I" + os.path.join(HERE, "..", "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + (DEVICE_FLAGS if src.endswith(".hip") else []) + \
        ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    return src, obj, r.returncode, out


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(8, os.cpu_count() or 1)
    objs = []
    with ThreadPoolExecutor(jobs) as ex:
        for src, obj, rc, out in ex.map(_compile, srcs):
            if rc != 0:
                raise RuntimeError("hipcc failed on %s:\n%s" % (src, out))
            if verbose and out.strip():
                print(out)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out_dir, driver_src, jobs=None):
    """The library's sources and a host driver built with AddressSanitizer and
    UBSan on the host code only (the device code is compiled as usual), linked
    into one executable in out_dir; returns its path.  For host-side checks on
    a machine without a GPU."""
    os.makedirs(out_dir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = ["--offload-arch=" + ARCH, "-O1", "-g", "-std=c++17", "-fPIC", "-I" + os.path.join(HERE, "..", "include")]

    def one(src):
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + flags + (DEVICE_FLAGS if src.endswith(".hip") else []) + san + \
            ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r.returncode, r.stderr

    objs = []
    with ThreadPoolExecutor(jobs or min(8, os.cpu_count() or 1)) as ex:
        for src, obj, rc, err in ex.map(one, srcs):
            if rc != 0:
                raise RuntimeError("hipcc (sanitized host) failed on %s:\n%s" % (src, err))
            objs.append(obj)
    clangxx = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/llvm/bin/clang++"
    drv_obj = os.path.join(out_dir, "driver.o")
    exe = os.path.join(out_dir, "driver")
    for cmd in ([clangxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                 "-I" + os.path.join(HERE, "..", "include"), "-c", driver_src, "-o", drv_obj],
                [clangxx, "-fsanitize=address,undefined", drv_obj] + objs +
                ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("sanitized driver build failed:\n" + r.stdout + r.stderr)
    return exe


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.v))
