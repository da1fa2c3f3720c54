"""Build libsgpe.so (HIP kernels for gfx950 + host C ABI) in-tree.

    python -m paper_2010_15069_amd.build

The library is linked against the same HIP runtime that PyTorch loads (its bundled
libamdhip64, SONAME libamdhip64.so.7) so that one process never holds two HIP runtimes; the
RUNPATH lists PyTorch's library directory first and /opt/rocm/lib second.
"""
from __future__ import annotations

import hashlib
import importlib.util
import os
import shutil
import subprocess
import sys
import tempfile

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
INCLUDE = os.path.join(REPO, "include")
LIB_NAME = "libsgpe.so"
LIB_PATH = os.path.join(PKG_DIR, LIB_NAME)

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# Packed fp32 instructions are disabled for all device code (see the kernels' header comments).
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")]


def source_hash() -> str:
    """Short hash of the native sources (kernels, host library, public header)."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".cpp")))
    for f in files:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(INCLUDE, "sgpe.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


# The sources the step kernels compile from (with the device compile flags): a record measured on
# these kernels stays valid while this hash is unchanged, whatever happens to the host library.
KERNEL_SOURCES = ("row_pass.hip", "col_pass.hip", "row_body.hpp", "col_body.hpp", "fft_device.hpp",
                  "sgpe_internal.hpp")


def kernel_hash() -> str:
    """Short hash of the step kernels' sources and device compile flags."""
    h = hashlib.sha256(" ".join(HIP_FLAGS).encode())
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _torch_lib_dir():
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return None
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None


def _run(cmd, cwd=None):
    proc = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host compilation pass does not know the packed-fp32 target feature; that note is noise
    out = "\n".join(l for l in proc.stdout.splitlines() if "packed-fp32-ops" not in l)
    if proc.returncode != 0:
        raise RuntimeError(f"command failed ({proc.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clangxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    torch_lib = _torch_lib_dir()
    hip_lib_dir = torch_lib or os.path.join(ROCM, "lib")
    hip_lib = os.path.join(hip_lib_dir, "libamdhip64.so")
    rpath = [d for d in (torch_lib, os.path.join(ROCM, "lib")) if d]
    incs = ["-I", INCLUDE, "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="sgpe_build_") as tmp:
        objs = []
        jobs = []
        # every HIP source (kernels, and host code that must share a translation unit with them)
        # and every host-only C++ source of csrc/; the largest first, so that it starts first
        hip_srcs = sorted((f for f in os.listdir(CSRC) if f.endswith(".hip")),
                          key=lambda f: -os.path.getsize(os.path.join(CSRC, f)))
        cpp_srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
        for src in hip_srcs:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            jobs.append(([hipcc, "-c"] + HIP_FLAGS + incs + [os.path.join(CSRC, src), "-o", obj], obj))
        for src in cpp_srcs:
            obj = os.path.join(tmp, src.replace(".cpp", ".o"))
            jobs.append(([hipcc, "-c", "-x", "c++"] + HOST_FLAGS + incs +
                         [os.path.join(CSRC, src), "-o", obj], obj))
        procs = []
        for cmd, name in jobs:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True),
                          cmd, name))
        for p, cmd, name in procs:
            out, _ = p.communicate()
            out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
            if p.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
            if verbose and out.strip():
                print(out)
            objs.append(name)
        link = [clangxx, "-shared", "-fPIC"] + objs + [hip_lib] + \
            [f"-Wl,-rpath,{d}" for d in rpath] + ["-o", os.path.join(tmp, LIB_NAME)]
        if verbose:
            print(" ".join(link), flush=True)
        _run(link)
        tmp_out = LIB_PATH + ".tmp"
        shutil.copyfile(os.path.join(tmp, LIB_NAME), tmp_out)
        os.replace(tmp_out, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
