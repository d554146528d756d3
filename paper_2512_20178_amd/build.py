"""Build libshiro.so (gfx950 HIP kernels + C ABI) in-tree with hipcc.

    python -m paper_2512_20178_amd.build

Every .hip file under csrc/ is compiled in parallel and linked into
paper_2512_20178_amd/libshiro.so.  Objects go to paper_2512_20178_amd/_build/.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libshiro.so")
OBJ = os.path.join(PKG, "_build")
ARCH = os.environ.get("SHIRO_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-fvisibility=hidden",
    # keep the compiler from forming packed-FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def source_hash() -> str:
    """sha256 (16 hex digits) of every source the library is built from: the
    HIP files, their headers and the C ABI header, in a fixed order."""
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp")))
    files.append(os.path.join(PKG, "..", "include", "shiro.h"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _buildinfo(digest: str) -> str:
    """A one-function object that stamps the source hash into the library."""
    src = os.path.join(OBJ, "buildinfo.cpp")
    with open(src, "w") as f:
        f.write('extern "C" __attribute__((visibility("default"))) const char* shiro_build_hash(void) {\n'
                f'  return "{digest}";\n}}\n')
    obj = src + ".o"
    r = subprocess.run([HIPCC, "-O2", "-fPIC", "-c", src, "-o", obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling the build stamp failed:\n{r.stderr}")
    return obj


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _stale(src: str, headers) -> bool:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *headers])


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source (or, with incremental, those newer than their
    object or than any header) and link libshiro.so."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    headers = sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + [os.path.join(PKG, "..", "include", "shiro.h")]
    todo = [f for f in srcs if not incremental or _stale(f, headers)]
    jobs = min(max(len(todo), 1), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(OBJ, os.path.basename(f) + ".o") for f in srcs]
    objs.append(_buildinfo(source_hash()))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
