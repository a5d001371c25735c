"""Build steps for the native parts, run in-tree.

* ``libefgen.so``  - seeded graph generators (g++, OpenMP)
* ``libef.so``     - the Expected Force library: HIP kernels for gfx950 plus the
                     C-ABI host code (hipcc)
* ``oracle/liboracle.so`` - the CPU oracle (gcc); built here only so that the
                     tests can load it, never called from the library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are kept out of every device build.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd, cwd=None):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return r


def build_gen():
    src = os.path.join(PKG, "gen", "gen.cpp")
    out = os.path.join(PKG, "gen", "libefgen.so")
    _run(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", src, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_oracle():
    """The CPU oracle (test infrastructure): every C source under oracle/."""
    d = os.path.join(ROOT, "oracle")
    srcs = sorted(os.path.join(d, f) for f in os.listdir(d) if f.endswith(".c"))
    out = os.path.join(d, "liboracle.so")
    _run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp"] + srcs + ["-lm",
          "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def lib_sources():
    d = os.path.join(PKG, "csrc")
    return sorted(os.path.join(d, f) for f in os.listdir(d)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def hip_runtime_dir():
    """Directory of the HIP runtime to link against. When PyTorch-ROCm is
    installed, its bundled libamdhip64.so is used, so that a Python process
    holds a single HIP runtime shared by torch (memory, streams) and this
    library; otherwise the ROCm installation's."""
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec and spec.submodule_search_locations:
        d = os.path.join(spec.submodule_search_locations[0], "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    return os.path.join(ROCM, "lib")


def build_lib(jobs=None):
    """Compiles every source of the library to an object (in parallel, in
    _build/), then links libef.so."""
    from concurrent.futures import ThreadPoolExecutor

    out = os.path.join(PKG, "libef.so")
    srcs = lib_sources()
    if not srcs:
        return None
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    obj_dir = os.path.join(ROOT, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    cflags = [f for f in HIP_FLAGS if f != "-shared"]
    objs = [os.path.join(obj_dir, os.path.basename(s) + ".o") for s in srcs]
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, [HIPCC] + cflags + inc + ["-c", s, "-o", o])
                  for s, o in zip(srcs, objs)]:
            f.result()
    rt = hip_runtime_dir()
    link = ["-no-hip-rt", "-L", rt, "-l:libamdhip64.so", f"-Wl,-rpath,{rt}",
            f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + link
         + ["-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_all():
    build_gen()
    build_oracle()
    build_lib()


if __name__ == "__main__":
    build_all()
    print("built")
