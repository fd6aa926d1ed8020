"""Build step of the HIP library: compiles csrc/ for gfx950 into libka.so
inside the package directory (in-tree, so the built object travels with the
source tree)."""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libka.so")
ARCH = os.environ.get("KA_OFFLOAD_ARCH", "gfx950")

SOURCES = ["host_setup.cpp", "gamma.hip", "transfer.hip", "dense64.hip", "sym.hip", "nonsym.hip", "api.hip", "eigs.hip", "serve.hip", "sample.hip", "capi.hip", "gamma_static.hip"]

HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             # no packed FP32 instructions in any generated code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if src.endswith(".cpp"):
        cmd = ["hipcc", "-O3", "-fPIC", "-std=c++17", "-c", path, "-o", obj]
    else:
        cmd = ["hipcc", "-x", "hip"] + HIP_FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    lines = [l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l and l.strip()]
    return src, r.returncode, "\n".join(lines), obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    errors = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        for src, rc, err, obj in ex.map(_compile, SOURCES):
            if rc != 0:
                errors.append(f"--- {src}\n{err}")
            elif verbose and err:
                print(f"--- {src}\n{err}", file=sys.stderr)
            objs.append(obj)
    if errors:
        raise RuntimeError("HIP build failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
