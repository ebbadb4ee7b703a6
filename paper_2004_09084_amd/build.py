"""Builds libqcmet.so (HIP kernels + host runtime + C ABI) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqcmet.so")
SOURCES = ["kernels.hip", "layer_f32.hip", "layer_f16.hip", "layer_f8.hip", "lds_sweeps.hip", "nms.hip", "framegen.hip",
           "noalloc.hip", "api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str, obj: str):
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in (res.stderr or "").splitlines() if "packed-fp32-ops" not in l and l.strip()]
    return cmd, res.returncode, noise


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links."""
    import concurrent.futures as cf
    import tempfile
    tmpdir = tempfile.mkdtemp(prefix="qcmet_build_")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
    workers = max(1, min(len(srcs), os.cpu_count() or 1, 8))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_compile, srcs, objs))
    failed = False
    for cmd, rc, noise in results:
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0 or (verbose and noise):
            sys.stderr.write("\n".join(noise) + "\n")
        failed |= rc != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + f".tmp{os.getpid()}"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stderr or "")
        raise RuntimeError(f"link failed ({res.returncode})")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(tmpdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
