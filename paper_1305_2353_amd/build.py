"""Build libctp.so (the HIP library) in-tree with hipcc for gfx950.

    python -m paper_1305_2353_amd.build

Every source under csrc/ is compiled on each call (a few seconds each) and
linked into paper_1305_2353_amd/libctp.so; the roofline probes under probe/
go into paper_1305_2353_amd/libctp_probe.so.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libctp.so")
PROBE_SRC = os.path.join(HERE, "probe", "probe.hip")
PROBE_OUT = os.path.join(HERE, "libctp_probe.so")
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-result",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    shutil.move(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    build_probe(verbose)
    return OUT


def build_probe(verbose=False):
    """The roofline probes (measured peaks), a library of their own."""
    tmp = PROBE_OUT + ".tmp"
    cmd = [HIPCC, *FLAGS, "-shared", PROBE_SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {PROBE_SRC}:\n{res.stdout}\n{res.stderr}")
    shutil.move(tmp, PROBE_OUT)
    if verbose:
        print(f"built {PROBE_OUT}")
    return PROBE_OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
