"""Build libgm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2302_05176_amd.build

The library is written next to this file so that it travels with the source
tree; nothing is installed.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgm.so")
SOURCES = ["gm_api.hip", "gm_plain.hip", "gm_fastgm.hip", "gm_estimators.hip", "gm_rates.hip",
           "gm_lsh.hip", "gm_tune.cpp", "gm_serve.cpp"]
HEADERS = ["gm_common.h", "gm_draw.h"]
ARCH = os.environ.get("GM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    # The draw specification is a fixed sequence of IEEE operations: no
    # compiler-fused multiply-adds, no fast-math.
    "-ffp-contract=off", "-fno-fast-math",
    # Packed FP32 instructions are kept out of the generated code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def command(out: str = LIB) -> list[str]:
    return ([hipcc(), f"--offload-arch={ARCH}"] + FLAGS +
            ["-I", os.path.join(ROOT, "include"), "-I", CSRC] +
            [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out])


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "gm.h")]
    return all(os.path.getmtime(d) <= t for d in deps)


OBJDIR = os.path.join(ROOT, "_build")


def _compile(src: str, obj: str, verbose: bool):
    flags = [f for f in FLAGS if f != "-shared"]
    cmd = ([hipcc(), f"--offload-arch={ARCH}"] + flags +
           ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj])
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every HIP source into libgm.so (always when force=True): one
    hipcc per source in parallel, then one link."""
    if not force and up_to_date():
        return LIB
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    tag = "%d" % os.getpid()
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + "." + tag + ".o") for s in SOURCES]
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(SOURCES, objs)))
    for src, res in zip(SOURCES, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libgm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
