"""Build the native libraries in-tree.

libggen.so  input generators (gcc, host only)
libgg.so    the traversal library: HIP kernels for gfx950 + C ABI (hipcc)
"""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
ARCH = os.environ.get("GG_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed fp32 instructions stay off in every HIP build of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    noise = "is not a recognized feature for this target"
    text = "\n".join(l for l in r.stdout.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{text}")
    return text


def build_gen() -> str:
    src = os.path.join(PKG, "gen", "ggen.c")
    out = os.path.join(PKG, "gen", "libggen.so")
    _run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread", src,
          "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def hip_sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build_gg() -> str:
    out = os.path.join(PKG, "libgg.so")
    srcs = hip_sources()
    if not srcs:
        raise RuntimeError("no HIP sources found")
    _run(["hipcc", *HIP_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", *srcs, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_all() -> list[str]:
    return [build_gen(), build_gg()]


if __name__ == "__main__":
    for p in build_all():
        print(p)
