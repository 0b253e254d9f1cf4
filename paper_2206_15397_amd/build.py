"""Build libkfac.so (HIP, gfx950) in-tree with hipcc.

Every .hip source under csrc/ is compiled for gfx950 only and linked into one shared
library next to this file.  Packed fp32 VALU instructions are disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkfac.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-source code-generation options.  The bf16 kernels keep their MFMA accumulators in
# ordinary VGPRs: the EA tile kernel's two register stages and its accumulators then fit
# one register file without copies between VGPRs and AGPRs.
FILE_FLAGS = {"kernels_bf16.hip": ["-mllvm", "--amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def source_hash() -> str:
    """Hash of every device/host source and header the library is built from, and the
    build flags: names the exact kernels a stored measurement was taken on."""
    import hashlib
    h = hashlib.sha256()
    inc = os.path.join(ROOT, "include")
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    files += sorted(os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join([ARCH, "-O3"] + DEVICE_FLAGS).encode())
    for k in sorted(FILE_FLAGS):
        h.update((k + " " + " ".join(FILE_FLAGS[k])).encode())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              "-I", os.path.join(ROOT, "include"), "-Wno-unused-result",
              f'-DKFAC_SRC_HASH="{source_hash()}"'] + DEVICE_FLAGS
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = common + FILE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            for _, p in procs:
                p.wait()
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        msg = "\n\n".join(f"{s}:\n{o}" for s, o in failed)
        raise RuntimeError("libkfac build failed:\n" + msg)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
