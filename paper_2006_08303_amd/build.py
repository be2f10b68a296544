"""Compile the HIP library for gfx950 (hipcc, in-tree).

Translation units: csrc/cip.hip (C ABI, plan, operators, row passes),
csrc/patch.hip (patch-dictionary MFMA kernels and their dictionary
learning), csrc/conv.hip (convolutional-dictionary kernels),
csrc/wavelet.hip (wavelet (x) DCT prior), csrc/server.hip (request server
on the plan API), csrc/static_solve.hip (reconstruction in a static device
buffer) and one csrc/col_pass.hip
instance per supported column length. They are compiled in
parallel and linked into paper_2006_08303_amd/libcip.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcip.so")
CSRC = os.path.join(HERE, "csrc")
SIZES = (16, 32, 64, 128, 256, 384, 512, 768, 1024, 1536, 2048)   # as in csrc/sizes.hpp
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    extra = [f"-D{d}" for d in defines]
    tmpdir = tempfile.mkdtemp(prefix="cipbuild_")
    jobs = [(os.path.join(CSRC, "cip.hip"), os.path.join(tmpdir, "cip.o"), []),
            (os.path.join(CSRC, "patch.hip"), os.path.join(tmpdir, "patch.o"), []),
            (os.path.join(CSRC, "conv.hip"), os.path.join(tmpdir, "conv.o"), []),
            (os.path.join(CSRC, "server.hip"), os.path.join(tmpdir, "server.o"), []),
            (os.path.join(CSRC, "wavelet.hip"), os.path.join(tmpdir, "wavelet.o"), []),
            (os.path.join(CSRC, "static_solve.hip"), os.path.join(tmpdir, "static_solve.o"), [])]
    for n in SIZES:
        jobs.append((os.path.join(CSRC, "col_pass.hip"), os.path.join(tmpdir, f"col_{n}.o"),
                     [f"-DCIP_COL_N={n}"]))
    procs = []
    for src, obj, d in jobs:
        cmd = [hipcc, *FLAGS, *extra, *d, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                            text=True)))
    failed = False
    for cmd, p in procs:
        outp, _ = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(outp)
    if failed:
        raise RuntimeError("hipcc failed compiling libcip")
    tmp = out + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for _, o, _ in jobs], "-o", tmp,
            "-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libcip.so")
    os.replace(tmp, out)
    for _, o, _ in jobs:
        os.remove(o)
    os.rmdir(tmpdir)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
