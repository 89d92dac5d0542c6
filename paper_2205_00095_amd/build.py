"""Build the gfx950 shared library ``libdgsrhd.so`` in-tree with hipcc.

Translation units: the host C-ABI layer, the adjoint layer and one kernel unit
per spatial dimension (``launch.hip`` compiled with ``-DDG_DIM=1/2/3``), built
in parallel, then linked with ``hipcc -shared``.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdgsrhd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP64 division without the range-scaling steps (all operands here are normal
    # numbers; quotients are unchanged on the tested data, ~5% fewer instructions)
    "-fapprox-func",
    "-Wno-unused-result",
]


# sources the forward element kernel is compiled from (with FLAGS): a measurement taken
# on one build is matched to the current sources through this digest
ELEMENT_KERNEL_SOURCES = ("kernels.hpp", "physics.hpp", "launch.hip", "launch.hpp")


def source_digest(files=ELEMENT_KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _units():
    units = [("dg_api.hip", "dg_api.o", []), ("adjoint.hip", "adjoint.o", [])]
    for d in (1, 2, 3):
        units.append(("launch.hip", f"launch_dim{d}.o", [f"-DDG_DIM={d}"]))
        units.append(("launch_adj.hip", f"launch_adj_dim{d}.o", [f"-DDG_DIM={d}"]))
        units.append(("launch_lim.hip", f"launch_lim_dim{d}.o", [f"-DDG_DIM={d}"]))
    return units


def build(verbose: bool = False, extra_flags=None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    t0 = time.time()
    procs = []
    for src, obj, defs in _units():
        cmd = [HIPCC, *FLAGS, *(extra_flags or []), *defs, "-c", os.path.join(CSRC, src),
               "-o", os.path.join(BUILD, obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for obj, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((obj, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        for obj, out in failed:
            sys.stderr.write(f"--- {obj} ---\n{out}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(o for o, _ in failed))
    objs = [os.path.join(BUILD, o) for _, o, _ in _units()]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
