"""Build the HIP library libmstruct.so for gfx950 in-tree (hipcc), and the
roofline calibration probes libmstruct_probe.so (not part of the library)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmstruct.so")
PROBE_OUT = os.path.join(HERE, "libmstruct_probe.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ("api.hip", "kernels.hip", "mlp.hip", "step_f64_lib.hip", "step_f64_synth.hip", "step_f64_paper.hip")
PROBE_SOURCES = ("probe.hip",)
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # keep packed-FP32 instructions out of the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


def _link(objs, out, verbose):
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + PROBE_SOURCES
    with ThreadPoolExecutor(len(srcs)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    _link([objs[s] for s in SOURCES], OUT, verbose)
    _link([objs[s] for s in PROBE_SOURCES], PROBE_OUT, verbose)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
