"""Build libmlcc3.so (HIP, gfx950) in-tree: python -m paper_2202_08612_amd.build"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SO = os.path.join(PKG, "libmlcc3.so")
ARCH = os.environ.get("MLCC3_OFFLOAD_ARCH", "gfx950")
SOURCES = ["gemm_f64.hip", "tile_gemm_f64.hip", "dcontract_mixed.hip", "dcontract_bf16.hip", "triples_kernels.hip", "mlcc3_abi.hip"]
FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
         # no packed-FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wno-unused-result"]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with tempfile.TemporaryDirectory() as td:
        procs, objs = [], []
        for s in srcs:
            obj = os.path.join(td, s.replace(".hip", ".o"))
            cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        failed = []
        for s, p in procs:
            out = p.communicate()[0].decode(errors="replace")
            lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
            if p.returncode != 0:
                failed.append(s)
                print("\n".join(lines), file=sys.stderr)
            elif verbose and lines:
                print("\n".join(lines))
        if failed:
            raise RuntimeError(f"hipcc failed for {failed}")
        tmp = SO + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        subprocess.check_call(cmd)
        os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
