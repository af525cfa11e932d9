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


# host-side sanitizer build (CPU checks of the orchestration in dry-run mode): every sanitizer
# flag applies to the host compilation only, the device code is built as usual
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
SO_SANITIZE = os.path.join(PKG, "libmlcc3_hostsan.so")


def build(verbose=False, sanitize=False, out=None):
    """Compile libmlcc3.so; sanitize=True builds libmlcc3_hostsan.so with AddressSanitizer and
    UndefinedBehaviorSanitizer in the host code (load it with the clang ASan runtime preloaded)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    so = out or (SO_SANITIZE if sanitize else SO)
    extra = SANITIZE_FLAGS if sanitize else []
    with tempfile.TemporaryDirectory() as td:
        procs, objs = [], []
        for s in srcs:
            obj = os.path.join(td, s.replace(".hip", ".o"))
            cmd = [hipcc, *FLAGS, *extra, "-c", os.path.join(CSRC, s), "-o", obj]
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
        tmp = so + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs]
        subprocess.check_call(cmd)
        os.replace(tmp, so)
    return so


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
