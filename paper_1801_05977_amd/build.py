"""Build libqpgf.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1801_05977_amd.build        # or __graft_entry__.build()

Each source is compiled to an object of its own (in parallel; every kernel and its
launcher live in one translation unit, so no relocatable device code is needed),
then the objects are linked into the shared library.
"""

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqpgf.so")
SOURCES = ["api.hip", "fill.hip", "fft.hip", "gather.hip", "mlp.hip", "surrogate.hip"]
ARCH = os.environ.get("QPGF_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _filter(out):
    return [l for l in out.strip().splitlines() if "packed-fp32-ops" not in l and "not a recognized feature" not in l]


def build(verbose=True):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="qpgf_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc, *FLAGS, "-c", "-o", obj, os.path.join(CSRC, src)]
            r = subprocess.run(cmd, capture_output=True, text=True)
            return src, obj, r.returncode, _filter(r.stdout + r.stderr), " ".join(cmd)

        with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
            results = list(ex.map(compile_one, SOURCES))
        errors = []
        for src, obj, rc, warn, cmd in results:
            if verbose:
                print(cmd, flush=True)
            if rc != 0:
                errors.append(f"{src}:\n" + "\n".join(warn))
            elif verbose and warn:
                print("\n".join(warn[:40]))
        if errors:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
        tmp = LIB + ".tmp"
        cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *[r[1] for r in results]]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + "\n".join(_filter(r.stdout + r.stderr)))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
