"""Build the LSNIF HIP library (``liblsnif.so``) for gfx950 with hipcc.

Each ``csrc/*.hip`` unit is compiled to an object in parallel and the objects
are linked into one shared library next to this file.  The float32 steps of
the walk and the grid indexing must not be contracted into fused
multiply-adds, hence ``-ffp-contract=off``; denormals are kept; packed FP32
instructions are disabled.
"""

import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblsnif.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fno-gpu-flush-denormals-to-zero", "-fhip-fp32-correctly-rounded-divide-sqrt",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def build(verbose=False):
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    tmp = tempfile.mkdtemp(prefix="lsnif_build_")
    objs, procs = [], []
    for s in srcs:
        o = os.path.join(tmp, os.path.basename(s) + ".o")
        objs.append(o)
        procs.append((s, subprocess.Popen([HIPCC, *FLAGS, "-c", s, "-o", o],
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature; that warning is expected
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {os.path.basename(s)}\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    out = LIB + f".{os.getpid()}.tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-o", out, *objs], check=True)
    os.replace(out, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(tmp)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
