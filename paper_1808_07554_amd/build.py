"""Build liblbtp.so (HIP, gfx950) in place next to this file.

Usage: python -m paper_1808_07554_amd.build   (or build() from Python).
Every source under csrc/ is compiled with hipcc for gfx950 only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbtp.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # no FMA contraction: every template instantiation of a sweep rounds the
    # same way, so ensemble members, checkpoints and single runs agree bitwise
    "-ffp-contract=off",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src, obj, verbose):
    cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-I", os.path.join(HERE, "..", "include"), "-c", "-o",
                                                             obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose=False, jobs=None):
    """Compile every source to an object in a temporary folder (in parallel),
    then link the shared library and move it into place."""
    import concurrent.futures
    import tempfile

    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 1, 16)
    with tempfile.TemporaryDirectory(prefix="lbtp_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(f)[:-4] + ".o") for f in srcs]
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda a: _compile(a[0], a[1], verbose), zip(srcs, objs)))
        tmp = LIB + ".tmp"
        cmd = [HIPCC] + FLAGS + ["-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
