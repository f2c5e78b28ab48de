"""Build the gfx950 C-ABI library libopo.so in-tree with hipcc.

The kernel instantiations are spread over several translation units
(csrc/k_*.hip) that compile in parallel; the host unit (csrc/opo.hip) holds the
C ABI. --sanitize builds the host code of every unit with AddressSanitizer and
UndefinedBehaviorSanitizer (device code is built as usual) into
libopo_sanitize.so, for the CPU test suite (OPO_LIB selects the library the
binding loads).

Usage: python -m paper_2410_02532_amd.build [--sanitize] [-j N]
"""
import argparse
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libopo.so")
LIB_SANITIZE = os.path.join(PKG, "libopo_sanitize.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

UNITS = ["opo.hip", "k_common.hip", "k_f32_pass.hip", "k_f64_pass.hip", "k_f32_mixed3.hip",
         "k_f32_mixed2.hip", "k_f64_mixed.hip", "k_resident.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
# host-side sanitizers only (each option applies to the host compilation)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build(verbose=False, sanitize=False, jobs=None):
    out = LIB_SANITIZE if sanitize else LIB
    extra = SANITIZE if sanitize else []
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="opo_build_") as tmpd:
        def compile_unit(unit):
            obj = os.path.join(tmpd, unit.replace(".hip", ".o"))
            cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, unit), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            return obj

        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(compile_unit, UNITS))
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + extra + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


def build_microbench(verbose=False):
    """Compile the stand-alone microbenchmarks (microbench/*.hip) as a build check; the
    executables go to a temporary directory (run them with the commands in their headers)."""
    mb = os.path.join(PKG, "microbench")
    with tempfile.TemporaryDirectory(prefix="opo_mb_") as tmpd:
        for f in sorted(os.listdir(mb)):
            if f.endswith(".hip"):
                cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
                       "-packed-fp32-ops", os.path.join(mb, f), "-o", os.path.join(tmpd, f[:-4])]
                if verbose:
                    print(" ".join(cmd), flush=True)
                subprocess.check_call(cmd)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--sanitize", action="store_true")
    ap.add_argument("-j", "--jobs", type=int, default=None)
    args = ap.parse_args()
    build(verbose=True, sanitize=args.sanitize, jobs=args.jobs)
    sys.exit(0)
