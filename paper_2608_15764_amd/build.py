"""Build libilpsweep.so for gfx950 in-tree with hipcc.

    python -m paper_2608_15764_amd.build [--asm]

Every HIP source is compiled with packed-FP32 code generation disabled
(the kernels never rely on v_pk_*_f32) and linked into
``paper_2608_15764_amd/libilpsweep.so``.  ``--asm`` also writes the device
assembly of every kernel source to ``_build/asm/`` for the ISA audit.
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libilpsweep.so")
ARCH = "gfx950"

SOURCES = ["kernels_plain.hip", "kernels_fused.hip", "kernels_lds.hip",
           "kernels_misc.hip", "kernels_chase.hip", "kernels_xcd.hip", "static_scratch.hip",
           "runtime.cpp", "plan.cpp"]

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         "-Wall", "-Wno-unused-command-line-argument"]


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    # hipcc's host pass does not know the packed-fp32 feature: harmless
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def compile_one(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    _run([hipcc(), *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
    return obj


def asm_one(src):
    out = os.path.join(BUILD, "asm", os.path.splitext(src)[0] + ".s")
    _run([hipcc(), *FLAGS, "-x", "hip", "--cuda-device-only", "-S",
          os.path.join(CSRC, src), "-o", out])
    return out


def build(asm=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(os.path.join(BUILD, "asm"), exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
        if asm:
            list(ex.map(asm_one, [s for s in SOURCES if s.endswith(".hip")]))
    tmp = LIB + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs,
          "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", action="store_true")
    ap.add_argument("-j", "--jobs", type=int, default=None)
    a = ap.parse_args(argv)
    print(build(asm=a.asm, jobs=a.jobs))


if __name__ == "__main__":
    sys.exit(main())
