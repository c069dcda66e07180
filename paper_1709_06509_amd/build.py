"""Build step: compiles the HIP library (gfx950) and the synthetic-input generator in-tree.

  libbpstereo.so   hipcc --offload-arch=gfx950, from csrc/*.hip and csrc/api.cpp
  synth/libsynth.so  gcc, from synth/synth.c

Every call rebuilds everything.  Packed FP32 instructions are disabled for all device
code (-packed-fp32-ops).
"""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbpstereo.so")
SYNTH_LIB = os.path.join(HERE, "synth", "libsynth.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-command-line-argument",
             "-I" + os.path.join(ROOT, "include")]


# Extra flags of single source files (none at present).
FILE_FLAGS = {}


def _run_all(cmds):
    procs = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for c in cmds]
    errs = []
    for c, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the device-only feature flag: harmless, filtered
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            errs.append(" ".join(c) + "\n" + "\n".join(lines))
        elif lines:
            print("\n".join(lines))
    if errs:
        raise RuntimeError("build failed:\n" + "\n\n".join(errs))


def build_synth():
    tmp = SYNTH_LIB + ".tmp"
    _run_all([["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-Wall", "-Wextra",
               "-o", tmp, os.path.join(HERE, "synth", "synth.c"), "-lm"]])
    os.replace(tmp, SYNTH_LIB)
    return SYNTH_LIB


def build_hip():
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip"))) + sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")))
    objs, cmds = [], []
    for s in srcs:
        o = os.path.join(BUILD_DIR, os.path.basename(s) + ".o")
        objs.append(o)
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        cmds.append([HIPCC] + HIP_FLAGS + FILE_FLAGS.get(os.path.basename(s), []) + lang + ["-c", s, "-o", o])
    _run_all(cmds)
    tmp = LIB + ".tmp"
    _run_all([[HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs])
    os.replace(tmp, LIB)
    return LIB


def build():
    build_synth()
    return build_hip()


if __name__ == "__main__":
    print(build())
