"""Compile the HIP sources into libtjm.so (gfx950), in-tree."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtjm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return out


def build(verbose=False):
    """Compile every HIP source and link libtjm.so; returns its path."""
    objs = []
    procs = []
    # the step kernels are one source compiled once per contraction precision
    units = [("tjm_step.hip", "tjm_step_f32", ["-DTJM_TC=float"]),
             ("tjm_step.hip", "tjm_step_f64", ["-DTJM_TC=double"]),
             ("tjm_kernels.hip", "tjm_kernels", []),
             ("tjm_noalloc.hip", "tjm_noalloc", []),
             ("tjm_api.cpp", "tjm_api", ["-x", "hip"]),
             ("tjm_server.cpp", "tjm_server", ["-x", "hip"]),
             ("tjm_tune.cpp", "tjm_tune", ["-x", "hip"])]
    for src, name, extra in units:
        obj = os.path.join(CSRC, name + ".o")
        cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write("\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l) + "\n")
            raise RuntimeError("build step failed: " + " ".join(cmd))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
