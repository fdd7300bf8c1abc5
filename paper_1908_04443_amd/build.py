"""Build the gfx950 library paper_1908_04443_amd/liblbm.so in-tree.

Every source under csrc/ is compiled by hipcc for gfx950 (device code) and
the host objects are linked with g++ against the HIP runtime that PyTorch
ships, so that one process holds a single HIP runtime when the library is
used next to torch.  Packed-FP32 code generation is disabled (see the
compile flags).  The kernel sources are compiled once per precision: the
FP64 objects without FMA contraction, so that they follow the rounding steps
of a plain scalar evaluation, the FP32 objects with contraction.
"""
import os
import subprocess
import sys
import sysconfig

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["api.cpp", "thermo.cpp", "geometry.cpp", "step2d.hip", "step_march.hip",
           "aux.hip", "adjoint2d.hip", "noalloc.hip"]
# kernels compiled once per precision: FP32 with FMA contraction, FP64 without
SPLIT = {"step2d.hip", "step_march.hip", "adjoint2d.hip"}
EXTRA_SOURCES = []

# a plain C program that uses the library through include/lbm.h only
DEMO_SRC = os.path.join(CSRC, "cabi_demo.c")
DEMO = os.path.join(HERE, "lbm_cabi_demo")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
          "-Wno-unused-variable", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-munsafe-fp-atomics"]


def torch_lib_dir():
    # locate torch's lib dir without importing torch (keeps the build fast)
    for base in (sysconfig.get_paths()["purelib"], sysconfig.get_paths()["platlib"]):
        d = os.path.join(base, "torch", "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    import torch  # fallback
    return os.path.join(os.path.dirname(torch.__file__), "lib")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    jobs_list = []
    for src in SOURCES + EXTRA_SOURCES:
        path = os.path.join(CSRC, src)
        stem = os.path.splitext(src)[0]
        if src in SPLIT:
            for prec, contract in ((4, "fast"), (8, "off")):
                flags = [f if f != "-ffp-contract=off" else f"-ffp-contract={contract}"
                         for f in COMMON]
                obj = os.path.join(BUILD, f"{stem}_f{8 * prec}.o")
                jobs_list.append(([HIPCC, *flags, *DEVICE, f"-DLBM_PREC={prec}", "-x", "hip",
                                   "-c", path, "-o", obj], obj, src))
        elif src.endswith(".hip"):
            obj = os.path.join(BUILD, stem + ".o")
            jobs_list.append(([HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", path, "-o", obj],
                              obj, src))
        else:
            obj = os.path.join(BUILD, stem + ".o")
            jobs_list.append(([HIPCC, *COMMON, "-c", path, "-o", obj], obj, src))
    for cmd, obj, src in jobs_list:
        objs.append(obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        if len(procs) >= jobs:
            p, s = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"compile failed: {s}")
    for p, s in procs:
        if p.wait() != 0:
            raise RuntimeError(f"compile failed: {s}")
    tlib = torch_lib_dir()
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-o", tmp, *objs, f"-L{tlib}", "-lamdhip64",
          f"-Wl,-rpath,{tlib}", "-Wl,--no-undefined", "-Wl,--disable-new-dtags"], verbose)
    os.replace(tmp, LIB)
    # the C demo: gcc, C11, HIP runtime C API; finds liblbm.so next to itself
    dtmp = DEMO + ".tmp"
    _run(["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
          "-I/opt/rocm/include", f"-I{INCLUDE}", DEMO_SRC, "-o", dtmp, f"-L{HERE}", "-llbm",
          f"-L{tlib}", "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN", f"-Wl,-rpath,{tlib}",
          "-Wl,--disable-new-dtags"], verbose)
    os.replace(dtmp, DEMO)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
