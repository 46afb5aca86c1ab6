"""Build libsym.so (HIP kernels + C ABI) for gfx950 with hipcc.

Every translation unit under csrc/ is compiled to an object in parallel (the two
heavy force kernels once per precision), then linked into
paper_1808_02281_amd/libsym.so; the benchmark's FMA-rate probe goes into a library of
its own, paper_1808_02281_amd/libsymprobe.so. Objects go to paper_1808_02281_amd/_build/.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsym.so")

ARCH = "gfx950"
# Packed FP32 instructions are switched off: hipcc would otherwise form v_pk_* FP32
# operations from plain float code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]

# (source, extra defines, object name)
UNITS = [
    ("abi.hip", [], "abi.o"),
    ("action.hip", [], "action.o"),
    ("layout.hip", [], "layout.o"),
    ("check.hip", [], "check.o"),
    ("leapfrog.hip", [], "leapfrog.o"),
    ("force_direct.hip", ["-DSYM_ONLY_F32"], "force_direct_f32.o"),
    ("force_direct.hip", ["-DSYM_ONLY_F64"], "force_direct_f64.o"),
    ("force_factored.hip", ["-DSYM_ONLY_F32"], "force_factored_f32.o"),
    ("force_factored.hip", ["-DSYM_ONLY_F64"], "force_factored_f64.o"),
    ("force_batch.hip", ["-DSYM_ONLY_F32"], "force_batch_f32.o"),
    ("force_batch.hip", ["-DSYM_ONLY_F64"], "force_batch_f64.o"),
    ("fat.hip", ["-DSYM_ONLY_F32"], "fat_f32.o"),
    ("fat.hip", ["-DSYM_ONLY_F64"], "fat_f64.o"),
    ("wilson.hip", [], "wilson.o"),
]
# The benchmark's FMA-rate probe: a library of its own, not part of libsym.so.
PROBE_UNIT = ("probe.hip", [], "probe.o")
PROBE_LIB = os.path.join(HERE, "libsymprobe.so")


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _headers_mtime():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs.append(os.path.join(os.path.dirname(HERE), "include", "sym.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(unit, force, verbose):
    src, defs, obj = unit
    src_p = os.path.join(CSRC, src)
    obj_p = os.path.join(BUILD, obj)
    if not force and os.path.exists(obj_p):
        newest = max(os.path.getmtime(src_p), _headers_mtime())
        if os.path.getmtime(obj_p) >= newest:
            return obj_p
    cmd = [_hipcc()] + FLAGS + defs + ["-c", src_p, "-o", obj_p + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(obj_p + ".tmp", obj_p)
    return obj_p


def build(force=True, verbose=False, jobs=None):
    """Compile and link libsym.so; returns its path. force=False reuses fresh objects."""
    sys.path.insert(0, CSRC)
    try:
        import gen_paths

        gen_paths.main()
    finally:
        sys.path.pop(0)
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, force, verbose), UNITS + [PROBE_UNIT]))
    for lib, parts in ((LIB, objs[:-1]), (PROBE_LIB, objs[-1:])):
        cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}"] + parts + ["-o", lib + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
