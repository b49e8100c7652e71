"""Build the HIP library in-tree for gfx950 (hipcc cross-compiles without a GPU)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_NAME = "libld_mi355x.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
SOURCES = ["csrc/ld_kernels.hip", "csrc/ld_resident.hip", "csrc/ld_fp64.hip", "csrc/ld_prox.hip", "csrc/ld_interm.hip", "csrc/ld_fsb.hip", "csrc/ld_sigmoid.hip", "csrc/ld_bab.hip", "csrc/ld_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {what} ({res.returncode}):\n{errs}")
    if verbose and errs.strip():
        print(errs, file=sys.stderr)


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (the translation units share no
    device symbols), link the shared library, then the C ABI host program."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="ld_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[hipcc] + HIPCC_FLAGS + ["-c"] + inc + [os.path.join(HERE, s), "-o", o] for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(lambda c: _run(c[0], c[1], verbose), zip(cmds, SOURCES)))
        tmp = LIB_PATH + ".tmp"
        _run([hipcc] + HIPCC_FLAGS + objs + ["-o", tmp], "link", verbose)
    os.replace(tmp, LIB_PATH)
    build_abi_program(hipcc)
    return LIB_PATH


# A host program that calls the library through include/ld.h only (tests/c).
ABI_PROGRAM_SRC = os.path.join(ROOT, "tests", "c", "ld_abi_run.cpp")
ABI_PROGRAM = os.path.join(ROOT, "tests", "c", "ld_abi_run")


def build_abi_program(hipcc: str) -> str:
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), ABI_PROGRAM_SRC,
           "-L", HERE, "-lld_mi355x", "-Wl,-rpath,$ORIGIN/../../paper_2104_06718_amd", "-o", ABI_PROGRAM]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc (C ABI program) failed ({res.returncode}):\n{res.stderr}")
    return ABI_PROGRAM


if __name__ == "__main__":
    print(build(verbose=True))
