"""Build the HIP library liblbm.so for gfx950 in place (paper_0812_1282_amd/).

    python -m paper_0812_1282_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lb_kernels.hip", "lb_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # Code object v5 loads under every ROCm 6/7 runtime, including the one
    # bundled with the PyTorch wheel that shares this process.
    "-mcode-object-version=5",
    # Same rounding in every template instance: contract a*b+c only within
    # one expression.
    "-ffp-contract=on",
    # No packed FP32 instructions in device code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# roctx ranges (host-side markers for the profiler's marker trace)
ROCM_LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "lib")
LINK = ["-L" + ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]
N_FORMATS = 6  # storage formats: one compilation unit of sweep kernels each


def units():
    """(object name, source, extra flags) of every compilation unit."""
    out = [("lb_api", "lb_api.hip", []), ("lb_kernels", "lb_kernels.hip", [])]
    out += [(f"lb_sweep{k}", "lb_kernels.hip", [f"-DLB_SWEEP_UNIT={k}"]) for k in range(N_FORMATS)]
    return out


def build(verbose: bool = False, jobs: int = None) -> str:
    """Compile the units in parallel into objects under a temporary folder,
    then link liblbm.so."""
    import concurrent.futures
    import tempfile
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = jobs or max(1, min(len(units()), os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmp:
        cmds = []
        for name, src, extra in units():
            obj = os.path.join(tmp, name + ".o")
            cmds.append((obj, [HIPCC] + FLAGS + extra + inc +
                         ["-c", os.path.join(CSRC, src), "-o", obj]))
        if verbose:
            for _, c in cmds:
                print(" ".join(c), flush=True)
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(lambda c: subprocess.run(c[1], capture_output=True, text=True),
                                  cmds))
        for (_, c), r in zip(cmds, results):
            if r.returncode != 0:
                sys.stderr.write(r.stderr)
                raise subprocess.CalledProcessError(r.returncode, c)
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + \
            [o for o, _ in cmds] + LINK
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
