"""Compile the CPU oracle (test infrastructure) into oracle/libhcoracle.so.

Two builds of the same source: a baseline x86-64 one and one that may use
AVX2 (the loops are plain C either way; -O3 lets the compiler vectorise them,
which changes no result: the arithmetic is integer, and the floating-point
features use no fast-math).  The loader picks the AVX2 build on a CPU that
has AVX2."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hc_oracle.c")
LIB = os.path.join(HERE, "libhcoracle.so")
LIB_AVX2 = os.path.join(HERE, "libhcoracle_avx2.so")


def _gcc(out, extra, verbose):
    cmd = ["gcc", "-O3", *extra, "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _gcc(LIB, [], verbose)
    _gcc(LIB_AVX2, ["-mavx2"], verbose)
    return LIB


def cpu_has_avx2() -> bool:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    return " avx2" in line
    except OSError:
        pass
    return False


def lib_path() -> str:
    """The build to load on this CPU."""
    return LIB_AVX2 if cpu_has_avx2() and os.path.exists(LIB_AVX2) else LIB


if __name__ == "__main__":
    print(build(verbose=True))
