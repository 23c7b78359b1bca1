"""Build the CPU oracle library (test infrastructure).

Compiles oracle/hydro_oracle.cpp with g++ into oracle/libhydro_oracle.so.
FP contraction is switched off so that every + and * rounds on its own, as
the source is written.

    python oracle/build_oracle.py               # optimised build
    python oracle/build_oracle.py --sanitize    # AddressSanitizer + UndefinedBehaviorSanitizer
                                                # build into oracle/libhydro_oracle_san.so (host only)

The sanitized library is loaded by a child process that preloads the ASan
runtime (tests/test_oracle_sanitize.py); it is never the library the other
tests use.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hydro_oracle.cpp")
LIB = os.path.join(HERE, "libhydro_oracle.so")
LIB_SAN = os.path.join(HERE, "libhydro_oracle_san.so")

FLAGS = ["-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def build(force: bool = True, sanitize: bool = False) -> str:
    lib = LIB_SAN if sanitize else LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["g++", *opt, *FLAGS, "-o", lib + ".tmp", SRC]
    subprocess.check_call(cmd)
    os.replace(lib + ".tmp", lib)
    return lib


def asan_runtime() -> str:
    """Path of g++'s AddressSanitizer runtime (to preload into a Python child)."""
    return subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv, sanitize="--sanitize" in sys.argv))
