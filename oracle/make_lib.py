"""Build step for the oracle library (test infrastructure): gcc, plain C99, FP64, no fast-math.

``build(sanitize=True)`` makes ``liboracle_san.so`` instead, with AddressSanitizer and
UndefinedBehaviorSanitizer (any report aborts the process).  ``oracle.lib()`` loads it when the
environment sets ``LDO_SANITIZE=1``; the ASan runtime must then be the first library loaded:

    LDO_SANITIZE=1 LD_PRELOAD="$(gcc -print-file-name=libasan.so)${LD_PRELOAD:+:$LD_PRELOAD}" \\
    ASAN_OPTIONS=detect_leaks=0 python -m pytest tests -m "not gpu" -k "oracle or gmrf_model"

(leak detection is off because the Python interpreter itself keeps allocations until exit).
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))

SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]


def lib_name(sanitize: bool) -> str:
    return os.path.join(_HERE, "liboracle_san.so" if sanitize else "liboracle.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    src = os.path.join(_HERE, "ldo.c")
    out = lib_name(sanitize)
    tmp = f"{out}.tmp{os.getpid()}"  # per process: parallel test workers may build at once
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc", "-std=c99", *opt, "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import sys

    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
