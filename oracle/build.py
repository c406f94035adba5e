"""Build ``liboracle.so`` from ``oracle.c`` with gcc (no HIP involved).

-O2 without fast-math and with -ffp-contract=off keeps every binary64
operation an IEEE round-to-nearest-even operation in source order.
"""
import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """liboracle.so, or with sanitize=True liboracle_san.so built with
    AddressSanitizer and UndefinedBehaviorSanitizer (for the CPU test run
    under the sanitizers)."""
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle_san.so" if sanitize else "liboracle.so")
    tmp = out + ".tmp"
    san = (["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
            "-fno-sanitize-recover=undefined"] if sanitize else [])
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"] + san + ["-o", tmp, src,
           "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
