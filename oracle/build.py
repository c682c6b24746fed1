"""Compile the plain-C FP64 oracle into ``oracle/liblwacm_oracle.so`` with gcc.

Test infrastructure: the product library never links or loads this.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lwacm_oracle.c")
LIB = os.path.join(HERE, "liblwacm_oracle.so")


def build(verbose: bool = False, out: str = LIB, sanitize: bool = False) -> str:
    """Compile the oracle to ``out``; ``sanitize`` adds AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only; load it with the sanitizer
    runtimes preloaded, see tests/test_sanitizers.py)."""
    tmp = out + ".tmp"
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    cmd = ["gcc"] + flags + ["-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
                             "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
