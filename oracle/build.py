"""Build the CPU oracle (test infrastructure only).

Compiles ``wenoiu_oracle.cpp`` with g++ into ``liboracle.so`` beside it:
plain C++17, -O2, no floating-point contraction and no fast-math, OpenMP
over independent grid lines only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wenoiu_oracle.cpp")
HDR = os.path.join(HERE, "wenoiu_oracle.hpp")
HDR2 = os.path.join(HERE, "flop_count.hpp")
HDR3 = os.path.join(HERE, "ad_types.hpp")
HDR4 = os.path.join(HERE, "multiblock.hpp")
HDR5 = os.path.join(HERE, "euler3d.hpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(SRC), os.path.getmtime(HDR), os.path.getmtime(HDR2), os.path.getmtime(HDR3),
            os.path.getmtime(HDR4), os.path.getmtime(HDR5)):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(out):
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only; every undefined-behaviour report is fatal), written to
    `out`.  Loaded into a Python process with the ASan runtime preloaded."""
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", out, SRC]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build())
