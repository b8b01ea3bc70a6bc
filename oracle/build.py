"""Compile the CPU oracle (plain C, gcc) into oracle/liborc.so and oracle/liborc_cs.so.

The second library is the same source built with complex arithmetic for
complex-step derivatives.  Test infrastructure only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> None:
    src = os.path.join(HERE, "orc.c")
    for out, extra in (("liborc.so", []), ("liborc_cs.so", ["-DORC_CSTEP"])):
        dst = os.path.join(HERE, out)
        tmp = f"{dst}.tmp{os.getpid()}"
        cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
               "-fno-fast-math", *extra, src, "-o", tmp, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, dst)  # a process that has the old library loaded keeps its copy


if __name__ == "__main__":
    build(verbose=True)
