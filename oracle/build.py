"""Builds the CPU oracle (test infrastructure) into oracle/liboracle32.so and liboracle64.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11",
         "-Wall", "-Wextra"]


def build(verbose: bool = False) -> None:
    src = os.path.join(HERE, "gi_oracle.c")
    for name, extra in (("liboracle32.so", []), ("liboracle64.so", ["-DORC_F64"])):
        out = os.path.join(HERE, name)
        tmp = out + ".tmp"
        cmd = ["gcc", *FLAGS, *extra, "-o", tmp, src, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


if __name__ == "__main__":
    build(verbose=True)
