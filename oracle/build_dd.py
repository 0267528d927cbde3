"""Build oracle/libddresid.so (the double-double residual kernel of the
reference solver) with gcc.  Test infrastructure only, built apart from the
HIP library and linked with nothing of it.

Usage: python -m oracle.build_dd
"""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ddresid.c")
LIB = os.path.join(HERE, "libddresid.so")


def build() -> str:
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("gcc not found: the oracle's double-double residual kernel needs a C compiler")
    tmp = LIB + ".tmp"
    # no contraction and no fast-math: the error-free transformations need
    # every product and sum rounded as written
    subprocess.run([cc, "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
