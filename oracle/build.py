"""Build step for the CPU oracle library (test infrastructure; see oracle/__init__.py)."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    srcs = sorted(os.path.join(_HERE, f) for f in os.listdir(_HERE) if f.endswith(".c"))
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-fopenmp", *srcs, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
