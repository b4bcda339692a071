"""Compile the oracle's C direct sums (dft.c) into a shared library next to it."""

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path():
    return os.path.join(_HERE, "liboracle_dft.so")


def build(force=True):
    out = lib_path()
    src = os.path.join(_HERE, "dft.c")
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out
