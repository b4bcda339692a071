"""Host-only code of the library built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on the CPU (tests/host/host_checks.cpp): the
ES-kernel quadrature and parameter tables, the amplitude-model frequency bins.
The oracle's C direct sums are built and run the same way on a small case."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("hostsan"))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_asan_ubsan(tmp_path_factory):
    out = os.path.join(_build_dir(tmp_path_factory), "host_checks")
    subprocess.run(["g++", "-std=c++17", *SAN, os.path.join(HERE, "host", "host_checks.cpp"), "-o", out],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([out], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks ok" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_direct_sums_under_asan_ubsan(tmp_path_factory):
    d = _build_dir(tmp_path_factory)
    drv = os.path.join(d, "drv.c")
    with open(drv, "w") as f:
        f.write(r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
void oracle_degrid(int64_t, int64_t, double, double, int, const double *, int64_t, const double *,
                   const double *, const double *, double *);
void oracle_grid(int64_t, int64_t, double, double, int, int64_t, const double *, const double *,
                 const double *, const double *, double *);
int main(void) {
    const int64_t n = 8, nv = 5;
    double img[64], u[5], v[5], w[5], vis[10], out[64];
    for (int i = 0; i < 64; ++i) img[i] = (i % 7) - 3.0;
    for (int k = 0; k < nv; ++k) { u[k] = 100.0 * k; v[k] = -50.0 * k; w[k] = 3.0 * k; }
    oracle_degrid(n, n, 1e-3, 1e-3, 1, img, nv, u, v, w, vis);
    oracle_grid(n, n, 1e-3, 1e-3, 1, nv, u, v, w, vis, out);
    /* adjointness in the real inner product: <R x, R x> = <x, R^+ R x> */
    double a = 0, b = 0;
    for (int k = 0; k < 2 * nv; ++k) a += vis[k] * vis[k];
    for (int i = 0; i < 64; ++i) b += img[i] * out[i];
    if (fabs(a - b) > 1e-10 * fabs(a)) { printf("adjointness %g %g\n", a, b); return 1; }
    printf("oracle ok\n");
    return 0;
}
''')
    out = os.path.join(d, "drv")
    subprocess.run(["gcc", "-std=c11", *SAN, drv, os.path.join(ROOT, "oracle", "dft.c"), "-lm", "-o", out],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([out], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle ok" in r.stdout
