"""The kernels' double-precision logarithms (csrc/perrk_log.h) compiled for the
host and checked against numpy's log / log1p: at most 4 units in the last
place for log and 6 for log1p over the whole double range, near 1 and at
subnormal arguments, with an exact reciprocal (6 and 10 with one that is off by
an ulp: the device refines the hardware reciprocal to within an ulp); zero,
negative, infinite and NaN arguments give -inf, NaN, inf and NaN."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r'''
#include <cmath>
#include "perrk_log.h"
struct Exact { double operator()(double v) const { return 1.0 / v; } };
struct OffByUlp { double operator()(double v) const { return std::nextafter(1.0 / v, v > 0 ? INFINITY : -INFINITY); } };
extern "C" {
void plog(const double *x, double *y, long n, int off) {
    for (long i = 0; i < n; ++i) y[i] = off ? perrk_log::log_f64(x[i], OffByUlp()) : perrk_log::log_f64(x[i], Exact());
}
void plog1p(const double *x, double *y, long n, int off) {
    for (long i = 0; i < n; ++i) y[i] = off ? perrk_log::log1p_f64(x[i], OffByUlp()) : perrk_log::log1p_f64(x[i], Exact());
}
}
'''


@pytest.fixture(scope="module")
def L():
    d = tempfile.mkdtemp()
    src, lib = os.path.join(d, "plog.cpp"), os.path.join(d, "plog.so")
    with open(src, "w") as f:
        f.write(SRC)
    subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", "-ffp-contract=off", "-I",
                           os.path.join(ROOT, "paper_2507_04991_amd", "csrc"), src, "-o", lib])
    return ctypes.CDLL(lib)


def run(L, fn, x, off):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    dp = ctypes.POINTER(ctypes.c_double)
    getattr(L, fn)(x.ctypes.data_as(dp), y.ctypes.data_as(dp), ctypes.c_long(len(x)), ctypes.c_int(off))
    return y


def ulps(y, ref):
    return np.abs(y - ref) / np.spacing(np.abs(ref))


@pytest.mark.parametrize("off", [0, 1])
def test_log_accuracy(L, off):
    rng = np.random.default_rng(off)
    x = np.concatenate([np.exp(rng.uniform(-744, 709, 200000)), rng.uniform(0.25, 4.0, 200000),
                        1.0 + rng.uniform(-1e-5, 1e-5, 50000), 2.0 ** rng.integers(-1074, 1023, 2000).astype(float),
                        np.array([1.0 + 2.0 ** -52, 1.0 - 2.0 ** -53, np.nextafter(0.0, 1.0), 1.7976931348623157e308])])
    ref = np.log(x)
    nz = ref != 0.0
    assert np.all(run(L, "plog", x[~nz], off) == 0.0)
    u = ulps(run(L, "plog", x[nz], off), ref[nz])
    assert u.max() <= (6.0 if off else 4.0), (u.max(), x[nz][np.argmax(u)])


@pytest.mark.parametrize("off", [0, 1])
def test_log1p_accuracy(L, off):
    rng = np.random.default_rng(10 + off)
    x = np.concatenate([rng.uniform(-0.999, 5.0, 200000), rng.uniform(-1e-2, 1e-2, 100000),
                        10.0 ** rng.uniform(-300, -1, 50000), -(10.0 ** rng.uniform(-300, -1, 50000)),
                        np.exp(rng.uniform(0, 700, 20000))])
    u = ulps(run(L, "plog1p", x, off), np.log1p(x))
    assert u.max() <= (10.0 if off else 6.0), (u.max(), x[np.argmax(u)])


def test_special_arguments(L):
    y = run(L, "plog", np.array([0.0, -0.0, -1.0, np.inf, -np.inf, np.nan]), 0)
    assert y[0] == -np.inf and y[1] == -np.inf and np.isnan(y[2]) and y[3] == np.inf
    assert np.isnan(y[4]) and np.isnan(y[5])
    z = run(L, "plog1p", np.array([0.0, -1.0, -2.0, np.inf]), 0)
    assert z[0] == 0.0 and z[1] == -np.inf and np.isnan(z[2]) and z[3] == np.inf
