"""The kernels' exponential and binary32 logarithm (csrc/device/coot_exp.h,
coot_log.h) built for the host with g++, so their arithmetic can be checked against
the oracle without a GPU."""
import ctypes
import os
import shutil
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEV = os.path.join(ROOT, "paper_2508_11385_amd", "csrc", "device")

SRC = r"""
#define __host__
#define __device__
#define __forceinline__ inline
#include "coot_exp.h"
#include "coot_log.h"
extern "C" void logf_n(const float* x, float* y, long n) { for (long i = 0; i < n; ++i) y[i] = coot::log_lf(x[i]); }
extern "C" void expf_n(const float* x, float* y, long n) { for (long i = 0; i < n; ++i) y[i] = coot::exp_cr<float>(x[i]); }
extern "C" void exp_n(const double* x, double* y, long n) { for (long i = 0; i < n; ++i) y[i] = coot::exp_cr<double>(x[i]); }
extern "C" void expf_rn_n(const float* x, float* y, long n) { for (long i = 0; i < n; ++i) y[i] = coot::exp_rn<float>(x[i]); }
extern "C" void exp_rn_n(const double* x, double* y, long n) { for (long i = 0; i < n; ++i) y[i] = coot::exp_rn<double>(x[i]); }
extern "C" long expf_fast_misses(const float* x, long n) {
  long m = 0;
  for (long i = 0; i < n; ++i) { bool ok; (void)coot::exp_fast<float>(x[i], ok); m += !ok; }
  return m;
}
"""


def build():
    """Compile and load the host library; None when g++ is missing."""
    gxx = shutil.which("g++")
    if not gxx:
        return None
    d = tempfile.mkdtemp()
    src = os.path.join(d, "e.cpp")
    so = os.path.join(d, "e.so")
    with open(src, "w") as f:
        f.write(SRC)
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-I", DEV, src, "-o", so],
                   check=True)
    L = ctypes.CDLL(so)
    for name in ("expf_n", "exp_n", "expf_rn_n", "exp_rn_n", "logf_n"):
        getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]
    L.expf_fast_misses.argtypes = [ctypes.c_void_p, ctypes.c_long]
    L.expf_fast_misses.restype = ctypes.c_long
    return L
