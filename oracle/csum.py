"""ctypes wrapper of the C oracle sums (csum.c) and their build (test infrastructure).

The C code computes the same definition as convolve.convolve_sampled (ring candidates narrowed by
the exact azimuth bound plus two pixels, then the exact chord test), in FP64 on OpenMP threads,
so that large samples (1e5 pixels at Nside 2048) and the CPU timing baseline are affordable.
It is pinned against the NumPy oracle in tests/test_oracle_csum.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csum.c")
LIB = os.path.join(HERE, "_csum.so")


def build(verbose: bool = False) -> str:
    """gcc -O2 -fopenmp (no fast-math, no FMA contraction): IEEE FP64 throughout."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_convolve_sampled.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_int,
                                                ip, ctypes.c_int64, dp, ip, ctypes.c_int]
        lib.oracle_convolve_sampled.restype = ctypes.c_int
        _lib = lib
    return _lib


def convolve_sampled(nside: int, table, theta_cut: float, x, pix, nthreads: int = 0):
    """y at the listed pixels: returns (y [nmaps, len(pix)], pair counts [len(pix)]). x: [npix] or
    [nmaps, npix] (any float dtype; promoted to FP64 exactly)."""
    lib = _load()
    xm = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    npix = 12 * int(nside) ** 2
    if xm.shape[1] != npix:
        raise ValueError("x must have 12 nside^2 columns")
    table = np.ascontiguousarray(table, dtype=np.float64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    out = np.empty((xm.shape[0], len(pix)))
    counts = np.empty(len(pix), dtype=np.int64)
    for m0 in range(0, xm.shape[0], 64):
        blk = np.ascontiguousarray(xm[m0:m0 + 64])
        yb = np.empty((blk.shape[0], len(pix)))
        rc = lib.oracle_convolve_sampled(int(nside), table.ctypes.data_as(dp), len(table), float(theta_cut),
                                         blk.ctypes.data_as(dp), blk.shape[0], pix.ctypes.data_as(ip), len(pix),
                                         yb.ctypes.data_as(dp), counts.ctypes.data_as(ip), int(nthreads))
        if rc != 0:
            raise ValueError("oracle_convolve_sampled: bad arguments")
        out[m0:m0 + blk.shape[0]] = yb
    return out, counts
