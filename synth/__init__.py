"""Seeded synthetic inputs (DEMs, rainfall, random draws) for flow routing.

This module holds no flow-routing arithmetic.  It is the one piece of code
shared by the GPU library's tests and benchmark and by the CPU oracle's tests:
both sides route exactly the same grids.

The DEM recipe stands in for the paper's Colorado DEM (Section 4): a
diamond-square fractal (Hurst 0.7) normalised to [0, 1], a planar tilt of
0.01 per row so that water drains toward row 0 along long trunk rivers, and
U[0, 1e-3) noise, evaluated in float64 and rounded once to float32.  Rainfall
is U[0, 1) with 24 random bits, so every value is exact in float32.
All randomness is counter-based SplitMix64 (see ``synth.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libfrsynth.so")

# Streams of the counter-based generator reserved for tests and benchmarks.
STREAM_FRACTAL, STREAM_NOISE, STREAM_RAIN = 0, 1, 2
STREAM_PICK, STREAM_NORMAL = 3, 4

# Default DEM recipe parameters.
HURST, TILT, NOISE = 0.7, 0.01, 1e-3


def build(force: bool = False) -> str:
    """Compile ``libfrsynth.so`` with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # SYNTH_LIB_PATH: a build of the same source to load instead (the test
        # suite's sanitizer run sets it).
        path = os.environ.get("SYNTH_LIB_PATH")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB):
                build()
        lib = ctypes.CDLL(path)
        i64, u64, vp, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double
        lib.syn_u64.restype = u64
        lib.syn_u64.argtypes = [u64, u64, u64]
        lib.syn_uniform.restype = None
        lib.syn_uniform.argtypes = [u64, u64, i64, i64, vp]
        lib.syn_u64_array.restype = None
        lib.syn_u64_array.argtypes = [u64, u64, i64, i64, vp]
        lib.syn_fractal.restype = ctypes.c_int
        lib.syn_fractal.argtypes = [u64, i64, i64, dbl, vp]
        lib.syn_dem.restype = ctypes.c_int
        lib.syn_dem.argtypes = [u64, i64, i64, dbl, dbl, dbl, vp]
        lib.syn_rain.restype = None
        lib.syn_rain.argtypes = [u64, i64, vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def fractal(seed: int, nrows: int, ncols: int, hurst: float = HURST) -> np.ndarray:
    """Diamond-square fractal cropped to nrows x ncols, normalised to [0, 1]."""
    out = np.empty((nrows, ncols), dtype=np.float64)
    if _load().syn_fractal(seed, nrows, ncols, hurst, _ptr(out)) != 0:
        raise MemoryError("synth: fractal lattice allocation failed")
    return out


def dem(seed: int, nrows: int, ncols: int, hurst: float = HURST, tilt: float = TILT,
        noise: float = NOISE) -> np.ndarray:
    """float32 DEM: fractal + tilt*row + U[0, noise), row 0 lowest on average."""
    z = np.empty((nrows, ncols), dtype=np.float32)
    if _load().syn_dem(seed, nrows, ncols, hurst, tilt, noise, _ptr(z)) != 0:
        raise MemoryError("synth: DEM allocation failed")
    return z


def rain(seed: int, nrows: int, ncols: int) -> np.ndarray:
    """float32 rainfall k * 2^-24, k uniform in [0, 2^24)."""
    r = np.empty((nrows, ncols), dtype=np.float32)
    _load().syn_rain(seed, nrows * ncols, _ptr(r))
    return r


def uniform(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """n uniform [0, 1) doubles at counter indices start .. start+n-1."""
    out = np.empty(n, dtype=np.float64)
    _load().syn_uniform(seed, stream, start, n, _ptr(out))
    return out


def u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().syn_u64_array(seed, stream, start, n, _ptr(out))
    return out


def integers(seed: int, stream: int, n: int, lo: int, hi: int, start: int = 0) -> np.ndarray:
    """n integers uniform in [lo, hi] (inclusive), by multiply-shift on 64-bit draws."""
    span = int(hi) - int(lo) + 1
    raw = u64(seed, stream, n, start)
    vals = [(int(x) * span) >> 64 for x in raw]
    return np.asarray(vals, dtype=np.int64) + int(lo)


def distinct_cells(seed: int, stream: int, count: int, ncells: int) -> np.ndarray:
    """``count`` distinct cell indices in [0, ncells), in draw order."""
    out, seen, i = [], set(), 0
    while len(out) < count:
        batch = integers(seed, stream, 4 * count, 0, ncells - 1, start=i)
        i += 4 * count
        for v in batch:
            v = int(v)
            if v not in seen:
                seen.add(v)
                out.append(v)
                if len(out) == count:
                    break
    return np.asarray(out, dtype=np.int64)


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """n standard normal doubles by Box-Muller on counter-based uniforms."""
    u = uniform(seed, stream, 2 * n)
    u1 = 1.0 - u[0::2]  # in (0, 1]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def batch_shapes(seed: int, ntiles: int, lo: int = 64, hi: int = 2048) -> list[tuple[int, int]]:
    """Side lengths of independent DEM tiles: rows and cols uniform in [lo, hi]."""
    v = integers(seed, STREAM_PICK, 2 * ntiles, lo, hi)
    return [(int(v[2 * i]), int(v[2 * i + 1])) for i in range(ntiles)]
