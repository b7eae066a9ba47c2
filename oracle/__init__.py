"""CPU oracle for flow routing -- TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library
and never imports it.  All arithmetic lives in ``oracle.c`` (plain C, float64
and uint64); this file only marshals numpy arrays.

Every function follows the paper (W. Bangerth, "Massively parallel flow
routing and drainage area determination"):

* ``receivers``        -- local flow routing, D8/D4 (Section 2.1)
* ``mfd_fractions``    -- local routing with several receivers (Appendix A)
* ``order``            -- high-to-low sort (Section 2.1)
* ``accumulate_*``     -- global flow routing / in-place triangular solve
                          (Section 2.1 listing, Section 3.1, Appendix A)
* ``adjoint_*``        -- transpose solve (I - W) rbar = qbar, the same sweep
                          run low-to-high (from eq. linear-system)
* ``apply_A_*``        -- matrix-free A x (Section 3.1, Appendix A)
* ``mass_*``           -- sink outflow versus total rain (Section 4)
* ``block_richardson`` -- the paper's parallel scheme run sequentially: block
                          Richardson iterations on (I+X) and (I-X)(I+X)
                          (Section 3.3, Appendix B)
* ``fill_depressions`` -- priority-flood depression filling, plain or with an
                          epsilon step so every cell drains (Section 4)

Pins: every function here is checked in ``tests/test_oracle_pins.py`` against
things other than itself (the paper's 3x3 example, brute force, library
solvers, closed forms).  The MFD slope-power law itself has no printed value
in the paper: its exponent is "parity unpinned" beyond the special cases
listed in that test file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

D8, MFD, D4 = 0, 1, 2
SINK = 0xFF
# Neighbour k -> (drow, dcol), row-major window order.
OFFSETS = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc: no fast-math, no FP contraction."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # ORACLE_LIB_PATH: a build of the same source to load instead (the test
        # suite's sanitizer run sets it).
        path = os.environ.get("ORACLE_LIB_PATH")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB):
                build()
        lib = ctypes.CDLL(path)
        i64, vp, dbl, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_int
        sig = {
            "or_receivers": [vp, i64, i64, ci, vp],
            "or_mfd_fractions": [vp, i64, i64, dbl, ci, vp, vp],
            "or_order": [vp, i64, vp],
            "or_accumulate_single": [vp, i64, i64, vp, vp, vp, vp],
            "or_accumulate_mfd": [vp, i64, i64, dbl, ci, vp, vp, vp],
            "or_adjoint_single": [vp, i64, i64, vp, vp, vp],
            "or_adjoint_mfd": [vp, i64, i64, dbl, vp, vp, vp],
            "or_apply_A_single": [vp, i64, i64, vp, vp],
            "or_apply_A_mfd": [vp, i64, i64, dbl, vp, vp],
            "or_mass_single": [vp, i64, vp, vp, vp],
            "or_mass_mfd": [vp, i64, i64, vp, vp, vp],
            "or_block_richardson": [vp, vp, i64, i64, dbl, vp, vp, i64, i64, ci, ci, vp, vp, vp],
            "or_fill_depressions": [vp, i64, i64, ci, ci, vp],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.restype = ci
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle: {name} failed with {rc}")


def receivers(z, rule: int = D8) -> np.ndarray:
    """Direction code 0..7 of each cell's receiver, 0xFF for sinks (D8 or D4)."""
    z = _f32(z)
    nr, nc = z.shape
    code = np.empty((nr, nc), dtype=np.uint8)
    _check(_load().or_receivers(_p(z), nr, nc, rule, _p(code)), "receivers")
    return code


def mfd_fractions(z, p: float = 1.1, frac32: bool = False):
    """(mask uint8[nr,nc], frac float64[nr,nc,8]) of the multiple-receiver split."""
    z = _f32(z)
    nr, nc = z.shape
    mask = np.empty((nr, nc), dtype=np.uint8)
    frac = np.empty((nr, nc, 8), dtype=np.float64)
    _check(_load().or_mfd_fractions(_p(z), nr, nc, p, int(frac32), _p(mask), _p(frac)), "mfd_fractions")
    return mask, frac


def order(z) -> np.ndarray:
    """Cell indices sorted by elevation descending, equal elevations by index."""
    z = _f32(z)
    out = np.empty(z.size, dtype=np.int64)
    _check(_load().or_order(_p(z), z.size, _p(out)), "order")
    return out


def accumulate_single(code, rain=None, order_=None, z=None, q=True, counts=True):
    """Single-receiver push: returns (q float64 or None, counts uint64 or None).

    ``order_`` is the high-to-low order; if absent it is computed from ``z``.
    """
    code = np.ascontiguousarray(code, dtype=np.uint8)
    nr, nc = code.shape
    if order_ is None:
        order_ = order(z)
    r = None if rain is None else _f32(rain)
    qo = np.empty((nr, nc), dtype=np.float64) if q else None
    co = np.empty((nr, nc), dtype=np.uint64) if counts else None
    _check(_load().or_accumulate_single(_p(code), nr, nc, _p(order_), _p(r), _p(qo), _p(co)),
           "accumulate_single")
    return qo, co


def accumulate_mfd(z, rain=None, p: float = 1.1, order_=None, frac32: bool = False) -> np.ndarray:
    z = _f32(z)
    nr, nc = z.shape
    if order_ is None:
        order_ = order(z)
    r = None if rain is None else _f32(rain)
    q = np.empty((nr, nc), dtype=np.float64)
    _check(_load().or_accumulate_mfd(_p(z), nr, nc, p, int(frac32), _p(order_), _p(r), _p(q)),
           "accumulate_mfd")
    return q


def block_richardson(z, block, rule: int = D8, rain=None, scheme: int = 0, p: float = 1.1,
                     max_iter: int = 100000, order_=None):
    """The paper's parallel scheme run sequentially (Section 3.3 "I+X"
    (scheme 0) and "(I-X)(I+X)" (scheme 1) iterations; Appendix B): blocks of
    block = (rows, cols) cells, D = every routing pair inside a block solved
    by the block's own high-to-low push, water passed across block
    boundaries between iterations.  Returns (q float64, counts uint64 (None
    for MFD), iterations until the iterate is exact)."""
    z = _f32(z)
    nr, nc = z.shape
    if order_ is None:
        order_ = order(z)
    code = receivers(z, rule) if rule != MFD else None
    r = None if rain is None else _f32(rain)
    q = np.empty((nr, nc), dtype=np.float64)
    co = np.empty((nr, nc), dtype=np.uint64) if code is not None else None
    it = ctypes.c_int(0)
    _check(_load().or_block_richardson(_p(code), _p(z), nr, nc, p, _p(order_), _p(r), int(block[0]),
                                       int(block[1]), int(scheme), int(max_iter), _p(q), _p(co),
                                       ctypes.addressof(it)), "block_richardson")
    return q, co, it.value


def fill_depressions(z, conn: int = 8, eps: bool = True) -> np.ndarray:
    """Filled float32 surface: boundary cells keep z; every other cell is
    raised to the lowest level (plus one float32 step per cell crossed when
    eps) at which it can drain to the boundary through ``conn``-neighbours."""
    z = _f32(z)
    nr, nc = z.shape
    out = np.empty((nr, nc), dtype=np.float32)
    rc = _load().or_fill_depressions(_p(z), nr, nc, int(conn), int(bool(eps)), _p(out))
    if rc == -5:
        raise ValueError("fill_depressions: non-finite elevation")
    _check(rc, "fill_depressions")
    return out


def adjoint_single(code, qbar, order_=None, z=None) -> np.ndarray:
    code = np.ascontiguousarray(code, dtype=np.uint8)
    nr, nc = code.shape
    if order_ is None:
        order_ = order(z)
    qb = np.ascontiguousarray(qbar, dtype=np.float64).reshape(nr, nc)
    rb = np.empty((nr, nc), dtype=np.float64)
    _check(_load().or_adjoint_single(_p(code), nr, nc, _p(order_), _p(qb), _p(rb)), "adjoint_single")
    return rb


def adjoint_mfd(z, qbar, p: float = 1.1, order_=None) -> np.ndarray:
    z = _f32(z)
    nr, nc = z.shape
    if order_ is None:
        order_ = order(z)
    qb = np.ascontiguousarray(qbar, dtype=np.float64).reshape(nr, nc)
    rb = np.empty((nr, nc), dtype=np.float64)
    _check(_load().or_adjoint_mfd(_p(z), nr, nc, p, _p(order_), _p(qb), _p(rb)), "adjoint_mfd")
    return rb


def apply_A_single(code, x) -> np.ndarray:
    code = np.ascontiguousarray(code, dtype=np.uint8)
    nr, nc = code.shape
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(nr, nc)
    y = np.empty((nr, nc), dtype=np.float64)
    _check(_load().or_apply_A_single(_p(code), nr, nc, _p(xx), _p(y)), "apply_A_single")
    return y


def apply_A_mfd(z, x, p: float = 1.1) -> np.ndarray:
    z = _f32(z)
    nr, nc = z.shape
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(nr, nc)
    y = np.empty((nr, nc), dtype=np.float64)
    _check(_load().or_apply_A_mfd(_p(z), nr, nc, p, _p(xx), _p(y)), "apply_A_mfd")
    return y


def mass_single(code, q, rain=None):
    code = np.ascontiguousarray(code, dtype=np.uint8)
    qq = np.ascontiguousarray(q, dtype=np.float64)
    r = None if rain is None else _f32(rain)
    out = np.zeros(2, dtype=np.float64)
    _check(_load().or_mass_single(_p(code), code.size, _p(r), _p(qq), _p(out)), "mass_single")
    return float(out[0]), float(out[1])


def mass_mfd(z, q, rain=None):
    z = _f32(z)
    nr, nc = z.shape
    qq = np.ascontiguousarray(q, dtype=np.float64)
    r = None if rain is None else _f32(rain)
    out = np.zeros(2, dtype=np.float64)
    _check(_load().or_mass_mfd(_p(z), nr, nc, _p(r), _p(qq), _p(out)), "mass_mfd")
    return float(out[0]), float(out[1])


def route(z, rule: int = D8, rain=None, p: float = 1.1):
    """Whole path for tests: receivers + high-to-low push.

    D8/D4 returns (code, q float64, counts uint64); MFD returns (mask, q).
    """
    o = order(z)
    if rule == MFD:
        mask, _ = mfd_fractions(z, p)
        return mask, accumulate_mfd(z, rain, p, o)
    code = receivers(z, rule)
    q, c = accumulate_single(code, rain, o)
    return code, q, c
