"""Flow routing on a gridded DEM for AMD MI355X (gfx950).

Python binding of ``libflowroute.so`` (C ABI in ``include/fr_api.h``).  Every
step of the computation runs in the library's HIP kernels; this module only
marshals torch tensors (device memory, streams) into the C calls.  There is
no CPU fallback: if the library is missing, importing the binding's compute
functions raises.

What it computes (W. Bangerth, "Massively parallel flow routing and drainage
area determination"): local flow routing (Section 2.1, Appendix A) and the
water q per cell solving (I - W^T) q = r (Section 2.2), plus the adjoint
solve for gradients with respect to the rain.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libflowroute.so")

# Constants mirrored from include/fr_api.h.
D8, MFD, D4 = 0, 1, 2
NONE, F32, F64 = 0, 1, 2
SINK = 0xFF
FN_ACCUMULATE, FN_ADJOINT, FN_BLOCK_ITER, FN_BLOCK_ITER_PRE, FN_FILL = 1, 2, 3, 4, 5
SCHEME_IX, SCHEME_IMX_IX = 0, 1
OK = 0
ERR_ARG, ERR_RULE, ERR_WORKSPACE, ERR_HIP = -1, -2, -3, -4
ERR_NONFINITE, ERR_NOTDAG, ERR_BADCODE, ERR_TOOLARGE = -5, -6, -7, -8
ERR_STALL, ERR_CAPACITY = -9, -10
PATH_AUTO, PATH_SWEEP, PATH_ENGINE, PATH_TILES = 0, 1, 2, 3
PATHS = {"auto": PATH_AUTO, "sweep": PATH_SWEEP, "engine": PATH_ENGINE, "tiles": PATH_TILES}

RULES = {"d8": D8, "mfd": MFD, "d4": D4}
EXPORTS = ["fr_receivers", "fr_accumulate", "fr_accumulate_adjoint", "fr_workspace_bytes",
           "fr_status_string", "fr_version", "fr_timing_enable", "fr_timing_last",
           "fr_batched_workspace_bytes", "fr_accumulate_batched", "fr_batch_autotune",
           "fr_accumulate_block_iterations", "fr_fill_depressions", "fr_set_accumulate_path",
           "fr_accumulate_noalloc", "fr_set_autotune_cache", "fr_served_by"]
SERVED = {0: "none", 1: "rows", 2: "tiles", 3: "row_sweep", 4: "sweep", 5: "engine"}
ORDER_GIVEN, ORDER_ROWS_DESC, ORDER_CELLS_DESC = 0, 1, 2


class Tile(ctypes.Structure):
    """``fr_tile`` of the C ABI (device pointers, shape, rule)."""
    _fields_ = [("z", ctypes.c_void_p), ("rain", ctypes.c_void_p), ("q_out", ctypes.c_void_p),
                ("counts_out", ctypes.c_void_p), ("code_out", ctypes.c_void_p), ("nrows", ctypes.c_int64),
                ("ncols", ctypes.c_int64), ("rule", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchPlan(ctypes.Structure):
    """``fr_batch_plan`` of the C ABI."""
    _fields_ = [("workers", ctypes.c_int32), ("order", ctypes.c_int32)]


class FlowRouteError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


_lib = None


def load_library() -> ctypes.CDLL:
    """Load ``libflowroute.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libflowroute.so not found at {LIB_PATH}; build it with "
                          f"`python -m paper_2606_12800_amd._build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, ci, cd, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.fr_receivers.argtypes = [vp, i64, i64, ci, vp, vp, vp]
    lib.fr_receivers.restype = ci
    lib.fr_accumulate.argtypes = [vp, vp, i64, i64, ci, cd, vp, ci, ci, vp, vp, vp, vp, vp, sz, vp]
    lib.fr_accumulate.restype = ci
    lib.fr_accumulate_adjoint.argtypes = [vp, vp, i64, i64, ci, cd, vp, ci, vp, vp, vp, sz, vp]
    lib.fr_accumulate_adjoint.restype = ci
    lib.fr_workspace_bytes.argtypes = [ci, i64, i64, ci, ci]
    lib.fr_workspace_bytes.restype = sz
    lib.fr_status_string.argtypes = [ci]
    lib.fr_status_string.restype = ctypes.c_char_p
    lib.fr_version.argtypes = []
    lib.fr_version.restype = ctypes.c_char_p
    lib.fr_timing_enable.argtypes = [ci]
    lib.fr_timing_enable.restype = ci
    lib.fr_timing_last.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float), ci]
    lib.fr_timing_last.restype = ci
    i32 = ctypes.c_int32
    lib.fr_batched_workspace_bytes.argtypes = [vp, i32]
    lib.fr_batched_workspace_bytes.restype = sz
    lib.fr_accumulate_batched.argtypes = [vp, i32, vp, vp, vp, sz, vp]
    lib.fr_accumulate_batched.restype = ci
    lib.fr_batch_autotune.argtypes = [vp, i32, vp, vp, sz, ci, vp, vp]
    lib.fr_batch_autotune.restype = ci
    lib.fr_accumulate_block_iterations.argtypes = [vp, vp, i64, i64, ci, cd, i64, i64, ci, vp, ci, ci, vp, vp, i32,
                                                   vp, vp, vp, sz, vp]
    lib.fr_accumulate_block_iterations.restype = ci
    lib.fr_fill_depressions.argtypes = [vp, i64, i64, ci, ci, vp, vp, vp, vp, sz, vp]
    lib.fr_fill_depressions.restype = ci
    lib.fr_set_accumulate_path.argtypes = [ci]
    lib.fr_set_accumulate_path.restype = ci
    lib.fr_accumulate_noalloc.argtypes = [vp, vp, i64, i64, ci, cd, vp, ci, ci, vp, vp, vp, vp, vp]
    lib.fr_accumulate_noalloc.restype = ci
    lib.fr_set_autotune_cache.argtypes = [ctypes.c_char_p]
    lib.fr_set_autotune_cache.restype = ci
    lib.fr_served_by.argtypes = [vp, sz, vp, vp]
    lib.fr_served_by.restype = ci
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load_library().fr_status_string(int(code)).decode()


def workspace_bytes(fn: int, nrows: int, ncols: int, rule: int, dtype: int) -> int:
    return int(load_library().fr_workspace_bytes(fn, nrows, ncols, rule, dtype))


def timing_enable(on: bool = True) -> None:
    """Record per-phase device times of subsequent library calls."""
    load_library().fr_timing_enable(1 if on else 0)


def timing_last() -> dict:
    """{phase name: milliseconds} of the most recent timed library call."""
    names = (ctypes.c_char_p * 8)()
    ms = (ctypes.c_float * 8)()
    k = load_library().fr_timing_last(names, ms, 8)
    if k < 0:
        raise FlowRouteError(k, "fr_timing_last")
    out = {}
    for i in range(k):
        key = names[i].decode()
        out[key] = out.get(key, 0.0) + float(ms[i])
    return out


@contextlib.contextmanager
def accumulate_path(path: str):
    """Within the block, fr_accumulate / fr_accumulate_adjoint take the given
    path ("auto", "sweep", "engine" or "tiles"; ``fr_set_accumulate_path``).  Every
    path computes the same solution; tests use this to cover the fallbacks."""
    lib = load_library()
    rc = lib.fr_set_accumulate_path(PATHS[path])
    if rc != OK:
        raise FlowRouteError(rc, "fr_set_accumulate_path")
    try:
        yield
    finally:
        lib.fr_set_accumulate_path(PATH_AUTO)


def served_by(ws: "Workspace | None" = None, device=None) -> str:
    """Which solver finished the most recent accumulate / adjoint call that
    used the workspace (``fr_served_by``): "rows", "tiles", "row_sweep",
    "sweep", "engine" or "none"."""
    w = ws or _default_ws
    if w.buf is None:
        return "none"
    dev = device if device is not None else w.buf.device
    out = ctypes.c_int32(0)
    rc = load_library().fr_served_by(_ptr(w.buf), w.buf.numel(), ctypes.byref(out), _stream(dev))
    if rc != OK:
        raise FlowRouteError(rc, "fr_served_by")
    return SERVED.get(out.value, "none")


def _rule(rule) -> int:
    if isinstance(rule, str):
        return RULES[rule.lower()]
    return int(rule)


def _dtype_code(dtype) -> int:
    if dtype is None:
        return NONE
    if dtype == torch.float32:
        return F32
    if dtype == torch.float64:
        return F64
    raise ValueError(f"unsupported dtype {dtype}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_grid(t: torch.Tensor, dtype: torch.dtype, name: str):
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D (nrows, ncols)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be C-contiguous")


class Workspace:
    """Device scratch buffer reused across calls (grows on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        return self.buf


_default_ws = Workspace()


def _raise_status(status: torch.Tensor, what: str):
    s = int(status.item())
    if s != OK:
        raise FlowRouteError(s, what)


def receivers(z: torch.Tensor, rule="d8", check: bool = True) -> torch.Tensor:
    """Local flow routing: uint8 codes (D8/D4 direction or MFD lower mask)."""
    _check_grid(z, torch.float32, "z")
    nr, nc = z.shape
    code = torch.empty((nr, nc), dtype=torch.uint8, device=z.device)
    status = torch.zeros(1, dtype=torch.int32, device=z.device)
    rc = load_library().fr_receivers(_ptr(z), nr, nc, _rule(rule), _ptr(code), _ptr(status),
                                     _stream(z.device))
    if rc != OK:
        raise FlowRouteError(rc, "fr_receivers")
    if check:
        _raise_status(status, "fr_receivers")
    return code


def accumulate(code: torch.Tensor, z: torch.Tensor | None = None, rain: torch.Tensor | None = None,
               rule="d8", dtype=torch.float32, counts: bool = False, mass: bool = False,
               p: float = 1.1, ws: Workspace | None = None, check: bool = True):
    """Global flow routing: returns (q, counts, mass) with None for what was not asked."""
    _check_grid(code, torch.uint8, "code")
    nr, nc = code.shape
    dev = code.device
    r = _rule(rule)
    if z is not None:
        _check_grid(z, torch.float32, "z")
    rdt = F32
    if rain is not None:
        if rain.dtype not in (torch.float32, torch.float64):
            raise TypeError("rain must be float32 or float64")
        _check_grid(rain, rain.dtype, "rain")
        rdt = _dtype_code(rain.dtype)
    dt = _dtype_code(dtype)
    q = None if dtype is None else torch.empty((nr, nc), dtype=dtype, device=dev)
    cnt = torch.empty((nr, nc), dtype=torch.uint64, device=dev) if counts else None
    m = torch.empty(2, dtype=torch.float64, device=dev) if mass else None
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = workspace_bytes(FN_ACCUMULATE, nr, nc, r, dt)
    buf = (ws or _default_ws).get(nbytes, dev)
    rc = load_library().fr_accumulate(_ptr(z), _ptr(code), nr, nc, r, p, _ptr(rain), rdt, dt, _ptr(q),
                                      _ptr(cnt), _ptr(m), _ptr(status), _ptr(buf), buf.numel(),
                                      _stream(dev))
    if rc != OK:
        raise FlowRouteError(rc, "fr_accumulate")
    if check:
        _raise_status(status, "fr_accumulate")
    return q, cnt, m


def adjoint(code: torch.Tensor, qbar: torch.Tensor, z: torch.Tensor | None = None, rule="d8",
            p: float = 1.1, ws: Workspace | None = None, check: bool = True) -> torch.Tensor:
    """Transpose solve (I - W) rbar = qbar; dtype follows qbar (float32 or float64)."""
    _check_grid(code, torch.uint8, "code")
    nr, nc = code.shape
    dev = code.device
    if qbar.dtype not in (torch.float32, torch.float64):
        raise TypeError("qbar must be float32 or float64")
    _check_grid(qbar, qbar.dtype, "qbar")
    if z is not None:
        _check_grid(z, torch.float32, "z")
    r = _rule(rule)
    dt = _dtype_code(qbar.dtype)
    rbar = torch.empty_like(qbar)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = workspace_bytes(FN_ADJOINT, nr, nc, r, dt)
    buf = (ws or _default_ws).get(nbytes, dev)
    rc = load_library().fr_accumulate_adjoint(_ptr(z), _ptr(code), nr, nc, r, p, _ptr(qbar), dt,
                                              _ptr(rbar), _ptr(status), _ptr(buf), buf.numel(),
                                              _stream(dev))
    if rc != OK:
        raise FlowRouteError(rc, "fr_accumulate_adjoint")
    if check:
        _raise_status(status, "fr_accumulate_adjoint")
    return rbar


def block_iterations(code: torch.Tensor, rain: torch.Tensor | None = None, rule="d8",
                     dtype=torch.float64, counts: bool = True, max_iter: int = 100000,
                     ws: Workspace | None = None, check: bool = True, scheme: str = "ix",
                     block=(256, 256)):
    """The paper's block Richardson iterations (``fr_accumulate_block_iterations``)
    with blocks of ``block`` = (rows, cols) cells, each solved exactly:
    scheme "ix" iterates on I+X, "imx_ix" on (I-X)(I+X).
    Returns (q float64 or None, counts or None, iterations until exact)."""
    schemes = {"ix": SCHEME_IX, "imx_ix": SCHEME_IMX_IX}
    if scheme not in schemes:
        raise ValueError(f"unknown scheme {scheme!r}")
    sch = schemes[scheme]
    _check_grid(code, torch.uint8, "code")
    nr, nc = code.shape
    dev = code.device
    r = _rule(rule)
    rdt = F32
    if rain is not None:
        if rain.dtype not in (torch.float32, torch.float64):
            raise TypeError("rain must be float32 or float64")
        _check_grid(rain, rain.dtype, "rain")
        rdt = _dtype_code(rain.dtype)
    if dtype not in (None, torch.float64):
        raise TypeError("block iterations compute float64 water (or counts only)")
    dt = _dtype_code(dtype)
    q = None if dtype is None else torch.empty((nr, nc), dtype=dtype, device=dev)
    cnt = torch.empty((nr, nc), dtype=torch.uint64, device=dev) if counts else None
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = workspace_bytes(FN_BLOCK_ITER if sch == SCHEME_IX else FN_BLOCK_ITER_PRE, nr, nc, r, dt)
    buf = (ws or _default_ws).get(nbytes, dev)
    iters = ctypes.c_int32(0)
    rc = load_library().fr_accumulate_block_iterations(None, _ptr(code), nr, nc, r, 0.0, int(block[0]),
                                                       int(block[1]), sch, _ptr(rain), rdt, dt, _ptr(q),
                                                       _ptr(cnt), int(max_iter), ctypes.byref(iters),
                                                       _ptr(status), _ptr(buf), buf.numel(), _stream(dev))
    if rc != OK:
        raise FlowRouteError(rc, "fr_accumulate_block_iterations")
    if check:
        _raise_status(status, "fr_accumulate_block_iterations")
    return q, cnt, iters.value


def fill_depressions(z: torch.Tensor, rule="d8", eps: bool = True, ws: Workspace | None = None,
                     check: bool = True, launches: bool = False):
    """Depression filling (``fr_fill_depressions``): the priority-flood
    surface, with one float32 step per cell crossed when ``eps`` so that the
    rule routes every cell to the boundary.  Returns the filled float32
    grid (and the number of tile launches when ``launches``)."""
    _check_grid(z, torch.float32, "z")
    nr, nc = z.shape
    dev = z.device
    r = _rule(rule)
    f = torch.empty_like(z)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = workspace_bytes(FN_FILL, nr, nc, r, F32)
    buf = (ws or _default_ws).get(nbytes, dev)
    n = ctypes.c_int32(0)
    rc = load_library().fr_fill_depressions(_ptr(z), nr, nc, r, int(bool(eps)), _ptr(f), ctypes.byref(n),
                                            _ptr(status), _ptr(buf), buf.numel(), _stream(dev))
    if rc != OK:
        raise FlowRouteError(rc, "fr_fill_depressions")
    if check:
        _raise_status(status, "fr_fill_depressions")
    return (f, n.value) if launches else f


def route(z: torch.Tensor, rain: torch.Tensor | None = None, rule="d8", dtype=torch.float32,
          counts: bool = False, mass: bool = False, p: float = 1.1):
    """Receivers + accumulation.  Returns (code, q, counts, mass)."""
    code = receivers(z, rule)
    zz = z if _rule(rule) == MFD else None
    q, cnt, m = accumulate(code, zz, rain, rule, dtype, counts, mass, p)
    return code, q, cnt, m


class FlowAccumulate(torch.autograd.Function):
    """q = A^{-1} r with A = I - W^T; backward gives dL/dr = A^{-T} dL/dq.

    ``rain`` float32 uses float-float accumulation with float32 output,
    float64 uses the float64 path.  The gradient with respect to the
    elevations is not defined here (routing is piecewise constant in z) and is
    returned as None.
    """

    @staticmethod
    def forward(ctx, rain, z, rule="mfd", p=1.1):
        code = receivers(z, rule)
        zz = z if _rule(rule) == MFD else None
        q, _, _ = accumulate(code, zz, rain.contiguous(), rule, rain.dtype, p=p)
        ctx.save_for_backward(code, z)
        ctx.rule, ctx.p = rule, p
        return q

    @staticmethod
    def backward(ctx, gq):
        code, z = ctx.saved_tensors
        zz = z if _rule(ctx.rule) == MFD else None
        rbar = adjoint(code, gq.contiguous(), zz, ctx.rule, ctx.p)
        return rbar, None, None, None


def set_autotune_cache(path: str | None) -> None:
    """File that keeps autotuned batch plans across processes (or None)."""
    rc = load_library().fr_set_autotune_cache(None if path is None else os.fsencode(path))
    if rc != OK:
        raise FlowRouteError(rc, "fr_set_autotune_cache")


class Batch:
    """A batch of independent tiles routed by one persistent launch
    (``fr_accumulate_batched``).  Each tile is given as its elevation tensor,
    rule, optional float32 rain, and the outputs to fill: ``q`` (float32 water,
    required for MFD) or ``counts`` (uint64 drainage counts, D8/D4).  The batch
    keeps the device copy of the tile table and the workspace, so it can be
    routed repeatedly (and captured in a HIP graph)."""

    def __init__(self, tiles, device=None):
        self.tiles = []
        arr = (Tile * max(len(tiles), 1))()
        for i, t in enumerate(tiles):
            z = t["z"]
            _check_grid(z, torch.float32, "z")
            rule = _rule(t.get("rule", "d8"))
            rain, q, cnt, code = t.get("rain"), t.get("q"), t.get("counts"), t.get("code")
            for name, x, dt in [("rain", rain, torch.float32), ("q", q, torch.float32), ("counts", cnt, torch.int64),
                                ("code", code, torch.uint8)]:
                if x is not None:
                    _check_grid(x, dt if name != "counts" else x.dtype, name)
                    if x.shape != z.shape:
                        raise ValueError(f"{name} shape differs from z")
                    if name == "counts" and x.dtype not in (torch.int64, torch.uint64):
                        raise TypeError("counts must be 64-bit integers")
            arr[i] = Tile(z.data_ptr(), rain.data_ptr() if rain is not None else None,
                          q.data_ptr() if q is not None else None, cnt.data_ptr() if cnt is not None else None,
                          code.data_ptr() if code is not None else None, z.shape[0], z.shape[1], rule, 0)
            self.tiles.append(t)
        self.n = len(tiles)
        self.device = device if device is not None else (tiles[0]["z"].device if tiles else torch.device("cuda"))
        lib = load_library()
        self.ws_bytes = int(lib.fr_batched_workspace_bytes(ctypes.addressof(arr), self.n))
        if self.n and self.ws_bytes == 0:
            raise FlowRouteError(ERR_ARG, "fr_batched_workspace_bytes")
        raw = bytes(memoryview(arr).cast("B"))[: ctypes.sizeof(Tile) * self.n]
        self.table = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device) if self.n else None
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.plan = None

    def run(self, check: bool = True, plan=None):
        """Enqueue the routing of every tile on the current stream."""
        if check:
            self.status.zero_()
        p = plan if plan is not None else self.plan
        rc = load_library().fr_accumulate_batched(
            _ptr(self.table), self.n, ctypes.byref(p) if p is not None else None, _ptr(self.status),
            _ptr(self.ws), self.ws_bytes, _stream(self.device))
        if rc != OK:
            raise FlowRouteError(rc, "fr_accumulate_batched")
        if check:
            _raise_status(self.status, "fr_accumulate_batched")

    def autotune(self, reps: int = 2) -> BatchPlan:
        """Pick the fastest schedule among the library's candidates (cached by
        the batch's shape signature; see ``set_autotune_cache``)."""
        plan = BatchPlan()
        self.status.zero_()
        rc = load_library().fr_batch_autotune(_ptr(self.table), self.n, _ptr(self.status), _ptr(self.ws),
                                              self.ws_bytes, reps, ctypes.byref(plan), _stream(self.device))
        if rc != OK:
            raise FlowRouteError(rc, "fr_batch_autotune")
        _raise_status(self.status, "fr_batch_autotune")
        self.plan = plan
        return plan
