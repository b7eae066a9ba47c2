"""C-ABI checks that need no GPU: the library loads, exports every symbol its
header declares, and rejects bad arguments on the host before any device
work is enqueued."""
import ctypes
import os
import re

import pytest

import paper_2606_12800_amd as fr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fr_api.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fr.LIB_PATH):
        from paper_2606_12800_amd import _build
        _build.build()
    return fr.load_library()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "fr_receivers" in names and "fr_accumulate" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(fr.EXPORTS) <= set(names)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    consts = dict((m.group(1), int(m.group(2), 0)) for m in
                  re.finditer(r"#define\s+(FR_[A-Z_0-9]+)\s+(-?(?:0x)?[0-9A-Fa-f]+)", text))
    assert consts["FR_D8"] == fr.D8 and consts["FR_MFD"] == fr.MFD and consts["FR_D4"] == fr.D4
    assert consts["FR_F32"] == fr.F32 and consts["FR_F64"] == fr.F64 and consts["FR_NONE"] == fr.NONE
    assert consts["FR_SINK"] == fr.SINK
    for name in ["ARG", "RULE", "WORKSPACE", "HIP", "NONFINITE", "NOTDAG", "BADCODE", "TOOLARGE", "STALL",
                 "CAPACITY"]:
        assert consts[f"FR_ERR_{name}"] == getattr(fr, f"ERR_{name}")
    for name in ["AUTO", "SWEEP", "ENGINE", "TILES"]:
        assert consts[f"FR_PATH_{name}"] == getattr(fr, f"PATH_{name}")
    served = {v: k for k, v in fr.SERVED.items()}
    for name in ["NONE", "ROWS", "TILES", "ROW_SWEEP", "SWEEP", "ENGINE"]:
        assert consts[f"FR_SERVED_{name}"] == served[name.lower()]


def test_status_strings(lib):
    for code in [0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10]:
        s = fr.status_string(code)
        assert s and s != "unknown status"
    assert fr.status_string(12345) == "unknown status"
    assert b"gfx950" in lib.fr_version()


def test_workspace_bytes(lib):
    a = fr.workspace_bytes(fr.FN_ACCUMULATE, 256, 256, fr.D8, fr.F32)
    b = fr.workspace_bytes(fr.FN_ACCUMULATE, 256, 256, fr.D8, fr.NONE)
    c = fr.workspace_bytes(fr.FN_ACCUMULATE, 256, 256, fr.MFD, fr.F32)
    assert a >= b > 0 and c > 0
    assert fr.workspace_bytes(fr.FN_ACCUMULATE, 256, 256, fr.MFD, fr.NONE) == 0
    assert fr.workspace_bytes(fr.FN_ADJOINT, 256, 256, fr.D8, fr.NONE) == 0
    assert fr.workspace_bytes(fr.FN_ADJOINT, 64, 64, fr.MFD, fr.F64) > 0
    assert fr.workspace_bytes(99, 64, 64, fr.D8, fr.F32) == 0
    assert fr.workspace_bytes(fr.FN_ACCUMULATE, -1, 64, fr.D8, fr.F32) == 0
    assert fr.workspace_bytes(fr.FN_ACCUMULATE, 64, 64, 7, fr.F32) == 0
    # too many cells for int32 indices
    assert fr.workspace_bytes(fr.FN_ACCUMULATE, 1 << 16, 1 << 16, fr.D8, fr.F32) == 0
    # grows linearly with the cell count
    big = fr.workspace_bytes(fr.FN_ACCUMULATE, 2048, 2048, fr.D8, fr.F32)
    assert big > 2048 * 2048 * 6


NULL = None
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def test_receivers_validation(lib):
    assert lib.fr_receivers(NULL, -1, 4, fr.D8, FAKE, NULL, NULL) == fr.ERR_ARG
    assert lib.fr_receivers(FAKE, 4, 4, 9, FAKE, NULL, NULL) == fr.ERR_RULE
    assert lib.fr_receivers(NULL, 4, 4, fr.D8, FAKE, NULL, NULL) == fr.ERR_ARG
    assert lib.fr_receivers(FAKE, 4, 4, fr.D8, NULL, NULL, NULL) == fr.ERR_ARG
    assert lib.fr_receivers(NULL, 0, 5, fr.D8, NULL, NULL, NULL) == fr.OK  # empty grid: no-op
    assert lib.fr_receivers(FAKE, 1 << 16, 1 << 16, fr.D8, FAKE, NULL, NULL) == fr.ERR_TOOLARGE


# Distinct fake buffers (an 8 x 8 grid's largest array is 512 bytes); the
# workspace's 2^40 bytes lie above all of them.
Z, CODE, RAIN, Q, CNT, MASS, WS = (ctypes.c_void_p(a) for a in
                                   (0x10000, 0x20000, 0x30000, 0x40000, 0x50000, 0x60000, 1 << 44))


def _acc(lib, z=Z, code=CODE, nr=8, nc=8, rule=fr.D8, p=1.1, rain=NULL, rdt=fr.F32, qdt=fr.F32,
         q=Q, cnt=NULL, mass=NULL, ws=WS, wsb=1 << 40):
    return lib.fr_accumulate(z, code, nr, nc, rule, p, rain, rdt, qdt, q, cnt, mass, NULL, ws, wsb, NULL)


def test_accumulate_validation(lib):
    assert _acc(lib, nr=-1) == fr.ERR_ARG
    assert _acc(lib, rule=5) == fr.ERR_RULE
    assert _acc(lib, qdt=7) == fr.ERR_ARG
    assert _acc(lib, qdt=fr.NONE) == fr.ERR_ARG            # q_out given but no dtype
    assert _acc(lib, q=NULL) == fr.ERR_ARG                  # dtype given but no q_out
    assert _acc(lib, qdt=fr.NONE, q=NULL, cnt=NULL) == fr.ERR_ARG  # nothing to compute
    assert _acc(lib, qdt=fr.NONE, q=NULL, cnt=FAKE, mass=FAKE) == fr.ERR_ARG
    assert _acc(lib, rule=fr.MFD, cnt=FAKE) == fr.ERR_RULE  # counts are single-receiver only
    assert _acc(lib, rule=fr.MFD, qdt=fr.NONE, q=NULL) == fr.ERR_RULE
    assert _acc(lib, rule=fr.MFD, p=0.0) == fr.ERR_ARG
    assert _acc(lib, rule=fr.MFD, p=float("nan")) == fr.ERR_ARG
    assert _acc(lib, rule=fr.MFD, z=NULL) == fr.ERR_ARG
    assert _acc(lib, code=NULL) == fr.ERR_ARG
    assert _acc(lib, rain=FAKE, rdt=3) == fr.ERR_ARG
    assert _acc(lib, ws=NULL) == fr.ERR_WORKSPACE
    need = fr.workspace_bytes(fr.FN_ACCUMULATE, 8, 8, fr.D8, fr.F32)
    assert _acc(lib, wsb=need - 1) == fr.ERR_WORKSPACE
    assert _acc(lib, nr=1 << 16, nc=1 << 16) == fr.ERR_TOOLARGE
    assert _acc(lib, nr=0, q=NULL, code=NULL, ws=NULL) == fr.OK  # empty grid: no-op
    # Outputs overlapping an input, the workspace or one another.
    assert _acc(lib, rain=Q) == fr.ERR_ARG                                    # in place over rain
    assert _acc(lib, rain=ctypes.c_void_p(0x40000 - 255)) == fr.ERR_ARG       # rain's last byte under q
    assert _acc(lib, q=CODE) == fr.ERR_ARG
    assert _acc(lib, q=Z, rule=fr.MFD) == fr.ERR_ARG
    assert _acc(lib, cnt=ctypes.c_void_p(0x40000 + 128)) == fr.ERR_ARG        # counts inside q
    assert _acc(lib, mass=ctypes.c_void_p(0x40000 + 252)) == fr.ERR_ARG       # mass over q's last word
    assert _acc(lib, q=ctypes.c_void_p((1 << 44) + 4096)) == fr.ERR_ARG       # q inside the workspace
    # Adjacent buffers are fine: validation goes on to the next check.
    assert _acc(lib, rain=ctypes.c_void_p(0x40000 - 256), ws=NULL) == fr.ERR_WORKSPACE
    assert _acc(lib, cnt=ctypes.c_void_p(0x40000 + 256), ws=NULL) == fr.ERR_WORKSPACE


def test_adjoint_validation(lib):
    def adj(z=FAKE, code=FAKE, nr=8, nc=8, rule=fr.D8, p=1.1, qb=FAKE, dt=fr.F32, rb=FAKE, ws=FAKE,
            wsb=1 << 40):
        return lib.fr_accumulate_adjoint(z, code, nr, nc, rule, p, qb, dt, rb, NULL, ws, wsb, NULL)
    assert adj(nr=-3) == fr.ERR_ARG
    assert adj(rule=4) == fr.ERR_RULE
    assert adj(dt=fr.NONE) == fr.ERR_ARG
    assert adj(qb=NULL) == fr.ERR_ARG
    assert adj(rb=NULL) == fr.ERR_ARG
    assert adj(rule=fr.MFD, z=NULL) == fr.ERR_ARG
    assert adj(rule=fr.MFD, p=-1.0) == fr.ERR_ARG
    assert adj(ws=NULL) == fr.ERR_WORKSPACE
    assert adj(nr=0) == fr.OK


def test_block_iterations_validation(lib):
    it = ctypes.c_int32(7)

    def bi(code=FAKE, nr=8, nc=8, rule=fr.D8, scheme=fr.SCHEME_IX, rain=NULL, rdt=fr.F32, qdt=fr.F64, q=FAKE,
           cnt=FAKE, max_iter=10, iters=ctypes.byref(it), ws=FAKE, wsb=1 << 40, br=256, bc=256):
        return lib.fr_accumulate_block_iterations(NULL, code, nr, nc, rule, 0.0, br, bc, scheme, rain, rdt, qdt, q,
                                                  cnt, max_iter, iters, NULL, ws, wsb, NULL)
    assert bi(nr=-1) == fr.ERR_ARG
    assert bi(br=0) == fr.ERR_ARG and bi(bc=-3) == fr.ERR_ARG
    assert bi(nr=600, nc=600, br=100) == fr.ERR_ARG          # block rows: a multiple of 16
    assert bi(nr=600, nc=600, bc=300) == fr.ERR_ARG          # block cols: a multiple of 256
    assert bi(iters=NULL) == fr.ERR_ARG
    assert bi(max_iter=0) == fr.ERR_ARG
    assert bi(rule=fr.MFD) == fr.ERR_RULE
    assert bi(scheme=2) == fr.ERR_ARG
    assert bi(rain=FAKE, rdt=fr.NONE) == fr.ERR_ARG
    assert bi(qdt=fr.F32) == fr.ERR_ARG                      # float64 water or counts only
    assert bi(q=NULL) == fr.ERR_ARG                          # dtype given but no q_out
    assert bi(qdt=fr.NONE, q=NULL, cnt=NULL) == fr.ERR_ARG   # nothing to compute
    assert bi(scheme=fr.SCHEME_IMX_IX, cnt=NULL) == fr.ERR_ARG  # converges on the counts
    assert bi(code=NULL) == fr.ERR_ARG
    assert bi(ws=NULL) == fr.ERR_WORKSPACE
    need = fr.workspace_bytes(fr.FN_BLOCK_ITER_PRE, 8, 8, fr.D8, fr.F64)
    assert bi(scheme=fr.SCHEME_IMX_IX, wsb=need - 1) == fr.ERR_WORKSPACE
    assert bi(nr=1 << 16, nc=1 << 16) == fr.ERR_TOOLARGE
    it.value = 7
    assert bi(nr=0, code=NULL, ws=NULL) == fr.OK and it.value == 0  # empty grid: no-op


def test_accumulate_path_selection(lib):
    assert lib.fr_set_accumulate_path(4) == fr.ERR_ARG
    assert lib.fr_set_accumulate_path(-1) == fr.ERR_ARG
    for p in (fr.PATH_ENGINE, fr.PATH_SWEEP, fr.PATH_TILES, fr.PATH_AUTO):
        assert lib.fr_set_accumulate_path(p) == fr.OK
    with fr.accumulate_path("engine"):
        pass  # restores the default on exit


def test_served_by_validation(lib):
    out = ctypes.c_int32(7)
    assert lib.fr_served_by(NULL, 1 << 20, ctypes.byref(out), NULL) == fr.ERR_ARG
    assert lib.fr_served_by(FAKE, 1 << 20, None, NULL) == fr.ERR_ARG
    assert lib.fr_served_by(FAKE, 256, ctypes.byref(out), NULL) == fr.ERR_ARG  # below one control block
    assert out.value == 7


def test_fill_validation(lib):
    n = ctypes.c_int32(5)

    def fill(z=FAKE, nr=8, nc=8, rule=fr.D8, eps=1, out=ctypes.c_void_p(0x2000), ws=FAKE, wsb=1 << 40):
        return lib.fr_fill_depressions(z, nr, nc, rule, eps, out, ctypes.byref(n), NULL, ws, wsb, NULL)
    assert fill(nr=-2) == fr.ERR_ARG
    assert fill(eps=2) == fr.ERR_ARG
    assert fill(rule=9) == fr.ERR_RULE
    assert fill(z=NULL) == fr.ERR_ARG
    assert fill(out=NULL) == fr.ERR_ARG
    assert fill(out=FAKE) == fr.ERR_ARG  # output aliases the elevations
    assert fill(ws=NULL) == fr.ERR_WORKSPACE
    assert fill(wsb=fr.workspace_bytes(fr.FN_FILL, 8, 8, fr.D8, fr.F32) - 1) == fr.ERR_WORKSPACE
    assert fill(nr=1 << 16, nc=1 << 16) == fr.ERR_TOOLARGE
    n.value = 5
    assert fill(nr=0, z=NULL, out=NULL, ws=NULL) == fr.OK and n.value == 0


def test_workspace_bytes_next_rows():
    a = fr.workspace_bytes(fr.FN_BLOCK_ITER, 300, 500, fr.D8, fr.F64)
    b = fr.workspace_bytes(fr.FN_BLOCK_ITER_PRE, 300, 500, fr.D8, fr.F64)
    assert a >= 300 * 500 * 16 and b >= 3 * 300 * 500 * 16
    assert fr.workspace_bytes(fr.FN_BLOCK_ITER, 300, 500, fr.MFD, fr.F64) == 0
    assert fr.workspace_bytes(fr.FN_BLOCK_ITER, 300, 500, fr.D8, fr.F32) == 0
    f = fr.workspace_bytes(fr.FN_FILL, 300, 500, fr.D4, fr.F32)
    tiles = ((300 + 61) // 62) * ((500 + 61) // 62)
    assert f >= 4 * (4 * tiles + 4)
    assert fr.workspace_bytes(fr.FN_FILL, 300, 500, fr.D8, fr.F64) == 0


def test_scheme_and_fn_constants_match_binding():
    text = open(HEADER).read()
    consts = dict((m.group(1), int(m.group(2), 0)) for m in
                  re.finditer(r"#define\s+(FR_[A-Z_0-9]+)\s+(-?(?:0x)?[0-9A-Fa-f]+)", text))
    assert consts["FR_SCHEME_IX"] == fr.SCHEME_IX and consts["FR_SCHEME_IMX_IX"] == fr.SCHEME_IMX_IX
    assert consts["FR_FN_BLOCK_ITER"] == fr.FN_BLOCK_ITER and consts["FR_FN_BLOCK_ITER_PRE"] == fr.FN_BLOCK_ITER_PRE
    assert consts["FR_FN_FILL"] == fr.FN_FILL
