"""fr_accumulate_noalloc: the accumulation entry point for callers that
cannot allocate (its scratch is a fixed array inside the library).  Called
through the C ABI twice in a row -- a D8 grid with float32 rain, counts and
mass, then a smaller MFD grid -- each result compared bit for bit with
fr_accumulate on a caller workspace (both are deterministic), the D8 counts
also with the oracle; a grid whose workspace exceeds the array is refused.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2606_12800_amd")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fr.load_library()
    yield


def P(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def noalloc(code, z, rain, rule, dtype, counts, mass):
    nr, nc = code.shape
    dev = code.device
    q = torch.empty((nr, nc), dtype=dtype, device=dev)
    cnt = torch.empty((nr, nc), dtype=torch.uint64, device=dev) if counts else None
    m = torch.empty(2, dtype=torch.float64, device=dev) if mass else None
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    rdt = fr.F32 if rain is None else fr._dtype_code(rain.dtype)
    rc = fr.load_library().fr_accumulate_noalloc(P(z), P(code), nr, nc, fr.RULES[rule], 1.1, P(rain), rdt,
                                                 fr._dtype_code(dtype), P(q), P(cnt), P(m), P(status),
                                                 fr._stream(dev))
    assert rc == fr.OK, fr.status_string(rc)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return q, cnt, m


def test_noalloc_two_calls_match_workspace_calls():
    # First call: D8, float32 rain, counts and mass.
    nr, nc = 900, 1100
    z_h = synth.dem(91, nr, nc)
    rain_h = synth.rain(91, nr, nc)
    z, rain = torch.from_numpy(z_h).cuda(), torch.from_numpy(rain_h).cuda()
    code = fr.receivers(z, "d8")
    q, cnt, m = noalloc(code, None, rain, "d8", torch.float32, True, True)
    q2, cnt2, m2 = fr.accumulate(code, None, rain, "d8", torch.float32, counts=True, mass=True)
    torch.cuda.synchronize()
    assert torch.equal(q.view(torch.int32), q2.view(torch.int32))
    assert torch.equal(cnt, cnt2)
    assert torch.equal(m.view(torch.int64), m2.view(torch.int64))
    _, cref = oracle.accumulate_single(oracle.receivers(z_h), None, z=z_h)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint64), cref)
    # Second call, smaller: MFD float32 (the array keeps the first call's
    # contents; the call clears what it needs).
    nr, nc = 260, 333
    z_h = synth.dem(92, nr, nc)
    z = torch.from_numpy(z_h).cuda()
    code = fr.receivers(z, "mfd")
    q, _, m = noalloc(code, z, None, "mfd", torch.float32, False, True)
    q2, _, m2 = fr.accumulate(code, z, None, "mfd", torch.float32, mass=True)
    torch.cuda.synchronize()
    assert torch.equal(q.view(torch.int32), q2.view(torch.int32))
    assert torch.equal(m.view(torch.int64), m2.view(torch.int64))
    qref = oracle.accumulate_mfd(z_h, None, 1.1)
    assert np.linalg.norm(q.cpu().numpy() - qref) / np.linalg.norm(qref) <= 1e-6


def test_noalloc_refuses_grids_beyond_its_array():
    lib = fr.load_library()
    nr = nc = 8192  # D8 with counts: well over the array's size
    need = fr.workspace_bytes(fr.FN_ACCUMULATE, nr, nc, fr.D8, fr.F32)
    assert need > (256 << 20)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the call is refused first
    rc = lib.fr_accumulate_noalloc(None, fake, nr, nc, fr.D8, 1.1, None, fr.F32, fr.F32, fake, fake, None, None,
                                   None)
    assert rc == fr.ERR_TOOLARGE
    # Argument errors as fr_accumulate; an empty grid is a no-op.
    assert lib.fr_accumulate_noalloc(None, fake, 8, 8, 7, 1.1, None, fr.F32, fr.F32, fake, None, None, None,
                                     None) == fr.ERR_RULE
    assert lib.fr_accumulate_noalloc(None, None, 0, 8, fr.D8, 1.1, None, fr.F32, fr.F32, None, None, None, None,
                                     None) == fr.OK
