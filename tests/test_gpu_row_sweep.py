"""The MFD row sweep (forward and adjoint) against the float64 oracle.

The row sweep serves an MFD call when no cell sends water into the row
before it in one of the two row orders.  Each strip of 32 columns is
computed with 16 ghost columns on each side; ghost columns are refreshed
from the neighbouring strip when values of unknown origin would reach the
owned columns.  These cases stress that exchange: many strips, ragged
widths, both row orientations, and same-row ramps longer than a strip, which
make a strip take the neighbour's values of the current row.  Every case is
also run with the general wavefront sweep forced, and the two must agree
with the oracle to the same bounds.
"""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nz = b != 0
    return float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) if nz.any() else 0.0


def relnorm(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def terrain(kind, nr, nc, seed):
    """float32 DEMs whose MFD masks send nothing against one row order."""
    rr, cc = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    noise = synth.uniform(seed, synth.STREAM_NOISE, nr * nc).reshape(nr, nc) * 1e-3
    # The benchmark's fractal, with a tilt steep enough for grids this small
    # (at 16384^2 the tilt of 0.01 already dominates the per-cell relief).
    if kind == "fractal":
        return synth.dem(seed, nr, nc, tilt=0.2)
    if kind == "fractal_flipped":
        return np.ascontiguousarray(synth.dem(seed, nr, nc, tilt=0.2)[::-1])
    if kind == "ramps":
        # Same-row ramps 150 columns long (longer than a strip and its ghost
        # columns), alternating direction, over a row tilt that dominates
        # every same-row drop.
        ramp = np.where((cc // 150) % 2 == 0, cc % 150, 149 - cc % 150) * 2e-5
        return (0.05 * rr + ramp + noise * 1e-3).astype(np.float32)
    if kind == "valleys":
        # Valleys 40 columns apart across the tilt: long same-row chains
        # toward each valley floor, both directions.
        v = np.abs(((cc + 7) % 40) - 20) * 1e-3
        return (0.03 * rr + v + noise).astype(np.float32)
    raise ValueError(kind)


CASES = [
    ("fractal", 150, 2000, 21),
    ("fractal_flipped", 150, 2000, 22),
    ("fractal", 64, 33, 23),
    ("fractal", 1, 1, 24),
    ("fractal", 1, 100, 25),
    ("fractal", 90, 1, 26),
    ("fractal", 2, 65, 27),
    ("fractal", 333, 257, 28),
    ("ramps", 120, 1000, 29),
    ("valleys", 200, 700, 30),
]


def _applicable(z):
    """True when the MFD masks send nothing against one row order (the row
    sweep then serves the call)."""
    nr = z.shape[0]
    if nr < 2:
        return True
    up = (z[:-1, :] < z[1:, :]).any() or (z[:-1, 1:] < z[1:, :-1]).any() or (z[:-1, :-1] < z[1:, 1:]).any()
    dn = (z[1:, :] < z[:-1, :]).any() or (z[1:, 1:] < z[:-1, :-1]).any() or (z[1:, :-1] < z[:-1, 1:]).any()
    return not (up and dn)


@pytest.mark.parametrize("path", ["auto", "sweep"])
@pytest.mark.parametrize("kind,nr,nc,seed", CASES)
def test_row_sweep_forward(kind, nr, nc, seed, path):
    print(f"row sweep forward {kind} {nr}x{nc} {path}", flush=True)
    z = terrain(kind, nr, nc, seed)
    assert _applicable(z)
    rain = synth.rain(seed, nr, nc)
    zt = dev(z)
    code = fr.receivers(zt, "mfd")
    qref = oracle.accumulate_mfd(z, rain, 1.1)
    with fr.accumulate_path(path):
        q32, _, m32 = fr.accumulate(code, zt, dev(rain), "mfd", torch.float32, mass=True)
        q64, _, m64 = fr.accumulate(code, zt, dev(rain), "mfd", torch.float64, mass=True)
        qu, _, _ = fr.accumulate(code, zt, None, "mfd", torch.float64)
        # The automatic choice takes the row sweep here; the forced wavefront
        # sweep finishes the call itself (or hands it to the engine).
        served = fr.served_by()
        assert served == "row_sweep" if path == "auto" else served in ("sweep", "engine")
    e32, e64 = relmax(host(q32), qref), relmax(host(q64), qref)
    print(f"  e_max32={e32:.2e} e_norm32={relnorm(host(q32), qref):.2e} e_max64={e64:.2e}", flush=True)
    assert e32 <= 1e-6
    assert e64 <= 1e-10
    assert relmax(host(qu), oracle.accumulate_mfd(z, None, 1.1)) <= 1e-10
    s, t = host(m64)
    assert abs(s - t) <= 1e-11 * t
    s, t = host(m32)
    assert abs(s - t) <= 1e-6 * t
    assert t == pytest.approx(float(rain.astype(np.float64).sum()), rel=1e-12)


@pytest.mark.parametrize("path", ["auto", "sweep"])
@pytest.mark.parametrize("kind,nr,nc,seed", CASES)
def test_row_sweep_adjoint(kind, nr, nc, seed, path):
    print(f"row sweep adjoint {kind} {nr}x{nc} {path}", flush=True)
    z = terrain(kind, nr, nc, seed)
    zt = dev(z)
    code = fr.receivers(zt, "mfd")
    qbar = synth.normal(seed, synth.STREAM_NORMAL, nr * nc).reshape(nr, nc)
    ref = oracle.adjoint_mfd(z, qbar, 1.1)
    with fr.accumulate_path(path):
        r64 = host(fr.adjoint(code, dev(qbar), zt, "mfd"))
        r32 = host(fr.adjoint(code, dev(qbar.astype(np.float32)), zt, "mfd"))
    ref32 = oracle.adjoint_mfd(z, qbar.astype(np.float32).astype(np.float64), 1.1)
    scale = np.abs(ref).max()
    print(f"  e64={np.max(np.abs(r64 - ref)) / scale:.2e} e32={relnorm(r32, ref32):.2e}", flush=True)
    assert np.max(np.abs(r64 - ref)) <= 1e-10 * scale
    assert relnorm(r32, ref32) <= 1e-6


def test_row_sweep_bits_repeat():
    """Which ghost columns are refreshed, and from what, depends only on the
    data: two routes give the same bits."""
    z = terrain("valleys", 400, 3000, 31)
    rain = synth.rain(31, 400, 3000)
    zt, rt = dev(z), dev(rain)
    code = fr.receivers(zt, "mfd")
    outs = []
    for _ in range(3):
        q, _, m = fr.accumulate(code, zt, rt, "mfd", torch.float32, mass=True)
        torch.cuda.synchronize()
        outs.append((q, m))
    for q, m in outs[1:]:
        assert torch.equal(q.view(torch.int32), outs[0][0].view(torch.int32))
        assert torch.equal(m.view(torch.int64), outs[0][1].view(torch.int64))


def test_row_sweep_declines_two_way_flow():
    """Terrain that drains both up and down the rows: the general sweep
    serves the call, with the same result bounds."""
    nr, nc = 200, 300
    rr, cc = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    noise = synth.uniform(32, synth.STREAM_NOISE, nr * nc).reshape(nr, nc) * 1e-3
    z = (1e-4 * (rr - 100) ** 2 + noise).astype(np.float32)
    assert not _applicable(z)
    rain = synth.rain(32, nr, nc)
    zt = dev(z)
    code = fr.receivers(zt, "mfd")
    q64, _, _ = fr.accumulate(code, zt, dev(rain), "mfd", torch.float64)
    assert fr.served_by() in ("sweep", "engine")
    assert relmax(host(q64), oracle.accumulate_mfd(z, rain, 1.1)) <= 1e-10


@pytest.mark.parametrize("path", ["auto", "sweep"])
def test_row_sweep_reports_bad_masks_and_nonfinite(path):
    """Invalid inputs give the same device errors on the row sweep as on
    the general sweep: a receiver that is not lower or lies off the grid
    (FR_ERR_BADCODE), a non-finite elevation or rain (FR_ERR_NONFINITE)."""
    nr, nc = 100, 300
    z = terrain("fractal", nr, nc, 33)
    assert _applicable(z)
    zt = dev(z)
    code = host(fr.receivers(zt, "mfd"))
    r = 50
    j = next(j for j in range(1, nc - 1) if z[r, j + 1] > z[r, j])
    cases = []
    c = code.copy()
    c[r, j] |= 1 << 4  # the higher right neighbour claimed as a receiver
    cases.append(("higher receiver", c, z, None, fr.ERR_BADCODE))
    c = code.copy()
    c[10, 0] |= 1 << 3  # a receiver left of column 0
    cases.append(("off the grid", c, z, None, fr.ERR_BADCODE))
    rain = synth.rain(33, nr, nc)
    rain[20, 30] = np.nan
    cases.append(("nan rain", code, z, rain, fr.ERR_NONFINITE))
    # A cell no neighbour sends to (a same-row peak in the highest row), so
    # that the infinite elevation is the only error.
    top = nr - 1
    k = next(k for k in range(1, nc - 1) if z[top, k] > z[top, k - 1] and z[top, k] > z[top, k + 1])
    z2 = z.copy()
    z2[top, k] = np.inf
    cases.append(("inf elevation", code, z2, None, fr.ERR_NONFINITE))
    with fr.accumulate_path(path):
        for name, c, zz, rr, err in cases:
            print(f"  {path}: {name}", flush=True)
            with pytest.raises(fr.FlowRouteError) as e:
                fr.accumulate(dev(c), dev(zz), None if rr is None else dev(rr), "mfd", torch.float64)
            assert e.value.code == err, name
