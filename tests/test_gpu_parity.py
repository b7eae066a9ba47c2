"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.

Bars (integer work bit-exact, floating point within stated tolerances):
  * receivers (D8/D4 codes, MFD masks): bit-exact;
  * D8/D4 uint64 counts: bit-exact;
  * float32 (float-float) water: max relative error <= 1e-6 per cell (D8),
    ||q - q*||_2 / ||q*||_2 <= 1e-6 (MFD), both against the float64 oracle;
  * float64 water: max relative error <= 1e-10 per cell;
  * mass balance: float64 path <= 1e-11 relative (the paper's figure,
    Section 4), float32 path <= 1e-6;
  * adjoint: same bars against the oracle's transpose solve.
Sizes span several 32 x 64 engine tiles and ragged tails.
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
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    b = np.asarray(b, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    nz = b != 0
    return float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) if nz.any() else 0.0


def relnorm(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_ACC_PATH = {"rows": "auto", "sweep": "sweep", "engine": "engine", "tiles": "tiles"}


@pytest.fixture(params=["rows", "sweep", "engine", "tiles"])
def d8path(request):
    """Single-receiver forward accumulation has four GPU paths: row sweeps
    with an exit forest (default), the tile forest (where the row sweeps'
    exit list overflows), the windowed wavefront sweep and the peeling
    engine (the fallback of the sweeps)."""
    with fr.accumulate_path(_ACC_PATH[request.param]):
        yield request.param


_SERVED = {"rows": "rows", "tiles": "tiles", "engine": "engine"}


def check_served(d8path):
    """The chosen single-receiver path served the last forward call (the
    wavefront sweep may hand over to the engine)."""
    got = fr.served_by()
    if d8path == "sweep":
        assert got in ("sweep", "engine")
    else:
        assert got == _SERVED[d8path]


@pytest.fixture(params=["rows", "sweep", "engine"])
def accpath(request):
    """MFD and adjoint accumulation: the automatic choice (the row sweep
    where no cell sends against a row order, else the wavefront sweep), the
    wavefront sweep forced, or the peeling engine."""
    with fr.accumulate_path(_ACC_PATH[request.param]):
        yield request.param


SHAPES = [(256, 256, 1), (97, 131, 7), (1, 1, 8), (1, 300, 9), (300, 1, 10), (64, 64, 11),
          (200, 1030, 12), (513, 777, 2)]


# ---------------------------------------------------------------------------
# Receivers


@pytest.mark.parametrize("nr,nc,seed", SHAPES)
@pytest.mark.parametrize("rule", ["d8", "d4", "mfd"])
def test_receivers_bitexact(nr, nc, seed, rule):
    print(f"receivers {rule} {nr}x{nc} seed {seed}", flush=True)
    z = synth.dem(seed, nr, nc)
    code = host(fr.receivers(dev(z), rule))
    if rule == "mfd":
        ref, _ = oracle.mfd_fractions(z)
    else:
        ref = oracle.receivers(z, oracle.D8 if rule == "d8" else oracle.D4)
    assert np.array_equal(code, ref)


@pytest.mark.parametrize("rule", ["d8", "d4", "mfd"])
def test_receivers_ties_plateaus_integer_dem(rule):
    vals = synth.integers(77, synth.STREAM_PICK, 150 * 203, 0, 12).reshape(150, 203)
    z = vals.astype(np.float32)
    z[40:60, 50:90] = 5.0  # plateau
    code = host(fr.receivers(dev(z), rule))
    if rule == "mfd":
        ref, _ = oracle.mfd_fractions(z)
    else:
        ref = oracle.receivers(z, oracle.D8 if rule == "d8" else oracle.D4)
    assert np.array_equal(code, ref)


def test_receivers_unaligned_width_and_flat():
    for nr, nc in [(33, 65), (5, 1027), (70, 3)]:
        z = synth.dem(3, nr, nc)
        assert np.array_equal(host(fr.receivers(dev(z), "d8")), oracle.receivers(z))
    flat = np.zeros((40, 70), dtype=np.float32)
    assert (host(fr.receivers(dev(flat), "d8")) == 0xFF).all()
    assert (host(fr.receivers(dev(flat), "mfd")) == 0).all()


# ---------------------------------------------------------------------------
# D8 / D4 accumulation


@pytest.mark.parametrize("nr,nc,seed", SHAPES)
@pytest.mark.parametrize("rule", ["d8", "d4"])
def test_counts_bitexact(nr, nc, seed, rule, d8path):
    print(f"counts {rule} {nr}x{nc} seed {seed}", flush=True)
    z = synth.dem(seed, nr, nc)
    code = fr.receivers(dev(z), rule)
    _, cnt, _ = fr.accumulate(code, None, None, rule, dtype=None, counts=True)
    check_served(d8path)
    _, ref = oracle.accumulate_single(host(code), None, z=z, q=False)
    got = host(cnt)
    assert np.array_equal(got, ref)
    assert int(got[host(code) == 0xFF].sum()) == nr * nc


@pytest.mark.parametrize("nr,nc,seed", [(256, 256, 1), (513, 777, 2), (97, 131, 7), (1, 300, 9)])
def test_d8_rain_float32_and_counts(nr, nc, seed, d8path):
    print(f"d8 rain f32 {nr}x{nc} seed {seed}", flush=True)
    z = synth.dem(seed, nr, nc)
    rain = synth.rain(seed, nr, nc)
    code = fr.receivers(dev(z), "d8")
    q, cnt, m = fr.accumulate(code, None, dev(rain), "d8", torch.float32, counts=True, mass=True)
    check_served(d8path)
    qref, cref = oracle.accumulate_single(host(code), rain, z=z)
    assert np.array_equal(host(cnt), cref)
    assert relmax(host(q), qref) <= 1e-6
    s, t = host(m)
    assert abs(s - t) <= 1e-6 * t
    assert t == pytest.approx(float(rain.astype(np.float64).sum()), rel=1e-12)


@pytest.mark.parametrize("nr,nc,seed", [(256, 256, 1), (513, 777, 2), (1, 300, 9), (300, 1, 10)])
def test_d8_float64(nr, nc, seed, d8path):
    z = synth.dem(seed, nr, nc)
    rain = synth.rain(seed, nr, nc)
    code = fr.receivers(dev(z), "d8")
    q, _, m = fr.accumulate(code, None, dev(rain), "d8", torch.float64, mass=True)
    check_served(d8path)
    qref, _ = oracle.accumulate_single(host(code), rain, z=z, counts=False)
    assert relmax(host(q), qref) <= 1e-10
    s, t = host(m)
    assert abs(s - t) <= 1e-11 * t


def test_d8_unit_rain_float32_equals_counts(d8path):
    z = synth.dem(1, 256, 256)
    code = fr.receivers(dev(z), "d8")
    q, cnt, _ = fr.accumulate(code, None, None, "d8", torch.float32, counts=True)
    # counts < 2^24 here, so float32 holds them exactly
    assert np.array_equal(host(q).astype(np.uint64), host(cnt))


@pytest.mark.parametrize("kind", ["rows_up", "cols_left", "cols_right", "diag", "bowl"])
def test_d8_terrain_orientations(kind, d8path):
    """Terrain draining against or across the sweep direction: every edge is
    then cut, so the exit forest carries the whole solve."""
    nr, nc = 300, 270
    rr, cc = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    noise = synth.uniform(9, synth.STREAM_NOISE, nr * nc).reshape(nr, nc) * 1e-3
    base = {"rows_up": -0.01 * rr, "cols_left": 0.01 * cc, "cols_right": -0.01 * cc,
            "diag": 0.01 * (rr + cc), "bowl": 1e-4 * ((rr - 150.5) ** 2 + (cc - 130.5) ** 2)}[kind]
    z = (base + noise).astype(np.float32)
    rain = synth.rain(9, nr, nc)
    code = fr.receivers(dev(z), "d8")
    q, cnt, _ = fr.accumulate(code, None, dev(rain), "d8", torch.float32, counts=True)
    qref, cref = oracle.accumulate_single(host(code), rain, z=z)
    assert np.array_equal(host(cnt), cref)
    assert relmax(host(q), qref) <= 1e-6


def test_d8_exit_list_overflow_takes_the_tile_forest():
    # Flow along rows only: every cell is an exit of the row sweep, more than
    # the exit list holds on a grid above 2^22 cells; the tile forest then
    # serves the call.
    nr, nc = 2100, 2100
    cc = np.arange(nc, dtype=np.float64)[None, :] * np.ones((nr, 1))
    noise = synth.uniform(3, synth.STREAM_NOISE, nr * nc).reshape(nr, nc) * 1e-3
    z = (0.01 * cc + noise).astype(np.float32)
    code = fr.receivers(dev(z), "d8")
    _, cnt, _ = fr.accumulate(code, None, None, "d8", None, counts=True)
    assert fr.served_by() == "tiles"
    _, cref = oracle.accumulate_single(host(code), None, z=z, q=False)
    assert np.array_equal(host(cnt), cref)


# ---------------------------------------------------------------------------
# MFD accumulation


@pytest.mark.parametrize("nr,nc,seed", [(256, 256, 3), (300, 517, 4), (97, 131, 7), (1, 200, 9),
                                        (200, 1, 10), (64, 65, 13), (700, 129, 14)])
def test_mfd_float32_float64(nr, nc, seed, accpath):
    print(f"mfd {nr}x{nc} seed {seed}", flush=True)
    z = synth.dem(seed, nr, nc)
    rain = synth.rain(seed, nr, nc)
    zt = dev(z)
    code = fr.receivers(zt, "mfd")
    qref = oracle.accumulate_mfd(z, rain, 1.1)
    q32, _, m32 = fr.accumulate(code, zt, dev(rain), "mfd", torch.float32, mass=True)
    q64, _, m64 = fr.accumulate(code, zt, dev(rain), "mfd", torch.float64, mass=True)
    q32, q64 = host(q32), host(q64)
    assert relnorm(q32, qref) <= 1e-6
    assert relmax(q64, qref) <= 1e-10
    s, t = host(m64)
    assert abs(s - t) <= 1e-11 * t
    s, t = host(m32)
    assert abs(s - t) <= 1e-6 * t
    print(f"  e_norm32={relnorm(q32, qref):.2e} e_max32={relmax(q32, qref):.2e} "
          f"e_max64={relmax(q64, qref):.2e}")


def test_mfd_unit_rain(accpath):
    z = synth.dem(3, 256, 300)
    zt = dev(z)
    code = fr.receivers(zt, "mfd")
    q, _, _ = fr.accumulate(code, zt, None, "mfd", torch.float64)
    assert relmax(host(q), oracle.accumulate_mfd(z, None, 1.1)) <= 1e-10


def _oriented_terrain(kind, nr, nc, seed):
    rr, cc = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    noise = synth.uniform(seed, synth.STREAM_NOISE, nr * nc).reshape(nr, nc) * 1e-3
    cr, ccen = (nr - 1) / 2 + 0.5, (nc - 1) / 2 + 0.5
    base = {"rows_down": 0.01 * rr, "rows_up": -0.01 * rr, "cols_left": 0.01 * cc,
            "cols_right": -0.01 * cc, "diag": 0.01 * (rr + cc), "antidiag": 0.01 * (rr - cc),
            "bowl": 1e-4 * ((rr - cr) ** 2 + (cc - ccen) ** 2),
            "ridge": -1e-4 * ((rr - cr) ** 2 + (cc - ccen) ** 2)}[kind]
    return (base + noise).astype(np.float32)


@pytest.mark.parametrize("kind", ["rows_down", "rows_up", "cols_left", "cols_right", "diag", "antidiag",
                                  "bowl", "ridge"])
def test_mfd_terrain_orientations(kind, accpath):
    """MFD on terrain draining along, against and across the row order, and
    toward / away from the centre: the sweep needs several passes in both
    directions and long chains across strip boundaries."""
    nr, nc = 190, 333
    print(f"mfd orientation {kind}", flush=True)
    z = _oriented_terrain(kind, nr, nc, 15)
    rain = synth.rain(15, nr, nc)
    zt = dev(z)
    code = fr.receivers(zt, "mfd")
    qref = oracle.accumulate_mfd(z, rain, 1.1)
    q64, _, m64 = fr.accumulate(code, zt, dev(rain), "mfd", torch.float64, mass=True)
    q32, _, _ = fr.accumulate(code, zt, dev(rain), "mfd", torch.float32)
    assert relmax(host(q64), qref) <= 1e-10
    assert relnorm(host(q32), qref) <= 1e-6
    s, t = host(m64)
    assert abs(s - t) <= 1e-11 * t
    qbar = synth.normal(15, synth.STREAM_NORMAL, nr * nc).reshape(nr, nc)
    ref = oracle.adjoint_mfd(z, qbar, 1.1)
    r64 = host(fr.adjoint(code, dev(qbar), zt, "mfd"))
    assert np.max(np.abs(r64 - ref)) <= 1e-10 * np.abs(ref).max()


def test_snake_path_many_passes(d8path):
    """A single river that reverses its row direction in every column: the
    wavefront sweep would need one pass per column, so it hands over to the
    peeling engine; every path must still give count = position + 1."""
    nr, nc = 40, 75
    code = np.empty((nr, nc), dtype=np.uint8)
    pos = np.empty((nr, nc), dtype=np.int64)
    for c in range(nc):
        for r in range(nr):
            down = c % 2 == 0
            last = (r == nr - 1) if down else (r == 0)
            code[r, c] = 4 if last else (6 if down else 1)
            pos[r, c] = c * nr + (r if down else nr - 1 - r)
    code[0 if nc % 2 == 0 else nr - 1, nc - 1] = 0xFF
    _, cnt, _ = fr.accumulate(dev(code), None, None, "d8", None, counts=True)
    assert np.array_equal(host(cnt), (pos + 1).astype(np.uint64))
    qbar = np.zeros((nr, nc))
    qbar[0 if nc % 2 == 0 else nr - 1, nc - 1] = 1.0
    rbar = host(fr.adjoint(dev(code), dev(qbar), None, "d8"))
    assert (rbar == 1.0).all()


# ---------------------------------------------------------------------------
# Adjoint


@pytest.mark.parametrize("rule", ["d8", "mfd"])
@pytest.mark.parametrize("nr,nc,seed", [(256, 256, 5), (97, 131, 7)])
def test_adjoint_matches_transpose_solve(rule, nr, nc, seed, accpath):
    print(f"adjoint {rule} {nr}x{nc}", flush=True)
    z = synth.dem(seed, nr, nc)
    zt = dev(z)
    code = fr.receivers(zt, rule)
    qbar = synth.normal(seed, synth.STREAM_NORMAL, nr * nc).reshape(nr, nc)
    if rule == "mfd":
        ref = oracle.adjoint_mfd(z, qbar, 1.1)
    else:
        ref = oracle.adjoint_single(host(code), qbar, z=z)
    r64 = host(fr.adjoint(code, dev(qbar), zt if rule == "mfd" else None, rule))
    r32 = host(fr.adjoint(code, dev(qbar.astype(np.float32)), zt if rule == "mfd" else None, rule))
    scale = np.abs(ref).max()
    assert np.max(np.abs(r64 - ref)) <= 1e-10 * scale
    ref32 = (oracle.adjoint_mfd(z, qbar.astype(np.float32).astype(np.float64), 1.1) if rule == "mfd"
             else oracle.adjoint_single(host(code), qbar.astype(np.float32).astype(np.float64), z=z))
    assert relnorm(r32, ref32) <= 1e-6
    # dot-product identity against the forward solve
    rain = synth.rain(seed, nr, nc).astype(np.float64)
    q, _, _ = fr.accumulate(code, zt if rule == "mfd" else None, dev(rain), rule, torch.float64)
    lhs = float((qbar * host(q)).sum())
    rhs = float((r64 * rain).sum())
    assert lhs == pytest.approx(rhs, rel=1e-10)


# ---------------------------------------------------------------------------
# Determinism, errors, degenerate inputs


def test_determinism_bits():
    z = synth.dem(2, 513, 777)
    rain = dev(synth.rain(2, 513, 777))
    zt = dev(z)
    for rule in ["d8", "mfd"]:
        code = fr.receivers(zt, rule)
        a, _, _ = fr.accumulate(code, zt, rain, rule, torch.float32)
        b, _, _ = fr.accumulate(code, zt, rain, rule, torch.float32)
        assert torch.equal(a, b)


def test_nonfinite_elevation_and_rain():
    z = synth.dem(1, 64, 128)
    z[10, 20] = np.nan
    with pytest.raises(fr.FlowRouteError) as e:
        fr.receivers(dev(z), "d8")
    assert e.value.code == fr.ERR_NONFINITE
    z = synth.dem(1, 64, 128)
    rain = synth.rain(1, 64, 128)
    rain[3, 3] = np.inf
    code = fr.receivers(dev(z), "d8")
    with pytest.raises(fr.FlowRouteError) as e:
        fr.accumulate(code, None, dev(rain), "d8", torch.float32)
    assert e.value.code == fr.ERR_NONFINITE


def test_cycle_and_bad_codes_reported(d8path):
    print(f"bad codes, path {d8path}", flush=True)
    code = np.full((8, 70), 0xFF, dtype=np.uint8)
    code[3, 5] = 4   # -> (3, 6)
    code[3, 6] = 3   # -> (3, 5): a 2-cycle
    code[6, 63] = 4  # crosses a tile boundary
    code[6, 64] = 3  # 2-cycle across tiles
    with pytest.raises(fr.FlowRouteError) as e:
        fr.accumulate(dev(code), None, None, "d8", None, counts=True)
    assert e.value.code == fr.ERR_NOTDAG
    code = np.full((8, 70), 0xFF, dtype=np.uint8)
    code[0, 0] = 0   # points off the grid
    with pytest.raises(fr.FlowRouteError) as e:
        fr.accumulate(dev(code), None, None, "d8", None, counts=True)
    assert e.value.code == fr.ERR_BADCODE
    code = np.full((8, 70), 0xFF, dtype=np.uint8)
    code[4, 4] = 17
    with pytest.raises(fr.FlowRouteError) as e:
        fr.accumulate(dev(code), None, None, "d8", None, counts=True)
    assert e.value.code == fr.ERR_BADCODE


def test_empty_grid():
    z = torch.empty((0, 5), dtype=torch.float32, device="cuda")
    code = fr.receivers(z, "d8")
    assert code.shape == (0, 5)
    q, cnt, m = fr.accumulate(code, None, None, "d8", torch.float32, counts=True, mass=True)
    assert q.numel() == 0 and cnt.numel() == 0
    assert host(m).tolist() == [0.0, 0.0]


def test_paper_3x3_example_on_gpu():
    # Section 2.1 worked example (constructed elevations reproduce the
    # printed routing list); unit rain gives w = [1,3,9,1,2,3,1,1,1].
    z = np.array([[38, 23, 14], [54, 33, 20], [59, 51, 31]], dtype=np.float32)
    code = fr.receivers(dev(z), "d8")
    assert host(code).ravel().tolist() == [4, 4, 255, 2, 2, 1, 2, 2, 1]
    q, cnt, _ = fr.accumulate(code, None, None, "d8", torch.float64, counts=True)
    assert host(q).ravel().tolist() == [1, 3, 9, 1, 2, 3, 1, 1, 1]
    assert host(cnt).ravel().tolist() == [1, 3, 9, 1, 2, 3, 1, 1, 1]


def test_autograd_gradcheck_and_fd():
    z = dev(synth.dem(5, 12, 16))
    for rule in ["mfd", "d8"]:
        rain = dev(synth.rain(5, 12, 16).astype(np.float64)).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda r: fr.FlowAccumulate.apply(r, z, rule), (rain,),
                                        eps=1.0, atol=1e-9, rtol=1e-9)
