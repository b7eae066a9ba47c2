"""Depression filling on the GPU (the priority-flood surface the paper fills
the DEM with before routing, Section 4) against the oracle's priority flood.

Every operation on the path is exact (order-preserving keys, min, max, one
float32 step), so the filled surface must match bit for bit: D8/MFD (8
neighbours) and D4 (4), plain and epsilon variants, ragged shapes across
several 62 x 62 tiles, thin grids that are all boundary, a crater and a
serpentine channel whose flood path crosses tile boundaries many times.  At
sizes the oracle cannot take, the fixed-point equation itself is checked at
every cell: it has exactly one solution, so that check is complete.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2606_12800_amd")

CONN = {"d8": 8, "d4": 4, "mfd": 8}


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fr.load_library()
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bits_equal(a, b):
    return np.array_equal(np.asarray(a, dtype=np.float32).view(np.uint32), np.asarray(b, dtype=np.float32).view(np.uint32))


def _pits(seed, nr, nc):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 40, size=(nr, nc)) * 0.25).astype(np.float32)


def _crater(nr, nc, spill_col):
    z = np.full((nr, nc), 100.0, dtype=np.float32)
    z[1:-1, 1:-1] = 1.0
    z[0, spill_col] = 7.0
    return z


def _serpentine(nr, nc, wall=90.0):
    """Low floor cut into lanes by walls with alternating gaps: the only
    way out winds through every lane, crossing tile rows many times."""
    z = np.full((nr, nc), 5.0, dtype=np.float32)
    for r in range(4, nr - 4, 6):
        z[r, :] = wall
        if (r // 6) % 2:
            z[r, 2:4] = 5.0
        else:
            z[r, nc - 4:nc - 2] = 5.0
    z[:, 0] = z[:, -1] = wall
    z[-1, :] = wall
    z[0, :] = wall
    z[0, 3] = 6.0
    return z


def _check(z, rule, eps):
    print(f"fill {rule} eps={eps} shape {z.shape}", flush=True)
    f, n = fr.fill_depressions(dev(z), rule, eps, launches=True)
    torch.cuda.synchronize()
    ref = oracle.fill_depressions(z, CONN[rule], eps)
    assert _bits_equal(f.cpu().numpy(), ref)
    return n


@pytest.mark.parametrize("rule", ["d8", "d4", "mfd"])
@pytest.mark.parametrize("eps", [True, False])
@pytest.mark.parametrize("seed,shape", [(1, (1, 1)), (2, (1, 70)), (3, (70, 2)), (4, (3, 3)), (5, (62, 62)),
                                        (6, (64, 64)), (7, (63, 125)), (8, (200, 300)), (9, (517, 333))])
def test_fill_matches_oracle(rule, eps, seed, shape):
    _check(synth.dem(seed, *shape, tilt=0.0), rule, eps)


@pytest.mark.parametrize("rule", ["d8", "d4"])
def test_fill_random_pits_and_crater(rule):
    for eps in (True, False):
        _check(_pits(21, 301, 157), rule, eps)
        _check(_crater(250, 390, 200), rule, eps)


@pytest.mark.parametrize("rule", ["d8", "d4"])
def test_fill_serpentine_many_tile_crossings(rule):
    z = _serpentine(400, 300)
    n = _check(z, rule, True)
    # The flood winds through ~66 lanes: many launches, each reaching the
    # tiles next to the last change.
    assert n > 3


def test_fill_then_route_drains_to_boundary():
    z = synth.dem(31, 400, 517, tilt=0.0)
    zf = fr.fill_depressions(dev(z), "d8", True)
    code0 = fr.receivers(dev(z), "d8").cpu().numpy()
    code, q, _, mass = fr.route(zf, dev(synth.rain(31, 400, 517)), "d8", torch.float64, mass=True)
    c = code.cpu().numpy()
    inner = np.zeros(z.shape, dtype=bool)
    inner[1:-1, 1:-1] = True
    assert np.any((code0 == fr.SINK) & inner)
    assert not np.any((c == fr.SINK) & inner)
    out, total = mass.cpu().tolist()
    assert abs(out - total) <= 1e-12 * total


def test_fill_errors_and_empty():
    z = synth.dem(41, 50, 60)
    z[10, 20] = np.nan
    with pytest.raises(fr.FlowRouteError) as e:
        fr.fill_depressions(dev(z), "d8")
    assert e.value.code == fr.ERR_NONFINITE
    e0 = fr.fill_depressions(torch.empty((0, 7), dtype=torch.float32, device="cuda"))
    assert e0.shape == (0, 7)
    with pytest.raises(ValueError):
        fr.fill_depressions(dev(np.zeros(5, dtype=np.float32)))
    lib = fr.load_library()
    zz = dev(synth.dem(42, 10, 10))
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    import ctypes
    rc = lib.fr_fill_depressions(zz.data_ptr(), 10, 10, fr.D8, 1, zz.data_ptr(), None, None, ws.data_ptr(), 4096,
                                 None)
    assert rc == fr.ERR_ARG  # output aliases the input
    out = torch.empty_like(zz)
    rc = lib.fr_fill_depressions(zz.data_ptr(), 10, 10, fr.D8, 2, out.data_ptr(), None, None, ws.data_ptr(), 4096,
                                 None)
    assert rc == fr.ERR_ARG  # eps not 0/1
    rc = lib.fr_fill_depressions(zz.data_ptr(), 10, 10, fr.D8, 1, out.data_ptr(), None, None, ws.data_ptr(), 1,
                                 None)
    assert rc == fr.ERR_WORKSPACE
    del ctypes


def _fixed_point_ok(z, f, conn, eps):
    """F = z on the boundary and F = max(z, min_n next(F_n)) inside, checked
    with torch on the device in float32 (exact operations)."""
    inf = torch.tensor(float("inf"), device=f.device)
    pad = torch.nn.functional.pad(f[None, None], (1, 1, 1, 1), value=float("inf"))[0, 0]
    nr, nc = f.shape
    m = torch.full_like(f, float("inf"))
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if (dr, dc) == (0, 0) or (conn == 4 and dr != 0 and dc != 0):
                continue
            m = torch.minimum(m, pad[1 + dr:1 + dr + nr, 1 + dc:1 + dc + nc])
    if eps:
        m = torch.nextafter(m, inf)
    want = torch.maximum(z, m)
    ok_in = torch.equal(f[1:-1, 1:-1], want[1:-1, 1:-1])
    ok_b = (torch.equal(f[0], z[0]) and torch.equal(f[-1], z[-1]) and torch.equal(f[:, 0], z[:, 0])
            and torch.equal(f[:, -1], z[:, -1]))
    return ok_in and ok_b


@pytest.mark.parametrize("rule,n", [("d8", 4096), ("d4", 2500)])
def test_fill_fixed_point_large(rule, n):
    print(f"fill fixed point {rule} {n}x{n}", flush=True)
    z = dev(synth.dem(51, n, n, tilt=0.0))
    f = fr.fill_depressions(z, rule, True)
    assert _fixed_point_ok(z, f, CONN[rule], True)
    assert bool((f >= z).all())


def test_fill_fixed_point_fullsize():
    """The bench's fill workload (43360^2 untilted DEM, seed 2, epsilon, 8
    neighbours), checked band by band against the fixed-point equation, which
    has exactly one solution."""
    n = 43360
    print(f"fill fixed point d8 {n}x{n}", flush=True)
    z = torch.from_numpy(synth.dem(2, n, n, tilt=0.0)).cuda()
    f = fr.fill_depressions(z, "d8", True)
    torch.cuda.synchronize()
    inf = torch.tensor(float("inf"), device=f.device)
    for r0 in range(0, n, 4096):
        r1 = min(r0 + 4096, n)
        a, b = max(r0 - 1, 0), min(r1 + 1, n)
        band = torch.nn.functional.pad(f[a:b][None, None], (1, 1, 1 if a == r0 else 0, 1 if b == r1 else 0),
                                       value=float("inf"))[0, 0]
        m = torch.full((r1 - r0, n), float("inf"), device=f.device)
        for dr in (-1, 0, 1):
            for dc in (-1, 0, 1):
                if (dr, dc) != (0, 0):
                    m = torch.minimum(m, band[1 + dr:1 + dr + (r1 - r0), 1 + dc:1 + dc + n])
        want = torch.maximum(z[r0:r1], torch.nextafter(m, inf))
        got = f[r0:r1]
        inner = torch.ones_like(got, dtype=torch.bool)
        inner[:, 0] = inner[:, -1] = False
        if r0 == 0:
            inner[0] = False
        if r1 == n:
            inner[-1] = False
        assert torch.equal(got[inner], want[inner]), r0
        assert torch.equal(got[~inner], z[r0:r1][~inner]), r0
        del band, m, want
    assert bool((f >= z).all())
    del z, f
    torch.cuda.empty_cache()


def test_filled_untilted_dem_routes_like_the_oracle():
    """The paper's workflow (Section 4): fill, then route.  An untilted
    4096^2 fractal DEM (seed 2), filled (epsilon variant, 8 neighbours) on
    the GPU and bit-exact against the oracle's priority flood, then routed
    D8 with float32 rain and counts.  Its flow runs in every direction: more
    than an eighth of the cells leave their row-sweep tile, which overflows
    the row sweeps' exit list at this size, so the tile forest serves the
    call -- counts bit-exact and water within 1e-6 of the oracle."""
    n = 4096
    print(f"fill + route untilted {n}^2", flush=True)
    z_h = synth.dem(2, n, n, tilt=0.0)
    rain_h = synth.rain(2, n, n)
    f = fr.fill_depressions(dev(z_h), "d8", eps=True)
    torch.cuda.synchronize()
    f_h = f.cpu().numpy()
    assert _bits_equal(f_h, oracle.fill_depressions(z_h, 8, True))
    code, q, cnt, mass = fr.route(f, dev(rain_h), "d8", torch.float32, counts=True, mass=True)
    torch.cuda.synchronize()
    assert fr.served_by() == "tiles"
    code_h = oracle.receivers(f_h)
    assert np.array_equal(code.cpu().numpy(), code_h)
    # Only boundary cells are sinks after filling.
    inner = code_h[1:-1, 1:-1]
    assert not (inner == 0xFF).any()
    exits = np.mean(~np.isin(code_h, [0, 1, 2]))
    print(f"  cells not draining to the row before: {exits:.3f}", flush=True)
    order = oracle.order(f_h)
    qref, _ = oracle.accumulate_single(code_h, rain_h, order)
    _, cref = oracle.accumulate_single(code_h, None, order)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint64), cref)
    qh = q.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(qh - qref) / qref) <= 1e-6
    s, t = mass.cpu().tolist()
    assert abs(s - t) <= 1e-6 * t
