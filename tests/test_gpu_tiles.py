"""GPU parity of the tile-forest path (single receivers, flow in every
direction): 32 x 64-cell tiles solved in LDS and joined by the exit forest.
It serves D8 / D4 calls whose cells drain to the previous row too rarely for
the row sweeps (predicted from a sample of the codes on grids of 2^18 cells
and more, or when their exit list overflows), and any call under the
"tiles" path choice.  The solution is the same unique one
(Section 2.2), so the bars are those of the other single-receiver paths:
counts bit-exact, float32 water within 1e-6 and float64 water within 1e-10
relative per cell of the float64 oracle, mass balance (Section 4) within
1e-6 / 1e-11.  Terrains: the paper's workflow (an untilted fractal DEM,
depression-filled), white noise (short paths, many pits), on grids of a few
million cells with ragged tile tails in both directions, and hand-made
codes where one exit gathers almost its whole ring (the most children an
exit can have); small and degenerate shapes run under the same path in the
general parity tests.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2606_12800_amd")

NR, NC = 2111, 2089  # 4,409,879 cells: 31 rows and 41 columns past the last full tile


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


def _case(kind, rule):
    """(elevations, codes, high-to-low order) of a seeded terrain."""
    conn = 8 if rule == "d8" else 4
    if kind == "filled":
        # The paper's workflow: an untilted fractal DEM, depression-filled.
        z = oracle.fill_depressions(synth.dem(52, NR, NC, tilt=0.0), conn, True)
    else:
        # White noise: short paths in every direction, many pits (sinks).
        z = synth.uniform(53, synth.STREAM_NOISE, NR * NC).reshape(NR, NC).astype(np.float32)
    code = oracle.receivers(z, oracle.D8 if rule == "d8" else oracle.D4)
    return z, code, oracle.order(z)


_CASES = {}


def case(kind, rule):
    if (kind, rule) not in _CASES:
        _CASES[(kind, rule)] = _case(kind, rule)
    return _CASES[(kind, rule)]


def _route(code, rain, rule, dtype, path="tiles"):
    with fr.accumulate_path(path):
        q, cnt, m = fr.accumulate(dev(code), rain=rain, rule=rule, dtype=dtype, counts=True,
                                  mass=dtype is not None)
        torch.cuda.synchronize()
    return q, cnt, m


@pytest.mark.parametrize("kind,rule", [("filled", "d8"), ("noise", "d8"), ("filled", "d4")])
@pytest.mark.parametrize("dtype,rain_kind", [(torch.float32, "f32"), (torch.float64, "f64"),
                                             (torch.float64, "f32"), (torch.float32, None), (None, None)])
def test_tiles_match_the_oracle(kind, rule, dtype, rain_kind):
    print(f"tiles {kind} {rule} {dtype} rain={rain_kind}", flush=True)
    z, code, order = case(kind, rule)
    rain_h = synth.rain(54, NR, NC)
    rain = None
    if rain_kind == "f32":
        rain = dev(rain_h)
    elif rain_kind == "f64":
        rain = dev(rain_h.astype(np.float64))
    q, cnt, m = _route(code, rain, rule, dtype)
    assert fr.served_by() == "tiles"
    qref, cref = oracle.accumulate_single(code, rain_h if rain_kind else None, order)
    assert np.array_equal(host(cnt), cref)
    if dtype is None:
        return
    tol = 1e-6 if dtype == torch.float32 else 1e-10
    assert relmax(host(q), qref) <= tol
    s, t = host(m).tolist()
    total = float(rain_h.astype(np.float64).sum()) if rain_kind else float(NR * NC)
    assert t == pytest.approx(total, rel=1e-12)
    assert abs(s - t) <= (1e-6 if dtype == torch.float32 else 1e-11) * t


def test_tiles_bits_repeat():
    """Fixed-order sums in the tiles and integer sums in the forest: every
    output repeats bit for bit."""
    _, code, _ = case("filled", "d8")
    rain = dev(synth.rain(55, NR, NC))
    outs = []
    for _ in range(3):
        q, cnt, m = _route(code, rain, "d8", torch.float32)
        assert fr.served_by() == "tiles"
        outs.append((q.view(torch.int32).clone(), cnt.clone(), m.view(torch.int64).clone()))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)


def test_overflow_takes_the_tile_forest():
    """Under the automatic choice: white noise on 3000 x 2900 cells drains to
    the previous row from too few cells, so the row sweeps' exit list (2^22
    entries and some slack here) overflows and the tile forest serves the
    call."""
    nr, nc = 3000, 2900
    z = synth.uniform(58, synth.STREAM_NOISE, nr * nc).reshape(nr, nc).astype(np.float32)
    code = oracle.receivers(z)
    assert np.sum(~np.isin(code, [0, 1, 2, 0xFF])) > 1.2 * 2**22
    rain_h = synth.rain(58, nr, nc)
    q, cnt, m = _route(code, dev(rain_h), "d8", torch.float32, path="auto")
    assert fr.served_by() == "tiles"
    qref, cref = oracle.accumulate_single(code, rain_h, oracle.order(z))
    assert np.array_equal(host(cnt), cref)
    assert relmax(host(q), qref) <= 1e-6
    s, t = host(m).tolist()
    assert abs(s - t) <= 1e-6 * t


@pytest.mark.parametrize("nr,nc,want", [(1024, 1536, "tiles"), (400, 500, "rows")])
def test_filled_grids_below_the_list_limit(nr, nc, want):
    """Under the automatic choice, on depression-filled DEMs below 2^22 cells
    (where the row sweeps' list holds every cell): from 2^18 cells on, the
    code sample predicts flow in every direction and the tile forest
    serves the call; smaller grids stay on the row sweeps.  Both against
    the oracle."""
    z = oracle.fill_depressions(synth.dem(59, nr, nc, tilt=0.0), 8, True)
    code = oracle.receivers(z)
    rain_h = synth.rain(59, nr, nc)
    q, cnt, m = _route(code, dev(rain_h), "d8", torch.float32, path="auto")
    assert fr.served_by() == want
    qref, cref = oracle.accumulate_single(code, rain_h, oracle.order(z))
    assert np.array_equal(host(cnt), cref)
    assert relmax(host(q), qref) <= 1e-6
    s, t = host(m).tolist()
    assert abs(s - t) <= 1e-6 * t


def test_tilted_terrain_stays_on_the_row_sweeps():
    z = synth.dem(56, NR, NC)
    code = oracle.receivers(z)
    assert np.mean(~np.isin(code, [0, 1, 2])) < 0.05
    q, cnt, _ = _route(code, None, "d8", torch.float32, path="auto")
    assert fr.served_by() == "rows"
    _, cref = oracle.accumulate_single(code, None, oracle.order(z))
    assert np.array_equal(host(cnt), cref)


def test_engine_path_still_selectable():
    _, code, order = case("noise", "d8")
    _, cnt, _ = _route(code, None, "d8", None, path="engine")
    assert fr.served_by() == "engine"
    _, cref = oracle.accumulate_single(code, None, order)
    assert np.array_equal(host(cnt), cref)


def _expect_status(code, rain, err):
    with fr.accumulate_path("tiles"), pytest.raises(fr.FlowRouteError) as e:
        fr.accumulate(dev(code), rain=rain, rule="d8", dtype=torch.float32, counts=True)
    assert e.value.code == err, fr.status_string(e.value.code)


def test_tiles_report_malformed_input():
    """Errors found on the tile path: a receiver off the grid or an unknown
    code (FR_ERR_BADCODE), a cycle inside a tile and one across a tile edge
    (FR_ERR_NOTDAG), non-finite rain (FR_ERR_NONFINITE)."""
    _, code, _ = case("noise", "d8")
    c = code.copy()
    c[NR - 1, 500] = 6  # below the last row
    print("tiles: off the grid", flush=True)
    _expect_status(c, None, fr.ERR_BADCODE)
    c = code.copy()
    c[700, 700] = 9
    print("tiles: unknown code", flush=True)
    _expect_status(c, None, fr.ERR_BADCODE)
    c = code.copy()
    c[40, 10], c[40, 11] = 4, 3  # right, left: a two-cell cycle inside tile (1, 0)
    print("tiles: cycle inside a tile", flush=True)
    _expect_status(c, None, fr.ERR_NOTDAG)
    c = code.copy()
    c[100, 63], c[100, 64] = 4, 3  # a cycle across the edge of tiles (3, 0) and (3, 1)
    print("tiles: cycle across tiles", flush=True)
    _expect_status(c, None, fr.ERR_NOTDAG)
    rain = synth.rain(57, NR, NC)
    rain[1234, 567] = np.inf
    print("tiles: non-finite rain", flush=True)
    _expect_status(code, dev(rain), fr.ERR_NONFINITE)


def _ring_funnel_codes():
    """D8 codes on 3 x 3 tiles (96 x 192 cells) where one exit of the middle
    tile gathers the whole middle tile and 195 exits of the ring around it:
    X = (32, 64), the middle tile's top-left cell, drains to (31, 63) and up
    column 63 to a sink at (0, 63); every other middle-tile cell drains
    toward X; every ring cell except (31, 63) drains into the middle tile;
    all other cells are sinks."""
    S = 0xFF
    UL, U, UR, L, R, DL, D = 0, 1, 2, 3, 4, 5, 6
    code = np.full((96, 192), S, dtype=np.uint8)
    r0, r1, c0, c1 = 32, 63, 64, 127  # the middle tile, inclusive
    for r in range(r0, r1 + 1):
        for c in range(c0, c1 + 1):
            code[r, c] = UL if (r > r0 and c > c0) else (L if r == r0 else U)
    code[r0, c0] = UL                    # X leaves its tile
    code[1:32, 63] = U                   # X's receiver and the path to the sink
    code[0, 63] = S
    code[31, c0:c1 + 1] = D              # top ring
    code[31, c1 + 1] = DL
    code[64, c0:c1 + 1] = U              # bottom ring
    code[64, c0 - 1] = UR
    code[64, c1 + 1] = UL
    code[r0:r1 + 1, c0 - 1] = R          # left ring
    code[r0:r1 + 1, c1 + 1] = L          # right ring
    return code


def _donors_first(code):
    """An order in which every cell follows all cells upstream of it: by
    decreasing number of steps to the cell's sink."""
    dr = np.array([-1, -1, -1, 0, 0, 1, 1, 1])
    dc = np.array([-1, 0, 1, -1, 1, -1, 0, 1])
    nr, nc = code.shape
    steps = np.zeros(nr * nc, dtype=np.int64)
    for i in range(nr * nc):
        r, c, s = i // nc, i % nc, 0
        while code[r, c] != 0xFF:
            k = int(code[r, c])
            r, c, s = r + dr[k], c + dc[k], s + 1
        steps[i] = s
    return np.argsort(-steps, kind="stable").astype(np.int64)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_exit_with_the_most_children(dtype):
    """The exit forest's sums add each child's total into its parent's low
    word without a carry, which holds while an exit has at most 196 children
    (one per cell of the ring around its tile).  Here one exit has 195, and
    the rain spans twenty binary orders of magnitude, so the low words of the
    fixed-point sums are full: values within the usual bars of the oracle,
    counts exact."""
    code = _ring_funnel_codes()
    order = _donors_first(code)
    n = code.size
    mant = synth.uniform(56, synth.STREAM_NOISE, n).astype(np.float64) + 0.5
    expo = synth.integers(57, synth.STREAM_PICK, n, -10, 11).astype(np.float64)
    rain_h = (mant * np.exp2(expo)).astype(np.float32).reshape(code.shape)
    q, cnt, m = _route(code, dev(rain_h), "d8", dtype)
    assert fr.served_by() == "tiles"
    qref, cref = oracle.accumulate_single(code, rain_h, order)
    assert cref[32, 64] == 32 * 64 + 195
    assert np.array_equal(host(cnt), cref)
    assert relmax(host(q), qref) <= (1e-6 if dtype == torch.float32 else 1e-10)
