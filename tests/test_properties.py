"""Property-based checks of the oracle over drawn grids (hypothesis,
derandomised so that every run draws the same cases).

Each property follows from the problem's definition, not from the oracle's
own code:
  * D8 / D4 receivers are strictly lower neighbours inside the grid, and a
    cell is a sink exactly when no neighbour is strictly lower (Section 2.1);
  * D8 counts equal the number of cells whose receiver path passes through
    the cell, found by walking every path (brute force);
  * water is conserved: the sinks receive all the rain (Section 4's check),
    for single receivers and for multiple-flow-direction fractions;
  * q is linear in r, and the transpose solve satisfies
    <qbar, q(r)> = <rbar(qbar), r> (the adjoint of (I - W^T) q = r,
    Section 2.2);
  * depression filling raises no cell below its elevation, leaves a filled
    surface unchanged, and (epsilon variant) leaves every interior cell a
    strictly lower neighbour, so D8 routing of it has sinks on the border
    only.
Grids are small (at most 40 x 40) so that the brute force stays cheap; the
terrains cover fractal DEMs with and without tilt, white noise, and
integer steps with ties and plateaus.
"""
import numpy as np
import pytest

import oracle
import synth

hyp = pytest.importorskip("hypothesis")
st = pytest.importorskip("hypothesis.strategies")
given, settings = hyp.given, hyp.settings

SETTINGS = settings(derandomize=True, max_examples=120, deadline=None)

DR8 = [-1, -1, -1, 0, 0, 1, 1, 1]
DC8 = [-1, 0, 1, -1, 1, -1, 0, 1]
D4_CODES = {1, 3, 4, 6}


def terrain(kind, seed, nr, nc):
    if kind == "dem":
        return synth.dem(seed, nr, nc)
    if kind == "dem_flat":
        return synth.dem(seed, nr, nc, tilt=0.0)
    if kind == "noise":
        return synth.uniform(seed, synth.STREAM_NOISE, nr * nc).reshape(nr, nc).astype(np.float32)
    return synth.integers(seed, synth.STREAM_PICK, nr * nc, 0, 4).reshape(nr, nc).astype(np.float32)


grids = st.tuples(st.sampled_from(["dem", "dem_flat", "noise", "steps"]), st.integers(0, 10_000),
                  st.integers(1, 40), st.integers(1, 40))


def lower_neighbours(z, r, c, rule):
    nr, nc = z.shape
    out = []
    for k in range(8):
        if rule == oracle.D4 and k not in D4_CODES:
            continue
        rr, cc = r + DR8[k], c + DC8[k]
        if 0 <= rr < nr and 0 <= cc < nc and z[rr, cc] < z[r, c]:
            out.append(k)
    return out


@SETTINGS
@given(grids, st.sampled_from([oracle.D8, oracle.D4]))
def test_receivers_are_strictly_lower_and_sinks_have_none(g, rule):
    kind, seed, nr, nc = g
    z = terrain(kind, seed, nr, nc)
    code = oracle.receivers(z, rule)
    for r in range(nr):
        for c in range(nc):
            low = lower_neighbours(z, r, c, rule)
            if code[r, c] == 0xFF:
                assert not low
            else:
                assert int(code[r, c]) in low


def walk_counts(code):
    """Counts by walking every cell's receiver path to its sink."""
    nr, nc = code.shape
    cnt = np.zeros((nr, nc), dtype=np.uint64)
    for r in range(nr):
        for c in range(nc):
            rr, cc, steps = r, c, 0
            while True:
                cnt[rr, cc] += 1
                k = int(code[rr, cc])
                if k == 0xFF:
                    break
                rr, cc = rr + DR8[k], cc + DC8[k]
                steps += 1
                assert steps <= nr * nc  # strictly lower receivers: no cycle
    return cnt


@SETTINGS
@given(grids, st.sampled_from([oracle.D8, oracle.D4]))
def test_d8_counts_equal_walked_paths(g, rule):
    kind, seed, nr, nc = g
    z = terrain(kind, seed, nr, nc)
    code = oracle.receivers(z, rule)
    _, cnt = oracle.accumulate_single(code, None, z=z, q=False)
    assert np.array_equal(cnt, walk_counts(code))


@SETTINGS
@given(grids)
def test_water_is_conserved_single_and_mfd(g):
    kind, seed, nr, nc = g
    z = terrain(kind, seed, nr, nc)
    rain = synth.rain(seed, nr, nc).astype(np.float64)
    total = float(rain.sum())
    code = oracle.receivers(z)
    q, _ = oracle.accumulate_single(code, rain, z=z, counts=False)
    assert float(q[code == 0xFF].sum()) == pytest.approx(total, rel=1e-12, abs=1e-300)
    qm = oracle.accumulate_mfd(z, rain)
    mask, _ = oracle.mfd_fractions(z)
    assert float(qm[mask == 0].sum()) == pytest.approx(total, rel=1e-12, abs=1e-300)
    # every cell holds at least its own rain (non-negative rain)
    assert np.all(q >= rain) and np.all(qm >= rain * (1 - 1e-15))


@SETTINGS
@given(grids, st.sampled_from(["d8", "mfd"]), st.integers(-3, 3), st.integers(-3, 3))
def test_linearity_and_adjoint_identity(g, rule, a, b):
    """Rain enters in float32 (the method's input precision), so the rain
    fields are small integers and multiples of 2^-10, whose combinations
    with small integer weights are exact in float32."""
    kind, seed, nr, nc = g
    z = terrain(kind, seed, nr, nc)
    n = nr * nc
    r1 = synth.integers(seed, synth.STREAM_PICK, n, -8, 9).reshape(nr, nc).astype(np.float64)
    r2 = synth.integers(seed + 1, synth.STREAM_PICK, n, 0, 1024).reshape(nr, nc).astype(np.float64) / 1024
    qbar = synth.normal(seed + 2, synth.STREAM_NORMAL, n).reshape(nr, nc)
    if rule == "d8":
        code = oracle.receivers(z)
        solve = lambda r: oracle.accumulate_single(code, r, z=z, counts=False)[0]  # noqa: E731
        rbar = oracle.adjoint_single(code, qbar, z=z)
    else:
        solve = lambda r: oracle.accumulate_mfd(z, r)  # noqa: E731
        rbar = oracle.adjoint_mfd(z, qbar)
    q1, q2 = solve(r1), solve(r2)
    lhs = solve(a * r1 + b * r2)
    scale = max(1.0, float(np.max(np.abs(a * q1))) + float(np.max(np.abs(b * q2))))
    assert np.max(np.abs(lhs - (a * q1 + b * q2))) <= 1e-12 * scale
    x, y = float(np.sum(qbar * q1)), float(np.sum(rbar * r1))
    assert x == pytest.approx(y, rel=1e-10, abs=1e-10 * float(np.sum(np.abs(qbar) * np.abs(q1))) + 1e-300)


@SETTINGS
@given(grids, st.sampled_from([8, 4]))
def test_fill_raises_only_is_idempotent_and_drains(g, conn):
    kind, seed, nr, nc = g
    z = terrain(kind, seed, nr, nc)
    f = oracle.fill_depressions(z, conn, True)
    assert np.all(f >= z)
    assert np.array_equal(oracle.fill_depressions(f, conn, True), f)
    code = oracle.receivers(f, oracle.D8 if conn == 8 else oracle.D4)
    sinks = np.argwhere(code == 0xFF)
    for r, c in sinks:
        assert r == 0 or c == 0 or r == nr - 1 or c == nc - 1
    # plain variant: no higher than the epsilon one, and still raises only
    fp = oracle.fill_depressions(z, conn, False)
    assert np.all(fp >= z) and np.all(fp <= f)
