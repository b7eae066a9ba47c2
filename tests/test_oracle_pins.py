"""Pins of the CPU oracle against things other than itself.

Each test ties an oracle function to something the paper or mathematics fixes:
the paper's 3x3 worked example (Section 2.1, Section 2.2), brute-force path
tracing, exact rational arithmetic, library solvers (numpy / scipy), closed
forms and conservation laws.  A plausible slip in the oracle -- a dropped
term, a wrong sign or index, a transposed operand, a reversed sort -- fails
at least one of them.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_3x3.json")
OFFS = oracle.OFFSETS


def _paper3x3():
    with open(GOLDEN) as f:
        return json.load(f)


def _node_to_cell(n):
    return (n - 1) // 3, (n - 1) % 3


def _target(code, r, c):
    cd = int(code[r, c])
    if cd == oracle.SINK:
        return None
    dr, dc = OFFS[cd]
    return r + dr, c + dc


# --------------------------------------------------------------------------
# Paper's 3x3 example (Section 2.1, Figure 3x3; Section 2.2).

def test_3x3_receivers_reproduce_printed_routing_list():
    g = _paper3x3()
    z = np.array(g["elevation_constructed"], dtype=np.float32)
    code = oracle.receivers(z)
    assert code.ravel().tolist() == g["d8_codes_constructed"]
    for src, dst in g["routing_list_printed"]:
        t = _target(code, *_node_to_cell(src))
        if dst is None:
            assert t is None
        else:
            assert t == _node_to_cell(dst)


def test_3x3_order_is_printed_high_to_low_order():
    g = _paper3x3()
    z = np.array(g["elevation_constructed"], dtype=np.float32)
    o = oracle.order(z)
    assert [int(i) + 1 for i in o] == g["high_to_low_order_printed"]


def test_3x3_accumulation_matches_printed_equations():
    g = _paper3x3()
    z = np.array(g["elevation_constructed"], dtype=np.float32)
    code = oracle.receivers(z)
    q, c = oracle.accumulate_single(code, None, z=z)
    assert q.ravel().tolist() == g["w_unit_rain_derived"]
    assert c.ravel().tolist() == g["w_unit_rain_derived"]
    # Arbitrary rain: evaluate the printed equations top to bottom.
    rain = synth.rain(11, 3, 3)
    r = {n: float(rain[_node_to_cell(n)]) for n in range(1, 10)}
    w = {}
    for n in g["high_to_low_order_printed"]:
        w[n] = r[n] + sum(w[m] for m in g["equations_printed"][f"w{n}"])
    q, _ = oracle.accumulate_single(code, rain, z=z, counts=False)
    for n in range(1, 10):
        assert q[_node_to_cell(n)] == pytest.approx(w[n], rel=1e-15)


def test_3x3_apply_A_is_printed_matrix():
    g = _paper3x3()
    z = np.array(g["elevation_constructed"], dtype=np.float32)
    code = oracle.receivers(z)
    A = np.zeros((9, 9))
    for j in range(9):
        e = np.zeros(9)
        e[j] = 1.0
        A[:, j] = oracle.apply_A_single(code, e.reshape(3, 3)).ravel()
    assert A.tolist() == np.array(g["matrix_A_printed_rows"], dtype=float).tolist()
    # The printed matrix times the derived unit-rain solution is the unit rain.
    w = np.array(g["w_unit_rain_derived"], dtype=float)
    assert (np.array(g["matrix_A_printed_rows"]) @ w).tolist() == [1.0] * 9


def test_3x3_printed_matrix_triangular_after_high_to_low_permutation():
    # Section 2.4: P A P^T is lower triangular for the high-to-low numbering.
    g = _paper3x3()
    A = np.array(g["matrix_A_printed_rows"], dtype=float)
    perm = [n - 1 for n in g["high_to_low_order_printed"]]
    Ad = A[np.ix_(perm, perm)]
    assert np.allclose(Ad, np.tril(Ad))
    w = spla.spsolve_triangular(sp.csr_matrix(Ad), np.ones(9), lower=True)
    assert np.allclose(w[np.argsort(perm)], g["w_unit_rain_derived"])


# --------------------------------------------------------------------------
# Receivers: exact rational steepest descent on integer DEMs.

def _exact_receiver(zi, r, c, nr, nc, rule=oracle.D8):
    best, best_s2 = None, None
    for k, (dr, dc) in enumerate(OFFS):
        if rule == oracle.D4 and dr != 0 and dc != 0:
            continue
        rr, cc = r + dr, c + dc
        if not (0 <= rr < nr and 0 <= cc < nc):
            continue
        d = int(zi[r][c]) - int(zi[rr][cc])
        if d <= 0:
            continue
        s2 = Fraction(d * d, 2) if (dr and dc) else Fraction(d * d)
        if best is None or s2 > best_s2:
            best, best_s2 = k, s2
    return oracle.SINK if best is None else best


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("rule", [oracle.D8, oracle.D4])
def test_receivers_exact_rational_integer_dem(seed, rule):
    nr, nc = 9 + seed, 13 - seed
    vals = synth.integers(100 + seed, synth.STREAM_PICK, nr * nc, 0, 60).reshape(nr, nc)
    z = vals.astype(np.float32)
    code = oracle.receivers(z, rule)
    for r in range(nr):
        for c in range(nc):
            assert code[r, c] == _exact_receiver(vals.tolist(), r, c, nr, nc, rule), (r, c)


def test_receivers_tilted_plane_and_cone():
    nr, nc = 17, 11
    rows = np.arange(nr, dtype=np.float32)[:, None] * np.ones((1, nc), dtype=np.float32)
    code = oracle.receivers(rows)
    assert (code[0] == oracle.SINK).all()
    assert (code[1:] == 1).all()  # neighbour (-1, 0)
    q, c = oracle.accumulate_single(code, None, z=rows)
    expect = (nr - np.arange(nr))[:, None] * np.ones((1, nc))
    assert (q == expect).all() and (c == expect.astype(np.uint64)).all()
    # Cone: everything drains to the apex.
    r0, c0 = 7, 4
    rr, cc = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    cone = ((rr - r0) ** 2 + (cc - c0) ** 2).astype(np.float32)
    code = oracle.receivers(cone)
    assert (code == oracle.SINK).sum() == 1 and code[r0, c0] == oracle.SINK
    _, c = oracle.accumulate_single(code, None, z=cone, q=False)
    assert int(c[r0, c0]) == nr * nc


def test_receivers_degenerate_shapes():
    for shape in [(1, 1), (1, 7), (7, 1), (2, 2)]:
        z = synth.dem(5, *shape)
        code = oracle.receivers(z)
        for r in range(shape[0]):
            for c in range(shape[1]):
                t = _target(code, r, c)
                if t is not None:
                    assert z[t] < z[r, c]
    flat = np.zeros((5, 6), dtype=np.float32)
    assert (oracle.receivers(flat) == oracle.SINK).all()
    q, c = oracle.accumulate_single(oracle.receivers(flat), None, z=flat)
    assert (q == 1).all() and (c == 1).all()


# --------------------------------------------------------------------------
# Order: library stable sort.

def test_order_matches_numpy_stable_argsort():
    z = synth.dem(3, 40, 50)
    z[3, :10] = z[3, 0]  # ties
    z[7, 5] = -0.0
    z[7, 6] = 0.0
    o = oracle.order(z)
    ref = np.argsort(-z.ravel().astype(np.float64), kind="stable")
    assert (o == ref).all()


# --------------------------------------------------------------------------
# D8 accumulation: brute-force path tracing.

def _trace_all(code, rain):
    nr, nc = code.shape
    q = np.zeros((nr, nc))
    cnt = np.zeros((nr, nc), dtype=np.int64)
    steps = 0
    for r in range(nr):
        for c in range(nc):
            cur = (r, c)
            while cur is not None:
                q[cur] += rain[r, c]
                cnt[cur] += 1
                steps += 1
                cur = _target(code, *cur)
    return q, cnt, steps


@pytest.mark.parametrize("seed,shape", [(1, (16, 16)), (2, (5, 23)), (3, (23, 5)), (4, (1, 30)),
                                        (5, (30, 1)), (6, (12, 12))])
def test_d8_push_equals_brute_force_tracing(seed, shape):
    z = synth.dem(seed, *shape)
    rain = synth.rain(seed, *shape)
    code = oracle.receivers(z)
    q, c = oracle.accumulate_single(code, rain, z=z)
    bq, bc, steps = _trace_all(code, rain)
    assert np.allclose(q, bq, rtol=1e-13, atol=0)
    assert (c.astype(np.int64) == bc).all()
    # Subtree identity: sum of counts = sum over cells of (path length + 1).
    assert int(c.sum()) == steps
    # Conservation: sinks receive all the water.
    s, t = oracle.mass_single(code, q, rain)
    assert s == pytest.approx(t, rel=1e-14)
    _, cc = oracle.accumulate_single(code, None, z=z, q=False)
    assert int(cc[code == oracle.SINK].sum()) == z.size


def test_d8_residual_is_zero_with_apply_A():
    z = synth.dem(9, 64, 48)
    rain = synth.rain(9, 64, 48)
    code = oracle.receivers(z)
    q, _ = oracle.accumulate_single(code, rain, z=z, counts=False)
    res = rain.astype(np.float64) - oracle.apply_A_single(code, q)
    assert np.abs(res).max() <= 1e-12 * q.max()


def test_d8_counts_on_benchmark_dem_256():
    # The 256x256 benchmark DEM (seed 1): receivers' targets are lower, sinks
    # absorb every cell exactly once, and counts obey the local balance.
    z = synth.dem(1, 256, 256)
    code = oracle.receivers(z)
    _, c = oracle.accumulate_single(code, None, z=z, q=False)
    assert int(c[code == oracle.SINK].sum()) == z.size
    inflow = np.zeros(z.shape, dtype=np.uint64)
    for k, (dr, dc) in enumerate(OFFS):
        src = np.argwhere(code == k)
        np.add.at(inflow, (src[:, 0] + dr, src[:, 1] + dc), c[src[:, 0], src[:, 1]])
    assert (c == inflow + 1).all()


# --------------------------------------------------------------------------
# MFD fractions: special cases of the slope-power law.

def test_mfd_fraction_invariants_and_limits():
    z = synth.dem(21, 20, 17)
    mask, f = oracle.mfd_fractions(z, 1.1)
    nr, nc = z.shape
    for r in range(nr):
        for c in range(nc):
            lower = [k for k, (dr, dc) in enumerate(OFFS)
                     if 0 <= r + dr < nr and 0 <= c + dc < nc and z[r + dr, c + dc] < z[r, c]]
            assert mask[r, c] == sum(1 << k for k in lower)
            if lower:
                assert f[r, c].sum() == pytest.approx(1.0, abs=1e-14)
                assert all(f[r, c, k] > 0 for k in lower)
            assert all(f[r, c, k] == 0 for k in range(8) if k not in lower)
    # p = 0: equal split among the lower neighbours.
    _, f0 = oracle.mfd_fractions(z, 0.0)
    m = np.array([[bin(v).count("1") for v in row] for row in mask])
    for k in range(8):
        sel = (mask >> k) & 1 == 1
        assert np.allclose(f0[..., k][sel], 1.0 / m[sel])
    # The largest fraction goes to the steepest receiver (exact rational
    # steepest descent on an integer DEM, ties to the lowest index).
    vals = synth.integers(22, synth.STREAM_PICK, 20 * 17, 0, 60).reshape(20, 17)
    _, fi = oracle.mfd_fractions(vals.astype(np.float32), 1.1)
    for r in range(20):
        for c in range(17):
            ex = _exact_receiver(vals.tolist(), r, c, 20, 17)
            if ex != oracle.SINK:
                assert int(np.argmax(fi[r, c])) == ex


def test_mfd_fraction_slope_uses_diagonal_distance():
    # Centre 10, cardinal neighbour 8 (drop 2), diagonal neighbour 6 (drop 4);
    # all others higher.  Slopes 2 and 4/sqrt(2) = 2 sqrt(2).
    z = np.full((3, 3), 50.0, dtype=np.float32)
    z[1, 1], z[0, 1], z[0, 0] = 10.0, 8.0, 6.0
    for p in (1.0, 1.1, 2.0):
        _, f = oracle.mfd_fractions(z, p)
        ratio = f[1, 1, 0] / f[1, 1, 1]
        assert ratio == pytest.approx(np.sqrt(2.0) ** p, rel=1e-14)
    # Two cardinal neighbours with equal drops split evenly.
    z = np.full((3, 3), 50.0, dtype=np.float32)
    z[1, 1], z[1, 0], z[1, 2] = 10.0, 7.0, 7.0
    _, f = oracle.mfd_fractions(z, 1.1)
    assert f[1, 1, 3] == 0.5 and f[1, 1, 4] == 0.5


# --------------------------------------------------------------------------
# MFD accumulation: library solvers.

def _W(mask_frac, shape):
    f = mask_frac
    nr, nc = shape
    n = nr * nc
    rows, cols, vals = [], [], []
    for r in range(nr):
        for c in range(nc):
            for k, (dr, dc) in enumerate(OFFS):
                if f[r, c, k] != 0.0:
                    rows.append(r * nc + c)
                    cols.append((r + dr) * nc + (c + dc))
                    vals.append(f[r, c, k])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.parametrize("seed,shape", [(31, (12, 12)), (32, (24, 24)), (33, (5, 19))])
def test_mfd_push_equals_dense_solve(seed, shape):
    z = synth.dem(seed, *shape)
    rain = synth.rain(seed, *shape)
    _, f = oracle.mfd_fractions(z, 1.1)
    W = _W(f, shape).toarray()
    n = z.size
    q_ref = np.linalg.solve(np.eye(n) - W.T, rain.ravel().astype(np.float64))
    q = oracle.accumulate_mfd(z, rain, 1.1)
    assert np.allclose(q.ravel(), q_ref, rtol=1e-12, atol=0)
    s, t = oracle.mass_mfd(z, q, rain)
    assert s == pytest.approx(t, rel=1e-13)
    # Residual with the matrix-free A of Appendix A.
    res = rain.astype(np.float64) - oracle.apply_A_mfd(z, q, 1.1)
    assert np.abs(res).max() <= 1e-12 * q.max()


def test_mfd_push_equals_sparse_lu_and_neumann_series():
    shape = (300, 330)  # ~1e5 cells
    z = synth.dem(34, *shape)
    _, f = oracle.mfd_fractions(z, 1.1)
    W = _W(f, shape)
    n = z.size
    r = np.ones(n)
    q_ref = spla.spsolve(sp.identity(n, format="csc") - W.T.tocsc(), r)
    q = oracle.accumulate_mfd(z, None, 1.1).ravel()
    assert np.max(np.abs(q - q_ref) / q_ref) < 1e-10
    # Neumann series sum_k (W^T)^k r terminates after the DAG depth.
    WT = W.T.tocsr()
    term, acc = r.copy(), r.copy()
    for _ in range(n):
        term = WT @ term
        if not term.any():
            break
        acc += term
    assert not term.any()
    assert np.max(np.abs(acc - q) / q) < 1e-10


# --------------------------------------------------------------------------
# Adjoint: brute force, dense transpose solve, dot-product identity.

def test_d8_adjoint_is_downstream_path_sum():
    z = synth.dem(41, 14, 19)
    code = oracle.receivers(z)
    qbar = synth.normal(41, synth.STREAM_NORMAL, z.size).reshape(z.shape)
    rb = oracle.adjoint_single(code, qbar, z=z)
    nr, nc = z.shape
    for r in range(nr):
        for c in range(nc):
            cur, s = (r, c), 0.0
            while cur is not None:
                s += qbar[cur]
                cur = _target(code, *cur)
            assert rb[r, c] == pytest.approx(s, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("seed,shape", [(42, (15, 15)), (43, (9, 26))])
def test_mfd_adjoint_equals_dense_transpose_solve(seed, shape):
    z = synth.dem(seed, *shape)
    _, f = oracle.mfd_fractions(z, 1.1)
    W = _W(f, shape).toarray()
    n = z.size
    qbar = synth.normal(seed, synth.STREAM_NORMAL, n)
    rb_ref = np.linalg.solve(np.eye(n) - W, qbar)
    rb = oracle.adjoint_mfd(z, qbar, 1.1).ravel()
    assert np.allclose(rb, rb_ref, rtol=1e-11, atol=1e-12)
    # <qbar, A^-1 r> = <A^-T qbar, r>
    rain = synth.rain(seed, *shape)
    q = oracle.accumulate_mfd(z, rain, 1.1).ravel()
    lhs = float(qbar @ q)
    rhs = float(rb @ rain.ravel().astype(np.float64))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_fp32_fraction_variant_is_close_to_fp64():
    z = synth.dem(44, 64, 64)
    q64 = oracle.accumulate_mfd(z, None, 1.1)
    q32 = oracle.accumulate_mfd(z, None, 1.1, frac32=True)
    assert np.max(np.abs(q32 - q64) / q64) < 1e-5


# ---------------------------------------------------------------------------
# The paper's parallel scheme (Section 3.3 "I+X" and "(I-X)(I+X)"; Appendix B):
# block Richardson iterations with per-block high-to-low solves.

def _block(shape, blk, r, c):
    nbc = (shape[1] + blk[1] - 1) // blk[1]
    return (r // blk[0]) * nbc + c // blk[1]


def _max_crossings_d8(code, blk):
    """Brute force: follow every cell's flow path to its sink, counting the
    pairs that cross a block boundary; the maximum over all paths."""
    best = 0
    for r in range(code.shape[0]):
        for c in range(code.shape[1]):
            cur, n = (r, c), 0
            while True:
                nxt = _target(code, *cur)
                if nxt is None:
                    break
                n += _block(code.shape, blk, *cur) != _block(code.shape, blk, *nxt)
                cur = nxt
            best = max(best, n)
    return best


def _max_crossings_mfd(z, blk):
    """Longest path, counted in block crossings, through the DAG of
    lower-neighbour edges (cells taken from high to low, plain Python)."""
    mask, _ = oracle.mfd_fractions(z, 1.1)
    nr, nc = z.shape
    cells = sorted(((float(z[r, c]), -(r * nc + c)) for r in range(nr) for c in range(nc)), reverse=True)
    L = np.zeros(z.shape, dtype=np.int64)
    for _, neg in cells:
        i = -neg
        r, c = divmod(i, nc)
        for k, (dr, dc) in enumerate(oracle.OFFSETS):
            if not (mask[r, c] >> k) & 1:
                continue
            rr, cc = r + dr, c + dc
            step = int(_block(z.shape, blk, r, c) != _block(z.shape, blk, rr, cc))
            L[rr, cc] = max(L[rr, cc], L[r, c] + step)
    return int(L.max())


@pytest.mark.parametrize("rule", [oracle.D8, oracle.D4, oracle.MFD])
def test_block_richardson_one_block_is_the_sequential_solve(rule):
    # One process: D = A, R = 0, so one iteration gives the exact solution,
    # and it is the high-to-low push itself (Section 3.2).
    z = synth.dem(61, 30, 37)
    rain = synth.rain(61, 30, 37)
    if rule == oracle.MFD:
        ref_q = oracle.accumulate_mfd(z, rain, 1.1)
        ref_c = None
    else:
        ref_q, _ = oracle.accumulate_single(oracle.receivers(z, rule), rain, z=z)
        _, ref_c = oracle.accumulate_single(oracle.receivers(z, rule), None, z=z)
    for scheme in (0, 1):
        q, cnt, it = oracle.block_richardson(z, (30, 37), rule, rain, scheme)
        assert it == 1
        assert np.array_equal(q, ref_q)
        if ref_c is not None:
            assert np.array_equal(cnt, ref_c)


@pytest.mark.parametrize("seed,shape,blk", [(62, (40, 33), (10, 11)), (63, (24, 50), (6, 7)),
                                            (64, (31, 31), (31, 4)), (65, (20, 20), (1, 1))])
@pytest.mark.parametrize("rule", [oracle.D8, oracle.D4])
def test_block_richardson_needs_crossings_plus_one_iterations(seed, shape, blk, rule):
    # Appendix B: with streams crossing block boundaries at most C times the
    # I+X iterate is exact after C+1 iterations and not before; the
    # (I-X)(I+X) scheme squares the iteration's error operator (about half
    # the iterations, Section 3.3): ceil((C+1)/2).
    z = synth.dem(seed, *shape)
    code = oracle.receivers(z, rule)
    C = _max_crossings_d8(code, blk)
    ref_q, ref_c = oracle.accumulate_single(code, synth.rain(seed, *shape), z=z)
    _, ref_c = oracle.accumulate_single(code, None, z=z)
    q, cnt, it0 = oracle.block_richardson(z, blk, rule, synth.rain(seed, *shape), 0)
    assert it0 == C + 1
    assert np.array_equal(cnt, ref_c)
    assert np.allclose(q, ref_q, rtol=1e-12, atol=0)
    q1, cnt1, it1 = oracle.block_richardson(z, blk, rule, synth.rain(seed, *shape), 1)
    assert it1 == (C + 2) // 2
    assert np.array_equal(cnt1, ref_c)
    assert np.allclose(q1, ref_q, rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed,shape,blk", [(66, (21, 18), (7, 6)), (67, (16, 30), (4, 10))])
def test_block_richardson_mfd_crossings_plus_one(seed, shape, blk):
    z = synth.dem(seed, *shape)
    C = _max_crossings_mfd(z, blk)
    ref = oracle.accumulate_mfd(z, None, 1.1)
    q, _, it0 = oracle.block_richardson(z, blk, oracle.MFD, None, 0)
    assert it0 == C + 1
    assert np.allclose(q, ref, rtol=1e-12, atol=0)
    q1, _, it1 = oracle.block_richardson(z, blk, oracle.MFD, None, 1)
    assert it1 == (C + 2) // 2
    assert np.allclose(q1, ref, rtol=1e-12, atol=0)


# --------------------------------------------------------------------------
# Depression filling (Section 4: priority flood before routing).

def _fill_relaxation(z, conn, eps):
    """Independent brute force: start from +inf inside, z on the boundary,
    and apply F <- max(z, min(F, next(F_n))) to every cell at once until
    nothing changes (Bellman-Ford order instead of the oracle's heap)."""
    z = np.asarray(z, dtype=np.float32) + np.float32(0.0)
    nr, nc = z.shape
    f = np.full((nr + 2, nc + 2), np.inf, dtype=np.float32)  # padded: off-grid = +inf
    inner = f[1:-1, 1:-1]
    inner[...] = np.inf
    bnd = np.zeros((nr, nc), dtype=bool)
    bnd[0, :] = bnd[-1, :] = bnd[:, 0] = bnd[:, -1] = True
    inner[bnd] = z[bnd]
    offs = [(dr, dc) for dr, dc in OFFS if conn == 8 or dr == 0 or dc == 0]
    while True:
        m = np.full((nr, nc), np.inf, dtype=np.float32)
        for dr, dc in offs:
            m = np.minimum(m, f[1 + dr:1 + dr + nr, 1 + dc:1 + dc + nc])
        if eps:
            m = np.nextafter(m, np.float32(np.inf))
        new = np.where(bnd, z, np.maximum(z, np.minimum(inner, m)))
        if np.array_equal(new, inner):
            return new
        inner[...] = new


def _fill_mst_bottleneck(z, conn):
    """Plain fill from a library minimum spanning tree: the filled level of
    a cell is the largest edge on its tree path to a virtual outside node,
    edges weighted max(z_u, z_v) between neighbours and z_b from each
    boundary cell (the minimax-path property of spanning trees)."""
    from scipy.sparse.csgraph import breadth_first_order, minimum_spanning_tree
    z = np.asarray(z, dtype=np.float64)
    nr, nc = z.shape
    n = nr * nc
    shift = 1.0 - z.min()  # csgraph drops zero weights: make all positive
    rows, cols, w = [], [], []
    for r in range(nr):
        for c in range(nc):
            i = r * nc + c
            for dr, dc in OFFS:
                if conn == 4 and dr != 0 and dc != 0:
                    continue
                rr, cc = r + dr, c + dc
                if 0 <= rr < nr and 0 <= cc < nc and rr * nc + cc > i:
                    rows.append(i)
                    cols.append(rr * nc + cc)
                    w.append(max(z[r, c], z[rr, cc]) + shift)
            if r in (0, nr - 1) or c in (0, nc - 1):
                rows.append(i)
                cols.append(n)
                w.append(z[r, c] + shift)
    g = sp.coo_matrix((w, (rows, cols)), shape=(n + 1, n + 1)).tocsr()
    t = minimum_spanning_tree(g)
    t = (t + t.T).tocsr()
    order_, pred = breadth_first_order(t, n, directed=False)
    level = np.zeros(n + 1)
    level[n] = -np.inf
    for v in order_[1:]:
        level[v] = max(level[pred[v]], t[pred[v], v])
    return (level[:n] - shift).reshape(nr, nc)


def _pit_dem(seed, nr, nc):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 12, size=(nr, nc)).astype(np.float32) * np.float32(0.5)


@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("seed,shape", [(1, (9, 11)), (2, (13, 7)), (3, (3, 20)), (4, (17, 17))])
def test_fill_plain_matches_spanning_tree_bottleneck(conn, seed, shape):
    z = _pit_dem(seed, *shape)
    f = oracle.fill_depressions(z, conn, eps=False)
    ref = _fill_mst_bottleneck(z, conn)
    assert np.array_equal(f.astype(np.float64), ref)


@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("seed,shape", [(5, (9, 11)), (6, (16, 23)), (7, (1, 9)), (8, (2, 2)), (9, (30, 4))])
def test_fill_matches_brute_force_relaxation(conn, seed, shape):
    z = _pit_dem(seed, *shape)
    for eps in (False, True):
        assert np.array_equal(oracle.fill_depressions(z, conn, eps), _fill_relaxation(z, conn, eps))
    zf = synth.dem(seed, 40, 37)
    assert np.array_equal(oracle.fill_depressions(zf, conn, True), _fill_relaxation(zf, conn, True))


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_crater_closed_form(conn):
    # Rim at 10 with one spill cell at 5 on the top edge, flat floor at 0:
    # the floor fills to 5, and with eps each floor cell sits one float32
    # step above the cell before it on a shortest hop path to the spill
    # (Chebyshev distance for 8 neighbours, Manhattan for 4).
    nr, nc, k = 9, 12, 4
    z = np.full((nr, nc), 10.0, dtype=np.float32)
    z[1:-1, 1:-1] = 0.0
    z[0, k] = 5.0
    plain = oracle.fill_depressions(z, conn, eps=False)
    assert np.all(plain[1:-1, 1:-1] == 5.0) and np.array_equal(plain[0], z[0])
    f = oracle.fill_depressions(z, conn, eps=True)
    for i in range(1, nr - 1):
        for j in range(1, nc - 1):
            d = max(i, abs(j - k)) if conn == 8 else i + abs(j - k)
            v = np.float32(5.0)
            for _ in range(d):
                v = np.nextafter(v, np.float32(np.inf))
            assert f[i, j] == v, (i, j)
    assert np.array_equal(f[[0, -1]], z[[0, -1]]) and np.array_equal(f[:, [0, -1]], z[:, [0, -1]])


@pytest.mark.parametrize("rule,conn", [(oracle.D8, 8), (oracle.D4, 4)])
def test_fill_invariants_and_drainage(rule, conn):
    z = synth.dem(11, 120, 97)
    f = oracle.fill_depressions(z, conn, True)
    assert np.all(f >= z)
    bnd = np.zeros(z.shape, dtype=bool)
    bnd[0, :] = bnd[-1, :] = bnd[:, 0] = bnd[:, -1] = True
    assert np.array_equal(f[bnd], z[bnd])
    # The DEM had interior pits; after filling every interior cell drains.
    code0 = oracle.receivers(z, rule)
    assert np.any((code0 == oracle.SINK) & ~bnd)
    code = oracle.receivers(f, rule)
    assert not np.any((code == oracle.SINK) & ~bnd)
    # Idempotent, and a surface that already drains is left alone.
    assert np.array_equal(oracle.fill_depressions(f, conn, True), f)
    plain = oracle.fill_depressions(z, conn, False)
    assert np.array_equal(oracle.fill_depressions(plain, conn, False), plain)
    assert np.all(f >= plain)
    rr, cc = np.mgrid[0:50, 0:60]
    tilt = (rr + 2 * cc).astype(np.float32)
    assert np.array_equal(oracle.fill_depressions(tilt, conn, True), tilt)
    # Tight: each raised cell sits one step above its lowest neighbour.
    pad = np.pad(f, 1, constant_values=np.inf)
    offs = [(dr, dc) for dr, dc in OFFS if conn == 8 or dr == 0 or dc == 0]
    m = np.min([pad[1 + dr:1 + dr + f.shape[0], 1 + dc:1 + dc + f.shape[1]] for dr, dc in offs], axis=0)
    raised = (f > z) & ~bnd
    assert np.any(raised)
    assert np.array_equal(f[raised], np.nextafter(m, np.float32(np.inf))[raised])
    # Section 4 check on the filled DEM: all rain leaves through the boundary.
    rain = synth.rain(11, *z.shape)
    q, _ = oracle.accumulate_single(code, rain, z=f)
    out, total = oracle.mass_single(code, q, rain)
    assert abs(out - total) <= 1e-12 * total


def test_fill_rejects_non_finite():
    z = np.zeros((4, 4), dtype=np.float32)
    z[2, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.fill_depressions(z)
