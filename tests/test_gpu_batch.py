"""Batched routing (one persistent launch for many tiles) against per-tile
results and the oracle.

Tiles of uneven shapes (1 row, 1 column, narrower than one strip, several
strips with ragged tails) and mixed rules: D8/D4 with uint64 counts or
float32 water, MFD with float32 water.  Bars as for single grids: codes and
counts bit-exact; float32 water within 1e-6 of the float64 oracle
(relative 2-norm for MFD, per cell for D8); MFD water bit-identical to the
single-grid wavefront sweep (same arithmetic in the same order).
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


def relnorm(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nz = b != 0
    return float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) if nz.any() else 0.0


SHAPES = [(1, 1), (1, 90), (90, 1), (37, 40), (64, 48), (65, 49), (200, 97), (333, 260), (128, 700),
          (511, 129), (96, 96), (300, 47)]


def make_tiles(shapes, seed0, with_rain):
    tiles, ref = [], []
    for i, (nr, nc) in enumerate(shapes):
        seed = seed0 + i
        z = synth.dem(seed, nr, nc)
        rule = ["d8", "mfd", "d4"][i % 3]
        rain = synth.rain(seed, nr, nc) if (with_rain and i % 2 == 0) else None
        t = {"z": dev(z), "rule": rule, "code": torch.empty((nr, nc), dtype=torch.uint8, device="cuda")}
        if rain is not None:
            t["rain"] = dev(rain)
        if rule == "mfd" or i % 4 == 1:
            t["q"] = torch.empty((nr, nc), dtype=torch.float32, device="cuda")
        else:
            t["counts"] = torch.empty((nr, nc), dtype=torch.int64, device="cuda")
        tiles.append(t)
        ref.append((z, rain))
    return tiles, ref


@pytest.mark.parametrize("with_rain", [False, True])
def test_batch_matches_oracle(with_rain):
    print(f"batch, rain={with_rain}", flush=True)
    tiles, ref = make_tiles(SHAPES, 500, with_rain)
    b = fr.Batch(tiles)
    b.run()
    for t, (z, rain) in zip(tiles, ref):
        rule = t["rule"]
        code = host(t["code"])
        rcode = oracle.receivers(z, oracle.D4 if rule == "d4" else oracle.D8) if rule != "mfd" else None
        if rule == "mfd":
            assert np.array_equal(code, host(fr.receivers(t["z"], "mfd")))
            qref = oracle.accumulate_mfd(z, rain, 1.1)
            assert relnorm(host(t["q"]), qref) <= 1e-6, z.shape
        else:
            assert np.array_equal(code, rcode), z.shape
            qref, cref = oracle.accumulate_single(code, rain, z=z)
            if "counts" in t:
                assert np.array_equal(host(t["counts"]).astype(np.uint64), cref), z.shape
            else:
                assert relmax(host(t["q"]), qref) <= 1e-6, z.shape


def test_batch_mfd_bitwise_equals_single_grid_sweep():
    shapes = [(300, 260), (129, 500), (64, 64)]
    tiles = []
    for i, (nr, nc) in enumerate(shapes):
        z = synth.dem(700 + i, nr, nc)
        tiles.append({"z": dev(z), "rule": "mfd", "rain": dev(synth.rain(700 + i, nr, nc)),
                      "q": torch.empty((nr, nc), dtype=torch.float32, device="cuda")})
    fr.Batch(tiles).run()
    for t in tiles:
        code = fr.receivers(t["z"], "mfd")
        q, _, _ = fr.accumulate(code, t["z"], t["rain"], "mfd", torch.float32)
        assert torch.equal(q, t["q"])


def test_batch_repeat_plans_and_graph_replay():
    tiles, _ = make_tiles(SHAPES[3:], 900, True)
    b = fr.Batch(tiles)
    b.run()
    first = [t.get("q", t.get("counts")).clone() for t in tiles]
    for plan in [fr.BatchPlan(0, fr.ORDER_GIVEN), fr.BatchPlan(64, fr.ORDER_ROWS_DESC), fr.BatchPlan(16, fr.ORDER_GIVEN)]:
        for t in tiles:
            t.get("q", t.get("counts")).zero_()
        b.run(plan=plan)
        for t, f in zip(tiles, first):
            assert torch.equal(t.get("q", t.get("counts")), f)
    # HIP graph: capture one routing, replay it with eager work in between.
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.run(check=False)  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            b.run(check=False)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for t in tiles:
            t.get("q", t.get("counts")).fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for t, f in zip(tiles, first):
            assert torch.equal(t.get("q", t.get("counts")), f), rep
    assert int(b.status.item()) == 0


def test_batch_errors_and_empty():
    b = fr.Batch([])
    b.run()
    z = synth.dem(3, 20, 30)
    z[4, 5] = np.nan
    b = fr.Batch([{"z": dev(z), "rule": "d8", "counts": torch.empty((20, 30), dtype=torch.int64, device="cuda")}])
    with pytest.raises(fr.FlowRouteError) as e:
        b.run()
    assert e.value.code == fr.ERR_NONFINITE
    with pytest.raises(fr.FlowRouteError):
        # a D8 tile needs exactly one of q / counts
        fr.Batch([{"z": dev(synth.dem(3, 8, 8)), "rule": "d8"}])


def test_batch_autotune_picks_a_plan_and_caches_it(tmp_path):
    path = str(tmp_path / "plans.txt")
    fr.set_autotune_cache(path)
    try:
        tiles, _ = make_tiles(SHAPES[5:9], 1200, False)
        b = fr.Batch(tiles)
        plan = b.autotune(reps=1)
        assert plan.workers > 0 and plan.order in (fr.ORDER_GIVEN, fr.ORDER_ROWS_DESC, fr.ORDER_CELLS_DESC)
        b.run()
        # The signature is cached: a batch of the same shapes gets the same
        # plan without timing, also from the file in a fresh cache.
        tiles2, _ = make_tiles(SHAPES[5:9], 1300, False)
        p2 = fr.Batch(tiles2).autotune(reps=1)
        assert (p2.workers, p2.order) == (plan.workers, plan.order)
        lines = open(path).read().split()
        assert len(lines) == 3 and int(lines[1]) == plan.workers and int(lines[2]) == plan.order
        # Every order runs and gives the same results.
        ref = [t["q"].clone() if "q" in t else t["counts"].clone() for t in tiles]
        for order in (fr.ORDER_GIVEN, fr.ORDER_ROWS_DESC, fr.ORDER_CELLS_DESC):
            b.run(plan=fr.BatchPlan(0, order))
            for t, r in zip(tiles, ref):
                assert torch.equal(t["q"] if "q" in t else t["counts"], r), order
    finally:
        fr.set_autotune_cache(None)


def test_batch_fullconfig_equals_single_grid_calls():
    """The bench's batched workload: 512 tiles, sides uniform in [64, 2048]
    (seed 4), tile i from seed 1000 + i, even tiles D8 with uint64 counts,
    odd tiles MFD with float32 water, unit rain, autotuned plan.  D8 counts
    bit-exact against single-grid calls (oracle-checked elsewhere); MFD water
    bitwise equal to the single-grid wavefront sweep."""
    shapes = synth.batch_shapes(4, 512)
    print(f"batched config: {len(shapes)} tiles, {sum(a * b for a, b in shapes) / 1e6:.1f} Mcells", flush=True)
    tiles = []
    for i, (nr, nc) in enumerate(shapes):
        t = {"z": dev(synth.dem(1000 + i, nr, nc)), "rule": "d8" if i % 2 == 0 else "mfd"}
        if i % 2 == 0:
            t["counts"] = torch.empty((nr, nc), dtype=torch.int64, device="cuda")
        else:
            t["q"] = torch.empty((nr, nc), dtype=torch.float32, device="cuda")
        tiles.append(t)
    b = fr.Batch(tiles)
    b.run(plan=b.autotune(reps=1))
    torch.cuda.synchronize()
    for i, t in enumerate(tiles):
        code = fr.receivers(t["z"], t["rule"])
        if i % 2 == 0:
            _, c, _ = fr.accumulate(code, None, None, "d8", None, counts=True)
            assert torch.equal(c.view(torch.int64), t["counts"]), i
        else:
            q, _, _ = fr.accumulate(code, t["z"], None, "mfd", torch.float32)
            assert torch.equal(q, t["q"]), i
    del tiles, b
    torch.cuda.empty_cache()
