"""Stream ordering: fr_receivers, fr_accumulate and fr_accumulate_adjoint
enqueue a fixed sequence of kernels and never wait for the host, so they can
be captured in a HIP graph.  Each case captures the calls once, replays the
graph several times with the program's own eager work (other routes,
synchronisations) in between, and checks every replay bit for bit against
an eager call on the same inputs -- also after new input values are copied
into the captured buffers.  The eager result itself is checked against the
oracle.  A second group runs the same route twice and compares the bits
(the D8 exit forest sums in exact integer arithmetic).
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


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nz = b != 0
    return float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz])))


def route_fn(z, rain, rule, dtype, counts, ws, mass=True):
    """One receivers + accumulate call pair on the current stream, no host
    synchronisation (status words are read after the replays)."""
    status = torch.zeros(1, dtype=torch.int32, device="cuda")

    def fn():
        code = fr.receivers(z, rule, check=False)
        zz = z if rule == "mfd" else None
        q, cnt, m = fr.accumulate(code, zz, rain, rule, dtype, counts=counts, mass=mass, ws=ws, check=False)
        return [x for x in (code, q, cnt, m) if x is not None]

    return fn, status


def capture(fn):
    """Warm up eagerly on a side stream (allocates the workspace), then
    capture fn() into a graph; returns (graph, captured outputs)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = fn()
    torch.cuda.synchronize()
    return g, out


def same_bits(a, b):
    return a.shape == b.shape and torch.equal(a.view(torch.uint8).flatten(), b.view(torch.uint8).flatten()) \
        if a.dtype != torch.uint8 else torch.equal(a, b)


def check_replays(g, out, eager_fn, swap=None):
    """Replays the graph three times, with eager routes in between, and once
    more after `swap()` changed the captured inputs' contents."""
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        ref = eager_fn()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert same_bits(a, b), f"replay {rep}: {a.dtype} differs from the eager call"
    if swap is not None:
        swap()
        g.replay()
        torch.cuda.synchronize()
        ref = eager_fn()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert same_bits(a, b), "replay after new inputs differs from the eager call"


CASES = [
    # name, shape, rule, dtype, counts, seed
    ("d8_f32_counts", (513, 777), "d8", torch.float32, True, 31),
    ("d8_f64_counts", (300, 1031), "d8", torch.float64, True, 32),
    ("d4_counts_only", (256, 256), "d4", None, True, 33),
    # Above 2^22 cells: the exit list holds an eighth of the cells and the
    # engine's gated fallback is part of the captured sequence.
    ("d8_f32_large", (2100, 2100), "d8", torch.float32, True, 34),
    ("mfd_f32", (384, 520), "mfd", torch.float32, False, 35),
    ("mfd_f64", (257, 300), "mfd", torch.float64, False, 36),
]


@pytest.mark.parametrize("name,shape,rule,dtype,counts,seed", CASES)
def test_graph_replay_equals_eager_route(name, shape, rule, dtype, counts, seed):
    print(f"capture {name} {shape}", flush=True)
    z_h = synth.dem(seed, *shape)
    rain_h = synth.rain(seed, *shape)
    z, rain = dev(z_h), dev(rain_h)
    ws = fr.Workspace()
    fn, _ = route_fn(z, rain, rule, dtype, counts, ws, mass=dtype is not None)
    g, out = capture(fn)
    ws_eager = fr.Workspace()
    eager_fn, _ = route_fn(z, rain, rule, dtype, counts, ws_eager, mass=dtype is not None)
    # The eager call against the oracle (so the replays are compared with a
    # checked result).
    ref = eager_fn()
    torch.cuda.synchronize()
    r = oracle.MFD if rule == "mfd" else (oracle.D4 if rule == "d4" else oracle.D8)
    if rule == "mfd":
        qref = oracle.accumulate_mfd(z_h, rain_h, 1.1)
        e = np.linalg.norm(ref[1].cpu().numpy().astype(np.float64) - qref) / np.linalg.norm(qref)
        assert e <= (1e-6 if dtype == torch.float32 else 1e-10)
    else:
        code_h = oracle.receivers(z_h, r)
        assert np.array_equal(ref[0].cpu().numpy(), code_h)
        qref, cref = oracle.accumulate_single(code_h, rain_h, z=z_h)
        k = 1
        if dtype is not None:
            assert relmax(ref[1].cpu().numpy(), qref) <= (1e-6 if dtype == torch.float32 else 1e-10)
            k = 2
        _, cref = oracle.accumulate_single(code_h, None, z=z_h)
        assert np.array_equal(ref[k].cpu().numpy().astype(np.uint64), cref)

    def swap():
        z2 = synth.dem(seed + 100, *shape)
        z.copy_(dev(z2))
        rain.copy_(dev(synth.rain(seed + 100, *shape)))

    check_replays(g, out, eager_fn, swap)


@pytest.mark.parametrize("rule,dtype,shape,seed", [("mfd", torch.float32, (300, 450), 41),
                                                   ("mfd", torch.float64, (200, 333), 42),
                                                   ("d8", torch.float64, (260, 515), 43)])
def test_graph_replay_equals_eager_adjoint(rule, dtype, shape, seed):
    print(f"capture adjoint {rule} {dtype} {shape}", flush=True)
    z_h = synth.dem(seed, *shape)
    z = dev(z_h)
    code = fr.receivers(z, rule)
    qbar_h = np.zeros(shape)
    cells = synth.distinct_cells(seed, synth.STREAM_PICK, 32, shape[0] * shape[1])
    qbar_h.reshape(-1)[cells] = synth.normal(seed, synth.STREAM_NORMAL, 32)
    qbar = dev(qbar_h).to(dtype)
    zz = z if rule == "mfd" else None
    ws = fr.Workspace()

    def fn():
        return [fr.adjoint(code, qbar, zz, rule, ws=ws, check=False)]

    g, out = capture(fn)
    ws_e = fr.Workspace()

    def eager_fn():
        return [fr.adjoint(code, qbar, zz, rule, ws=ws_e)]

    ref = eager_fn()[0].cpu().numpy().astype(np.float64)
    if rule == "mfd":
        want = oracle.adjoint_mfd(z_h, qbar.cpu().numpy().astype(np.float64), 1.1)
    else:
        want = oracle.adjoint_single(oracle.receivers(z_h), qbar.cpu().numpy().astype(np.float64), z=z_h)
    e = np.linalg.norm(ref - want) / np.linalg.norm(want)
    assert e <= (1e-6 if dtype == torch.float32 else 1e-10)

    def swap():
        qbar.mul_(-0.5)

    check_replays(g, out, eager_fn, swap)


@pytest.mark.parametrize("path", ["engine", "sweep", "tiles"])
def test_graph_replay_forced_paths(path):
    """The other paths captured on their own: the engine is one persistent
    launch behind the control block's gate; the sweep runs its passes under
    device control; the tile forest (on a filled DEM, flow in every
    direction) joins its tiles with a persistent work queue."""
    print(f"capture forced path {path}", flush=True)
    shape = (300, 517)
    z_h = synth.dem(44, *shape) if path != "tiles" else oracle.fill_depressions(
        synth.dem(44, *shape, tilt=0.0), 8, True)
    rain_h = synth.rain(44, *shape)
    z, rain = dev(z_h), dev(rain_h)
    with fr.accumulate_path(path):
        ws = fr.Workspace()
        fn, _ = route_fn(z, rain, "d8", torch.float32, True, ws)
        g, out = capture(fn)
        ws_e = fr.Workspace()
        eager_fn, _ = route_fn(z, rain, "d8", torch.float32, True, ws_e)
        check_replays(g, out, eager_fn)
    _, cref = oracle.accumulate_single(oracle.receivers(z_h), None, z=z_h)
    assert np.array_equal(out[2].cpu().numpy().astype(np.uint64), cref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("tilt", [0.01, 0.0])
def test_d8_route_bits_repeat(dtype, tilt):
    """Two routes of the same DEM give the same bits.  The untilted DEM
    drains in every direction: about 60% of its cells are exits, so the
    forest is large and many exits share ancestors."""
    n = 2048
    print(f"determinism d8 {dtype} tilt {tilt} {n}^2", flush=True)
    z = dev(synth.dem(45, n, n, tilt=tilt))
    rain = dev(synth.rain(45, n, n))
    code = fr.receivers(z, "d8")
    outs = []
    for _ in range(3):
        q, cnt, m = fr.accumulate(code, None, rain, "d8", dtype, counts=True, mass=True)
        torch.cuda.synchronize()
        outs.append((q, cnt, m))
    for q, cnt, m in outs[1:]:
        assert same_bits(q, outs[0][0])
        assert torch.equal(cnt, outs[0][1])
        assert same_bits(m, outs[0][2])
