"""Full-size checks at the benchmark's launch configuration: the 43,360 x
43,360 (1.88e9-cell) D8 route with float32 rain and uint64 counts, and the
paper's own grid shape, 57,345 x 32,769 (Section 4; rows not 4-cell
aligned, so the unaligned load and store variants run).

The oracle cannot route 1.88e9 cells within a test, so the checks are
(a) receivers bit-exact against the oracle on sampled row bands (a cell's
    receiver depends only on its 3x3 neighbourhood, so the oracle routes a
    3-row slab and its middle row is exact);
(b) properties that hold at any size and, together, determine the solution:
    every cell's count equals 1 + the counts of its donors (the local
    balance of (I - W^T) q = r, Section 2.2), the same for the float32
    water within float tolerance, all cells drain to sinks (sum over sinks =
    N), and the float64 mass balance of Section 4.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2606_12800_amd")

OFFS = oracle.OFFSETS


@pytest.fixture(scope="module", params=[(43360, 43360), (57345, 32769)], ids=["43360sq", "paper_shape"])
def routed(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nr, nc = request.param
    print(f"generating {nr}x{nc} DEM", flush=True)
    z_h = synth.dem(2, nr, nc)
    rain_h = synth.rain(2, nr, nc)
    z = torch.from_numpy(z_h).cuda()
    rain = torch.from_numpy(rain_h).cuda()
    print(f"routing {nr}x{nc}", flush=True)
    code, q, cnt, mass = fr.route(z, rain, "d8", torch.float32, counts=True, mass=True)
    torch.cuda.synchronize()
    yield z_h, rain_h, z, rain, code, q, cnt, mass
    del z, rain, code, q, cnt
    torch.cuda.empty_cache()


def test_fullsize_receivers_sampled_rows(routed):
    z_h, _, _, _, code, _, _, _ = routed
    N = z_h.shape[0]
    rows = sorted(set([0, 1, N // 2, N - 2, N - 1] + synth.integers(8, synth.STREAM_PICK, 20, 1, N - 2).tolist()))
    for r in rows:
        lo, hi = max(r - 1, 0), min(r + 2, N)
        ref = oracle.receivers(z_h[lo:hi])[r - lo]
        got = code[r].cpu().numpy()
        # The slab has no rows beyond it; only its middle row (or a grid
        # border row) sees its full neighbourhood.
        assert np.array_equal(got, ref), r


def test_fullsize_counts_local_balance_and_sinks(routed):
    _, _, _, _, code, _, cnt, _ = routed
    N, NC = code.shape
    c = cnt.view(torch.int64)
    for r0 in range(0, N, 4096):
        r1 = min(r0 + 4096, N)
        a, b = max(r0 - 1, 0), min(r1 + 1, N)
        band_code, band_c = code[a:b], c[a:b]
        out = torch.zeros_like(band_c)
        n_r = b - a
        for k, (dr, dc) in enumerate(OFFS):
            src_r = slice(max(-dr, 0), n_r - max(dr, 0))
            dst_r = slice(max(dr, 0), n_r - max(-dr, 0))
            src_c = slice(max(-dc, 0), NC - max(dc, 0))
            dst_c = slice(max(dc, 0), NC - max(-dc, 0))
            m = band_code[src_r, src_c] == k
            out[dst_r, dst_c] += torch.where(m, band_c[src_r, src_c], torch.zeros((), dtype=torch.int64, device=c.device))
        inner = slice(r0 - a, r0 - a + (r1 - r0))
        assert torch.equal(band_c[inner], out[inner] + 1), (r0, r1)
    assert int(c[code == 0xFF].sum().item()) == N * NC


def test_fullsize_water_local_balance_and_mass(routed):
    _, rain_h, _, rain, code, q, _, mass = routed
    N, NC = code.shape
    for r0 in range(0, N, 4096):
        r1 = min(r0 + 4096, N)
        a, b = max(r0 - 1, 0), min(r1 + 1, N)
        band_code, band_q = code[a:b], q[a:b].double()
        out = torch.zeros_like(band_q)
        n_r = b - a
        for k, (dr, dc) in enumerate(OFFS):
            src_r = slice(max(-dr, 0), n_r - max(dr, 0))
            dst_r = slice(max(dr, 0), n_r - max(-dr, 0))
            src_c = slice(max(-dc, 0), NC - max(dc, 0))
            dst_c = slice(max(dc, 0), NC - max(-dc, 0))
            m = band_code[src_r, src_c] == k
            out[dst_r, dst_c] += torch.where(m, band_q[src_r, src_c], torch.zeros((), dtype=torch.float64, device=q.device))
        inner = slice(r0 - a, r0 - a + (r1 - r0))
        expect = out[inner] + rain[r0:r1].double()
        # (a cell with zero rain and no donors holds exactly zero)
        rel = ((band_q[inner] - expect).abs() / expect.clamp(min=1e-30)).max().item()
        # q is float32 rounded from a float-float value; its donors are too.
        assert rel <= 1e-6, (r0, r1, rel)
    s, t = mass.cpu().numpy()
    assert abs(s - t) <= 1e-6 * t
    assert t == pytest.approx(float(rain_h.astype(np.float64).sum()), rel=1e-12)
