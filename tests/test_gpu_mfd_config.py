"""MFD at its benchmark configuration: a 16384 x 16384 DEM (seed 3), unit
rain, slope exponent p = 1.1 (Appendix A), float32 (float-float sums) and
float64 paths.

The oracle's push takes minutes at this size, so the checks are properties
that hold at any size and determine the solution:
  * the float64 result satisfies the local balance of (I - W^T) q = r at
    every cell, q(c) = r(c) + sum over donors d of f(d -> c) q(d), with the
    fractions f computed here in float64 from the elevations by the
    slope-power law (Section 2.2; Appendix A): relative residual <= 1e-11;
  * the float32 result is within 1e-6 (2-norm) of the float64 one;
  * mass balance (Section 4): water leaving through sinks equals the total
    rain, within 1e-11 (float64) and 1e-6 (float32).
"""
import math

import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2606_12800_amd")

N = 16384
P_EXP = 1.1
OFFS = oracle.OFFSETS


@pytest.fixture(scope="module")
def routed():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"mfd config: generating {N}x{N} DEM (seed 3)", flush=True)
    z = torch.from_numpy(synth.dem(3, N, N)).cuda()
    print("mfd config: routing float32 and float64", flush=True)
    _, q32, _, m32 = fr.route(z, None, "mfd", torch.float32, mass=True)
    _, q64, _, m64 = fr.route(z, None, "mfd", torch.float64, mass=True)
    torch.cuda.synchronize()
    yield z, q32, q64, m32, m64
    del z, q32, q64
    torch.cuda.empty_cache()


def _shift(a, dr, dc, fill):
    """b[i, j] = a[i + dr, j + dc], `fill` where that lies outside a."""
    b = torch.full_like(a, fill)
    nr, nc = a.shape
    b[max(-dr, 0):nr - max(dr, 0), max(-dc, 0):nc - max(dc, 0)] = \
        a[max(dr, 0):nr - max(-dr, 0), max(dc, 0):nc - max(-dc, 0)]
    return b


def test_mfd_config_local_balance_float64(routed):
    z, _, q64, _, _ = routed
    band = 2048
    worst = 0.0
    for r0 in range(0, N, band):
        r1 = min(r0 + band, N)
        # Donors of the band's cells lie one row outside it; their fractions
        # need their own neighbours, one row further.
        a, b = max(r0 - 2, 0), min(r1 + 2, N)
        zb = z[a:b].double()
        inf = float("inf")
        # Weights of each cell toward each neighbour k: s^p over strictly
        # lower neighbours, s = drop / distance; neighbours off the grid do
        # not exist (off-band rows at the grid edge are off the grid).
        w = []
        for dr, dc in OFFS:
            zn = _shift(zb, dr, dc, inf)
            if a == 0 and dr < 0:
                zn[0] = inf
            if b == N and dr > 0:
                zn[-1] = inf
            dist = math.sqrt(2.0) if dr != 0 and dc != 0 else 1.0
            s = torch.where(zn < zb, (zb - zn) / dist, torch.zeros_like(zb))
            w.append(torch.where(s > 0, torch.pow(s, P_EXP), torch.zeros_like(zb)))
        wsum = sum(w)
        qb = q64[a:b]
        inflow = torch.zeros_like(zb)
        for k, (dr, dc) in enumerate(OFFS):
            # Neighbour n = c + (dr, dc) gives c the share of direction 7 - k.
            share = torch.where(wsum > 0, w[7 - k] / wsum, torch.zeros_like(zb))
            inflow += _shift(share * qb, dr, dc, 0.0)
        lo, hi = r0 - a, r0 - a + (r1 - r0)
        res = (qb[lo:hi] - 1.0 - inflow[lo:hi]).abs() / qb[lo:hi]
        worst = max(worst, res.max().item())
        del zb, w, wsum, inflow, res
    print(f"  float64 local-balance residual (relative, max) {worst:.3e}")
    assert worst <= 1e-11


def test_mfd_config_float32_and_mass(routed):
    _, q32, q64, m32, m64 = routed
    e = (torch.linalg.vector_norm(q32.double() - q64) / torch.linalg.vector_norm(q64)).item()
    emax = ((q32.double() - q64).abs() / q64).max().item()
    print(f"  float32 vs float64: relative 2-norm {e:.3e}, max per cell {emax:.3e}")
    assert e <= 1e-6
    # Per cell: the float32 fractions (a few ulp each) compound along flow
    # paths of ~16k cells; reported, and held to 1e-5.
    assert emax <= 1e-5
    s64, t64 = m64.cpu().tolist()
    s32, t32 = m32.cpu().tolist()
    assert t64 == float(N * N) and t32 == float(N * N)
    assert abs(s64 - t64) <= 1e-11 * t64
    assert abs(s32 - t32) <= 1e-6 * t32
