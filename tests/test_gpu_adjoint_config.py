"""The adjoint at its benchmark configuration: MFD on a 4096 x 4096 DEM
(seed 5), loss L(r) = sum_g w_g q_g over 64 distinct gauge cells (seed 6),
w ~ N(0, 1); the gradient dL/dr is the transpose solve (I - W) rbar = qbar
with qbar = sum_g w_g e_g (the adjoint of Section 2.2's (I - W^T) q = r).

Checks:
  * rbar (float64 GPU) against the oracle's transpose solve, <= 1e-10 of
    max |rbar|; the float32 (float-float) adjoint within 1e-6 (2-norm), the
    tolerance the method's float32 results are held to;
  * central finite differences on 100 cells -- 50 uniform over the grid, 50
    from the support of rbar -- with the float64 forward solve on the GPU.
    q is linear in r, so with step h = 1 the difference quotient equals the
    derivative up to rounding: agreement to 1e-9 of max |rbar|.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2606_12800_amd")

N = 4096


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("adjoint config: generating 4096^2 DEM", flush=True)
    z = synth.dem(5, N, N)
    zt = torch.from_numpy(z).cuda()
    code = fr.receivers(zt, "mfd")
    cells = synth.distinct_cells(6, synth.STREAM_PICK, 64, N * N)
    w = synth.normal(6, synth.STREAM_NORMAL, 64)
    qbar = np.zeros(N * N)
    qbar[cells] = w
    qbar = qbar.reshape(N, N)
    rbar = fr.adjoint(code, torch.from_numpy(qbar).cuda(), zt, "mfd")
    torch.cuda.synchronize()
    return z, zt, code, cells, w, qbar, rbar.cpu().numpy()


def test_adjoint_config_vs_oracle(setup):
    z, zt, code, cells, w, qbar, rbar = setup
    print("adjoint config: oracle transpose solve", flush=True)
    ref = oracle.adjoint_mfd(z, qbar, 1.1)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.max(np.abs(rbar - ref)) <= 1e-10 * scale
    r32 = fr.adjoint(code, torch.from_numpy(qbar.astype(np.float32)).cuda(), zt, "mfd")
    ref32 = oracle.adjoint_mfd(z, qbar.astype(np.float32).astype(np.float64), 1.1)
    a = r32.cpu().numpy().astype(np.float64)
    e32 = np.linalg.norm(a - ref32) / np.linalg.norm(ref32)
    print(f"  float32 adjoint: relative 2-norm error {e32:.3e}")
    # The float32 fractions are corrected so that every cell passes on
    # exactly the water it holds (float-float), which keeps the error at a
    # few float32 ulp; measured 3.3e-8.
    assert e32 <= 1e-6


def test_adjoint_config_central_differences(setup):
    z, zt, code, cells, w, qbar, rbar = setup
    support = np.flatnonzero(rbar.ravel() != 0)
    uni = synth.integers(7, synth.STREAM_PICK, 50, 0, N * N - 1)
    pick = synth.integers(8, synth.STREAM_PICK, 50, 0, len(support) - 1)
    probe = np.concatenate([uni, support[pick]])
    rain = torch.from_numpy(synth.rain(5, N, N).astype(np.float64)).cuda()
    gauge = torch.from_numpy(cells).cuda()
    wt = torch.from_numpy(w).cuda()

    def loss(r):
        q, _, _ = fr.accumulate(code, zt, r, "mfd", torch.float64)
        return float((q.view(-1)[gauge] * wt).sum().item())

    scale = np.abs(rbar).max()
    print(f"adjoint config: {len(probe)} central differences", flush=True)
    worst = 0.0
    for i in probe:
        r = rain.clone()
        r.view(-1)[int(i)] += 1.0
        lp = loss(r)
        r.view(-1)[int(i)] -= 2.0
        lm = loss(r)
        fd = (lp - lm) / 2.0
        worst = max(worst, abs(fd - rbar.ravel()[int(i)]))
    print(f"  max |FD - rbar| = {worst:.3e} (max |rbar| {scale:.3e})")
    assert worst <= 1e-9 * scale
