"""The paper's block iterations (Section 3.3 "I+X" and "(I-X)(I+X)",
Appendix B) on the GPU.

fr_accumulate_block_iterations runs w <- D^-1 (r + R w) (scheme "ix") or
w <- w + (I - X)(b - (I + X) w) (scheme "imx_ix") with D^-1 the exact solve
of every block of block = (rows, cols) cells: D holds every routing pair
inside a block, R every pair between blocks -- the paper's splitting.
Checks against the oracle's block iteration with the same blocks
(oracle.block_richardson, the per-block high-to-low push): the iteration
count (C + 1 for "ix", ceil((C + 1) / 2) for "imx_ix", C the most block
crossings along a flow path), float64 water against the direct solve and
counts bit-exact.

Water tolerance.  Scheme "ix" adds the same positive terms as the direct
solve in another order: <= 1e-10 per cell, the float64 bar.  Scheme
"imx_ix" also forms the residual b - w + D^-1 R w, a difference of values
as large as the cell's own water, whose rounding (a few eps q per
iteration) is carried downstream by the next solves: at most about
eps * iterations * A relative to q for a cell draining A cells.  With
A <= 5.3e3 and <= 15 iterations here that is 9e-12: the same 1e-10 bar.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2606_12800_amd")

# Block shapes (rows, cols): multiples of 16 rows and 256 columns, or the
# whole extent; several tiles per block where the shapes allow it.
BLOCKS = [(256, 256), (128, 512), (64, 256), (512, 100000)]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fr.load_library()
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("seed,shape", [(71, (600, 700)), (72, (513, 259)), (73, (1, 900)), (74, (777, 1)),
                                        (75, (300, 1031))])
@pytest.mark.parametrize("rule", ["d8", "d4"])
@pytest.mark.parametrize("block", BLOCKS)
def test_block_iterations_match_oracle(seed, shape, rule, block):
    print(f"block iterations {rule} seed {seed} shape {shape} block {block}", flush=True)
    r = oracle.D8 if rule == "d8" else oracle.D4
    z = synth.dem(seed, *shape)
    rain = synth.rain(seed, *shape)
    code_h = oracle.receivers(z, r)
    ref_q, _ = oracle.accumulate_single(code_h, rain, z=z)
    _, ref_c = oracle.accumulate_single(code_h, None, z=z)
    _, _, ref_it = oracle.block_richardson(z, block, r, None, 0)
    code = fr.receivers(dev(z), rule)
    assert np.array_equal(code.cpu().numpy(), code_h)
    q, cnt, it = fr.block_iterations(code, dev(rain), rule, block=block)
    torch.cuda.synchronize()
    qh = q.cpu().numpy()
    assert np.max(np.abs(qh - ref_q) / np.maximum(ref_q, 1e-300)) <= 1e-10
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint64), ref_c)
    assert it == ref_it
    # Same counts as the main path (exit forest instead of iterations).
    _, c2, _ = fr.accumulate(code, None, None, rule, None, counts=True)
    assert torch.equal(c2, cnt)


def test_block_iterations_counts_only_and_unit_rain():
    z = synth.dem(76, 520, 300)
    code = fr.receivers(dev(z), "d8")
    _, cnt, it = fr.block_iterations(code, None, "d8", dtype=None)
    q, cnt2, it2 = fr.block_iterations(code, None, "d8")
    assert it == it2 and torch.equal(cnt, cnt2)
    # Unit rain: the water is the cell count.
    assert torch.equal(q, cnt.to(torch.float64))


def test_block_iterations_errors():
    z = synth.dem(77, 64, 64)
    code = fr.receivers(dev(z), "d8")
    with pytest.raises(fr.FlowRouteError) as e:
        fr.block_iterations(fr.receivers(dev(z), "mfd"), None, "mfd")
    assert e.value.code == fr.ERR_RULE
    with pytest.raises(TypeError):
        fr.block_iterations(code, None, "d8", dtype=torch.float32)
    # An iteration budget below C + 1 leaves no fixed point: reported.
    big = synth.dem(78, 900, 300)
    bcode = fr.receivers(dev(big), "d8")
    _, _, it = fr.block_iterations(bcode, None, "d8")
    # Block shapes the row-sweep tiles cannot form.
    with pytest.raises(fr.FlowRouteError) as e:
        fr.block_iterations(bcode, None, "d8", block=(100, 256))
    assert e.value.code == fr.ERR_ARG
    assert it >= 3
    with pytest.raises(fr.FlowRouteError) as e:
        fr.block_iterations(bcode, None, "d8", max_iter=it - 2)
    assert e.value.code == fr.ERR_NOTDAG
    # Empty grid.
    q, cnt, it = fr.block_iterations(torch.empty((0, 5), dtype=torch.uint8, device="cuda"), None, "d8")
    assert it == 0 and q.numel() == 0


@pytest.mark.parametrize("seed,shape", [(81, (600, 700)), (82, (513, 259)), (83, (1, 900)), (84, (777, 1)),
                                        (85, (300, 1031))])
@pytest.mark.parametrize("rule", ["d8", "d4"])
@pytest.mark.parametrize("block", BLOCKS[:2])
def test_preconditioned_block_iterations_match_oracle(seed, shape, rule, block):
    print(f"(I-X)(I+X) block iterations {rule} seed {seed} shape {shape} block {block}", flush=True)
    r = oracle.D8 if rule == "d8" else oracle.D4
    z = synth.dem(seed, *shape)
    rain = synth.rain(seed, *shape)
    code_h = oracle.receivers(z, r)
    ref_q, _ = oracle.accumulate_single(code_h, rain, z=z)
    _, ref_c = oracle.accumulate_single(code_h, None, z=z)
    _, _, ref_it = oracle.block_richardson(z, block, r, None, 1)
    _, _, ix_it = oracle.block_richardson(z, block, r, None, 0)
    code = fr.receivers(dev(z), rule)
    q, cnt, it = fr.block_iterations(code, dev(rain), rule, scheme="imx_ix", block=block)
    torch.cuda.synchronize()
    qh = q.cpu().numpy()
    assert np.max(np.abs(qh - ref_q) / np.maximum(ref_q, 1e-300)) <= 1e-10
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint64), ref_c)
    assert it == ref_it
    # Appendix B: the (I-X)(I+X) error operator is X^2, so ceil((C+1)/2).
    assert it == (ix_it + 1) // 2


def test_preconditioned_block_iterations_counts_only_and_errors():
    z = synth.dem(86, 900, 300)
    code = fr.receivers(dev(z), "d8")
    _, cnt, it = fr.block_iterations(code, None, "d8", dtype=None, scheme="imx_ix")
    _, cnt2, it2 = fr.block_iterations(code, None, "d8", dtype=None)
    assert torch.equal(cnt, cnt2) and it < it2
    # Convergence is decided on the counts: they are required.
    with pytest.raises(fr.FlowRouteError) as e:
        fr.block_iterations(code, None, "d8", counts=False, scheme="imx_ix")
    assert e.value.code == fr.ERR_ARG
    with pytest.raises(ValueError):
        fr.block_iterations(code, None, "d8", scheme="jacobi")
    if it >= 3:
        with pytest.raises(fr.FlowRouteError) as e:
            fr.block_iterations(code, None, "d8", max_iter=it - 2, scheme="imx_ix")
        assert e.value.code == fr.ERR_NOTDAG
    q, cnt, it = fr.block_iterations(torch.empty((3, 0), dtype=torch.uint8, device="cuda"), None, "d8",
                                     scheme="imx_ix")
    assert it == 0 and q.numel() == 0


def test_block_iterations_fullsize_counts_equal_main_path():
    """The bench's block-iteration workload: D8 unit-rain counts on the
    43360^2 DEM (seed 2) by I+X block iterations with blocks of 4096 x 4096
    cells (121 blocks, the paper's per-process subdomains), bit-exact
    against the main path's counts (which the full-size tests check cell by
    cell)."""
    n = 43360
    print(f"block iterations d8 {n}x{n} blocks 4096x4096", flush=True)
    code = fr.receivers(torch.from_numpy(synth.dem(2, n, n)).cuda(), "d8")
    torch.cuda.synchronize()
    _, cnt, it = fr.block_iterations(code, None, "d8", dtype=None, block=(4096, 4096))
    _, c2, _ = fr.accumulate(code, None, None, "d8", None, counts=True)
    print(f"iterations {it}", flush=True)
    assert it > 1 and torch.equal(cnt, c2)
    del code, cnt, c2
    fr._default_ws.buf = None
    torch.cuda.empty_cache()
