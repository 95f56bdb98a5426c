"""The allocation-free entry point (dedisp_execute_noalloc) against
dedisp_execute on the same plans and inputs, bit for bit: two calls in a
row on one plan, the second with a smaller input, where the first is split
into time slices by the fixed scratch; then an 8-bit plan with a kill mask,
16-bit outputs and a row stride, also sliced."""
import numpy as np
import pytest

from paper_1201_5380_amd import Plan, synth
from paper_1201_5380_amd._native import DedispError

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 128 << 20


def _compare(plan, inp, nsamps, stride, cuda):
    import torch
    nout = nsamps - plan.max_delay
    width = stride or nout
    want = torch.full((plan.ndm, width), -1, dtype=plan.output_dtype(), device=cuda)
    got = torch.full((plan.ndm, width), -1, dtype=plan.output_dtype(), device=cuda)
    plan.execute(inp, nsamps, out=want, out_row_stride=stride)
    plan.execute_noalloc(inp, got, nsamps, out_row_stride=stride)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    return nout


def test_noalloc_equals_execute_two_calls(native, cuda):
    import torch
    rng = np.random.default_rng(7)
    plan = Plan(1024, 64e-6, 1581.8, -0.390625, 2).set_dm_list(synth.dm_list_linear(1024, 1000.0))
    n1 = 1 << 19
    raw = torch.from_numpy(rng.integers(0, 256, size=n1 * plan.row_bytes, dtype=np.uint8)).to(cuda)
    # the first call's scratch (two bit planes per channel, 2^19 samples,
    # each row with at least 16 bytes of window margin) exceeds the fixed
    # array, so it runs in more than one time slice
    assert 2 * 1024 * (n1 // 8 + 16) > SCRATCH_BYTES
    print(f"no-alloc call 1: 2-bit 1024 ch, {n1} samples, tile {plan.tile_config()}", flush=True)
    _compare(plan, raw, n1, 0, cuda)
    n2 = (1 << 17) + 777
    print(f"no-alloc call 2: {n2} samples", flush=True)
    _compare(plan, raw[: n2 * plan.row_bytes], n2, 0, cuda)


def test_noalloc_8bit_killmask_narrow_output_stride(native, cuda):
    import torch
    rng = np.random.default_rng(11)
    nchans, nsamps = 512, 300_000
    plan = Plan(nchans, 64e-6, 1581.8, -0.78125, 8).set_dm_list(synth.dm_list_linear(96, 400.0))
    mask = np.ones(nchans, dtype=np.int32)
    mask[rng.choice(nchans, 37, replace=False)] = 0
    plan.set_killmask(mask).set_output_format(16, 2)
    assert (nchans - 37 + 7) // 8 * 8 * nsamps > SCRATCH_BYTES     # live rows, padded to 8
    raw = torch.from_numpy(rng.integers(0, 256, size=nsamps * nchans, dtype=np.uint8)).to(cuda)
    print(f"no-alloc 8-bit: {nchans} ch, {nsamps} samples, tile {plan.tile_config()}", flush=True)
    nout = _compare(plan, raw, nsamps, nsamps - plan.max_delay + 5, cuda)
    assert nout > 0
    print("no-alloc 8-bit smaller input", flush=True)
    _compare(plan, raw[: 50_000 * nchans], 50_000, 0, cuda)


def test_noalloc_needs_built_tables_and_direct_mode(native, cuda):
    import torch
    plan = Plan(256, 64e-6, 1500.0, -1.0, 8).set_dm_list(synth.dm_list_linear(40, 50.0))
    n = 8192
    inp = torch.zeros(n * 256, dtype=torch.uint8, device=cuda)
    out = torch.empty((plan.ndm, n - plan.max_delay), dtype=torch.int32, device=cuda)
    with pytest.raises(DedispError, match="UNSUPPORTED"):
        plan.execute_noalloc(inp, out, n)          # tables not built yet
    plan.execute(inp, n, out=out)
    plan.execute_noalloc(inp, out, n)
    plan.set_tree(8)
    with pytest.raises(DedispError, match="UNSUPPORTED"):
        plan.execute_noalloc(inp, out, n)
    torch.cuda.synchronize()

