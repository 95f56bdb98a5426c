"""GPU parity of sub-band dedispersion (Section 4) against the oracle, bit for bit.

The library runs the corner turn, then step 1 (every sub-band at every
nominal DM, one grouped launch of the tiled kernel writing byte or 16-bit
sums into an intermediate scratch) and step 2 (every nominal DM's trials over the
sub-band series, a second grouped launch).  Outputs are compared whole with
the oracle's two-step definition.
"""
import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Plan, synth, tile_configs

pytestmark = pytest.mark.gpu

SENTINEL = 0x5EEDF00D


def _run(plan, packed, nsamps, dev, width):
    import torch
    inp = torch.from_numpy(np.ascontiguousarray(packed.reshape(-1))).to(dev)
    out = torch.full((plan.ndm, width), SENTINEL, dtype=torch.int32, device=dev)
    plan.execute(inp, nsamps, out=out, out_row_stride=width)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def _codes(rng, nsamps, nchans, nbits):
    if nbits == 2:
        c = rng.integers(0, 4, size=(nsamps, nchans), dtype=np.uint8)
        c[::89] = 3
    else:
        c = np.clip(np.rint(rng.normal(128, 40, size=(nsamps, nchans))), 0, 255).astype(np.uint8)
        c[::89] = 255
    return c


@pytest.mark.parametrize("nbits,nchans,nsub,ngroup,ndm,nsamps", [
    (2, 256, 8, 8, 70, 20011),      # byte-lane intermediate sums (at most 24)
    (2, 256, 32, 16, 64, 16003),    # byte intermediate sums (at most 96) read as 8-bit codes
    (2, 256, 16, 8, 48, 14009),     # byte intermediate sums (at most 48) read as 8-bit codes
    (2, 512, 128, 8, 40, 16007),    # 16-bit intermediate sums (at most 384)
    (8, 128, 16, 5, 43, 15007),     # 8-bit codes: 16-bit sums, last group short
    (2, 192, 8, 4, 33, 17001),      # 24 sub-bands: zero padding rows in step 2
])
def test_subband_every_shape_bit_exact(native, cuda, nbits, nchans, nsub, ngroup, ndm, nsamps):
    dt, f_top, df = 64e-6, 1581.8, -400.0 / nchans
    dms = synth.dm_list_linear(ndm, 600.0)
    rng = np.random.default_rng(nchans * 7 + nsub)
    codes = _codes(rng, nsamps, nchans, nbits)
    packed = synth.pack(codes, nbits)
    plan = Plan(nchans, dt, f_top, df, nbits).set_dm_list(dms)
    plan.set_subband(nsub, ngroup)
    want = oracle.dedisperse_subband(packed, nsamps, nchans, nbits, dt, f_top, df, dms, nsub, ngroup)
    nout = want.shape[1]
    assert np.all(plan.output_lengths(nsamps) == nout)
    width = nout + 3
    ran = 0
    seen = set()
    for cfg in tile_configs():
        key = tuple(sorted(cfg.items()))
        if cfg["kind"] != 0 or key in seen:
            continue
        seen.add(key)
        try:
            plan.set_tile_config(cfg)
        except Exception:
            continue
        got = _run(plan, packed, nsamps, cuda, width)
        assert np.array_equal(got[:, :nout], want), cfg
        assert np.all(got[:, nout:] == SENTINEL)
        ran += 1
    assert ran >= 3


def test_subband_kill_mask_and_direct_reduction(native, cuda):
    nbits, nchans, nsamps = 2, 512, 15013
    dt, f_top, df = 64e-6, 1581.8, -400.0 / nchans
    dms = synth.dm_list_linear(96, 500.0)
    rng = np.random.default_rng(17)
    codes = _codes(rng, nsamps, nchans, nbits)
    packed = synth.pack(codes, nbits)
    mask = (rng.random(nchans) < 0.75).astype(np.int32)
    plan = Plan(nchans, dt, f_top, df, nbits).set_dm_list(dms)
    plan.set_killmask(mask)
    plan.set_subband(16, 12)
    want = oracle.dedisperse_subband(packed, nsamps, nchans, nbits, dt, f_top, df, dms, 16, 12,
                                     mask=mask)
    got = _run(plan, packed, nsamps, cuda, want.shape[1])
    assert np.array_equal(got, want)
    # one trial per nominal DM: the sub-band result is the direct transform
    plan.set_subband(16, 1)
    n1 = int(plan.output_lengths(nsamps)[0])
    got1 = _run(plan, packed, nsamps, cuda, n1)
    plan.set_subband(0, 0)
    direct = _run(plan, packed, nsamps, cuda, nsamps - plan.max_delay)
    assert np.array_equal(got1, direct[:, :n1])


def test_survey_beam_subband_full_size(native, cuda):
    """The benchmark's survey beam with 32-channel sub-bands and 32 trials per
    nominal DM, whole, against the oracle's two steps."""
    import torch
    b = synth.survey_beam()
    plan = Plan(b.nchans, b.dt, b.f_top, b.df, b.nbits).set_dm_list(b.dms)
    otab, _ = oracle.delay_table(b.nchans, b.dt, b.f_top, b.df, b.dms)
    b.inject(lambda i: otab[i])
    packed = b.packed()
    plan.set_subband(32, 32)
    want = oracle.dedisperse_subband(packed, b.nsamps, b.nchans, b.nbits, b.dt, b.f_top, b.df,
                                     b.dms, 32, 32)
    nout = want.shape[1]
    inp = torch.from_numpy(packed.reshape(-1)).to(cuda)
    out = torch.empty((plan.ndm, nout), dtype=torch.int32, device=cuda)
    plan.execute(inp, b.nsamps, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("nchans,nsub,ngroup,ndm", [(512, 32, 8, 40), (1024, 32, 32, 96)])
def test_subband_tuned_intermediate_width_bit_exact(native, cuda, nchans, nsub, ngroup, ndm):
    """2-bit codes in 32-channel sub-bands give sums up to 96: the tuner times
    both intermediate widths (bytes read as 8-bit codes, 16-bit values) and
    keeps the faster, starting from 16-bit sums (16 sub-bands, 8 trials per
    nominal DM) or from bytes (32 and 32).  The transform matches the oracle
    before and after tuning."""
    import torch
    nbits, nsamps = 2, 24007
    dt, f_top, df = 64e-6, 1581.8, -400.0 / nchans
    dms = synth.dm_list_linear(ndm, 400.0)
    rng = np.random.default_rng(nchans + ngroup)
    packed = synth.pack(_codes(rng, nsamps, nchans, nbits), nbits)
    want = oracle.dedisperse_subband(packed, nsamps, nchans, nbits, dt, f_top, df, dms, nsub, ngroup)
    plan = Plan(nchans, dt, f_top, df, nbits).set_dm_list(dms)
    plan.set_subband(nsub, ngroup)
    nout = want.shape[1]
    width = nout + 3
    assert np.array_equal(_run(plan, packed, nsamps, cuda, width)[:, :nout], want)
    inp = torch.from_numpy(np.ascontiguousarray(packed.reshape(-1))).to(cuda)
    out = torch.empty((plan.ndm, width), dtype=torch.int32, device=cuda)
    assert plan.tune(inp, out, nsamps, out_row_stride=width) > 0
    got = _run(plan, packed, nsamps, cuda, width)
    assert np.array_equal(got[:, :nout], want)
    assert np.all(got[:, nout:] == SENTINEL)


@pytest.mark.parametrize("nchans,nsub,ngroup,ndm", [(1024, 32, 32, 80), (1024, 64, 64, 100), (512, 16, 32, 70)])
def test_subband_step2_as_row_combination_bit_exact(native, cuda, nchans, nsub, ngroup, ndm):
    """Byte sub-band sums with whole blocks of 32 trials per nominal DM
    (ngroup a multiple of 32) over a narrow DM range: step 2 runs as the
    combination of per-sub-band rows staged in LDS (sums up to 96 added two
    terms at a time as bytes, up to 192 one at a time, up to 48 two at a
    time), with a ragged last nominal DM, a kill mask, and 16-bit outputs in
    a wider row stride, bit for bit against the oracle."""
    import torch
    nbits, nsamps = 2, 30011
    dt, f_top, df = 64e-6, 1581.8, -400.0 / nchans
    dms = np.linspace(0.0, 40.0, ndm)
    rng = np.random.default_rng(nchans + nsub + ngroup)
    codes = _codes(rng, nsamps, nchans, nbits)
    codes[5000:9000] = 3
    packed = synth.pack(codes, nbits)
    mask = (rng.random(nchans) < 0.93).astype(np.int32)
    want = oracle.dedisperse_subband(packed, nsamps, nchans, nbits, dt, f_top, df, dms, nsub, ngroup, mask=mask)
    plan = Plan(nchans, dt, f_top, df, nbits).set_dm_list(dms).set_killmask(mask)
    plan.set_subband(nsub, ngroup)
    nout = want.shape[1]
    width = nout + 5
    got = _run(plan, packed, nsamps, cuda, width)
    assert np.array_equal(got[:, :nout], want)
    assert np.all(got[:, nout:] == SENTINEL)
    plan.set_output_format(16, 1)
    inp = torch.from_numpy(np.ascontiguousarray(packed.reshape(-1))).to(cuda)
    out = torch.full((plan.ndm, width), 0x7777, dtype=plan.output_dtype(), device=cuda)
    plan.execute(inp, nsamps, out=out, out_row_stride=width)
    torch.cuda.synchronize()
    got16 = out.cpu().numpy().view(np.uint16)
    assert np.array_equal(got16[:, :nout], oracle.reduce_output(want, 16, 1))
    assert np.all(got16[:, nout:] == 0x7777)
