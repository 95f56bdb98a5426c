"""GPU parity: the HIP kernels against the CPU oracle, bit for bit.

Every test dedisperses seeded synthetic input on the GPU through the C ABI and
compares with the oracle on the same bytes: whole outputs at sizes the
oracle finishes in seconds (several time tiles, several DM blocks, ragged
tails).  The benchmark's full sizes are compared in test_gpu_full_size.py.
"""
import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Plan, synth, tile_configs

pytestmark = pytest.mark.gpu


def _to_gpu(arr, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr)).to(dev)


def _out_np(t):
    return t.cpu().numpy().view(np.uint32)


def _run(plan, packed, nsamps, dev, cfg=None, stride=0):
    import torch
    if cfg is not None:
        plan.set_tile_config(cfg)
    inp = _to_gpu(packed.reshape(-1), dev)
    nout = nsamps - plan.max_delay
    if stride:
        out = torch.full((plan.ndm, stride), -1, dtype=torch.int32, device=dev)
        plan.execute(inp, nsamps, out=out, out_row_stride=stride)
    else:
        out = plan.execute(inp, nsamps)
    torch.cuda.synchronize()
    o = _out_np(out)
    if stride:
        assert np.all(o[:, nout:] == 0xFFFFFFFF), "wrote past nout"
        o = o[:, :nout]
    return o


def _plan_for(beam):
    return Plan(beam.nchans, beam.dt, beam.f_top, beam.df, beam.nbits).set_dm_list(beam.dms)


def _configs_for(plan):
    """Every compiled shape usable for this plan's bit depth (tiled ones that fit + untiled)."""
    out, seen_untiled = [], False
    for c in tile_configs():
        if c["kind"] == 1:
            if seen_untiled:
                continue
            seen_untiled = True
        try:
            plan.set_tile_config(c)
        except Exception:
            continue
        got = plan.tile_config()
        if c["kind"] == 1 or (got["kind"] == 0 and got["waves"] == c["waves"]
                              and got["dms_per_wave"] == c["dms_per_wave"]
                              and got["words_per_lane"] == c["words_per_lane"]
                              and got["chunk_chans"] == c["chunk_chans"]):
            out.append(c)
    return out


def test_tiny_every_shape_bit_exact(native, cuda):
    b = synth.tiny_beam()
    table, mx = oracle.delay_table(b.nchans, b.dt, b.f_top, b.df, b.dms)
    b.inject(lambda i: table[i])
    want = oracle.dedisperse(b.packed(), b.nsamps, b.nchans, b.nbits, table)
    plan = _plan_for(b)
    cfgs = _configs_for(plan)
    assert len(cfgs) >= 3
    for cfg in cfgs:
        got = _run(plan, b.packed(), b.nsamps, cuda, cfg)
        assert np.array_equal(got, want), cfg
    assert np.unravel_index(int(got.argmax()), got.shape) == (16, 1000)


@pytest.mark.parametrize("nbits,nchans,ndm,nsamps", [
    (2, 1024, 64, 24576),      # survey band, 64 DMs over [0, 1000): 4 DM blocks, ragged tail
    (2, 256, 40, 9000),        # ndm not a multiple of any DM block
    (8, 512, 48, 12000),
    (8, 1024, 33, 7000)])
def test_survey_like_every_shape_bit_exact(native, cuda, nbits, nchans, ndm, nsamps):
    rng = np.random.default_rng(nbits * 7 + nchans + ndm)
    if nbits == 2:
        codes = synth.two_bit_codes(rng, nsamps, nchans)
    else:
        codes = synth.eight_bit_noise(rng, nsamps, nchans, 128.0, 20.0)
    df = -400.0 / nchans
    dms = synth.dm_list_linear(ndm, 1000.0 * ndm / 64 if nsamps > 20000 else 300.0)
    table, mx = oracle.delay_table(nchans, 64e-6, 1581.8, df, dms)
    assert nsamps > mx
    packed = synth.pack(codes, nbits)
    want = oracle.dedisperse(packed, nsamps, nchans, nbits, table)
    plan = Plan(nchans, 64e-6, 1581.8, df, nbits).set_dm_list(dms)
    assert np.array_equal(plan.delay_table(), table)
    cfgs = _configs_for(plan)
    for cfg in cfgs:
        if cfg["kind"] == 1 and nchans * ndm * nsamps > 5e8:
            continue
        got = _run(plan, packed, nsamps, cuda, cfg)
        assert np.array_equal(got, want), cfg


@pytest.mark.parametrize("nbits", [2, 8])
def test_ragged_edges_and_strides(native, cuda, nbits):
    nchans, ndm = 64, 7
    rng = np.random.default_rng(11 + nbits)
    dms = synth.dm_list_linear(ndm, 200.0)
    plan = Plan(nchans, 64e-6, 1500.0, -1.0, nbits).set_dm_list(dms)
    mx = plan.max_delay
    table = plan.delay_table()
    for nsamps in (mx + 1, mx + 3, mx + 4, mx + 1279, mx + 1281, mx + 5000):
        maxc = 255 if nbits == 8 else 3
        codes = rng.integers(0, maxc + 1, size=(nsamps, nchans), dtype=np.uint8)
        packed = synth.pack(codes, nbits)
        want = oracle.dedisperse(packed, nsamps, nchans, nbits, table)
        for stride in (0, nsamps - mx + 3, nsamps - mx + 8):
            got = _run(plan, packed, nsamps, cuda, None, stride)
            assert np.array_equal(got, want), (nsamps, stride)


def test_unsorted_and_repeated_dms(native, cuda):
    nchans, nsamps = 256, 6000
    rng = np.random.default_rng(12)
    dms = rng.permutation(np.concatenate([synth.dm_list_linear(30, 150.0), [75.0, 75.0, 0.0]]))
    plan = Plan(nchans, 64e-6, 1500.0, -0.5, 2).set_dm_list(dms)
    table = plan.delay_table()
    codes = synth.two_bit_codes(rng, nsamps, nchans)
    packed = synth.pack(codes, 2)
    want = oracle.dedisperse(packed, nsamps, nchans, 2, table)
    assert plan.tile_config()["kind"] == 0
    assert np.array_equal(_run(plan, packed, nsamps, cuda), want)


def test_huge_dm_gap_uses_untiled_kernel(native, cuda):
    nchans, nsamps = 64, 40000
    dms = np.array([0.0, 5000.0, 10.0, 4000.0])
    plan = Plan(nchans, 64e-6, 1500.0, -1.0, 8).set_dm_list(dms)
    assert plan.tile_config()["kind"] == 1
    table = plan.delay_table()
    codes = np.random.default_rng(13).integers(0, 256, size=(nsamps, nchans), dtype=np.uint8)
    want = oracle.dedisperse(codes, nsamps, nchans, 8, table)
    assert np.array_equal(_run(plan, codes, nsamps, cuda), want)


@pytest.mark.parametrize("nbits", [2, 8])
def test_impulse_probe_recovers_delay_table(native, cuda, nbits):
    """x = 1 at (t*, c*) only: out[d][t] = 1 exactly at t = t* - delay[d][c*]."""
    nchans, ndm = 128, 20
    dms = synth.dm_list_linear(ndm, 400.0)
    plan = Plan(nchans, 64e-6, 1500.0, -1.0, nbits).set_dm_list(dms)
    table = plan.delay_table()
    mx = plan.max_delay
    nsamps = 2 * mx + 3000
    nout = nsamps - mx
    for cstar in (0, 5, 63, 64, 127):
        for tstar in (mx + 1000, 7, nsamps - 1):
            codes = np.zeros((nsamps, nchans), dtype=np.uint8)
            codes[tstar, cstar] = 1
            got = _run(plan, synth.pack(codes, nbits), nsamps, cuda)
            want = np.zeros_like(got)
            for d in range(ndm):
                t = tstar - table[d, cstar]
                if 0 <= t < nout:
                    want[d, t] = 1
            assert np.array_equal(got, want), (cstar, tstar)


def test_extreme_codes_do_not_overflow_packed_lanes(native, cuda):
    """All-maximum input: every output equals max_code * nchans exactly."""
    for nbits, nchans in ((2, 1024), (8, 4096)):
        maxc = 3 if nbits == 2 else 255
        dms = synth.dm_list_linear(16, 100.0)
        plan = Plan(nchans, 64e-6, 1500.0, -0.09765625 * 4096 / nchans, nbits).set_dm_list(dms)
        nsamps = plan.max_delay + 2000
        codes = np.full((nsamps, nchans), maxc, dtype=np.uint8)
        for cfg in _configs_for(plan):
            got = _run(plan, synth.pack(codes, nbits), nsamps, cuda, cfg)
            assert np.all(got == maxc * nchans), cfg


def test_determinism(native, cuda):
    b = synth.survey_beam(seed=3, nsamps=40000, nchans=512, ndm=64, npulses=0)
    plan = _plan_for(b)
    packed = b.packed()
    a = _run(plan, packed, b.nsamps, cuda)
    c = _run(plan, packed, b.nsamps, cuda)
    assert np.array_equal(a, c)


@pytest.mark.parametrize("nbits,nchans", [(2, 256), (8, 192)])
def test_kill_mask_every_shape(native, cuda, nbits, nchans):
    """Killed channels are left out of the sum (oracle: each term times mask[c])."""
    rng = np.random.default_rng(60 + nbits)
    nsamps = 9000
    dms = synth.dm_list_linear(40, 300.0)
    df = -400.0 / nchans
    maxc = 3 if nbits == 2 else 255
    codes = rng.integers(0, maxc + 1, size=(nsamps, nchans), dtype=np.uint8)
    packed = synth.pack(codes, nbits)
    plan = Plan(nchans, 64e-6, 1581.8, df, nbits).set_dm_list(dms)
    table = plan.delay_table()
    masks = []
    m = (rng.random(nchans) < 0.7).astype(np.int32)
    m[0] = 0
    m[-1] = 0
    if m.sum() % 2 == 0:                       # an odd number of live channels
        m[nchans // 2] ^= 1
    masks.append(m)
    one = np.zeros(nchans, np.int32)
    one[nchans // 3] = 1
    masks.append(one)
    masks.append(np.zeros(nchans, np.int32))
    for mask in masks:
        plan.set_killmask(mask)
        want = oracle.dedisperse(packed, nsamps, nchans, nbits, table, mask=mask)
        cfgs = _configs_for(plan) if mask.sum() > 1 else [None]
        for cfg in cfgs:
            got = _run(plan, packed, nsamps, cuda, cfg)
            assert np.array_equal(got, want), (int(mask.sum()), cfg)
    plan.set_killmask(None)
    assert np.array_equal(_run(plan, packed, nsamps, cuda),
                          oracle.dedisperse(packed, nsamps, nchans, nbits, table))


@pytest.mark.parametrize("nchans,fmt", [(16, 4), (1344, 4), (1360, 0)])
def test_two_bit_scratch_format_by_channel_count(native, cuda, nchans, fmt):
    """2-bit codes are summed as bit planes while 3 x (channels rounded up to
    32) fits the planes' 12 bit levels (up to 1344 channels) and as nibbles
    beyond; both bit-exact on every shape, including all-maximum codes whose
    sums reach the top level (3 x 1344 = 4032)."""
    rng = np.random.default_rng(nchans)
    dms = synth.dm_list_linear(40, 200.0)
    df = -400.0 / nchans
    plan = Plan(nchans, 64e-6, 1581.8, df, 2).set_dm_list(dms)
    assert plan.tile_config()["sample_format"] == fmt
    table = plan.delay_table()
    nsamps = plan.max_delay + 7000
    for codes in (synth.two_bit_codes(rng, nsamps, nchans), np.full((nsamps, nchans), 3, np.uint8)):
        packed = synth.pack(codes, 2)
        want = oracle.dedisperse(packed, nsamps, nchans, 2, table)
        for cfg in _configs_for(plan):
            if cfg["kind"] == 1 and nchans > 64:
                continue
            got = _run(plan, packed, nsamps, cuda, cfg)
            assert np.array_equal(got, want), cfg


def test_two_bit_wide_dm_steps_fall_back_within_planes(native, cuda):
    """A DM list whose blocks spread too far for the 3-word plane windows runs
    on the 1-word plane shapes (or the untiled kernel), still bit-exact."""
    nchans, nsamps = 256, 60000
    dms = np.arange(48) * 10.0
    plan = Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, 2).set_dm_list(dms)
    table = plan.delay_table()
    assert nsamps > plan.max_delay + 1000
    codes = synth.two_bit_codes(np.random.default_rng(77), nsamps, nchans)
    packed = synth.pack(codes, 2)
    want = oracle.dedisperse(packed, nsamps, nchans, 2, table)
    cfg = plan.tile_config()
    assert cfg["kind"] == 0 and cfg["sample_format"] == 4 and cfg["words_per_lane"] == 1
    got = _run(plan, packed, nsamps, cuda)
    assert np.array_equal(got, want), cfg
