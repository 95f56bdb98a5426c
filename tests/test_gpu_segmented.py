"""GPU parity of the segmented bit-plane layout (sample_format 5) against the
oracle, bit for bit.

In this layout the outputs of a transform are cut into 32 segments of
S = ceil(nout / 32) samples and bit i of a scratch word holds segment i, so
every edge of the segment arithmetic is exercised here: outputs shorter than
one segment row (nout < 32), lengths one either side of a multiple of 32 and
of a whole tile, DM counts that leave a ragged last block, killed channels,
narrow outputs with a row stride, stream pushes (each push is its own
segmented transform over [history | chunk]) and the allocation-free entry
point's time slices.  The layout stages a DM block's whole delay spread in
words, so it runs only on fine DM grids like the survey's (steps of about
one unit of DM over a 400 MHz band at 1.4 GHz; the cases below use steps of
0.9), and only on launches of at least 8 max_delays of outputs (shorter
ones take the plain planes; the zero-DM cases have no delays at all).
"""
import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Plan, Stream, synth, tile_configs

pytestmark = pytest.mark.gpu


def _seg_configs():
    cfgs = [c for c in tile_configs() if c["kind"] == 0 and c["sample_format"] == 5]
    assert cfgs, "no segmented bit-plane shape compiled"
    return cfgs


def _use(plan, cfg):
    plan.set_tile_config(cfg)
    got = plan.tile_config()
    assert got["sample_format"] == 5 and got["words_per_lane"] == cfg["words_per_lane"], got


def _gpu(arr, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr).reshape(-1)).to(dev)


def _np(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("extra", [1, 5, 31, 32, 33, 6143, 6145, 40000])
@pytest.mark.parametrize("zero_dms", [True, False])
def test_segmented_lengths_bit_exact(native, cuda, extra, zero_dms):
    """Every segmented shape, nout = extra outputs per DM (1 .. several tiles).
    A launch shorter than 8 max_delays takes the plain planes, so the short
    lengths run the segmented layout only with an all-zero DM list (no
    delays); with the fine grid they check the fallback."""
    import torch
    nchans, ndm = 96, 37                      # 96 channels: three 32-channel units; 37 DMs: ragged block
    rng = np.random.default_rng(500 + extra)
    dms = np.zeros(ndm) if zero_dms else synth.dm_list_linear(ndm, 0.9 * ndm)
    plan = Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, 2).set_dm_list(dms)
    table = plan.delay_table()
    nsamps = plan.max_delay + extra
    print(f"segmented lengths: nout {extra}, nsamps {nsamps}", flush=True)
    packed = synth.pack(synth.two_bit_codes(rng, nsamps, nchans), 2)
    want = oracle.dedisperse(packed, nsamps, nchans, 2, table)
    inp = _gpu(packed, cuda)
    for cfg in _seg_configs():
        _use(plan, cfg)
        stride = extra + 5
        out = torch.full((ndm, stride), -1, dtype=torch.int32, device=cuda)
        plan.execute(inp, nsamps, out=out, out_row_stride=stride)
        torch.cuda.synchronize()
        o = _np(out)
        assert np.all(o[:, extra:] == 0xFFFFFFFF), ("wrote past nout", cfg)
        assert np.array_equal(o[:, :extra], want), cfg


def test_segmented_survey_band_all_max_codes_and_killmask(native, cuda):
    """1344 channels of code 3 reach the top bit level (3 x 1344 = 4032); then
    a kill mask compacts the live channels (padding rows up to a multiple of 32)."""
    nchans, ndm = 1344, 20
    plan = Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, 2).set_dm_list(synth.dm_list_linear(ndm, 0.9 * ndm))
    table = plan.delay_table()
    nsamps = plan.max_delay + 9000
    codes = np.full((nsamps, nchans), 3, np.uint8)
    packed = synth.pack(codes, 2)
    inp = _gpu(packed, cuda)
    want = oracle.dedisperse(packed, nsamps, nchans, 2, table)
    assert want.max() == 3 * nchans
    for cfg in _seg_configs():
        _use(plan, cfg)
        got = _np(plan.execute(inp, nsamps))
        assert np.array_equal(got, want), cfg
    rng = np.random.default_rng(9)
    codes = synth.two_bit_codes(rng, nsamps, nchans)
    packed = synth.pack(codes, 2)
    inp = _gpu(packed, cuda)
    mask = (rng.random(nchans) > 0.3).astype(np.int32)
    plan.set_killmask(mask)
    want = oracle.dedisperse(packed, nsamps, nchans, 2, table, mask=mask)
    for cfg in _seg_configs():
        _use(plan, cfg)
        got = _np(plan.execute(inp, nsamps))
        assert np.array_equal(got, want), cfg


@pytest.mark.parametrize("nbits_out,shift", [(8, 3), (16, 0)])
def test_segmented_narrow_outputs(native, cuda, nbits_out, shift):
    import torch
    nchans, ndm = 256, 18
    rng = np.random.default_rng(nbits_out)
    plan = Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, 2).set_dm_list(synth.dm_list_linear(ndm, 0.9 * ndm))
    plan.set_output_format(nbits_out, shift)
    table = plan.delay_table()
    nsamps = plan.max_delay + 7001
    packed = synth.pack(synth.two_bit_codes(rng, nsamps, nchans), 2)
    want = oracle.reduce_output(oracle.dedisperse(packed, nsamps, nchans, 2, table), nbits_out, shift)
    inp = _gpu(packed, cuda)
    nout = nsamps - plan.max_delay
    npdt = np.uint8 if nbits_out == 8 else np.uint16
    for cfg in _seg_configs():
        _use(plan, cfg)
        stride = nout + 7
        fill = 255 if nbits_out == 8 else -1
        out = torch.full((ndm, stride), fill, dtype=plan.output_dtype(), device=cuda)
        plan.execute(inp, nsamps, out=out, out_row_stride=stride)
        torch.cuda.synchronize()
        o = out.cpu().numpy().view(npdt)
        assert np.all(o[:, nout:] == npdt((1 << nbits_out) - 1)), ("wrote past nout", cfg)
        assert np.array_equal(o[:, :nout], want), cfg


def test_segmented_stream_pushes_equal_one_shot(native, cuda):
    import torch
    nchans = 512
    rng = np.random.default_rng(31)
    plan = Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, 2).set_dm_list(synth.dm_list_linear(24, 0.9 * 24))
    _use(plan, _seg_configs()[0])
    mx = plan.max_delay
    # pushes of at least 8 max_delays of outputs run segmented, the rest plain
    lengths = [mx // 3, 7, 9 * mx, 1, 12 * mx + 5, 1300, 20 * mx + 1, mx + 3]
    total = sum(lengths)
    packed = synth.pack(synth.two_bit_codes(rng, total, nchans), 2).reshape(total, -1)
    s = Stream(plan)
    outs, pos = [], 0
    for L in lengths:
        t = _gpu(packed[pos:pos + L], cuda)
        pos += L
        out = torch.full((plan.ndm, L + mx), -1, dtype=torch.int32, device=cuda)
        n, _ = s.push(t, out=out, out_row_stride=out.shape[1], nsamps=L)
        torch.cuda.synchronize()
        o = _np(out)
        assert np.all(o[:, n:] == 0xFFFFFFFF)
        outs.append(o[:, :n])
    got = np.concatenate(outs, axis=1)
    want = oracle.dedisperse(packed.reshape(-1), total, nchans, 2, plan.delay_table())
    assert np.array_equal(got, want)


def test_segmented_noalloc_slices_equal_execute(native, cuda):
    """The allocation-free entry point on a segmented shape: an input whose
    scratch exceeds the fixed array is cut into time slices, each its own
    segmented transform; then a smaller input in one slice (short enough to
    take the plain planes)."""
    import torch
    rng = np.random.default_rng(8)
    plan = Plan(1024, 64e-6, 1581.8, -0.390625, 2).set_dm_list(synth.dm_list_linear(256, 0.9 * 256))
    _use(plan, _seg_configs()[0])
    for n in (1 << 19, 40000):
        raw = torch.from_numpy(rng.integers(0, 256, size=n * plan.row_bytes, dtype=np.uint8)).to(cuda)
        nout = n - plan.max_delay
        want = torch.full((plan.ndm, nout), -1, dtype=torch.int32, device=cuda)
        got = torch.full((plan.ndm, nout), -1, dtype=torch.int32, device=cuda)
        print(f"segmented no-alloc: {n} samples", flush=True)
        plan.execute(raw, n, out=want)
        plan.execute_noalloc(raw, got, n)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        # and the segmented transform against the oracle on sampled DM rows
        rows = [0, 1, 127, 255]
        table = plan.delay_table()
        packed = raw.cpu().numpy()
        exp = oracle.dedisperse(packed, n, 1024, 2, table[rows], max_delay=plan.max_delay)
        assert np.array_equal(_np(want)[rows], exp)


def _fine_plan(nbits, nchans, ndm):
    return Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, nbits).set_dm_list(synth.dm_list_linear(ndm, 0.9 * ndm))


def _codes(rng, n, nchans, nbits):
    if nbits == 2:
        return synth.two_bit_codes(rng, n, nchans)
    return synth.eight_bit_noise(rng, n, nchans, 128.0, 16.0)


def test_segmented_multi_beam_push_many(native, cuda):
    """Streams on the segmented shape beside plain bit-plane (16-wave) and
    8-bit (8-wave) streams: every tick launches the three multi-beam kernel
    classes, and each stream's concatenated outputs equal its one-shot
    oracle transform."""
    import torch
    from paper_1201_5380_amd import push_many
    seg = _seg_configs()[0]
    specs = [(2, 1024, 24, "seg"), (2, 512, 20, "plane"), (8, 256, 16, None), (2, 256, 30, "seg")]
    plans, streams, packs, pos = [], [], [], []
    for i, (nb, nc, nd, kind) in enumerate(specs):
        p = _fine_plan(nb, nc, nd)
        if kind == "seg":
            _use(p, seg)
        elif kind == "plane":
            p.set_tile_config(dict(seg, sample_format=4))
            assert p.tile_config()["sample_format"] == 4 and p.tile_config()["waves"] == 16
        plans.append(p)
        streams.append(Stream(p))
        n = 40 * p.max_delay + 7000
        packs.append(synth.pack(_codes(np.random.default_rng(60 + i), n, nc, nb), nb).reshape(n, -1))
        pos.append(0)
    outs = [[] for _ in specs]
    rng = np.random.default_rng(5)
    for step in range(6):
        chunks, bufs, active = [], [], []
        for i, p in enumerate(plans):
            L = min(int(rng.integers(1, 12 * p.max_delay)), packs[i].shape[0] - pos[i])
            if L <= 0:
                continue
            chunks.append(_gpu(packs[i][pos[i]:pos[i] + L], cuda))
            bufs.append(torch.full((p.ndm, L + p.max_delay), -1, dtype=torch.int32, device=cuda))
            active.append(i)
            pos[i] += L
        print(f"push_many step {step}: streams {active}", flush=True)
        n_outs = push_many([streams[i] for i in active], chunks, bufs,
                           out_row_strides=[b.shape[1] for b in bufs])
        torch.cuda.synchronize()
        for i, b, n in zip(active, bufs, n_outs):
            o = _np(b)
            assert np.all(o[:, n:] == 0xFFFFFFFF)
            outs[i].append(o[:, :n])
    for i, p in enumerate(plans):
        got = np.concatenate(outs[i], axis=1)
        want = oracle.dedisperse(packs[i][:pos[i]].reshape(-1), pos[i], p.nchans, p.nbits, p.delay_table())
        assert np.array_equal(got, want), specs[i]


def test_segmented_batch_from_tune_cache(native, cuda, tmp_path):
    """A batch whose bit-plane beams are pinned to the segmented shape through
    the tune cache (the library's own entries, rewritten), on every replay of
    the captured graph."""
    import json
    import torch
    from paper_1201_5380_amd import Batch
    seg = _seg_configs()[0]
    beams, refs = [], []
    for i, (nb, nc, nd) in enumerate([(2, 1024, 24), (8, 256, 16), (2, 512, 33), (2, 256, 17)]):
        p = _fine_plan(nb, nc, nd)
        n = p.max_delay + 5000 + 1111 * i
        packed = synth.pack(_codes(np.random.default_rng(80 + i), n, nc, nb), nb)
        out = torch.full((p.ndm, n - p.max_delay), -1, dtype=torch.int32, device=cuda)
        beams.append((p, _gpu(packed, cuda), n, out, 0))
        refs.append(oracle.dedisperse(packed, n, nc, nb, p.delay_table()))
    cache = tmp_path / "tune.json"
    Batch(beams, tune_cache_path=str(cache)).execute()
    torch.cuda.synchronize()
    entries = json.load(open(cache))
    pinned = 0
    for k, v in entries.items():
        if k.startswith("multi:") and "nbits=2,fmt=4," in k:
            entries[k] = [0, seg["waves"], seg["dms_per_wave"], seg["words_per_lane"], seg["chunk_chans"],
                          v[5] if len(v) > 5 else 0.0, 5]
            pinned += 1
    assert pinned == 3, entries
    json.dump(entries, open(cache, "w"))
    batch = Batch(beams, tune_cache_path=str(cache))
    for rep in range(3):
        for _, _, _, out, _ in beams:
            out.fill_(-1)
        torch.cuda.synchronize()
        batch.execute(graph=(rep != 1))
        torch.cuda.synchronize()
        for (p, _, n, out, _), want in zip(beams, refs):
            assert np.array_equal(_np(out), want), (rep, p.nchans, p.nbits)
