"""GPU parity of the systems forms: streams, multi-stream pushes and batches.

Streams: the outputs of successive pushes, concatenated, must equal the
oracle's one-shot transform of the concatenated input, for chunkings that
include chunks shorter than the largest delay.  Batches: every beam equals
its own oracle transform, on every replay of the captured graph.
"""
import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Batch, Plan, Stream, push_many, synth

pytestmark = pytest.mark.gpu


def _gpu(arr, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr).reshape(-1)).to(dev)


def _np(t):
    return t.cpu().numpy().view(np.uint32)


def _stream_case(nbits, nchans, ndm, dm_max, seed):
    rng = np.random.default_rng(seed)
    plan = Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, nbits).set_dm_list(
        synth.dm_list_linear(ndm, dm_max))
    return plan, rng


def _codes(rng, nsamps, nchans, nbits):
    if nbits == 2:
        return synth.two_bit_codes(rng, nsamps, nchans)
    return synth.eight_bit_noise(rng, nsamps, nchans, 128.0, 16.0)


def _run_stream(stream, plan, packed_rows, lengths, dev, misalign=False):
    """Push chunks of the given lengths; return the concatenated outputs."""
    import torch
    rb = plan.row_bytes
    outs, pos = [], 0
    for L in lengths:
        chunk = packed_rows[pos:pos + L]
        pos += L
        flat = np.ascontiguousarray(chunk).reshape(-1)
        if misalign:
            buf = torch.zeros(flat.size + 1, dtype=torch.uint8, device=dev)
            buf[1:] = torch.from_numpy(flat).to(dev)
            t = buf[1:]
        else:
            t = _gpu(flat, dev)
        out = torch.full((plan.ndm, max(L, 1) + plan.max_delay), -1, dtype=torch.int32, device=dev)
        n, _ = stream.push(t, out=out, out_row_stride=out.shape[1], nsamps=L)
        torch.cuda.synchronize()
        o = _np(out)
        assert np.all(o[:, n:] == 0xFFFFFFFF), "wrote past n_out"
        outs.append(o[:, :n])
        assert n == (0 if stream.state()[1] <= plan.max_delay else min(L, stream.state()[1] - plan.max_delay))
    return np.concatenate(outs, axis=1)


@pytest.mark.parametrize("nbits,nchans,misalign", [(2, 1024, False), (8, 256, False),
                                                   (2, 512, True), (8, 64, True)])
def test_stream_concatenation_equals_one_shot(native, cuda, nbits, nchans, misalign):
    plan, rng = _stream_case(nbits, nchans, 24, 300.0, nbits * 100 + nchans)
    mx = plan.max_delay
    lengths = [max(1, mx // 3), max(1, mx // 3), 7, mx + 5, 1, 3 * mx, 1300, 17, 2 * mx + 1]
    total = sum(lengths)
    codes = _codes(rng, total, nchans, nbits)
    packed = synth.pack(codes, nbits)
    s = Stream(plan)
    got = _run_stream(s, plan, packed, lengths, cuda, misalign)
    table = plan.delay_table()
    want = oracle.dedisperse(packed, total, nchans, nbits, table)
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    assert s.state() == (mx, total)


def test_stream_checkpoint_and_restore(native, cuda):
    plan, rng = _stream_case(2, 512, 16, 400.0, 5)
    mx = plan.max_delay
    lengths = [mx // 2, mx, 999, 2 * mx, 5000]
    total = sum(lengths)
    packed = synth.pack(_codes(rng, total, 512, 2), 2)
    ref = Stream(plan)
    whole = _run_stream(ref, plan, packed, lengths, cuda)
    a = Stream(plan)
    first = _run_stream(a, plan, packed[: sum(lengths[:3])], lengths[:3], cuda)
    hist = a.get_history()
    rows, seen = a.state()
    assert hist.shape == (rows, plan.row_bytes)
    assert np.array_equal(hist, packed[seen - rows: seen].reshape(rows, plan.row_bytes))
    b = Stream(plan)
    b.set_history(hist, seen)
    second = _run_stream(b, plan, packed[sum(lengths[:3]):], lengths[3:], cuda)
    assert np.array_equal(np.concatenate([first, second], axis=1), whole)


def test_stream_reset_and_invalid_history(native, cuda):
    from paper_1201_5380_amd import DedispError
    plan, _ = _stream_case(8, 64, 8, 100.0, 6)
    s = Stream(plan)
    with pytest.raises(DedispError):
        s.set_history(np.zeros((plan.max_delay + 1, plan.row_bytes), np.uint8), plan.max_delay + 1)
    with pytest.raises(DedispError):
        s.set_history(np.zeros((3, plan.row_bytes), np.uint8), plan.max_delay + 10)
    s.reset()
    assert s.state() == (0, 0)


# 16-wave shapes, compiled into the second multi-beam kernel class
_WIDE = {2: dict(kind=0, waves=16, dms_per_wave=1, words_per_lane=3, chunk_chans=32),
         8: dict(kind=0, waves=16, dms_per_wave=2, words_per_lane=5, chunk_chans=64)}


@pytest.mark.parametrize("wide", [False, True])
def test_push_many_equals_each_stream_alone(native, cuda, wide):
    """Chunks of several streams in one batched launch equal the one-shot
    transform of each stream; with `wide`, every other stream uses a 16-wave
    shape, so one tick launches both multi-beam kernel classes."""
    import torch
    specs = [(2, 1024, 32, 1000.0), (8, 512, 20, 300.0), (2, 256, 48, 100.0), (8, 1024, 8, 50.0),
             (2, 1024, 32, 1000.0), (8, 512, 24, 60.0), (8, 256, 16, 40.0)]
    plans, rngs, streams, packs, pos = [], [], [], [], []
    for i, (nb, nc, nd, dmx) in enumerate(specs):
        p, r = _stream_case(nb, nc, nd, dmx, 40 + i)
        if wide and i % 2 == 0 and p.tile_config()["kind"] == 0:
            p.set_tile_config(_WIDE[nb])
        plans.append(p)
        streams.append(Stream(p))
        n = 3 * p.max_delay + 9000
        packs.append(synth.pack(_codes(r, n, nc, nb), nb))
        pos.append(0)
    if wide:
        # 2- and 8-bit beams on 16-wave shapes beside 8-wave ones
        waves = [(p.nbits, p.tile_config()["waves"]) for p in plans if p.tile_config()["kind"] == 0]
        assert {(2, 16), (8, 16), (8, 8)} <= set(waves), waves
    outs = [[] for _ in specs]
    rng = np.random.default_rng(77)
    for step in range(5):
        chunks, bufs, active = [], [], []
        for i, p in enumerate(plans):
            L = int(rng.integers(1, p.max_delay + 3000))
            L = min(L, packs[i].shape[0] - pos[i])
            if L <= 0:
                continue
            chunks.append(_gpu(packs[i][pos[i]:pos[i] + L], cuda))
            bufs.append(torch.full((p.ndm, L + p.max_delay), -1, dtype=torch.int32, device=cuda))
            active.append((i, L))
            pos[i] += L
        n_outs = push_many([streams[i] for i, _ in active], chunks, bufs,
                           out_row_strides=[b.shape[1] for b in bufs])
        torch.cuda.synchronize()
        for (i, L), b, n in zip(active, bufs, n_outs):
            outs[i].append(_np(b)[:, :n])
    for i, p in enumerate(plans):
        got = np.concatenate(outs[i], axis=1)
        n = pos[i]
        want = oracle.dedisperse(packs[i][:n], n, p.nchans, p.nbits, p.delay_table())
        assert np.array_equal(got, want), specs[i]


def test_batch_small_every_beam_and_replay(native, cuda, tmp_path):
    """13 beams of the batched workload, shortened so the oracle runs whole.

    Each beam keeps its channel count, bit depth and DM step but only the
    first 24-40 trials of its DM list; a 14th beam has a DM list with huge
    gaps and runs on the untiled kernel inside the same batch.
    """
    import torch
    beams, refs = [], []
    for b in range(14):
        prm = synth.batch_beam_params(b % 13)
        rng = np.random.default_rng(b)
        if b < 13:
            dms = synth.dm_list_linear(prm["ndm"], prm["dm_max"])[: 24 + 8 * (b % 3)]
        else:
            dms = np.array([0.0, 900.0, 30.0, 1200.0])
        plan = Plan(prm["nchans"], prm["dt"], prm["f_top"], prm["df"], prm["nbits"]).set_dm_list(dms)
        n = plan.max_delay + 2000 + 777 * b
        packed = synth.pack(_codes(rng, n, prm["nchans"], prm["nbits"]), prm["nbits"])
        out = torch.full((plan.ndm, n - plan.max_delay), -1, dtype=torch.int32, device=cuda)
        beams.append((plan, _gpu(packed, cuda), n, out, 0))
        refs.append(oracle.dedisperse(packed, n, plan.nchans, plan.nbits, plan.delay_table()))
    kinds = [p.tile_config()["kind"] for p, *_ in beams]
    assert kinds[:13] == [0] * 13 and kinds[13] == 1
    cache = str(tmp_path / "tune.json")
    batch = Batch(beams, tune_cache_path=cache)
    for rep in range(4):
        for _, _, _, out, _ in beams:
            out.fill_(-1)
        torch.cuda.synchronize()
        batch.execute(graph=(rep != 1))
        torch.cuda.synchronize()
        x = torch.arange(1000, device=cuda).sum()        # eager work between replays
        assert int(x) == 499500
        for (plan, _, n, out, _), want in zip(beams, refs):
            assert np.array_equal(_np(out), want), (rep, plan.nchans, plan.nbits)
    # 2-bit beams have several candidate shapes, so tuning wrote the cache;
    # a second batch over the same shapes reads it back
    import json
    assert len(json.load(open(cache))) >= 1
    Batch(beams, tune_cache_path=cache).execute()
    torch.cuda.synchronize()


def test_stream_with_kill_mask(native, cuda):
    plan, rng = _stream_case(2, 512, 16, 300.0, 91)
    mask = (rng.random(512) < 0.5).astype(np.int32)
    plan.set_killmask(mask)
    mx = plan.max_delay
    lengths = [mx // 2, mx, 4000, 77, 2 * mx]
    total = sum(lengths)
    packed = synth.pack(_codes(rng, total, 512, 2), 2)
    got = _run_stream(Stream(plan), plan, packed, lengths, cuda)
    want = oracle.dedisperse(packed, total, 512, 2, plan.delay_table(), mask=mask)
    assert np.array_equal(got, want)
