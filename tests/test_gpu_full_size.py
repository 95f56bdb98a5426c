"""GPU parity at the benchmark's full sizes, whole outputs (eq. direct, Section 2.1).

* Survey beam (2-bit, 1024 channels, 2^19 samples, 1024 DMs): the oracle's
  whole output against the tuned launch the benchmark times and against every
  compiled 2-bit tile shape that fits, so whichever shape the tuner picks on
  a given run has been compared element by element.
* Large beam (8-bit, 4096 channels, 2^20 samples, 2048 DMs): whole DM-row
  slices -- the first rows, a middle block and the last 64 rows (the last DM
  block of every shape, ragged or not) -- over the whole time range, for the
  tuned shape and every compiled 8-bit shape.
* Batched workload (13 beams at full size): the first and the last DM rows
  of every beam (the last block of any shape) over the whole time range.
* Streaming service at its configured scale (32 streams, 1024 DMs, chunks of
  U[2^14, 2^18] samples, two chunks per stream): every request's output in
  the mix equals the same stream pushed alone, compared on the device; the
  shortest stream is also compared whole with the oracle.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Batch, Plan, Stream, synth, tile_configs

# the oracle's share of these tests takes tens of seconds on the host
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _shapes(plan, nbits):
    """Every compiled tiled shape of this bit depth that the plan accepts as is."""
    out = []
    for c in tile_configs():
        if c["kind"] != 0:
            continue
        try:
            plan.set_tile_config(c)
        except Exception:
            continue
        got = plan.tile_config()
        if got["kind"] == 0 and all(got[k] == c[k] for k in
                                    ("waves", "dms_per_wave", "words_per_lane", "chunk_chans")):
            out.append(dict(c))
    return out


def _key(c):
    return tuple(c[k] for k in ("waves", "dms_per_wave", "words_per_lane", "chunk_chans"))


def test_survey_beam_whole_output_every_shape(native, cuda):
    import torch
    b = synth.survey_beam()
    plan = Plan(b.nchans, b.dt, b.f_top, b.df, b.nbits).set_dm_list(b.dms)
    table, mx = oracle.delay_table(b.nchans, b.dt, b.f_top, b.df, b.dms)
    assert mx == 20456 and np.array_equal(plan.delay_table(), table)
    b.inject(lambda i: table[i])
    packed = b.packed()
    nout = b.nsamps - mx
    t0 = time.perf_counter()
    want = oracle.dedisperse(packed, b.nsamps, b.nchans, b.nbits, table)
    _say(f"survey oracle: {want.shape} in {time.perf_counter() - t0:.1f} s")
    want_dev = torch.from_numpy(want.view(np.int32)).to(cuda)
    del want
    inp = torch.from_numpy(packed.reshape(-1)).to(cuda)
    out = torch.empty((plan.ndm, nout), dtype=torch.int32, device=cuda)
    plan.tune(inp, out, b.nsamps)
    tuned = plan.tile_config()
    shapes = _shapes(plan, 2)
    assert _key(tuned) in {_key(c) for c in shapes}
    for cfg in [tuned] + shapes:
        plan.set_tile_config(cfg)
        out.fill_(-1)
        plan.execute(inp, b.nsamps, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, want_dev), cfg
        _say(f"survey beam whole output equal: {_key(cfg)}")
    # pulses at their trials and times (the paper's Fig. 1 check)
    for p in b.pulses:
        lo, hi = max(0, p.t0 - 100), min(nout, p.t0 + 101)
        win = want_dev[:, lo:hi]
        k = int(torch.argmax(win.reshape(-1)))
        assert (k // (hi - lo), k % (hi - lo) + lo) == (p.dm_index, p.t0), p


def test_large_beam_whole_row_slices_every_shape(native, cuda):
    import torch
    t0 = time.perf_counter()
    b = synth.large_beam()
    _say(f"large beam input {b.codes.shape} made in {time.perf_counter() - t0:.1f} s")
    plan = Plan(b.nchans, b.dt, b.f_top, b.df, b.nbits).set_dm_list(b.dms)
    table, mx = oracle.delay_table(b.nchans, b.dt, b.f_top, b.df, b.dms)
    assert mx == 58003 and np.array_equal(plan.delay_table(), table)
    ndm, nout = len(b.dms), b.nsamps - mx
    rows = np.concatenate([np.arange(0, 32), np.arange(ndm // 2 - 16, ndm // 2 + 16),
                           np.arange(ndm - 64, ndm)])
    packed = b.packed()
    t0 = time.perf_counter()
    want = oracle.dedisperse(packed, b.nsamps, b.nchans, 8, table[rows], max_delay=mx)
    _say(f"large beam oracle: {want.shape} in {time.perf_counter() - t0:.1f} s")
    want_dev = torch.from_numpy(want.view(np.int32)).to(cuda)
    del want
    inp = torch.from_numpy(packed.reshape(-1)).to(cuda)
    del b, packed
    rows_dev = torch.from_numpy(rows).to(cuda)
    out = torch.empty((ndm, nout), dtype=torch.int32, device=cuda)
    plan.tune(inp, out, 1 << 20)
    tuned = plan.tile_config()
    shapes = _shapes(plan, 8)
    assert _key(tuned) in {_key(c) for c in shapes}
    for cfg in [tuned] + shapes:
        plan.set_tile_config(cfg)
        out.fill_(-1)
        plan.execute(inp, 1 << 20, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out.index_select(0, rows_dev), want_dev), cfg
        _say(f"large beam rows equal: {_key(cfg)}")
    # the DM 0 row is the plain channel sum over every output
    chansum = inp.view(1 << 20, -1)[:nout].sum(dim=1, dtype=torch.int32)
    assert torch.equal(out[0], chansum)


def test_batch_full_size_first_and_last_rows(native, cuda):
    import torch
    beams, refs = [], []
    for bi in range(13):
        beam = synth.batch_beam(bi)
        plan = Plan(beam.nchans, beam.dt, beam.f_top, beam.df, beam.nbits).set_dm_list(beam.dms)
        packed = beam.packed()
        n = beam.nsamps
        out = torch.full((plan.ndm, n - plan.max_delay), -1, dtype=torch.int32, device=cuda)
        beams.append((plan, torch.from_numpy(packed.reshape(-1)).to(cuda), n, out, 0))
        refs.append((packed, n))
    batch = Batch(beams)
    for rep in range(2):
        for *_, out, _ in beams:
            out.fill_(-1)
        torch.cuda.synchronize()
        batch.execute()
        torch.cuda.synchronize()
        if rep == 0:
            continue
        for (plan, _, n, out, _), (packed, _) in zip(beams, refs):
            rows = np.concatenate([np.arange(0, 32), np.arange(plan.ndm - 48, plan.ndm)])
            want = oracle.dedisperse(packed, n, plan.nchans, plan.nbits, plan.delay_table()[rows],
                                     max_delay=plan.max_delay)
            got = out.index_select(0, torch.from_numpy(rows).to(cuda)).cpu().numpy().view(np.uint32)
            assert np.array_equal(got, want), (plan.nchans, plan.nbits, n, plan.ndm)
            _say(f"batch beam {plan.nchans} ch {plan.nbits}-bit {n} samples {plan.ndm} DMs: equal")


def test_serving_scale_alone_equals_in_the_mix(native, cuda):
    import torch
    from paper_1201_5380_amd.serve import DONE, GpuExecutor, Server
    nstreams, nchans = 32, 1024
    plan = Plan(nchans, 64e-6, 1581.8, -0.390625, 2).set_dm_list(synth.dm_list_linear(1024, 1000.0))
    rb = plan.row_bytes
    lens = [synth.stream_chunk_lengths(s, 2) for s in range(nstreams)]
    t0 = time.perf_counter()
    data = []
    for s in range(nstreams):
        codes = synth.blockwise_codes([1000 + s], int(lens[s].sum()), nchans, 2)
        data.append(synth.pack(codes, 2).reshape(-1, rb))
        del codes
    _say(f"serving inputs made in {time.perf_counter() - t0:.1f} s")
    chunks = [[data[s][:lens[s][0]], data[s][lens[s][0]:]] for s in range(nstreams)]

    ex = GpuExecutor([plan] * nstreams, device=cuda, max_chunk=1 << 18)
    ex.tune(1 << 18)
    srv = Server(ex, nstreams, budget_bytes=64 << 30, max_tick=16, max_inflight_ticks=4).start()
    rate = nstreams * 4.0 / (((1 << 14) + (1 << 18)) / 2 * 64e-6)
    t_arr, _ = synth.poisson_arrivals(2 * nstreams, rate, nstreams, seed=5)
    order = [(s, k) for k in range(2) for s in np.random.default_rng(5).permutation(nstreams)]
    reqs = {}
    t0 = time.perf_counter()
    for ta, (s, k) in zip(t_arr, order):
        delay = t0 + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        reqs[(int(s), k)] = srv.submit(int(s), chunks[s][k])
    srv.drain(timeout=600)
    srv.stop()
    st = srv.stats()
    _say(f"serving mix: {st['requests_done']} requests in {st['ticks']} ticks, "
         f"mean tick {st['mean_tick_size']:.2f}, peak device bytes {st['peak_device_bytes']}")
    assert st["requests_done"] == 2 * nstreams
    assert st["peak_device_bytes"] <= 64 << 30
    for s in range(nstreams):
        alone = Stream(plan)
        for k in range(2):
            r = reqs[(s, k)]
            assert r.status == DONE
            dev = torch.from_numpy(np.ascontiguousarray(chunks[s][k]).reshape(-1)).to(cuda)
            L = chunks[s][k].shape[0]
            out = torch.empty((plan.ndm, L), dtype=torch.int32, device=cuda)
            n, _ = alone.push(dev, out=out, out_row_stride=L)
            torch.cuda.synchronize()
            assert n == r.n_out
            assert torch.equal(out[:, :n], r.out[:, :n]), (s, k)
            if s != int(np.argmin([len(d) for d in data])):
                r.out = None                      # free as we go
            del dev, out
        alone.close()
    # the shortest stream against the oracle, whole
    s = int(np.argmin([len(d) for d in data]))
    x = data[s]
    t0 = time.perf_counter()
    want = oracle.dedisperse(x, x.shape[0], nchans, 2, plan.delay_table())
    _say(f"stream {s} oracle: {want.shape} in {time.perf_counter() - t0:.1f} s")
    got = np.concatenate([reqs[(s, k)].out[:, :reqs[(s, k)].n_out].cpu().numpy().view(np.uint32)
                          for k in range(2)], axis=1)
    assert np.array_equal(got, want)
