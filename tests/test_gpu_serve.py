"""The streaming service on the GPU: every request's output is bit-identical
whether its stream runs alone (one push per chunk, nothing else on the
device) or in the mix (continuous batching with other streams' chunks in the
same multi-beam launches); one stream is also checked against the oracle."""
import time

import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Plan, Stream, synth
from paper_1201_5380_amd.serve import DONE, GpuExecutor, Server

pytestmark = pytest.mark.gpu


def test_alone_equals_in_the_mix(native, cuda):
    import torch
    nstreams = 6
    dms = synth.dm_list_linear(64, 1000.0)
    specs = [(1024, 2), (1024, 2), (512, 2), (1024, 8), (256, 8), (1024, 2)]
    plans = [Plan(nc, 64e-6, 1581.8, -400.0 / nc, nb).set_dm_list(dms[: 32 + 8 * (i % 3)])
             for i, (nc, nb) in enumerate(specs)]
    rng = np.random.default_rng(2024)
    chunks = [[] for _ in range(nstreams)]
    order = []
    for k in range(36):
        sid = int(rng.integers(0, nstreams))
        p = plans[sid]
        L = int(rng.integers(1 << 10, 1 << 14))
        if p.nbits == 2:
            codes = synth.two_bit_codes(rng, L, p.nchans)
        else:
            codes = synth.eight_bit_noise(rng, L, p.nchans, 128.0, 16.0)
        chunks[sid].append(synth.pack(codes, p.nbits).reshape(L, p.row_bytes))
        order.append((sid, len(chunks[sid]) - 1))

    ex = GpuExecutor(plans, max_chunk=1 << 14)
    ex.tune(1 << 14)            # tuned shapes, possibly of either multi-beam class
    srv = Server(ex, nstreams, budget_bytes=8 << 30, max_tick=4, max_inflight_ticks=3).start()
    reqs = {}
    for i, (sid, j) in enumerate(order):
        reqs[(sid, j)] = srv.submit(sid, chunks[sid][j])
        if i % 5 == 0:
            time.sleep(0.002)
    srv.drain(timeout=120)
    srv.stop()
    st = srv.stats()
    assert st["requests_done"] == len(order)
    assert st["mean_tick_size"] > 1.0, "no batching happened"

    for sid, p in enumerate(plans):
        alone = Stream(p)
        for j, data in enumerate(chunks[sid]):
            r = reqs[(sid, j)]
            assert r.status == DONE
            dev = torch.from_numpy(data.reshape(-1)).to(cuda)
            out = torch.empty((p.ndm, data.shape[0]), dtype=torch.int32, device=cuda)
            n, _ = alone.push(dev, out=out, out_row_stride=data.shape[0])
            torch.cuda.synchronize()
            assert n == r.n_out
            if n:
                assert torch.equal(out[:, :n], r.out[:, :n]), (sid, j)
    # stream 2 (512 channels) against the oracle, whole
    p = plans[2]
    x = np.concatenate(chunks[2])
    want = oracle.dedisperse(x, x.shape[0], p.nchans, p.nbits, p.delay_table())
    got = np.concatenate([reqs[(2, j)].out[:, : reqs[(2, j)].n_out].cpu().numpy().view(np.uint32)
                          for j in range(len(chunks[2]))], axis=1)
    assert np.array_equal(got, want)
