"""GPU parity of time-scrunching (Section 2.1) against the oracle, bit for bit.

Trials beyond the diagonal DM are dedispersed from s-sample sums at s times
the sampling time.  The library runs each factor group through its own
corner turn (which forms the sums) and the tiled kernel in the group's
sample format: nibbles (s = 1, 2-bit), bytes (s = 1, 8-bit), small byte sums
(2-bit, s <= 8) and 16-bit sums (2-bit, s >= 16; 8-bit, s >= 2).  Every row
is compared with the oracle's scrunched transform over its valid length, and
the rest of the row must be left untouched.
"""
import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Plan, synth, tile_configs

pytestmark = pytest.mark.gpu

SENTINEL = 0x5EEDF00D


def _dm_list_every_factor(nchans, dt, f_top, df, per_group, max_factor):
    """DMs on both sides of every power-of-two multiple of the diagonal up to max_factor."""
    diag = oracle.diagonal_dm(nchans, dt, f_top, df)
    dms = [np.linspace(0.0, diag, per_group)]
    k = 1
    while k < max_factor:
        dms.append(np.linspace(diag * k * 1.0001, diag * 2 * k, per_group))
        k *= 2
    return np.concatenate(dms)


def _run(plan, packed, nsamps, dev, width):
    import torch
    inp = torch.from_numpy(np.ascontiguousarray(packed.reshape(-1))).to(dev)
    out = torch.full((plan.ndm, width), SENTINEL, dtype=torch.int32, device=dev)
    plan.execute(inp, nsamps, out=out, out_row_stride=width)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def _check_rows(got, want, nout):
    for d in range(got.shape[0]):
        n = int(nout[d])
        assert np.array_equal(got[d, :n], want[d, :n]), f"row {d} (n={n})"
        assert np.all(got[d, n:] == SENTINEL), f"row {d} written past its length"


def _shape_configs():
    seen, out = set(), []
    for c in tile_configs():
        key = tuple(sorted(c.items()))
        if key not in seen:
            seen.add(key)
            out.append(c)
    return out


@pytest.mark.parametrize("nbits,nchans,nsamps,max_factor", [
    (2, 256, 30011, 64),
    (8, 128, 20005, 16),
])
def test_scrunched_every_shape_bit_exact(native, cuda, nbits, nchans, nsamps, max_factor):
    dt, f_top, df = 64e-6, 1581.8, -400.0 / nchans
    dms = _dm_list_every_factor(nchans, dt, f_top, df, 6, max_factor)
    rng = np.random.default_rng(nchans + nbits)
    codes = (rng.integers(0, 4, size=(nsamps, nchans), dtype=np.uint8) if nbits == 2 else
             np.clip(np.rint(rng.normal(128, 40, size=(nsamps, nchans))), 0, 255).astype(np.uint8))
    codes[::97] = 3 if nbits == 2 else 255          # saturated rows stress the packed lanes
    packed = synth.pack(codes, nbits)
    plan = Plan(nchans, dt, f_top, df, nbits).set_dm_list(dms)
    factors = plan.default_scrunch_factors(max_factor)
    assert set(factors.tolist()) == {1 << k for k in range(max_factor.bit_length())}
    plan.set_scrunching(factors)
    want, nout = oracle.dedisperse_scrunched(packed, nsamps, nchans, nbits, dt, f_top, df,
                                             dms, factors)
    assert np.array_equal(plan.output_lengths(nsamps), nout)
    width = int(nout.max()) + 5
    ran = 0
    for cfg in _shape_configs():
        try:
            plan.set_tile_config(cfg)
        except Exception:
            continue
        got = _run(plan, packed, nsamps, cuda, width)
        _check_rows(got, want, nout)
        ran += 1
    assert ran >= 4


def test_scrunched_with_kill_mask_and_unsorted_dms(native, cuda):
    nbits, nchans, nsamps = 2, 512, 24007
    dt, f_top, df = 64e-6, 1581.8, -400.0 / nchans
    dms = _dm_list_every_factor(nchans, dt, f_top, df, 5, 32)
    dms = dms[np.random.default_rng(1).permutation(len(dms))]
    rng = np.random.default_rng(11)
    codes = rng.integers(0, 4, size=(nsamps, nchans), dtype=np.uint8)
    packed = synth.pack(codes, nbits)
    mask = (rng.random(nchans) < 0.8).astype(np.int32)
    plan = Plan(nchans, dt, f_top, df, nbits).set_dm_list(dms)
    factors = plan.default_scrunch_factors(32)
    plan.set_scrunching(factors)
    plan.set_killmask(mask)
    want, nout = oracle.dedisperse_scrunched(packed, nsamps, nchans, nbits, dt, f_top, df,
                                             dms, factors, mask=mask)
    got = _run(plan, packed, nsamps, cuda, int(nout.max()))
    _check_rows(got, want, nout)
    # switching scrunching off gives the plain masked transform again
    plan.set_scrunching(None)
    table, mx = oracle.delay_table(nchans, dt, f_top, df, dms)
    got = _run(plan, packed, nsamps, cuda, nsamps - mx)
    assert np.array_equal(got, oracle.dedisperse(packed, nsamps, nchans, nbits, table, mask=mask))


def test_survey_beam_scrunched_full_size_sampled(native, cuda):
    """The benchmark's survey beam with the default factors (up to 64): sampled
    outputs of every group against the oracle, and each injected pulse found
    at its trial and at its time in the group's resolution."""
    import torch
    b = synth.survey_beam()
    plan = Plan(b.nchans, b.dt, b.f_top, b.df, b.nbits).set_dm_list(b.dms)
    otab, _ = oracle.delay_table(b.nchans, b.dt, b.f_top, b.df, b.dms)
    b.inject(lambda i: otab[i])
    packed = b.packed()
    factors = plan.default_scrunch_factors(64)
    assert np.array_equal(factors, oracle.scrunch_factors(b.nchans, b.dt, b.f_top, b.df, b.dms, 64))
    plan.set_scrunching(factors)
    nout = plan.output_lengths(b.nsamps)
    inp = torch.from_numpy(packed.reshape(-1)).to(cuda)
    out = torch.empty((plan.ndm, int(nout.max())), dtype=torch.int32, device=cuda)
    plan.execute(inp, b.nsamps, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(5)
    d = rng.integers(0, plan.ndm, size=6000)
    t = (rng.random(6000) * nout[d]).astype(np.int64)
    d = np.concatenate([d, [0, 1023, 1023]])
    t = np.concatenate([t, [0, 0, nout[1023] - 1]])
    want = oracle.dedisperse_scrunched_points(packed, b.nsamps, b.nchans, b.nbits, b.dt, b.f_top,
                                              b.df, b.dms, factors, d, t)
    assert np.array_equal(got[d, t], want)
    for p in b.pulses:
        s = int(factors[p.dm_index])
        tc = p.t0 // s
        lo, hi = max(0, tc - 50), tc + 51
        dl, dh = max(0, p.dm_index - 20), min(plan.ndm, p.dm_index + 21)
        rows = [r for r in range(dl, dh) if factors[r] == s]
        win = np.stack([got[r, lo:min(hi, int(nout[r]))] for r in rows]).astype(np.int64)
        rr, tt = np.unravel_index(int(win.argmax()), win.shape)
        # at resolution s neighbouring trials differ by less than one sample in
        # the lowest channel once s exceeds the per-trial delay step there, so
        # the peak may sit that many trials away
        step = (otab[min(p.dm_index + 1, plan.ndm - 1), -1] - otab[max(p.dm_index - 1, 0), -1]) / 2.0
        tol = 1 + int(np.ceil(s / max(step, 1e-9)))
        assert abs(rows[rr] - p.dm_index) <= tol and abs(tt + lo - tc) <= 1, (p, s, tol)
