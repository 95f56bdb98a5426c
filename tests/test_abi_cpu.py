"""Host-side checks of the C ABI that need no GPU.

The library computes its delay table on the host with its own code; it must
be identical, entry for entry, to the oracle's.  Argument validation happens
before any HIP call, so every error path is testable here.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import Plan, synth, tile_configs
from paper_1201_5380_amd._native import DedispError, SIGNATURES, lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "dedisp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dedisp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(native):
    declared = _declared_functions()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(native, name), name
        assert name in SIGNATURES, name


def test_binding_covers_only_declared_symbols():
    assert sorted(SIGNATURES) == _declared_functions()


WORKLOADS = {
    "tiny": (64, 8, 64e-6, 1500.0, -1.0, 32, 100.0),
    "survey": (1024, 2, 64e-6, 1581.8, -0.390625, 1024, 1000.0),
    "large": (4096, 8, 54.6e-6, 1500.0, -0.09765625, 2048, 2000.0),
    "batch-512": (512, 2, 64e-6, 1581.8, -0.78125, 700, 1234.5),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_delay_table_identical_to_oracle(native, name):
    nchans, nbits, dt, f0, df, ndm, dm_max = WORKLOADS[name]
    dms = synth.dm_list_linear(ndm, dm_max)
    plan = Plan(nchans, dt, f0, df, nbits).set_dm_list(dms)
    want, mx = oracle.delay_table(nchans, dt, f0, df, dms)
    got = plan.delay_table()
    assert np.array_equal(got, want)
    assert plan.max_delay == mx


def test_delay_table_arbitrary_dm_order(native):
    rng = np.random.default_rng(0)
    dms = rng.uniform(0, 900, size=77)
    plan = Plan(256, 64e-6, 1400.0, -0.5, 2).set_dm_list(dms)
    want, mx = oracle.delay_table(256, 64e-6, 1400.0, -0.5, dms)
    assert np.array_equal(plan.delay_table(), want) and plan.max_delay == mx


@pytest.mark.parametrize("args", [
    (0, 64e-6, 1500.0, -1.0, 8), (64, 64e-6, 1500.0, -1.0, 4), (6, 64e-6, 1500.0, -1.0, 2),
    (64, 0.0, 1500.0, -1.0, 8), (64, 64e-6, -5.0, -1.0, 8), (64, 64e-6, 1500.0, 0.0, 8),
    (64, 64e-6, 1500.0, 1.0, 8), (64, 64e-6, 50.0, -1.0, 8), (64, float("nan"), 1500.0, -1.0, 8),
    (64, 64e-6, float("inf"), -1.0, 8)])
def test_plan_create_rejects(native, args):
    with pytest.raises(DedispError) as ei:
        Plan(*args)
    assert ei.value.status == -1


@pytest.mark.parametrize("dms", [[], [1.0, -1.0], [float("nan")], [float("inf")], [1e12]])
def test_set_dm_list_rejects(native, dms):
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    with pytest.raises(DedispError) as ei:
        plan.set_dm_list(dms)
    assert ei.value.status == -1


def test_queries_before_dm_list(native):
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    v = ctypes.c_int()
    assert lib().dedisp_get_max_delay(plan.handle, ctypes.byref(v)) == -2
    assert lib().dedisp_execute(plan.handle, ctypes.c_void_p(16), 1000, ctypes.c_void_p(16), 0,
                                None) == -2


def test_execute_validation_precedes_hip(native):
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8).set_dm_list(synth.dm_list_linear(32, 100.0))
    L = lib()
    p16 = ctypes.c_void_p(1 << 20)
    assert L.dedisp_execute(plan.handle, None, 5000, p16, 0, None) == -1
    assert L.dedisp_execute(plan.handle, p16, 5000, None, 0, None) == -1
    assert L.dedisp_execute(plan.handle, p16, 250, p16, 0, None) == -3      # nsamps <= max_delay
    assert L.dedisp_execute(plan.handle, p16, 5000, p16, 10, None) == -1   # stride < nout
    assert L.dedisp_status_string(-3) == b"DEDISP_ERR_TOO_FEW_SAMPLES"


def test_tile_configs_listed(native):
    cfgs = tile_configs()
    assert any(c["kind"] == 0 for c in cfgs) and any(c["kind"] == 1 for c in cfgs)
    for c in cfgs:
        if c["kind"] == 0:
            assert c["words_per_lane"] % 2 == 1 and c["chunk_chans"] % 4 == 0


def test_huge_dm_gap_falls_back_to_untiled(native):
    plan = Plan(1024, 64e-6, 1581.8, -0.390625, 2).set_dm_list([0.0, 3000.0] * 8)
    assert plan.tile_config()["kind"] == 1
    plan2 = Plan(1024, 64e-6, 1581.8, -0.390625, 2).set_dm_list(synth.dm_list_linear(1024, 1000.0))
    assert plan2.tile_config()["kind"] == 0


def test_set_tile_config_rejects_unknown_shape(native):
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    with pytest.raises(DedispError):
        plan.set_tile_config(dict(kind=0, waves=3, dms_per_wave=4, words_per_lane=5, chunk_chans=32))


def test_stream_and_batch_validation_precedes_hip(native):
    L = lib()
    out = ctypes.c_void_p()
    assert L.dedisp_stream_create(None, ctypes.byref(out)) == -1
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    assert L.dedisp_stream_create(plan.handle, ctypes.byref(out)) == -2      # no DM list
    assert L.dedisp_stream_create(plan.handle, None) == -1
    n = ctypes.c_size_t(7)
    assert L.dedisp_stream_push(None, None, 0, None, 0, ctypes.byref(n), None) == -1
    assert L.dedisp_stream_reset(None) == -1
    assert L.dedisp_stream_reserve(None, 1 << 10) == -1
    from paper_1201_5380_amd._native import BeamStruct
    arr = (BeamStruct * 1)()
    assert L.dedisp_batch_create(arr, 1, None, None, ctypes.byref(out)) == -1   # NULL fields
    arr[0].plan = plan.handle.value
    arr[0].d_in = 1 << 20
    arr[0].d_out = 1 << 20
    arr[0].nsamps = 10
    assert L.dedisp_batch_create(arr, 1, None, None, ctypes.byref(out)) == -2   # no DM list
    plan.set_dm_list([0.0, 50.0])
    assert L.dedisp_batch_create(arr, 1, None, None, ctypes.byref(out)) == -3   # too few samples
    assert L.dedisp_batch_create(arr, 0, None, None, ctypes.byref(out)) == -1


# ---------------------------------------------------------------------------
# time-scrunching: host logic against the oracle (no GPU needed)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(WORKLOADS))
def test_diagonal_dm_and_default_factors_match_oracle(native, name):
    nchans, nbits, dt, f0, df, ndm, dm_max = WORKLOADS[name]
    dms = synth.dm_list_linear(ndm, dm_max)
    plan = Plan(nchans, dt, f0, df, nbits).set_dm_list(dms)
    assert plan.diagonal_dm() == oracle.diagonal_dm(nchans, dt, f0, df)
    for mf in (1, 2, 8, 64):
        assert np.array_equal(plan.default_scrunch_factors(mf),
                              oracle.scrunch_factors(nchans, dt, f0, df, dms, mf))


def test_single_channel_has_no_diagonal(native):
    plan = Plan(4, 64e-6, 1500.0, -1.0, 2).set_dm_list([0.0])
    assert plan.diagonal_dm() > 0
    one = Plan(1, 64e-6, 1500.0, -1.0, 8)
    assert np.isinf(one.diagonal_dm())


def test_output_lengths_match_oracle_groups(native):
    nchans, nbits, dt, f0, df, ndm, dm_max = WORKLOADS["survey"]
    dms = synth.dm_list_linear(ndm, dm_max)
    plan = Plan(nchans, dt, f0, df, nbits).set_dm_list(dms)
    nsamps = 1 << 19
    assert np.all(plan.output_lengths(nsamps) == nsamps - plan.max_delay)
    factors = plan.default_scrunch_factors(64)
    plan.set_scrunching(factors)
    got = plan.output_lengths(nsamps)
    for s in sorted(set(factors.tolist())):
        rows = np.nonzero(factors == s)[0]
        _, mx = oracle.delay_table(nchans, dt * s, f0, df, dms[rows])
        assert np.all(got[rows] == nsamps // s - mx), s
    assert plan.nout(nsamps) == got.max()
    # unsorted lists and arbitrary (valid) factors
    rng = np.random.default_rng(3)
    perm = rng.permutation(ndm)
    plan.set_dm_list(dms[perm])
    f2 = (2 ** rng.integers(0, 7, size=ndm)).astype(np.int32)
    plan.set_scrunching(f2)
    got = plan.output_lengths(nsamps)
    for s in sorted(set(f2.tolist())):
        rows = np.nonzero(f2 == s)[0]
        _, mx = oracle.delay_table(nchans, dt * s, f0, df, dms[perm][rows])
        assert np.all(got[rows] == nsamps // s - mx)


def test_scrunching_validation_precedes_hip(native):
    L = lib()
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    f = np.ones(4, np.int32)
    fp = f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert L.dedisp_set_scrunching(plan.handle, fp) == -2                  # no DM list
    plan.set_dm_list([0.0, 100.0, 200.0, 300.0])
    for bad in ([1, 3, 1, 1], [1, 1, 0, 1], [128, 1, 1, 1], [-2, 1, 1, 1]):
        b = np.array(bad, np.int32)
        assert L.dedisp_set_scrunching(plan.handle, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == -1
    out = np.zeros(4, np.int32)
    assert L.dedisp_default_scrunch_factors(plan.handle, 3, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == -1
    assert L.dedisp_default_scrunch_factors(plan.handle, 128, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == -1
    plan.set_scrunching([1, 2, 4, 8])
    mx8 = oracle.delay_table(64, 64e-6 * 8, 1500.0, -1.0, np.array([300.0]))[1]
    p16 = ctypes.c_void_p(1 << 20)
    n_small = 8 * (mx8 + 1) - 1                                             # group 8 has no output
    assert L.dedisp_execute(plan.handle, p16, n_small, p16, 0, None) == -3
    nout = (ctypes.c_size_t * 4)()
    assert L.dedisp_get_output_lengths(plan.handle, n_small, nout) == -3
    lens = plan.output_lengths(5000)
    assert L.dedisp_execute(plan.handle, p16, 5000, p16, int(lens.max()) - 1, None) == -1  # stride
    # streams and batches refuse a scrunching plan before touching the device
    h = ctypes.c_void_p()
    assert L.dedisp_stream_create(plan.handle, ctypes.byref(h)) == -6
    from paper_1201_5380_amd._native import BeamStruct
    arr = (BeamStruct * 1)()
    arr[0].plan = plan.handle.value
    arr[0].d_in = 1 << 20
    arr[0].d_out = 1 << 20
    arr[0].nsamps = 5000
    assert L.dedisp_batch_create(arr, 1, None, None, ctypes.byref(h)) == -6
    # off again: every row back to full resolution
    plan.set_scrunching(None)
    assert np.all(plan.output_lengths(5000) == 5000 - plan.max_delay)
    plan.set_scrunching([1, 1, 1, 1])
    assert np.all(plan.output_lengths(5000) == 5000 - plan.max_delay)
    assert L.dedisp_stream_create(plan.handle, None) == -1


# ---------------------------------------------------------------------------
# sub-band dedispersion: host logic against the oracle (no GPU needed)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,nsub,ngroup", [("survey", 32, 32), ("survey", 16, 7), ("tiny", 8, 4),
                                              ("large", 64, 16), ("batch-512", 8, 1)])
def test_subband_output_lengths_match_oracle(native, name, nsub, ngroup):
    nchans, nbits, dt, f0, df, ndm, dm_max = WORKLOADS[name]
    dms = synth.dm_list_linear(ndm, dm_max)
    plan = Plan(nchans, dt, f0, df, nbits).set_dm_list(dms)
    plan.set_subband(nsub, ngroup)
    tab, _ = oracle.delay_table(nchans, dt, f0, df, dms)
    tnom, _ = oracle.delay_table(nchans, dt, f0, df, oracle.subband_nominal_dms(dms, ngroup))
    nsamps = 1 << 20
    _, nout = oracle.subband_lengths(nsamps, nchans, nsub, tnom, tab)
    assert np.all(plan.output_lengths(nsamps) == nout)
    assert plan.nout(nsamps) == nout
    plan.set_subband(0, 0)
    assert np.all(plan.output_lengths(nsamps) == nsamps - plan.max_delay)


def test_subband_validation_precedes_hip(native):
    L = lib()
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    assert L.dedisp_set_subband(plan.handle, 8, 4) == -2                    # no DM list
    plan.set_dm_list(synth.dm_list_linear(32, 100.0))
    for nsub, ngroup in ((4, 4), (12, 4), (24, 4), (0, 4), (8, 0), (-8, 2)):
        assert L.dedisp_set_subband(plan.handle, nsub, ngroup) == -1, (nsub, ngroup)
    wide = Plan(512, 64e-6, 1500.0, -0.5, 8).set_dm_list([0.0, 10.0])
    assert L.dedisp_set_subband(wide.handle, 256, 1) == -6                  # 255*256 > 16 bits
    assert L.dedisp_set_subband(plan.handle, 8, 4) == 0
    # exclusive with time-scrunching, both ways
    f = np.array([1] * 16 + [2] * 16, np.int32)
    assert L.dedisp_set_scrunching(plan.handle, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == -6
    p16 = ctypes.c_void_p(1 << 20)
    assert L.dedisp_execute(plan.handle, p16, 100, p16, 0, None) == -3      # too short
    lens = plan.output_lengths(5000)
    assert L.dedisp_execute(plan.handle, p16, 5000, p16, int(lens[0]) - 1, None) == -1
    assert L.dedisp_execute(plan.handle, ctypes.c_void_p((1 << 20) + 2), 5000, p16, 0, None) == -1
    h = ctypes.c_void_p()
    assert L.dedisp_stream_create(plan.handle, ctypes.byref(h)) == -6
    plan.set_subband(0, 0)
    plan.set_scrunching(f)
    assert L.dedisp_set_subband(plan.handle, 8, 4) == -6
    # a new DM list clears both modes
    plan.set_dm_list(synth.dm_list_linear(32, 100.0))
    assert np.all(plan.output_lengths(5000) == 5000 - plan.max_delay)


def test_output_format_validation(native):
    L = lib()
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    nb, sh = ctypes.c_int(), ctypes.c_int()
    assert L.dedisp_get_output_format(plan.handle, ctypes.byref(nb), ctypes.byref(sh)) == 0
    assert (nb.value, sh.value) == (32, 0)
    for bad in ((12, 0), (0, 0), (64, 0), (8, -1), (16, 32)):
        assert L.dedisp_set_output_format(plan.handle, *bad) == -1, bad
    plan.set_output_format(8, 3)
    assert L.dedisp_get_output_format(plan.handle, ctypes.byref(nb), ctypes.byref(sh)) == 0
    assert (nb.value, sh.value) == (8, 3)
    import torch
    assert plan.output_dtype() == torch.uint8


# ---------------------------------------------------------------------------
# piecewise linear tree: host logic against the oracle (no GPU needed)
# ---------------------------------------------------------------------------

def _tree_diag(nchans, nsub, dt, f0, df):
    k = 4.148808e3 / dt
    fb, fa = f0 + nchans * df, f0 + (nchans - nsub) * df
    return (nsub - 0.5) / (k * (1 / fb ** 2 - 1 / f0 ** 2) - k * (1 / fa ** 2 - 1 / f0 ** 2))


@pytest.mark.parametrize("nchans,nbits,nsub,reach", [(1024, 2, 32, 0.99), (512, 2, 8, 0.99),
                                                     (256, 8, 64, 0.99), (128, 8, 128, 0.99),
                                                     (1024, 2, 32, 30.0), (256, 8, 16, 4.5)])
def test_tree_output_lengths_match_oracle(native, nchans, nbits, nsub, reach):
    """Outputs exist for t < nsamps - (P + 1)(nsub - 1) - max dt'', P the largest
    pass (0 up to the diagonal), as the oracle's tables give."""
    dt, f0, df = 64e-6, 1581.8, -400.0 / nchans
    dms = np.linspace(0.0, reach * _tree_diag(nchans, nsub, dt, f0, df), 50)
    plan = Plan(nchans, dt, f0, df, nbits).set_dm_list(dms).set_tree(nsub)
    dp, dd = oracle.tree_dm_tables(nchans, dt, f0, df, nsub, dms)
    npass = int(dp.max()) // nsub + 1
    assert (npass == 1) == (reach < 1)
    nsamps = 1 << 18
    assert np.all(plan.output_lengths(nsamps) == nsamps - npass * (nsub - 1) - dd.max())
    plan.set_tree(0)
    assert np.all(plan.output_lengths(nsamps) == nsamps - plan.max_delay)


@pytest.mark.parametrize("nbits,nsub,maxf", [(2, 32, 64), (2, 16, 8), (8, 16, 4)])
def test_scrunched_tree_output_lengths_match_oracle(native, nbits, nsub, maxf):
    """Scrunching then the tree: row d has nsamps // s - (P_s + 1)(nsub - 1) - max dt''_s
    outputs, from its factor group's tables at s*dt."""
    nchans, dt, f0, df = 1024, 64e-6, 1581.8, -0.390625
    dms = synth.dm_list_linear(300, 1000.0)
    plan = Plan(nchans, dt, f0, df, nbits).set_dm_list(dms)
    factors = plan.default_scrunch_factors(maxf)
    plan.set_scrunching(factors).set_tree(nsub)
    nsamps = 1 << 18
    want = np.zeros(len(dms), dtype=np.int64)
    for s in sorted(set(factors.tolist())):
        idx = np.nonzero(factors == s)[0]
        dp, dd = oracle.tree_dm_tables(nchans, dt * s, f0, df, nsub, dms[idx])
        want[idx] = nsamps // s - (int(dp.max()) // nsub + 1) * (nsub - 1) - int(dd.max())
    assert np.array_equal(plan.output_lengths(nsamps), want)
    assert plan.nout(nsamps) == want.max()


def test_scrunched_tree_validation(native):
    L = lib()
    nchans, dt, f0, df = 1024, 64e-6, 1581.8, -0.390625
    dms = synth.dm_list_linear(64, 1000.0)
    plan = Plan(nchans, dt, f0, df, 8).set_dm_list(dms)
    plan.set_scrunching(plan.default_scrunch_factors(16))
    assert L.dedisp_set_tree(plan.handle, 32) == -6         # 255 * 16 * 32 > 65535
    assert L.dedisp_set_tree(plan.handle, 8) == 0           # 255 * 16 * 8 fits
    f = plan.default_scrunch_factors(16).astype(np.int32)
    assert L.dedisp_set_scrunching(plan.handle, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == -6
    assert L.dedisp_set_scrunching(plan.handle, None) == -6            # the tree sits on the groups
    assert plan.output_lengths(1 << 18).min() > 0
    plan.set_tree(0)
    plan.set_scrunching(None)
    assert np.all(plan.output_lengths(1 << 18) == (1 << 18) - plan.max_delay)


def test_tree_validation_precedes_hip(native):
    L = lib()
    nchans, dt, f0, df = 256, 64e-6, 1581.8, -400.0 / 256
    plan = Plan(nchans, dt, f0, df, 2)
    assert L.dedisp_set_tree(plan.handle, 16) == -2                        # no DM list
    diag = _tree_diag(nchans, 16, dt, f0, df)
    plan.set_dm_list(np.linspace(0, 0.9 * diag, 10))
    for bad in (4, 12, 256, 3, -16):
        assert L.dedisp_set_tree(plan.handle, bad) == -1, bad
    plan.set_dm_list(np.linspace(0, 1.5 * diag, 10))
    assert L.dedisp_set_tree(plan.handle, 16) == 0                          # a second pass
    plan.set_dm_list(np.linspace(0, 0.9 * diag, 10))
    assert L.dedisp_set_tree(plan.handle, 16) == 0
    f = np.array([1] * 5 + [2] * 5, np.int32)
    assert L.dedisp_set_scrunching(plan.handle, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == -6
    assert L.dedisp_set_subband(plan.handle, 16, 2) == -6
    p16 = ctypes.c_void_p(1 << 20)
    assert L.dedisp_execute(plan.handle, p16, 10, p16, 0, None) == -3
    h = ctypes.c_void_p()
    assert L.dedisp_stream_create(plan.handle, ctypes.byref(h)) == -6
    plan.set_tree(0)
    assert np.all(plan.output_lengths(5000) == 5000 - plan.max_delay)


def test_noalloc_execute_validation_precedes_hip(native):
    L = lib()
    plan = Plan(64, 64e-6, 1500.0, -1.0, 8)
    p16 = ctypes.c_void_p(1 << 20)
    assert L.dedisp_execute_noalloc(plan.handle, p16, 5000, p16, 0, None) == -2   # no DM list
    plan.set_dm_list(synth.dm_list_linear(32, 100.0))
    assert L.dedisp_execute_noalloc(None, p16, 5000, p16, 0, None) == -1
    assert L.dedisp_execute_noalloc(plan.handle, None, 5000, p16, 0, None) == -1
    assert L.dedisp_execute_noalloc(plan.handle, p16, 5000, None, 0, None) == -1
    assert L.dedisp_execute_noalloc(plan.handle, p16, 250, p16, 0, None) == -3   # nsamps <= max_delay
    assert L.dedisp_execute_noalloc(plan.handle, p16, 5000, p16, 10, None) == -1  # stride < nout
    plan.set_tree(8)
    assert L.dedisp_execute_noalloc(plan.handle, p16, 5000, p16, 0, None) == -6


def _shape(cfg):
    return tuple(cfg[k] for k in ("waves", "dms_per_wave", "words_per_lane", "chunk_chans", "sample_format"))


def test_segmented_plane_shapes_selected_by_sample_format(native):
    """On a bit-plane plan the tile config's sample_format picks the segmented
    layout (5) or the plain planes (anything else) for the same wave shape;
    host-only (the shape is resolved without the device)."""
    segs = [c for c in tile_configs() if c["kind"] == 0 and c["sample_format"] == 5]
    assert segs
    plan = Plan(1024, 64e-6, 1581.8, -0.390625, 2).set_dm_list(synth.dm_list_linear(1024, 1000.0))
    for c in segs:
        plan.set_tile_config(c)
        assert _shape(plan.tile_config()) == _shape(c)
        plain = dict(c, sample_format=4)
        if any(_shape(p) == _shape(plain) for p in tile_configs()):
            plan.set_tile_config(plain)
            assert plan.tile_config()["sample_format"] == 4
        plan.set_tile_config(dict(c, sample_format=-1))
        assert plan.tile_config()["sample_format"] != 5


def test_segmented_shape_falls_back_when_the_spread_does_not_fit(native):
    """A DM block's delay spread is staged in words on the segmented planes:
    with DM steps of 15 (survey band) it exceeds the 512-word LDS rows, and
    the plan resolves to another tiled shape (host-only)."""
    seg = [c for c in tile_configs() if c["kind"] == 0 and c["sample_format"] == 5][0]
    plan = Plan(1024, 64e-6, 1581.8, -0.390625, 2).set_dm_list(synth.dm_list_linear(64, 1000.0))
    plan.set_tile_config(seg)
    got = plan.tile_config()
    assert got["kind"] == 0 and got["sample_format"] == 4


def test_segmented_shape_not_offered_to_other_formats(native):
    """8-bit and nibble plans have no segmented shapes: such a config is
    rejected as an unknown shape."""
    seg = [c for c in tile_configs() if c["kind"] == 0 and c["sample_format"] == 5][0]
    for nchans, nbits in ((256, 8), (2048, 2)):
        plan = Plan(nchans, 64e-6, 1581.8, -400.0 / nchans, nbits).set_dm_list(synth.dm_list_linear(16, 16.0))
        with pytest.raises(DedispError):
            plan.set_tile_config(seg)
