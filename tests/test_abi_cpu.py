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
