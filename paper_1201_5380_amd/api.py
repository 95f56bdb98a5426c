"""Python binding of the C ABI in include/dedisp.h.

Thin wrappers that marshal torch tensors (device memory) and streams into the
library's plain-pointer entry points; every step of the transform runs in the
HIP kernels.  Output buffers are torch.int32 tensors holding the library's
uint32 sums (every sum is below 2^31: at most 255 * nchans), or uint8 /
int16 (holding uint16) tensors under a reduced output format.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np

from . import _native
from ._native import TileConfig, check, lib


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t):
    return ctypes.c_void_p(int(t.data_ptr()))


def tile_configs():
    """Every tile shape compiled into the library."""
    out = []
    for i in range(lib().dedisp_tile_config_count()):
        c = TileConfig()
        check(lib().dedisp_tile_config_get(i, ctypes.byref(c)), "dedisp_tile_config_get")
        out.append(c.as_dict())
    return out


class Plan:
    """Observing set-up, DM list and device delay tables (``dedisp_plan``)."""

    def __init__(self, nchans: int, dt: float, f_top: float, df: float, nbits: int):
        self._h = ctypes.c_void_p()
        check(lib().dedisp_plan_create(ctypes.byref(self._h), int(nchans), float(dt),
                                       float(f_top), float(df), int(nbits)),
              "dedisp_plan_create")
        self.nchans, self.nbits = int(nchans), int(nbits)
        self.dt, self.f_top, self.df = float(dt), float(f_top), float(df)
        self.ndm = 0

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().dedisp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def row_bytes(self) -> int:
        return self.nchans * self.nbits // 8

    def set_dm_list(self, dms: Sequence[float]):
        arr = np.ascontiguousarray(dms, dtype=np.float64)
        check(lib().dedisp_set_dm_list(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       int(arr.shape[0])), "dedisp_set_dm_list")
        self.ndm = int(arr.shape[0])
        self._scrunched = False
        self._subband = False
        self._tree = False
        return self

    def set_killmask(self, mask):
        """0/1 per channel (None = all channels on)."""
        if mask is None:
            check(lib().dedisp_set_killmask(self._h, None), "dedisp_set_killmask")
            return self
        m = np.ascontiguousarray(mask, dtype=np.int32)
        if m.shape != (self.nchans,):
            raise ValueError("kill mask needs one entry per channel")
        check(lib().dedisp_set_killmask(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
              "dedisp_set_killmask")
        return self

    # ------------------------------------------------ time-scrunching

    def diagonal_dm(self) -> float:
        v = ctypes.c_double()
        check(lib().dedisp_get_diagonal_dm(self._h, ctypes.byref(v)), "dedisp_get_diagonal_dm")
        return float(v.value)

    def default_scrunch_factors(self, max_factor: int = 64) -> np.ndarray:
        out = np.zeros(self.ndm, dtype=np.int32)
        check(lib().dedisp_default_scrunch_factors(self._h, int(max_factor),
                                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
              "dedisp_default_scrunch_factors")
        return out

    def set_scrunching(self, factors):
        """Per-trial factors (powers of two up to 64); None switches scrunching off."""
        if factors is None:
            check(lib().dedisp_set_scrunching(self._h, None), "dedisp_set_scrunching")
            self._scrunched = False
            return self
        f = np.ascontiguousarray(factors, dtype=np.int32)
        if f.shape != (self.ndm,):
            raise ValueError("one scrunch factor per trial DM")
        check(lib().dedisp_set_scrunching(self._h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
              "dedisp_set_scrunching")
        self._scrunched = bool((f > 1).any())
        return self

    def set_output_format(self, nbits: int = 32, shift: int = 0):
        """Outputs as min(sum >> shift, 2^nbits - 1) in uint8 / uint16 / uint32."""
        check(lib().dedisp_set_output_format(self._h, int(nbits), int(shift)),
              "dedisp_set_output_format")
        self.out_nbits, self.out_shift = int(nbits), int(shift)
        return self

    def output_dtype(self):
        """torch dtype of output buffers (uint16 outputs are held as int16)."""
        import torch
        return {8: torch.uint8, 16: torch.int16, 32: torch.int32}[getattr(self, "out_nbits", 32)]

    def set_tree(self, nsub: int):
        """Piecewise linear tree over sub-bands of nsub channels (0 = off)."""
        check(lib().dedisp_set_tree(self._h, int(nsub)), "dedisp_set_tree")
        self._tree = bool(nsub)
        return self

    def set_subband(self, nsub: int, ngroup: int):
        """Sub-band dedispersion with nsub channels per sub-band and ngroup
        trials per nominal DM; (0, 0) switches it off."""
        check(lib().dedisp_set_subband(self._h, int(nsub), int(ngroup)), "dedisp_set_subband")
        self._subband = bool(nsub)
        return self

    def output_lengths(self, nsamps: int) -> np.ndarray:
        out = np.zeros(self.ndm, dtype=np.uintp)
        check(lib().dedisp_get_output_lengths(self._h, int(nsamps),
                                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_size_t))),
              "dedisp_get_output_lengths")
        return out.astype(np.int64)

    @property
    def max_delay(self) -> int:
        v = ctypes.c_int()
        check(lib().dedisp_get_max_delay(self._h, ctypes.byref(v)), "dedisp_get_max_delay")
        return int(v.value)

    def delay_table(self) -> np.ndarray:
        out = np.zeros((self.ndm, self.nchans), dtype=np.int32)
        check(lib().dedisp_get_delay_table(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
              "dedisp_get_delay_table")
        return out

    def set_tile_config(self, cfg: dict):
        c = TileConfig(**cfg)
        check(lib().dedisp_set_tile_config(self._h, ctypes.byref(c)), "dedisp_set_tile_config")

    def tile_config(self) -> dict:
        c = TileConfig()
        check(lib().dedisp_get_tile_config(self._h, ctypes.byref(c)), "dedisp_get_tile_config")
        return c.as_dict()

    def nout(self, nsamps: int) -> int:
        """Longest output row for nsamps input rows."""
        if getattr(self, "_scrunched", False) or getattr(self, "_subband", False) or \
                getattr(self, "_tree", False):
            return int(self.output_lengths(nsamps).max())
        return int(nsamps) - self.max_delay

    def alloc_output(self, nsamps: int, device="cuda"):
        import torch
        return torch.empty((self.ndm, self.nout(nsamps)), dtype=self.output_dtype(), device=device)

    def _check_input(self, inp, nsamps):
        if nsamps is None:
            nsamps = inp.numel() // self.row_bytes
        if inp.numel() < nsamps * self.row_bytes:
            raise ValueError("input holds fewer than nsamps rows")
        if not inp.is_contiguous():
            raise ValueError("input must be contiguous")
        return int(nsamps)

    def execute(self, inp, nsamps: int | None = None, out=None, out_row_stride: int = 0,
                stream=None):
        """Dedisperse ``nsamps`` rows of device tensor ``inp``; returns the output tensor."""
        nsamps = self._check_input(inp, nsamps)
        if out is None:
            out = self.alloc_output(nsamps, inp.device)
            out_row_stride = 0
        check(lib().dedisp_execute(self._h, _ptr(inp), nsamps, _ptr(out), int(out_row_stride),
                                   _stream_handle(stream)), "dedisp_execute")
        return out

    def execute_noalloc(self, inp, out, nsamps: int | None = None, out_row_stride: int = 0,
                        stream=None):
        """The direct transform into caller-given ``out`` with no device
        allocation (``dedisp_execute_noalloc``): the plan's device tables must
        already be built (``execute`` or ``tune`` ran after the last change)."""
        nsamps = self._check_input(inp, nsamps)
        check(lib().dedisp_execute_noalloc(self._h, _ptr(inp), nsamps, _ptr(out), int(out_row_stride),
                                           _stream_handle(stream)), "dedisp_execute_noalloc")
        return out

    def tune(self, inp, out, nsamps: int | None = None, out_row_stride: int = 0,
             cache_path: str | None = None, stream=None) -> float:
        nsamps = self._check_input(inp, nsamps)
        ms = ctypes.c_float()
        check(lib().dedisp_tune(self._h, _ptr(inp), nsamps, _ptr(out), int(out_row_stride),
                                _stream_handle(stream),
                                cache_path.encode() if cache_path else None, ctypes.byref(ms)),
              "dedisp_tune")
        return float(ms.value)


class Stream:
    """An unbounded input stream with device-resident history (``dedisp_stream``)."""

    def __init__(self, plan: Plan):
        self.plan = plan
        self._h = ctypes.c_void_p()
        check(lib().dedisp_stream_create(plan.handle, ctypes.byref(self._h)), "dedisp_stream_create")

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().dedisp_stream_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_chunk: int):
        """Size the stream's scratch for pushes of up to max_chunk rows with the
        plan's current tile shape (synchronous; call after tuning the plan)."""
        check(lib().dedisp_stream_reserve(self._h, int(max_chunk)), "dedisp_stream_reserve")

    def push(self, chunk, out=None, out_row_stride: int = 0, nsamps: int | None = None,
             stream=None):
        """Push a device chunk; returns (n_out, out) where out[:, :n_out] is new output."""
        if nsamps is None:
            nsamps = chunk.numel() // self.plan.row_bytes
        n_out = ctypes.c_size_t()
        outp = _ptr(out) if out is not None else ctypes.c_void_p()
        check(lib().dedisp_stream_push(self._h, _ptr(chunk), int(nsamps), outp,
                                       int(out_row_stride), ctypes.byref(n_out),
                                       _stream_handle(stream)), "dedisp_stream_push")
        return int(n_out.value), out

    def device_bytes(self) -> int:
        """Device memory the stream holds between pushes: history + scratch."""
        n = ctypes.c_size_t()
        check(lib().dedisp_stream_get_device_bytes(self._h, ctypes.byref(n)),
              "dedisp_stream_get_device_bytes")
        return int(n.value)

    def state(self):
        h = ctypes.c_size_t()
        t = ctypes.c_uint64()
        check(lib().dedisp_stream_get_state(self._h, ctypes.byref(h), ctypes.byref(t)),
              "dedisp_stream_get_state")
        return int(h.value), int(t.value)

    def get_history(self) -> np.ndarray:
        rows, _ = self.state()
        buf = np.zeros(max(1, rows * self.plan.row_bytes), dtype=np.uint8)
        n = ctypes.c_size_t()
        check(lib().dedisp_stream_get_history(self._h, buf.ctypes.data_as(ctypes.c_void_p),
                                              ctypes.byref(n)), "dedisp_stream_get_history")
        return buf[: int(n.value) * self.plan.row_bytes].reshape(int(n.value), self.plan.row_bytes)

    def set_history(self, rows: np.ndarray, total_rows: int):
        rows = np.ascontiguousarray(rows, dtype=np.uint8)
        n = rows.shape[0] if rows.ndim == 2 else rows.size // self.plan.row_bytes
        check(lib().dedisp_stream_set_history(self._h, rows.ctypes.data_as(ctypes.c_void_p), int(n),
                                              int(total_rows)), "dedisp_stream_set_history")

    def reset(self):
        check(lib().dedisp_stream_reset(self._h), "dedisp_stream_reset")


def push_many(streams: Sequence[Stream], chunks, outs, out_row_strides=None, stream=None):
    """Push one chunk into each of several streams with a single launch; returns n_outs."""
    n = len(streams)
    hs = (ctypes.c_void_p * n)(*[s.handle.value for s in streams])
    cs = (ctypes.c_void_p * n)(*[int(c.data_ptr()) for c in chunks])
    ns = (ctypes.c_size_t * n)(*[c.numel() // s.plan.row_bytes for c, s in zip(chunks, streams)])
    os_ = (ctypes.c_void_p * n)(*[int(o.data_ptr()) if o is not None else 0 for o in outs])
    st = (ctypes.c_size_t * n)(*(out_row_strides or [0] * n))
    nouts = (ctypes.c_size_t * n)()
    check(lib().dedisp_stream_push_many(hs, cs, ns, os_, st, nouts, n, _stream_handle(stream)),
          "dedisp_stream_push_many")
    return [int(v) for v in nouts]


class Batch:
    """A fixed set of beams run as one multi-beam, graph-captured launch (``dedisp_batch``)."""

    def __init__(self, beams, tune_cache_path: str | None = None, stream=None):
        """``beams``: sequence of (plan, input tensor, nsamps, output tensor, out_row_stride)."""
        n = len(beams)
        arr = (_native.BeamStruct * n)()
        self._keep = []
        for i, (plan, inp, nsamps, out, stride) in enumerate(beams):
            arr[i].plan = plan.handle.value
            arr[i].d_in = int(inp.data_ptr())
            arr[i].nsamps = int(nsamps)
            arr[i].d_out = int(out.data_ptr())
            arr[i].out_row_stride = int(stride)
            self._keep.append((plan, inp, out))
        self._h = ctypes.c_void_p()
        check(lib().dedisp_batch_create(arr, n, tune_cache_path.encode() if tune_cache_path else None,
                                        _stream_handle(stream), ctypes.byref(self._h)),
              "dedisp_batch_create")

    def execute(self, stream=None, graph: bool = True):
        fn = lib().dedisp_batch_execute if graph else lib().dedisp_batch_execute_direct
        check(fn(self._h, _stream_handle(stream)), "dedisp_batch_execute")

    def close(self):
        if self._h:
            lib().dedisp_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
