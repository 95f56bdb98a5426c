"""Seeded synthetic filterbank inputs for the direct dedispersion transform.

This module only makes input data: quantised noise, the packed time-major
byte layout, linear trial-DM lists and pulse trails placed at per-channel
offsets that the caller supplies.  It holds none of the transform's
arithmetic: it never evaluates a dispersion delay.  Both the GPU library and
the CPU oracle consume the same bytes, so a test can give both sides exactly
the same input.

Layout of a packed filterbank (the input format of the whole package):
``nsamps`` rows, one per time sample, each ``nchans * nbits / 8`` bytes,
channel fastest.  For 2-bit data channel ``c`` sits in byte ``c // 4`` at
bits ``[2*(c % 4), 2*(c % 4) + 1]`` (least-significant pair first).  Channel 0
is the top of the band (frequency ``f_top``); channel ``c`` is at
``f_top + c * df`` with ``df < 0``.

Random streams are numpy ``default_rng(seed)`` (PCG64), drawn in row blocks of
``BLOCK_ROWS`` rows so that arbitrarily large inputs can be produced with
bounded host memory; the block size is part of the recipe.  The large beam and
the batched beams draw every block from a generator of its own,
``default_rng([*key, block])``, so their blocks are made on several host
threads at once.
"""
from __future__ import annotations

import hashlib
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

BLOCK_ROWS = 1 << 14

# 2-bit levels: probabilities {0.16, 0.34, 0.34, 0.16} are realised exactly
# by thresholding a uniform integer in [0, 100) at 16, 50 and 84.
_TWO_BIT_THRESHOLDS = (16, 50, 84)


def dm_list_linear(ndm: int, dm_max: float) -> np.ndarray:
    """``ndm`` trial DMs ``i * dm_max / ndm`` for ``i = 0..ndm-1`` (endpoint excluded)."""
    step = float(dm_max) / int(ndm)
    return np.arange(int(ndm), dtype=np.float64) * step


def two_bit_codes(rng: np.random.Generator, nsamps: int, nchans: int) -> np.ndarray:
    """2-bit codes 0..3 with probabilities 0.16/0.34/0.34/0.16, uint8 [nsamps][nchans]."""
    out = np.empty((nsamps, nchans), dtype=np.uint8)
    t1, t2, t3 = _TWO_BIT_THRESHOLDS
    for r0 in range(0, nsamps, BLOCK_ROWS):
        r1 = min(nsamps, r0 + BLOCK_ROWS)
        u = rng.integers(0, 100, size=(r1 - r0, nchans), dtype=np.uint8)
        blk = out[r0:r1]
        np.greater_equal(u, t1, out=blk, casting="unsafe")
        blk += (u >= t2)
        blk += (u >= t3)
    return out


def eight_bit_noise(rng: np.random.Generator, nsamps: int, nchans: int,
                    mean: float, sd: float) -> np.ndarray:
    """Gaussian noise ``rint(mean + sd * z)`` clipped to [0, 255], uint8 [nsamps][nchans]."""
    out = np.empty((nsamps, nchans), dtype=np.uint8)
    for r0 in range(0, nsamps, BLOCK_ROWS):
        r1 = min(nsamps, r0 + BLOCK_ROWS)
        z = rng.standard_normal(size=(r1 - r0, nchans), dtype=np.float32)
        z *= np.float32(sd)
        z += np.float32(mean)
        np.rint(z, out=z)
        np.clip(z, 0.0, 255.0, out=z)
        out[r0:r1] = z.astype(np.uint8)
    return out


def _two_bit_block(rng: np.random.Generator, out: np.ndarray) -> None:
    t1, t2, t3 = _TWO_BIT_THRESHOLDS
    u = rng.integers(0, 100, size=out.shape, dtype=np.uint8)
    np.greater_equal(u, t1, out=out, casting="unsafe")
    out += (u >= t2)
    out += (u >= t3)


def _eight_bit_block(rng: np.random.Generator, out: np.ndarray, mean: float, sd: float) -> None:
    z = rng.standard_normal(size=out.shape, dtype=np.float32)
    z *= np.float32(sd)
    z += np.float32(mean)
    np.rint(z, out=z)
    np.clip(z, 0.0, 255.0, out=z)
    out[...] = z.astype(np.uint8)


def blockwise_codes(key, nsamps: int, nchans: int, nbits: int, mean: float = 128.0,
                    sd: float = 16.0, threads: int | None = None) -> np.ndarray:
    """Codes uint8 [nsamps][nchans]: block b (rows b*BLOCK_ROWS ...) drawn from
    ``default_rng([*key, b])`` -- 2-bit levels as in ``two_bit_codes``, or
    8-bit ``rint(mean + sd * z)`` clipped to [0, 255] -- on several threads."""
    key = [int(k) for k in (key if isinstance(key, (list, tuple)) else [key])]
    out = np.empty((nsamps, nchans), dtype=np.uint8)
    nblk = (nsamps + BLOCK_ROWS - 1) // BLOCK_ROWS

    def one(b):
        rng = np.random.default_rng(key + [b])
        blk = out[b * BLOCK_ROWS:min(nsamps, (b + 1) * BLOCK_ROWS)]
        if nbits == 2:
            _two_bit_block(rng, blk)
        else:
            _eight_bit_block(rng, blk, mean, sd)

    n = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, n)) as ex:
        list(ex.map(one, range(nblk)))
    return out


def pack(codes: np.ndarray, nbits: int) -> np.ndarray:
    """Pack unsigned codes [nsamps][nchans] into the time-major byte layout.

    8-bit: the codes themselves.  2-bit: four channels per byte, channel
    ``4j + k`` at bits ``[2k, 2k+1]`` of byte ``j``.
    """
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    if nbits == 8:
        return codes
    if nbits != 2:
        raise ValueError("nbits must be 2 or 8")
    nsamps, nchans = codes.shape
    if nchans % 4:
        raise ValueError("2-bit data needs nchans % 4 == 0")
    v = codes.reshape(nsamps, nchans // 4, 4)
    packed = v[..., 0] | (v[..., 1] << 2) | (v[..., 2] << 4) | (v[..., 3] << 6)
    return np.ascontiguousarray(packed.astype(np.uint8))


def inject_trail(codes: np.ndarray, t0: int, offsets: np.ndarray, *,
                 add: int | None = None, set_to: int | None = None,
                 max_code: int = 255) -> None:
    """Place a one-sample pulse along ``(t0 + offsets[c], c)`` in place.

    ``offsets`` is one integer per channel (the trail shape is the caller's
    business).  Either ``add`` counts (clipped at ``max_code``) or ``set_to``
    a fixed code.  Samples past the end of the data are skipped.
    """
    nsamps, nchans = codes.shape
    offsets = np.asarray(offsets, dtype=np.int64)
    assert offsets.shape == (nchans,)
    rows = t0 + offsets
    ok = (rows >= 0) & (rows < nsamps)
    ch = np.arange(nchans)[ok]
    rows = rows[ok]
    if set_to is not None:
        codes[rows, ch] = set_to
    else:
        v = codes[rows, ch].astype(np.int64) + int(add)
        codes[rows, ch] = np.minimum(v, max_code).astype(np.uint8)


def sha256(buf: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(buf).view(np.uint8)).hexdigest()


@dataclass
class Pulse:
    dm_index: int
    t0: int


@dataclass
class Beam:
    """One synthetic beam: observing parameters, DM trials and unpacked codes."""
    name: str
    nchans: int
    nbits: int
    dt: float
    f_top: float
    df: float
    dms: np.ndarray
    codes: np.ndarray                   # uint8 [nsamps][nchans], unpacked
    pulses: list = field(default_factory=list)   # pulses still to be injected
    pulse_add: int | None = None
    pulse_set: int | None = None

    @property
    def nsamps(self) -> int:
        return int(self.codes.shape[0])

    def inject(self, delay_row_for_dm_index) -> None:
        """Inject every pending pulse; ``delay_row_for_dm_index(i)`` gives the trail offsets."""
        max_code = 255 if self.nbits == 8 else 3
        for p in self.pulses:
            inject_trail(self.codes, p.t0, delay_row_for_dm_index(p.dm_index),
                         add=self.pulse_add, set_to=self.pulse_set, max_code=max_code)

    def packed(self) -> np.ndarray:
        return pack(self.codes, self.nbits)


def tiny_beam(seed: int = 0, nsamps: int = 4096) -> Beam:
    """8-bit, 64 channels, dt 64 us, f_top 1500 MHz, df -1 MHz, 32 DMs in [0, 100).

    Noise N(128, 16) rounded and clipped; one pulse at DM trial 16 (DM 50),
    t0 = 1000, +40 counts with clipping.
    """
    rng = np.random.default_rng(seed)
    codes = eight_bit_noise(rng, nsamps, 64, 128.0, 16.0)
    return Beam("tiny-8bit-64ch", 64, 8, 64e-6, 1500.0, -1.0, dm_list_linear(32, 100.0),
                codes, [Pulse(16, 1000)], pulse_add=40)


def survey_beam(seed: int = 1, nsamps: int = 1 << 19, nchans: int = 1024,
                ndm: int = 1024, npulses: int = 8, max_delay_hint: int = 20456) -> Beam:
    """2-bit, HTRU-like: f_top 1581.8 MHz, df -0.390625 MHz, dt 64 us, DMs in [0, 1000).

    Pulses: trial index uniform over the DM list, t0 uniform in
    ``[0, nsamps - max_delay_hint)``; the trail is set to code 3.
    """
    rng = np.random.default_rng(seed)
    codes = two_bit_codes(rng, nsamps, nchans)
    prng = np.random.default_rng([seed, 7])
    hi = max(1, nsamps - max_delay_hint)
    pulses = [Pulse(int(prng.integers(0, ndm)), int(prng.integers(0, hi)))
              for _ in range(npulses)]
    df = -400.0 / nchans
    return Beam(f"survey-2bit-{nchans}ch", nchans, 2, 64e-6, 1581.8, df,
                dm_list_linear(ndm, 1000.0), codes, pulses, pulse_set=3)


def large_beam(seed: int = 2, nsamps: int = 1 << 20, nchans: int = 4096, ndm: int = 2048) -> Beam:
    """8-bit, 4096 channels, dt 54.6 us, f_top 1500 MHz, df -0.09765625 MHz, DMs in [0, 2000).

    Noise rint(N(128, 20)) clipped to [0, 255], block b from default_rng([seed, b])."""
    codes = blockwise_codes([seed], nsamps, nchans, 8, 128.0, 20.0)
    return Beam(f"large-8bit-{nchans}ch", nchans, 8, 54.6e-6, 1500.0, -400.0 / nchans,
                dm_list_linear(ndm, 2000.0 * ndm / 2048.0), codes, [])


def batch_beam_params(b: int) -> dict:
    """Shape of beam ``b`` of the batched 13-beam workload (no samples drawn).

    Even ``b``: 1024 channels, 8-bit, N(128, 16).  Odd ``b``: 512 channels,
    2-bit levels.  ``default_rng(b)`` draws Nt in [2^16, 2^19], ndm in
    [256, 1024] and DM_max in [300, 1500]; BW is 400 MHz below 1581.8 MHz.
    """
    rng = np.random.default_rng(b)
    nsamps = int(rng.integers(1 << 16, (1 << 19) + 1))
    ndm = int(rng.integers(256, 1025))
    dm_max = float(rng.uniform(300.0, 1500.0))
    nchans = 1024 if b % 2 == 0 else 512
    nbits = 8 if b % 2 == 0 else 2
    return dict(nsamps=nsamps, ndm=ndm, dm_max=dm_max, nchans=nchans, nbits=nbits,
                dt=64e-6, f_top=1581.8, df=-400.0 / nchans, seed=b)


def batch_beam(b: int, nsamps: int | None = None) -> Beam:
    """Beam ``b`` of the batched workload: block k of its codes from
    default_rng([b, 11, k]); 8-bit noise N(128, 16) or 2-bit levels."""
    p = batch_beam_params(b)
    n = p["nsamps"] if nsamps is None else int(nsamps)
    codes = blockwise_codes([p["seed"], 11], n, p["nchans"], p["nbits"], 128.0, 16.0)
    return Beam(f"batch-{b}", p["nchans"], p["nbits"], p["dt"], p["f_top"], p["df"],
                dm_list_linear(p["ndm"], p["dm_max"]), codes, [])


def stream_chunk_lengths(stream: int, nchunks: int, lo: int = 1 << 14, hi: int = 1 << 18) -> np.ndarray:
    rng = np.random.default_rng([1000 + stream, 3])
    return rng.integers(lo, hi + 1, size=nchunks)


def stream_codes(stream: int, nsamps: int, nchans: int = 1024) -> np.ndarray:
    """2-bit level codes for one stream of the streaming workload (seed 1000 + stream)."""
    return two_bit_codes(np.random.default_rng(1000 + stream), nsamps, nchans)


def poisson_arrivals(n: int, rate_hz: float, nstreams: int, seed: int = 5):
    """Arrival times (s) of ``n`` chunks at aggregate ``rate_hz`` and the stream each belongs to."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    return np.cumsum(gaps), rng.integers(0, nstreams, size=n)
