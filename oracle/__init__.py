"""CPU oracle for the direct dedispersion transform (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library; see
``dedisp_oracle.c`` for the definitions it implements and the readings of the
paper it fixes.  Functions take and return numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_partial_delay.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, _f64p]
    lib.oracle_delay_table.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _f64p, ctypes.c_int, _i32p, _i32p]
    lib.oracle_dedisperse.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      _i32p, ctypes.c_int, ctypes.c_int32, _u32p,
                                      ctypes.c_int64, ctypes.c_int, _i32p]
    lib.oracle_dedisperse_points.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                             _i32p, ctypes.c_int, ctypes.c_int32, _i64p, _i64p,
                                             ctypes.c_int64, _u32p, ctypes.c_int, _i32p]
    lib.oracle_diagonal_dm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _f64p]
    lib.oracle_scrunch_factor.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_scrunch.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, _u32p]
    lib.oracle_dedisperse_values.argtypes = [_u32p, ctypes.c_int64, ctypes.c_int, _i32p,
                                             ctypes.c_int, ctypes.c_int32, _u32p,
                                             ctypes.c_int64, ctypes.c_int, _i32p]
    lib.oracle_dedisperse_scrunched_points.argtypes = [
        _u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int,
        ctypes.c_int32, _i64p, _i64p, ctypes.c_int64, _u32p, ctypes.c_int, _i32p]
    lib.oracle_subband_lengths.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _i32p,
                                           ctypes.c_int, _i32p, ctypes.c_int, _i64p, _i64p]
    lib.oracle_subband_step1.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_int64, _u32p,
                                         ctypes.c_int, _i32p]
    lib.oracle_subband_step2.argtypes = [_u32p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int64, _u32p, ctypes.c_int64,
                                         ctypes.c_int]
    lib.oracle_reduce_output.argtypes = [_u32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p]
    lib.oracle_tree.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                _u32p, _i32p]
    lib.oracle_tree_combine_tables.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int, _f64p, ctypes.c_int,
                                               _i32p, _i32p]
    lib.oracle_tree_combine.argtypes = [_u32p, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _i32p,
                                        _i32p, ctypes.c_int, ctypes.c_int64, _u32p]
    lib.oracle_tree_imposed.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, _u32p, _i32p]
    lib.oracle_tree_dm_tables.argtypes = lib.oracle_tree_combine_tables.argtypes
    lib.oracle_tree_imposed_values.argtypes = [_u32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, _u32p, _i32p]
    lib.oracle_tree_combine_passes.argtypes = [_u32p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                               ctypes.c_int, _i32p, _i32p, ctypes.c_int, ctypes.c_int64,
                                               _u32p]
    for f in ("oracle_tree", "oracle_tree_combine_tables", "oracle_tree_combine",
              "oracle_tree_imposed", "oracle_tree_dm_tables", "oracle_tree_combine_passes",
              "oracle_tree_imposed_values",
              "oracle_reduce_output", "oracle_subband_lengths", "oracle_subband_step1", "oracle_subband_step2",
              "oracle_dedisperse_scrunched_points", "oracle_partial_delay", "oracle_delay_table", "oracle_dedisperse",
              "oracle_dedisperse_points", "oracle_max_threads", "oracle_diagonal_dm",
              "oracle_scrunch_factor", "oracle_scrunch", "oracle_dedisperse_values"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def partial_delay(nchans, dt, f_top, df) -> np.ndarray:
    """Delta T(nu) in samples per unit DM, float64 [nchans]."""
    out = np.zeros(nchans, dtype=np.float64)
    _check(_load().oracle_partial_delay(nchans, dt, f_top, df, _ptr(out, _f64p)), "partial_delay")
    return out


def delay_table(nchans, dt, f_top, df, dms):
    """(int32 [ndm][nchans] delay table, max_delay)."""
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    ndm = int(dms.shape[0])
    table = np.zeros((max(ndm, 1), nchans), dtype=np.int32)
    mx = ctypes.c_int32(0)
    _check(_load().oracle_delay_table(nchans, dt, f_top, df, _ptr(dms, _f64p), ndm,
                                      _ptr(table, _i32p), ctypes.byref(mx)), "delay_table")
    return table, int(mx.value)


def _mask_arg(mask, nchans):
    if mask is None:
        return None, None
    m = np.ascontiguousarray(mask, dtype=np.int32)
    if m.shape != (nchans,):
        raise OracleError("mask must have one entry per channel")
    return m, _ptr(m, _i32p)


def dedisperse(packed, nsamps, nchans, nbits, table, max_delay=None, nthreads=0, mask=None):
    """Full transform: uint32 [ndm][nsamps - max_delay] (optional 0/1 channel kill mask)."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    table = np.ascontiguousarray(table, dtype=np.int32)
    ndm = int(table.shape[0])
    if max_delay is None:
        max_delay = int(table.max())
    nout = int(nsamps) - int(max_delay)
    if nout <= 0:
        raise OracleError("too few samples")
    if packed.size < int(nsamps) * nchans * nbits // 8:
        raise OracleError("input too short")
    out = np.zeros((ndm, nout), dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    _check(_load().oracle_dedisperse(_ptr(packed, _u8p), int(nsamps), nchans, nbits,
                                     _ptr(table, _i32p), ndm, int(max_delay),
                                     _ptr(out, _u32p), nout, int(nthreads), mp), "dedisperse")
    return out


def dedisperse_points(packed, nsamps, nchans, nbits, table, d_idx, t_idx, max_delay=None,
                      nthreads=0, mask=None):
    """The transform at the listed (d, t) points only: uint32 [npts]."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    table = np.ascontiguousarray(table, dtype=np.int32)
    d_idx = np.ascontiguousarray(d_idx, dtype=np.int64)
    t_idx = np.ascontiguousarray(t_idx, dtype=np.int64)
    if max_delay is None:
        max_delay = int(table.max())
    if packed.size < int(nsamps) * nchans * nbits // 8:
        raise OracleError("input too short")
    out = np.zeros(d_idx.shape[0], dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    _check(_load().oracle_dedisperse_points(_ptr(packed, _u8p), int(nsamps), nchans, nbits,
                                            _ptr(table, _i32p), int(table.shape[0]),
                                            int(max_delay), _ptr(d_idx, _i64p),
                                            _ptr(t_idx, _i64p), int(d_idx.shape[0]),
                                            _ptr(out, _u32p), int(nthreads), mp),
           "dedisperse_points")
    return out


# ---------------------------------------------------------------- time-scrunching


def diagonal_dm(nchans, dt, f_top, df) -> float:
    """The band's diagonal DM: one sample of delay between its last two channels."""
    v = ctypes.c_double()
    _check(_load().oracle_diagonal_dm(nchans, dt, f_top, df, ctypes.byref(v)), "diagonal_dm")
    return float(v.value)


def scrunch_factor(dm, dm_diag, max_factor) -> int:
    return int(_load().oracle_scrunch_factor(float(dm), float(dm_diag), int(max_factor)))


def scrunch(packed, nsamps, nchans, nbits, s):
    """Scrunched samples: uint32 [nsamps // s][nchans], each the sum of s samples."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    if packed.size < int(nsamps) * nchans * nbits // 8:
        raise OracleError("input too short")
    out = np.zeros((max(int(nsamps) // int(s), 1), nchans), dtype=np.uint32)
    _check(_load().oracle_scrunch(_ptr(packed, _u8p), int(nsamps), nchans, nbits, int(s),
                                  _ptr(out, _u32p)), "scrunch")
    return out[: int(nsamps) // int(s)]


def dedisperse_values(x, table, max_delay=None, nthreads=0, mask=None):
    """Direct transform of unpacked time-major values x [n][nchans]: uint32 [ndm][n - max_delay]."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    n, nchans = x.shape
    table = np.ascontiguousarray(table, dtype=np.int32)
    ndm = int(table.shape[0])
    if max_delay is None:
        max_delay = int(table.max())
    nout = n - int(max_delay)
    if nout <= 0:
        raise OracleError("too few samples")
    out = np.zeros((ndm, nout), dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    _check(_load().oracle_dedisperse_values(_ptr(x, _u32p), n, nchans, _ptr(table, _i32p), ndm,
                                            int(max_delay), _ptr(out, _u32p), nout,
                                            int(nthreads), mp), "dedisperse_values")
    return out


def scrunch_factors(nchans, dt, f_top, df, dms, max_factor):
    """Per-trial scrunch factors for a DM list."""
    dd = diagonal_dm(nchans, dt, f_top, df)
    return np.array([scrunch_factor(dm, dd, max_factor) for dm in dms], dtype=np.int32)


def dedisperse_scrunched(packed, nsamps, nchans, nbits, dt, f_top, df, dms, factors,
                         nthreads=0, mask=None):
    """The time-scrunched transform: each factor group dedispersed at its own
    resolution.  Returns (out, nout) with out uint32 [ndm][max nout] (row d
    valid up to nout[d], zero after) and nout int64 [ndm]."""
    dms = np.asarray(dms, dtype=np.float64)
    factors = np.asarray(factors, dtype=np.int64)
    groups = {}
    for s in sorted(set(int(v) for v in factors)):
        rows = np.nonzero(factors == s)[0]
        table, mx = delay_table(nchans, dt * s, f_top, df, dms[rows])
        n_s = int(nsamps) // s
        if n_s - mx <= 0:
            raise OracleError("too few samples for scrunch group %d" % s)
        x = scrunch(packed, nsamps, nchans, nbits, s)
        groups[s] = (rows, dedisperse_values(x, table, mx, nthreads, mask))
    width = max(g[1].shape[1] for g in groups.values())
    out = np.zeros((len(dms), width), dtype=np.uint32)
    nout = np.zeros(len(dms), dtype=np.int64)
    for s, (rows, o) in groups.items():
        out[rows, : o.shape[1]] = o
        nout[rows] = o.shape[1]
    return out, nout


def dedisperse_scrunched_points(packed, nsamps, nchans, nbits, dt, f_top, df, dms, factors,
                                d_idx, t_idx, nthreads=0, mask=None):
    """The time-scrunched transform at the listed (d, t') points only: uint32 [npts]."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    if packed.size < int(nsamps) * nchans * nbits // 8:
        raise OracleError("input too short")
    dms = np.asarray(dms, dtype=np.float64)
    factors = np.asarray(factors, dtype=np.int64)
    d_idx = np.asarray(d_idx, dtype=np.int64)
    t_idx = np.asarray(t_idx, dtype=np.int64)
    out = np.zeros(d_idx.shape[0], dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    for s in sorted(set(int(v) for v in factors)):
        rows = np.nonzero(factors == s)[0]
        table, mx = delay_table(nchans, dt * s, f_top, df, dms[rows])
        local = np.full(len(dms), -1, dtype=np.int64)
        local[rows] = np.arange(len(rows))
        sel = np.nonzero(factors[d_idx] == s)[0]
        if sel.size == 0:
            continue
        dl = np.ascontiguousarray(local[d_idx[sel]])
        tl = np.ascontiguousarray(t_idx[sel])
        o = np.zeros(sel.size, dtype=np.uint32)
        _check(_load().oracle_dedisperse_scrunched_points(
            _ptr(packed, _u8p), int(nsamps), nchans, nbits, s, _ptr(table, _i32p),
            int(table.shape[0]), int(mx), _ptr(dl, _i64p), _ptr(tl, _i64p), int(sel.size),
            _ptr(o, _u32p), int(nthreads), mp), "dedisperse_scrunched_points")
        out[sel] = o
    return out


# ---------------------------------------------------------------- sub-band dedispersion


def subband_nominal_dms(dms, ngroup):
    """The nominal DM of every group of ngroup consecutive trials: its first trial."""
    dms = np.asarray(dms, dtype=np.float64)
    return dms[::int(ngroup)].copy()


def subband_lengths(nsamps, nchans, nsub, tab_nom, tab):
    tab_nom = np.ascontiguousarray(tab_nom, dtype=np.int32)
    tab = np.ascontiguousarray(tab, dtype=np.int32)
    l1, no = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().oracle_subband_lengths(int(nsamps), nchans, int(nsub), _ptr(tab_nom, _i32p),
                                          int(tab_nom.shape[0]), _ptr(tab, _i32p), int(tab.shape[0]),
                                          ctypes.byref(l1), ctypes.byref(no)), "subband_lengths")
    return int(l1.value), int(no.value)


def dedisperse_subband(packed, nsamps, nchans, nbits, dt, f_top, df, dms, nsub, ngroup,
                       nthreads=0, mask=None, return_intermediate=False):
    """Two-step sub-band transform: uint32 [ndm][nout] (and S [nsb][nnom][len1])."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    if packed.size < int(nsamps) * nchans * nbits // 8:
        raise OracleError("input too short")
    dms = np.asarray(dms, dtype=np.float64)
    tab, _ = delay_table(nchans, dt, f_top, df, dms)
    nom = subband_nominal_dms(dms, ngroup)
    tab_nom, _ = delay_table(nchans, dt, f_top, df, nom)
    len1, nout = subband_lengths(nsamps, nchans, nsub, tab_nom, tab)
    nsb = nchans // nsub
    S = np.zeros((nsb, len(nom), len1), dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    _check(_load().oracle_subband_step1(_ptr(packed, _u8p), int(nsamps), nchans, nbits, int(nsub),
                                        _ptr(tab_nom, _i32p), len(nom), len1, _ptr(S, _u32p),
                                        int(nthreads), mp), "subband_step1")
    out = np.zeros((len(dms), nout), dtype=np.uint32)
    _check(_load().oracle_subband_step2(_ptr(S, _u32p), nsb, len(nom), len1, nchans, int(nsub),
                                        _ptr(tab, _i32p), len(dms), int(ngroup), nout,
                                        _ptr(out, _u32p), nout, int(nthreads)), "subband_step2")
    return (out, S) if return_intermediate else out


def subband_effective_delays(nchans, dt, f_top, df, dms, nsub, ngroup):
    """E[d][c] = dt(d, n*nsub) + dt(m, c) - dt(m, n*nsub): the delay each input sample of the
    two-step method is taken at (n = c // nsub, m = d // ngroup)."""
    dms = np.asarray(dms, dtype=np.float64)
    tab, _ = delay_table(nchans, dt, f_top, df, dms)
    tab_nom, _ = delay_table(nchans, dt, f_top, df, subband_nominal_dms(dms, ngroup))
    first = (np.arange(nchans) // nsub) * nsub
    m = np.arange(len(dms)) // ngroup
    return (tab[:, first] + tab_nom[m] - tab_nom[m][:, first]).astype(np.int64)


# ---------------------------------------------------------------- output bit depth


def reduce_output(sums, nbits, shift=0):
    """min(sums >> shift, 2^nbits - 1) as uint8 / uint16 / uint32 (same shape)."""
    sums = np.ascontiguousarray(sums, dtype=np.uint32)
    dtype = {8: np.uint8, 16: np.uint16, 32: np.uint32}.get(int(nbits))
    if dtype is None:
        raise OracleError("nbits must be 8, 16 or 32")
    out = np.zeros(sums.shape, dtype=dtype)
    _check(_load().oracle_reduce_output(_ptr(sums, _u32p), int(sums.size), int(nbits), int(shift),
                                        out.ctypes.data_as(ctypes.c_void_p)), "reduce_output")
    return out


# ---------------------------------------------------------------- tree dedispersion


def tree(packed, nsamps, nchans, nbits, k, mask=None):
    """k steps of the tree algorithm: uint32 [nchans][nsamps - (2^k - 1)]; row b*2^k + d'
    holds the block of 2^k channels starting at b*2^k at tree DM d'."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    if packed.size < int(nsamps) * nchans * nbits // 8:
        raise OracleError("input too short")
    n_out = int(nsamps) - ((1 << int(k)) - 1)
    if n_out <= 0:
        raise OracleError("too few samples")
    out = np.zeros((nchans, n_out), dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    _check(_load().oracle_tree(_ptr(packed, _u8p), int(nsamps), nchans, nbits, int(k),
                               _ptr(out, _u32p), mp), "tree")
    return out


def tree_imposed(packed, nsamps, nchans, nbits, k, slope, mask=None):
    """Stage 1 with an imposed delay of `slope` samples per channel within every block
    of 2^k channels (Section 3, computing larger DMs): uint32
    [nchans][nsamps - (slope + 1)(2^k - 1)]."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    if packed.size < int(nsamps) * nchans * nbits // 8:
        raise OracleError("input too short")
    n_out = int(nsamps) - (int(slope) + 1) * ((1 << int(k)) - 1)
    if n_out <= 0:
        raise OracleError("too few samples")
    out = np.zeros((nchans, n_out), dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    _check(_load().oracle_tree_imposed(_ptr(packed, _u8p), int(nsamps), nchans, nbits, int(k),
                                       int(slope), _ptr(out, _u32p), mp), "tree_imposed")
    return out


def tree_imposed_values(x, k, slope, mask=None):
    """tree_imposed over unpacked time-major values x [nsamps][nchans] (e.g. scrunched
    samples): uint32 [nchans][nsamps - (slope + 1)(2^k - 1)]."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    nsamps, nchans = x.shape
    n_out = nsamps - (int(slope) + 1) * ((1 << int(k)) - 1)
    if n_out <= 0:
        raise OracleError("too few samples")
    out = np.zeros((nchans, n_out), dtype=np.uint32)
    m, mp = _mask_arg(mask, nchans)
    _check(_load().oracle_tree_imposed_values(_ptr(x, _u32p), nsamps, nchans, int(k), int(slope),
                                              _ptr(out, _u32p), mp), "tree_imposed_values")
    return out


def tree_dm_tables(nchans, dt, f_top, df, nsub, dms):
    """(d'_n(d), dt''_n(d)) as int32 [ndm][nchans / nsub] each, d' unrestricted."""
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    nsb = nchans // nsub
    dp = np.zeros((len(dms), nsb), dtype=np.int32)
    dd = np.zeros((len(dms), nsb), dtype=np.int32)
    _check(_load().oracle_tree_dm_tables(nchans, dt, f_top, df, int(nsub), _ptr(dms, _f64p),
                                         len(dms), _ptr(dp, _i32p), _ptr(dd, _i32p)),
           "tree_dm_tables")
    return dp, dd


def tree_combine_tables(nchans, dt, f_top, df, nsub, dms):
    """(d'_n(d), dt''_n(d)) as int32 [ndm][nchans / nsub] each."""
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    nsb = nchans // nsub
    dp = np.zeros((len(dms), nsb), dtype=np.int32)
    dd = np.zeros((len(dms), nsb), dtype=np.int32)
    _check(_load().oracle_tree_combine_tables(nchans, dt, f_top, df, int(nsub), _ptr(dms, _f64p),
                                              len(dms), _ptr(dp, _i32p), _ptr(dd, _i32p)),
           "tree_combine_tables")
    return dp, dd


def _piecewise_tree(stage1, nsamps, nchans, dt, f_top, df, dms, nsub):
    """Stage 2 over the passes stage1(p) -> [nchans][>= len1] returns."""
    k = int(nsub).bit_length() - 1
    if (1 << k) != int(nsub):
        raise OracleError("nsub must be a power of two")
    dp, dd = tree_dm_tables(nchans, dt, f_top, df, nsub, dms)
    npass = int(dp.max()) // int(nsub) + 1
    len1 = int(nsamps) - npass * (int(nsub) - 1)
    nout = len1 - int(dd.max())
    if len1 <= 0 or nout <= 0:
        raise OracleError("too few samples")
    out = np.zeros((len(dms), nout), dtype=np.uint32)
    if npass == 1:
        S = np.ascontiguousarray(stage1(0)[:, :len1])
        _check(_load().oracle_tree_combine(_ptr(S, _u32p), nchans, len1, int(nsub), _ptr(dp, _i32p),
                                           _ptr(dd, _i32p), len(dms), nout, _ptr(out, _u32p)),
               "tree_combine")
        return out
    S = np.zeros((npass, nchans, len1), dtype=np.uint32)
    for p in range(npass):
        S[p] = stage1(p)[:, :len1]
    _check(_load().oracle_tree_combine_passes(_ptr(S, _u32p), npass, nchans, len1, int(nsub),
                                              _ptr(dp, _i32p), _ptr(dd, _i32p), len(dms), nout,
                                              _ptr(out, _u32p)), "tree_combine_passes")
    return out


def dedisperse_piecewise_tree(packed, nsamps, nchans, nbits, dt, f_top, df, dms, nsub, mask=None):
    """Piecewise linear tree (Section 3): stage 1 = log2(nsub) tree steps, stage 2 = the
    sub-band combination.  Trials past the piecewise diagonal use further passes with an
    imposed delay (pass p: p samples per channel within each sub-band), sub-band n of
    trial d taking pass d'_n(d) // nsub.  uint32 [ndm][nout], nout = nsamps -
    (P + 1)(nsub - 1) - max dt'' with P the largest pass."""
    k = int(nsub).bit_length() - 1
    if int(nsub) != 1 << k:
        raise OracleError("nsub must be a power of two")
    return _piecewise_tree(lambda p: (tree(packed, nsamps, nchans, nbits, k, mask=mask) if p == 0 else
                                      tree_imposed(packed, nsamps, nchans, nbits, k, p, mask=mask)),
                           nsamps, nchans, dt, f_top, df, dms, nsub)


def dedisperse_piecewise_tree_scrunched(packed, nsamps, nchans, nbits, dt, f_top, df, dms, nsub,
                                       factors, mask=None):
    """The tree on time-scrunched data (Section 3, computing larger DMs with
    time-scrunching): the trials of scrunch factor s go through the piecewise tree
    (with its passes) over the s-sample sums (scrunch) at resolution s*dt.  Returns a
    list of uint32 rows, trial d's of length nsamps // s - (P_s + 1)(nsub - 1) -
    max dt''_s over its group."""
    dms = np.asarray(dms, dtype=np.float64)
    factors = np.asarray(factors)
    k = int(nsub).bit_length() - 1
    rows = [None] * len(dms)
    for s in sorted(set(int(f) for f in factors)):
        idx = np.nonzero(factors == s)[0]
        x = scrunch(packed, nsamps, nchans, nbits, s)
        n = x.shape[0]
        got = _piecewise_tree(lambda p: tree_imposed_values(x, k, p, mask=mask), n, nchans, dt * s,
                              f_top, df, dms[idx], nsub)
        for j, d in enumerate(idx):
            rows[d] = got[j]
    return rows
