"""MI355X (gfx950) direct incoherent dedispersion.

The transform of Barsdell et al. (2012), Section 2.1, eq. direct, computed by
hand-written HIP kernels behind the C ABI in include/dedisp.h.  This package
holds the library sources (csrc/), its build script, a ctypes binding and the
seeded synthetic-input generator.  Importing it does not load the library;
the first call does, and fails loudly if it has not been built.
"""
from .api import Batch, Plan, Stream, push_many, tile_configs  # noqa: F401
from ._native import DedispError, lib  # noqa: F401
