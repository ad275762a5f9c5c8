"""Relative-binned BNS likelihood on MI355X: Python binding of librbl.so."""
from .rbl import (Event, LogLikeFn, bin_edges, profile_enable, profile_read, profile_read_summary,  # noqa: F401
                  ref_search, strain)
from ._lib import RblError, EXPORTS, LIB_PATH  # noqa: F401
from .serve import Server, clock_ns  # noqa: F401
from .mala import Mala  # noqa: F401
